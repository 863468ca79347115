"""MI355X (gfx950) recursive skeletonization for the 2D Stokes double layer.

The solver is the C-ABI library `librs_mi355x.so` (declared in include/rs.h);
this package only marshals arguments to it.  Importing the package does not
load the library; the first `RSSolver` does, and raises if it was not built.
"""

from .binding import (RSSolver, RSError, library_path, load_library, exported_symbols,  # noqa: F401
                      factor_batch, solve_batch, update_moved_nodes_batch, close_all, reset_tuning)
