"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/rs.h declares, and rejects invalid input before
touching the device."""

import os
import re

import numpy as np
import pytest

from paper_2001_11619_amd import RSSolver, RSError, load_library
from paper_2001_11619_amd.binding import default_params
from workloads import workload_small

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = load_library()
    names = _declared()
    assert "rs_build_tree" in names and "rs_update_moved_nodes" in names
    for n in names:
        assert hasattr(lib, n), n


def test_default_params():
    p = default_params()
    assert p.lambda_ == -0.5 and p.tol == 1e-10 and p.leaf_size == 64
    assert p.n_proxy == 64 and p.proxy_ratio == 1.5 and p.rcond_min == 1e-12
    assert p.precision == 0 and p.refine_tol == 1e-8 and p.refine_max == 0
    assert p.has_root == 0 and p.solve_graph == 1 and p.mixed_rcond_min == 1e-4 and p.apply_shape == -1
    assert p.refine_update == 1 and p.kernel == 0


def _geom():
    return workload_small(seed=11, n_outer=64, n_holes=1, nodes_per_hole=32, radius=3.0)


@pytest.mark.parametrize("bad", ["nan_xy", "normal_len", "weight", "curve_id", "tol", "empty_hole",
                                 "mixed_rcond", "refine_update", "kernel"])
def test_invalid_input_rejected(bad):
    g = _geom()
    xy, nrm, w, kap, cid = g.xy.copy(), g.normal.copy(), g.weight.copy(), g.curvature.copy(), g.curve_id.copy()
    kw = {}
    if bad == "nan_xy":
        xy[3, 0] = np.nan
    elif bad == "normal_len":
        nrm[5] *= 1.001
    elif bad == "weight":
        w[7] = -1.0
    elif bad == "curve_id":
        cid[0] = 5
    elif bad == "tol":
        kw["tol"] = -1.0
    elif bad == "mixed_rcond":
        kw["mixed_rcond_min"] = float("nan")
    elif bad == "refine_update":
        kw["refine_update"] = 2
    elif bad == "kernel":
        kw["kernel"] = 2
    elif bad == "empty_hole":
        cid[cid == 1] = 0
        cid[0] = 2           # hole 1 has no nodes, hole 2 has one
    with pytest.raises(RSError) as e:
        RSSolver(xy, nrm, w, kap, cid, **kw)
    assert e.value.name == "RS_ERR_ARG"


def test_fixed_root_must_contain_nodes():
    g = _geom()
    with pytest.raises(RSError) as e:
        RSSolver.from_geometry(g, root=(0.0, 0.0, 1.0))
    assert e.value.name == "RS_ERR_OUT_OF_ROOT"


def test_laplace_kernel_rejects_holes():
    """The Laplace Neumann kernel has no augmentation: a direct call with holes
    is refused before anything reaches the device."""
    import ctypes

    from paper_2001_11619_amd.binding import _dptr, _iptr, load_library

    g = _geom()
    lib = load_library()
    p = default_params()
    p.kernel = 1
    h = ctypes.c_void_p()
    cid = np.ascontiguousarray(g.curve_id, dtype=np.int32)
    st = lib.rs_build_tree(ctypes.byref(p), g.n_nodes, _dptr(np.ascontiguousarray(g.xy)),
                           _dptr(np.ascontiguousarray(g.normal)), _dptr(g.weight), _dptr(g.curvature),
                           _iptr(cid), int(cid.max()), None, ctypes.byref(h))
    assert st == 1 and not h.value          # RS_ERR_ARG, no context
