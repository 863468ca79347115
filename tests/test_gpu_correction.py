"""The float32 image of the operator that refinement uses for the image A dx of
a correction (rs_params.refine_update), and the certified residual it feeds.

* The image against the oracle's exact operator, element by element: every
  node's two rows differ from the exact A x by at most the bound the kernel
  reports for that node and column (a wrong sign, a dropped term or a
  mis-mapped MFMA lane breaks this by orders of magnitude), and the bound is
  not vacuous (error / bound and bound / |A x| both stay small).  Ragged sizes
  (targets and sources not multiples of the tiles, 5 and 20 columns: a partial
  and two column blocks), and sampled rows at the 131072-node size in the
  benchmark's 16-column shape.
* Refinement with updated residuals converges to the same solution as with
  exact residuals, and the residual it reports bounds the exact one (computed
  after the solve with the exact float64 apply).
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import stokes
from workloads import (boundary_data, exterior_forces_for_geometry, workload_circle10_8holes,
                       workload_circle40_64holes, workload_small)


def _solver(g, **kw):
    import torch

    assert torch.cuda.is_available()
    from paper_2001_11619_amd import RSSolver

    return RSSolver.from_geometry(g, **kw)


def _check_within_bound(y32, bound, yo, n2):
    err = np.abs(y32[:n2] - yo[:n2])
    err_node = np.maximum(err[0::2], err[1::2])                  # (N, ncols)
    assert np.all(err_node <= bound), float(np.max(err_node / bound))
    scale = np.abs(yo[:n2]).max(axis=0)
    assert np.all(bound.max(axis=0) <= 1e-3 * scale)             # the bound is informative
    assert np.abs(y32[n2:] - yo[n2:]).max(initial=0.0) <= 1e-12 * max(np.abs(yo[n2:]).max(initial=0.0), 1.0)
    return float(np.median(err_node / bound))


@pytest.mark.parametrize("ncols", [5, 20])
def test_f32_image_within_bound(ncols):
    g = workload_small(seed=17, n_outer=250, n_holes=3, nodes_per_hole=70, radius=3.0)
    assert g.n_nodes % 64 != 0 and g.n_nodes > 128
    rng = np.random.Generator(np.random.PCG64(ncols))
    X = rng.standard_normal((g.n_system, ncols))
    s = _solver(g, leaf_size=32)
    y32, bound = s.apply_f32(X)
    yo = stokes.apply_system(g, X)
    med = _check_within_bound(y32, bound, yo, g.n_dofs)
    print("float32 image, %d columns: median error / bound %.2e" % (ncols, med), flush=True)
    assert med < 0.1


def _oracle_rows(g, nodes, X):
    """Rows 2i, 2i+1 (i in nodes) of the augmented operator times X, from the
    oracle's entries: (lam I + D + N) over every column, plus H lambda."""
    n2 = g.n_dofs
    rdofs = np.stack([2 * nodes, 2 * nodes + 1], axis=1).reshape(-1)
    A = stokes.operator_entries(g, rdofs, np.arange(n2), -0.5)
    Y = A @ X[:n2]
    for h in range(g.n_holes):
        c = g.hole_xy[h]
        S = stokes.stokeslet_blocks(g.xy[nodes], c[None, :], np.ones(1))[:, 0]    # (m, 2, 2)
        R = stokes.rotlet_columns(g.xy[nodes], c)                                   # (m, 2)
        Hh = np.concatenate([S.reshape(-1, 2),
                             R.reshape(-1, 1)], axis=1)                             # (2m, 3)
        Y += Hh @ X[n2 + 3 * h:n2 + 3 * h + 3]
    return Y


def test_f32_image_within_bound_full_size_sampled():
    g = workload_circle40_64holes()
    rng = np.random.Generator(np.random.PCG64(7))
    X = rng.standard_normal((g.n_system, 16))
    s = _solver(g)
    y32, bound = s.apply_f32(X)
    nodes = np.unique(np.concatenate([[0, 1, g.n_nodes - 1, 16383, 16384],
                                      rng.choice(g.n_nodes, 27, replace=False)]))
    yo = _oracle_rows(g, nodes, X)
    rows = np.stack([2 * nodes, 2 * nodes + 1], axis=1).reshape(-1)
    err = np.abs(y32[rows] - yo)
    err_node = np.maximum(err[0::2], err[1::2])
    assert np.all(err_node <= bound[nodes]), float(np.max(err_node / bound[nodes]))
    rel = float(np.max(err / np.abs(yo).max(axis=0)))
    print("float32 image at 131072 nodes, %d sampled nodes: max relative error %.2e, "
          "median error / bound %.2e" % (nodes.size, rel, float(np.median(err_node / bound[nodes]))), flush=True)
    assert rel < 1e-5
    # the Psi^T rows are float64
    ye = s.apply(X)
    n2 = g.n_dofs
    assert np.abs(y32[n2:] - ye[n2:]).max() <= 1e-12 * np.abs(ye[n2:]).max()


def test_f32_image_rejects_close_nodes():
    from paper_2001_11619_amd import RSError

    g = workload_small(seed=11, n_outer=64, n_holes=1, nodes_per_hole=32, radius=3.0)
    xy = g.xy.copy()
    t = np.array([-g.normal[0, 1], g.normal[0, 0]])
    xy[1] = xy[0] + 1e-9 * t                      # a node 1e-9 from its neighbour
    from paper_2001_11619_amd import RSSolver

    s = RSSolver(xy, g.normal, g.weight, g.curvature, g.curve_id, g.hole_xy, leaf_size=16)
    with pytest.raises(RSError) as e:
        s.apply_f32(np.ones(g.n_system))
    assert e.value.name == "RS_ERR_ARG"


@pytest.mark.parametrize("precision,tol", [(1, 1e-7), (1, 1e-6), (2, 1e-6)])
def test_updated_refinement_certified(precision, tol):
    g = workload_circle10_8holes()
    f = boundary_data(g, exterior_forces_for_geometry(g, 4, seed=2))
    rhs = np.vstack([f, np.zeros((3 * g.n_holes, f.shape[1]))])
    out = {}
    for upd in (1, 0):
        s = _solver(g, tol=tol, precision=precision, refine_max=20, refine_tol=1e-8, refine_update=upd).factor()
        x, res = s.solve(f, residual=True)
        r = rhs - s.apply(x)                                        # exact float64 residual
        true = np.linalg.norm(r, axis=0) / np.linalg.norm(f, axis=0)
        out[upd] = (x, res, true, s.stats()["refine_iters"])
        assert np.all(res <= 1e-8)
        assert np.all(true <= res * (1 + 1e-6))                     # the reported residual bounds the exact one
    x1, res1, true1, it1 = out[1]
    x0, res0, true0, it0 = out[0]
    print("precision %d tol %g: updated residuals %d iterations (reported %.2e, exact %.2e), exact residuals %d"
          % (precision, tol, it1, res1.max(), true1.max(), it0), flush=True)
    assert it1 <= it0 + 1
    rel = np.linalg.norm(x1 - x0, axis=0) / np.linalg.norm(x0, axis=0)
    assert np.all(rel <= 1e-7)
