"""Iterative refinement and mixed precision (the float64 residual of the exact
operator with the factorization as inner solver).

Bar after refinement (north-star): max-column relative residual <= 1e-8 and
||x - x_ref|| / ||x_ref|| <= 1e-8, with x_ref from the oracle: the dense LU on
the small case, and the oracle's RS at tolerance 1e-13 (residual ~1e-11) on
the 12288-node workload.  The mixed path's parity with the oracle is only
through these solutions and residuals (its float32 factors have no oracle
counterpart)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import stokes
from oracle.rs import RSFactorization, RSParams
from workloads import boundary_data, exterior_forces_for_geometry, workload_circle10_8holes, workload_small


def _solver(g, **kw):
    import torch

    assert torch.cuda.is_available()
    from paper_2001_11619_amd import RSSolver

    return RSSolver.from_geometry(g, **kw)


def _rel(a, b):
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-7), (1, 1e-5), (2, 1e-6), (2, 1e-5)])
def test_refined_matches_dense_small(precision, tol):
    g = workload_small(seed=11, n_outer=256, n_holes=2, nodes_per_hole=128, radius=3.0)
    f = boundary_data(g, exterior_forces_for_geometry(g, 3, seed=5))
    xd = stokes.dense_solve(g, f)
    s = _solver(g, leaf_size=32, tol=tol, precision=precision, refine_max=30, refine_tol=1e-12).factor()
    x, res = s.solve(f, residual=True)
    assert np.all(res <= 1e-12)
    assert np.all(_rel(x, xd) < 1e-10)
    assert 1 <= s.stats()["refine_iters"] <= 30


def test_mixed_circle10_8holes():
    g = workload_circle10_8holes()
    f = boundary_data(g, exterior_forces_for_geometry(g, 4, seed=2))
    ref = RSFactorization(g, RSParams(tol=1e-13)).factor().solve(f)
    s = _solver(g, tol=1e-7, precision=1, refine_max=20, refine_tol=1e-8).factor()
    x, res = s.solve(f, residual=True)
    assert np.all(res <= 1e-8)
    assert np.all(_rel(x, ref) <= 1e-8)
    it_mixed = s.stats()["refine_iters"]
    p = _solver(g, tol=1e-10, precision=0, refine_max=20, refine_tol=1e-8).factor()
    xp, resp = p.solve(f, residual=True)
    assert np.all(resp <= 1e-8)
    assert np.all(_rel(xp, ref) <= 1e-8)
    assert p.stats()["refine_iters"] <= it_mixed


def test_noconv_reported():
    from paper_2001_11619_amd import RSError

    g = workload_small(seed=11, n_outer=256, n_holes=2, nodes_per_hole=128, radius=3.0)
    f = boundary_data(g, exterior_forces_for_geometry(g, 1, seed=5))
    s = _solver(g, leaf_size=32, tol=1e-4, precision=1, refine_max=1, refine_tol=1e-14).factor()
    with pytest.raises(RSError) as e:
        s.solve(f)
    assert e.value.name == "RS_ERR_NOCONV"


def test_graph_refinement_matches_eager():
    """Refinement replayed as a captured HIP graph (device-side convergence
    test) gives bitwise the iterates of the iterations launched one by one:
    over several replays with other device work and waits between them, after
    a new factorization (recapture) and for another number of columns."""
    from workloads import workload_small

    g = workload_small(seed=11, n_outer=256, n_holes=2, nodes_per_hole=128, radius=3.0)
    kw = dict(leaf_size=32, tol=1e-5, precision=1, refine_max=20, refine_tol=1e-10)
    se = _solver(g, solve_graph=0, **kw).factor()
    sg = _solver(g, solve_graph=1, **kw).factor()
    f = boundary_data(g, exterior_forces_for_geometry(g, 3, seed=2))
    xe, re = se.solve(f, residual=True)
    ie = se.stats()["refine_iters"]
    assert ie >= 3                      # several graph launches (two iterations each)
    rng = np.random.Generator(np.random.PCG64(1))
    for rep in range(4):
        xg, rg = sg.solve(f, residual=True)
        assert np.array_equal(xg, xe) and np.array_equal(rg, re)
        assert sg.stats()["refine_iters"] == ie
        sg.apply(rng.standard_normal((g.n_system, 2)))     # eager work between replays
    sg.factor()
    assert np.array_equal(sg.solve(f), xe)
    f1 = f[:, :1]
    assert np.array_equal(sg.solve(f1), se.solve(f1))


def test_solve_batch_matches_single():
    """The interleaved batched solve returns each context's own solution."""
    import torch

    from paper_2001_11619_amd import factor_batch, solve_batch
    from workloads import random_holes_geometry, single_ellipse

    geoms = [random_holes_geometry(41 + i, 5.0, 512, [128] * (i + 1)) for i in range(3)]
    geoms.append(single_ellipse(600, 1.0, 0.5))
    kw = dict(leaf_size=32, tol=1e-7, precision=1, refine_max=20, refine_tol=1e-9)
    batch = [_solver(gg, **kw) for gg in geoms]
    factor_batch(batch)
    fs = [boundary_data(gg, exterior_forces_for_geometry(gg, 3, seed=3)) for gg in geoms]
    f_dev = [torch.tensor(np.ascontiguousarray(ff.T), dtype=torch.float64, device="cuda") for ff in fs]
    x_dev = [torch.empty((3, gg.n_system), dtype=torch.float64, device="cuda") for gg in geoms]
    torch.cuda.synchronize()
    solve_batch(batch, f_dev, x_dev)
    for gg, s, ff, xd in zip(geoms, batch, fs, x_dev):
        alone = _solver(gg, **kw).factor()
        assert np.array_equal(xd.cpu().numpy().T, alone.solve(ff))


@pytest.mark.parametrize("thr", [2.0, 1e-1, 1e-2, 1e-3, 0.0])
def test_mixed_boxes_float_and_double(thr):
    """Mixed precision where the rcond threshold splits the boxes between float
    copies and float64 factors (thr > 1 keeps every box in float64, 0 puts every
    box in float): the border stage and the refined solve handle both kinds in
    one factorization.  With every box in float64 the solve is the float64 one
    bitwise."""
    g = workload_small(seed=11, n_outer=256, n_holes=2, nodes_per_hole=128, radius=3.0)
    f = boundary_data(g, exterior_forces_for_geometry(g, 3, seed=5))
    xd = stokes.dense_solve(g, f)
    s = _solver(g, leaf_size=32, tol=1e-7, precision=1, mixed_rcond_min=thr, refine_max=30,
                refine_tol=1e-12).factor()
    x, res = s.solve(f, residual=True)
    assert np.all(res <= 1e-12)
    assert np.all(_rel(x, xd) < 1e-10)
    if thr > 1.0:
        p = _solver(g, leaf_size=32, tol=1e-7, precision=0, refine_max=30, refine_tol=1e-12).factor()
        assert np.array_equal(p.solve(f), x)


def test_graph_skips_converged_iterations():
    """With two refinement iterations per graph launch, an odd number of needed
    corrections leaves a converged iteration in the last launch: it changes
    nothing (x, the reported iterations and residual equal those of the eager
    loop, which stops at convergence)."""
    g = workload_small(seed=11, n_outer=256, n_holes=2, nodes_per_hole=128, radius=3.0)
    f = boundary_data(g, exterior_forces_for_geometry(g, 2, seed=5))
    runs = {}
    for graph in (0, 1):
        s = _solver(g, leaf_size=32, tol=1e-6, precision=1, refine_max=20, refine_tol=1e-10,
                    solve_graph=graph).factor()
        x, res = s.solve(f, residual=True)
        runs[graph] = (x, res, s.stats()["refine_iters"])
    assert np.array_equal(runs[0][0], runs[1][0])
    assert runs[0][2] == runs[1][2]
    assert np.all(runs[1][1] <= 1e-10)


def test_graph_recaptured_after_buffers_grow():
    """A captured refinement graph holds device addresses.  An operator apply
    with more columns than the captured solve grows (reallocates) the apply's
    scratch; the next refined solve with the captured column count must
    capture again, and equal the iterations launched one by one bitwise."""
    g = workload_small(seed=11, n_outer=256, n_holes=2, nodes_per_hole=128, radius=3.0)
    kw = dict(leaf_size=32, tol=1e-6, precision=1, refine_max=20, refine_tol=1e-10)
    sg = _solver(g, solve_graph=1, **kw).factor()
    se = _solver(g, solve_graph=0, **kw).factor()
    f = boundary_data(g, exterior_forces_for_geometry(g, 1, seed=2))
    xe = se.solve(f)
    assert np.array_equal(sg.solve(f), xe)
    rng = np.random.Generator(np.random.PCG64(3))
    for ncols in (4, 9):
        sg.apply(rng.standard_normal((g.n_system, ncols)))
        assert np.array_equal(sg.solve(f), xe)
    # a direct solve with more columns grows the solve's vectors too
    sg2 = _solver(g, solve_graph=1, **kw).factor()
    assert np.array_equal(sg2.solve(f), xe)
    f7 = boundary_data(g, exterior_forces_for_geometry(g, 7, seed=4))
    sg2.solve(f7)
    assert np.array_equal(sg2.solve(f), xe)


def test_float32_bulk_is_float32():
    """The float32 bulk form (precision 2) really computes its entries and
    Schur complements in float32: its direct solution differs from the
    float64-factorization form's at float32 level (same tolerance, same
    tree), while both refine to the dense solution."""
    g = workload_small(seed=11, n_outer=256, n_holes=2, nodes_per_hole=128, radius=3.0)
    f = boundary_data(g, exterior_forces_for_geometry(g, 2, seed=5))
    xd = stokes.dense_solve(g, f)
    x = {}
    for prec in (1, 2):
        s = _solver(g, leaf_size=32, tol=1e-6, precision=prec).factor()
        x[prec] = s.solve(f)
    d = np.abs(x[2] - x[1]).max() / np.abs(x[1]).max()
    assert 1e-9 < d < 1e-3, d
    for prec in (1, 2):
        assert np.abs(x[prec] - xd).max() / np.abs(xd).max() < 1e-3
