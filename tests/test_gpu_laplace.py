"""The Laplace Neumann formulation of Section 4.4.1 on the device
(rs_params.kernel = 1) against the oracle's dense operator.

* The exact apply, element by element (the dense operator's rows; the
  uncoupled second unknown of every node gives lambda x).
* The direct solve at ID tolerance 1e-10 and the refined solve against the
  oracle's dense LU solve, element by element, at a ragged size spanning
  several leaves, with the eq. (neumanndata) flux and random data.
* Evaluation of S mu and its x-derivative at interior points.
* The 16384-node workload of the section (2/3 of the nodes on the outer
  starfish, 1/6 per hole): sampled operator rows, and an exact harmonic
  field reproduced up to one constant.
* A circle, where every entry of -D is the same, so that blocks of rows of the
  ID matrices are exactly rank-deficient (regression: their row reduction
  once produced NaN from reflectors of subnormal rounding residue).
* Moving the holes along their path (theta_1, theta_2): an update, alone and
  as a batch of related geometries, equals a fresh factorization bitwise.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import laplace as L
from workloads import starfish_geometry

ROOT = (0.0, 0.0, 2.6)     # a square holding every starfish of the workload


def _solver(g, **kw):
    import torch

    assert torch.cuda.is_available()
    from paper_2001_11619_amd import RSSolver

    kw.setdefault("root", ROOT)
    return RSSolver.from_geometry(g, kernel=1, **kw)


def _embed(f):
    from paper_2001_11619_amd import RSSolver

    return RSSolver.embed_scalar(f)


def _harmonic(g):
    srcs = np.array([[1.6, 0.3], [-0.2, 1.7], g.hole_xy[0], g.hole_xy[1]])
    q = np.array([0.7, -0.4, 1.1, -0.5])
    a = np.array([0.3, -0.8])

    def grad(x):
        r = x[:, None, :] - srcs[None]
        return (q[None, :, None] * r / (r * r).sum(-1)[..., None]).sum(1) + a

    def u(x):
        r = x[:, None, :] - srcs[None]
        return (q[None] * 0.5 * np.log((r * r).sum(-1))).sum(1) + x @ a

    return u, grad


TARGETS = np.array([[0.0, 0.3], [0.2, -0.4], [-0.6, 0.1], [0.35, 0.45], [0.0, 0.0]])


@pytest.mark.parametrize("ncols", [1, 5, 20])
def test_apply_matches_oracle(ncols):
    g = starfish_geometry(1003)
    rng = np.random.Generator(np.random.PCG64(ncols))
    X = rng.standard_normal((2 * g.n_nodes, ncols))
    y = _solver(g, leaf_size=32).apply(X).reshape(2 * g.n_nodes, ncols)
    A = L.operator_matrix(g)
    ye = A @ X[0::2]
    scale = (np.abs(A) @ np.abs(X[0::2])).max(axis=0)
    assert np.all(np.abs(y[0::2] - ye).max(axis=0) <= 1e-14 * scale)
    assert np.array_equal(y[1::2], -0.5 * X[1::2])


@pytest.mark.parametrize("n,leaf", [(1003, 32), (2400, 64)])
def test_direct_solve_matches_oracle(n, leaf):
    g = starfish_geometry(n)
    rng = np.random.Generator(np.random.PCG64(n))
    F = np.stack([L.neumann_data(g.curve_id), rng.standard_normal(g.n_nodes)], axis=1)
    s = _solver(g, leaf_size=leaf, tol=1e-10).factor()
    x, res = s.solve(_embed(F), residual=True)
    mu = x[0::2]
    assert np.abs(x[1::2]).max() <= 1e-14 * np.abs(mu).max()        # the uncoupled unknowns stay 0
    # the uncoupled unknowns: x = b / lambda there, the density unaffected
    Fe = _embed(F)
    Fe[1::2] = rng.standard_normal(F.shape)
    x2 = s.solve(Fe)
    assert np.array_equal(x2[0::2], mu) and np.array_equal(x2[1::2], Fe[1::2] / -0.5)
    mo = L.solve(g, F)
    err = np.abs(mu - mo).max(axis=0) / np.abs(mo).max(axis=0)
    print("Laplace direct solve N=%d: element-wise error %s, residual %s, ranks at the leaves %d"
          % (n, err, res, int(s.stats()["max_rank"])), flush=True)
    assert np.all(err < 1e-8), err
    assert np.all(res < 1e-8), res


def test_refined_mixed_solve_matches_oracle():
    g = starfish_geometry(2400)
    f = L.neumann_data(g.curve_id)
    s = _solver(g, leaf_size=32, tol=1e-6, precision=1, refine_max=10, refine_tol=1e-11).factor()
    x, res = s.solve(_embed(f), residual=True)
    mo = L.solve(g, f)
    err = np.abs(x[0::2] - mo).max() / np.abs(mo).max()
    print("Laplace refined mixed solve: %d iterations, residual %.2e, element-wise error %.2e"
          % (s.stats()["refine_iters"], res[0], err), flush=True)
    assert res[0] <= 1e-11 and err < 1e-9


def test_refined_float32_bulk_solve_matches_oracle():
    """The float32 bulk form (precision 2: float32 entries from box-local
    offsets, FP32 matrix-core Schur complements) refined to 1e-11."""
    g = starfish_geometry(2400)
    f = L.neumann_data(g.curve_id)
    s = _solver(g, leaf_size=32, tol=1e-6, precision=2, refine_max=12, refine_tol=1e-11).factor()
    x, res = s.solve(_embed(f), residual=True)
    mo = L.solve(g, f)
    err = np.abs(x[0::2] - mo).max() / np.abs(mo).max()
    print("Laplace refined float32 bulk solve: %d iterations, residual %.2e, element-wise error %.2e"
          % (s.stats()["refine_iters"], res[0], err), flush=True)
    assert res[0] <= 1e-11 and err < 1e-9


def test_circle_rank_deficient_blocks():
    from workloads import Geometry, starfish_nodes

    n = 512
    xy, nrm, w, kap = starfish_nodes(n, 1.0, 0.0, 5, 0.0, 0.0, 0.0, False)
    g = Geometry(xy=xy, normal=nrm, weight=w, curvature=kap, curve_id=np.zeros(n, np.int32),
                 hole_xy=np.zeros((0, 2)), curves=[])
    f = np.random.Generator(np.random.PCG64(1)).standard_normal(n)
    s = _solver(g, leaf_size=32, root=(0.0, 0.0, 2.2)).factor()
    x = s.solve(_embed(f))
    mo = L.solve(g, f)
    assert np.abs(x[0::2] - mo).max() < 1e-9 * np.abs(mo).max()


def test_evaluate_matches_oracle():
    g = starfish_geometry(1003)
    rng = np.random.Generator(np.random.PCG64(3))
    X = _embed(rng.standard_normal((g.n_nodes, 3)))
    s = _solver(g, leaf_size=32)
    U = s.evaluate(TARGETS, X)                       # (M, 2, 3)
    mu = X[0::2]
    u = L.single_layer(g, mu, TARGETS)
    dx = L.single_layer_dx(g, mu, TARGETS)
    assert np.abs(U[:, 0, :] - u).max() <= 1e-13 * np.abs(u).max()
    assert np.abs(U[:, 1, :] - dx).max() <= 1e-13 * np.abs(dx).max()


def test_full_size_workload():
    g = starfish_geometry(16384)
    u, grad = _harmonic(g)
    F = np.stack([L.neumann_data(g.curve_id), -(grad(g.xy) * g.normal).sum(1)], axis=1)
    s = _solver(g, tol=1e-10).factor()
    x, res = s.solve(_embed(F), residual=True)
    mu = x[0::2]
    rng = np.random.Generator(np.random.PCG64(9))
    rows = np.unique(np.concatenate([[0, 1, 10922, 10923, 13653, 16383],
                                     rng.choice(g.n_nodes, 40, replace=False)]))
    R = L.operator_rows(g, rows) @ mu - F[rows]
    print("Laplace 16384 nodes: residual %s, sampled row residual %.2e" % (res, np.abs(R).max()), flush=True)
    assert np.all(res < 1e-8)
    assert np.abs(R).max() < 1e-8 * np.abs(F).max()
    d = L.single_layer(g, mu[:, 1], TARGETS) - u(TARGETS)
    assert d.max() - d.min() < 1e-8
    U = s.evaluate(TARGETS, x[:, 1])
    assert np.abs(U[:, 1] - grad(TARGETS)[:, 0]).max() < 1e-8


def _moved(g0, g1):
    moved = np.nonzero(np.any(g0.xy != g1.xy, axis=1))[0].astype(np.int32)
    return (moved, g1.xy[moved], g1.normal[moved], g1.weight[moved], g1.curvature[moved])


def test_hole_move_update_equals_fresh():
    g0 = starfish_geometry(4096, 0.0, np.pi)
    s = _solver(g0, leaf_size=32).factor()
    f = _embed(L.neumann_data(g0.curve_id))
    for t1, t2 in [(0.05, np.pi), (0.05, np.pi - 0.1), (0.6, 2.0)]:
        g1 = starfish_geometry(4096, t1, t2)
        s.update_moved_nodes(*_moved(g0, g1))
        fresh = _solver(g1, leaf_size=32).factor()
        assert np.array_equal(s.solve(f), fresh.solve(f))
        g0 = g1


def test_batch_of_related_geometries():
    """The finite-difference stencil of one optimisation step: theta moved by
    +-h and +-2h in each coordinate, updated together in one batch."""
    from paper_2001_11619_amd import update_moved_nodes_batch

    t = (0.4, 3.0)
    h = 0.02
    base = starfish_geometry(4096, *t)
    shifts = [(k * h, 0.0) for k in (-2, -1, 1, 2)] + [(0.0, k * h) for k in (-2, -1, 1, 2)]
    solvers = [_solver(base, leaf_size=32).factor() for _ in shifts]
    geoms = [starfish_geometry(4096, t[0] + a, t[1] + b) for a, b in shifts]
    update_moved_nodes_batch(solvers, [_moved(base, gk) for gk in geoms])
    f = _embed(L.neumann_data(base.curve_id))
    errs = []
    for k, (sk, gk) in enumerate(zip(solvers, geoms)):
        fresh = _solver(gk, leaf_size=32).factor()
        x = sk.solve(f)
        assert np.array_equal(x, fresh.solve(f))
        if k in (0, 7):   # two of the stencil's geometries against the oracle's dense solve
            mo = L.solve(gk, L.neumann_data(gk.curve_id))
            errs.append(np.abs(x[0::2] - mo).max() / np.abs(mo).max())
    print("Laplace batch update: element-wise error against the dense solve %s" % errs, flush=True)
    assert max(errs) < 1e-8


def test_hole_delete_and_insert_update_equals_fresh():
    """Curves deleted and inserted (rs_update_geometry, N changes) with the
    Laplace kernel: bitwise the fresh factorization of the new boundary, and
    within 1e-8 of the oracle's dense solve."""
    from workloads import Geometry, starfish_nodes

    def geom(xy, nrm, w, kap, cid):
        return Geometry(xy=np.ascontiguousarray(xy), normal=np.ascontiguousarray(nrm), weight=w, curvature=kap,
                        curve_id=cid.astype(np.int32), hole_xy=np.zeros((0, 2)), curves=[])

    g0 = starfish_geometry(3000, 0.4, 3.0)
    s = _solver(g0, leaf_size=32).factor()
    rng = np.random.Generator(np.random.PCG64(21))
    # delete the second hole
    keep = np.nonzero(g0.curve_id != 2)[0]
    g1 = geom(g0.xy[keep], g0.normal[keep], g0.weight[keep], g0.curvature[keep], g0.curve_id[keep])
    # insert a third hole on the holes' path at polar angle 1.8
    th = 1.8
    rr = 0.5 * (1.0 + 0.25 * np.cos(5 * th))
    hx, hn, hw, hk = starfish_nodes(420, 0.16, 0.25, 5, th, rr * np.cos(th), rr * np.sin(th), True)
    g2 = geom(np.vstack([g1.xy, hx]), np.vstack([g1.normal, hn]), np.concatenate([g1.weight, hw]),
              np.concatenate([g1.curvature, hk]), np.concatenate([g1.curve_id, np.full(420, 2)]))
    steps = [(g1, keep), (g2, np.concatenate([np.arange(g1.n_nodes), np.full(420, -1)]))]
    for g, oon in steps:
        s.update_geometry(g.xy, g.normal, g.weight, g.curvature, g.curve_id, oon)
        fresh = _solver(g, leaf_size=32).factor()
        f = rng.standard_normal(g.n_nodes)
        x = s.solve(_embed(f))
        assert np.array_equal(x, fresh.solve(_embed(f)))
        mo = L.solve(g, f)
        err = np.abs(x[0::2] - mo).max() / np.abs(mo).max()
        print("Laplace curve update to %d nodes: element-wise error %.2e, recompressed %d boxes"
              % (g.n_nodes, err, s.stats()["boxes_recomputed"]), flush=True)
        assert err < 1e-8
