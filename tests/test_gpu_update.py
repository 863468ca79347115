"""GPU updating (Section 2.8) through rs_update_moved_nodes.

The paper's claim, with the root square kept: an updated factorization is
exactly the one a fresh factorization of the new geometry gives.  Checked
bitwise against a fresh GPU factorization (same root), against the oracle's
own update to the float64 parity bar, over several successive moves, and for
the degenerate update that moves nothing."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle.rs import RSFactorization, RSParams
from workloads import boundary_data, exterior_forces_for_geometry, move_hole, random_holes_geometry


def _solver(g, **kw):
    import torch

    assert torch.cuda.is_available()
    from paper_2001_11619_amd import RSSolver

    return RSSolver.from_geometry(g, **kw)


def _elem(x, xo, n2):
    """Element-wise error of the densities and of the border unknowns, each
    relative to the largest entry of its part of the reference."""
    em = np.max(np.abs(x[:n2] - xo[:n2]).max(axis=0) / np.abs(xo[:n2]).max(axis=0))
    eb = np.max(np.abs(x[n2:] - xo[n2:]).max(axis=0) / np.abs(xo[n2:]).max(axis=0))
    return float(em), float(eb)


def _moved_args(g, moved):
    return (moved, g.xy[moved], g.normal[moved], g.weight[moved], g.curvature[moved])


def test_update_equals_fresh_factorization_bitwise():
    g = random_holes_geometry(21, 6.0, 1024, [256] * 6)
    s = _solver(g, leaf_size=32).factor()
    root = tuple(s.boxes()["geom"][0])
    rng = np.random.Generator(np.random.PCG64(5))
    orc = RSFactorization(g, RSParams(leaf_size=32, pivot="key20")).factor()
    for step in range(3):
        g2, moved = move_hole(g, 1 + step, rng, radius=6.0)
        s.update_moved_nodes(*_moved_args(g2, moved), hole_xy=g2.hole_xy)
        st = s.stats()
        g2.root = np.array(root)
        fresh = _solver(g2, leaf_size=32, root=root).factor()
        f = boundary_data(g2, exterior_forces_for_geometry(g2, 3, seed=step))
        xu = s.solve(f)
        xf = fresh.solve(f)
        assert np.array_equal(xu, xf)
        nb = int(np.sum(fresh.boxes()["n"][1:] > 0))
        assert 0 < st["boxes_recomputed"] < 0.6 * nb
        rec = orc.update(g2, moved)
        assert sum(orc.fac[b].I.size > 0 for b in rec) == st["boxes_recomputed"]
        em, eb = _elem(xu, orc.solve(f), g2.n_dofs)
        assert em < 1e-10 and eb < 1e-10, (em, eb)
        g = g2


def test_update_nothing_moved():
    g = random_holes_geometry(22, 6.0, 512, [128] * 3)
    s = _solver(g, leaf_size=32).factor()
    f = boundary_data(g, exterior_forces_for_geometry(g, 2, seed=1))
    x0 = s.solve(f)
    s.update_moved_nodes(np.zeros(0, np.int32), np.zeros((0, 2)), np.zeros((0, 2)), np.zeros(0), np.zeros(0))
    assert s.stats()["boxes_recomputed"] == 0
    assert np.array_equal(s.solve(f), x0)


def test_update_out_of_root_rejected():
    from paper_2001_11619_amd import RSError

    g = random_holes_geometry(22, 6.0, 512, [128] * 3)
    s = _solver(g, leaf_size=32).factor()
    with pytest.raises(RSError) as e:
        s.update_moved_nodes(np.array([3], np.int32), np.array([[100.0, 0.0]]), g.normal[3:4],
                             g.weight[3:4], g.curvature[3:4])
    assert e.value.name == "RS_ERR_OUT_OF_ROOT"


def test_batch_factor_equals_single():
    """Level-synchronous factorization of several geometries in shared launches
    gives each geometry exactly its own factorization."""
    from paper_2001_11619_amd import factor_batch
    from workloads import single_ellipse, workload_small

    geoms = [random_holes_geometry(31 + i, 5.0, 512 + 128 * i, [128 + 64 * i] * (i + 1)) for i in range(3)]
    geoms.append(single_ellipse(700, 1.0, 0.5))
    geoms.append(workload_small(seed=11, n_outer=256, n_holes=2, nodes_per_hole=128, radius=3.0))
    batch = [_solver(g, leaf_size=32) for g in geoms]
    factor_batch(batch)
    for g, s in zip(geoms, batch):
        f = boundary_data(g, exterior_forces_for_geometry(g, 2, seed=7))
        alone = _solver(g, leaf_size=32).factor()
        assert np.array_equal(s.solve(f), alone.solve(f))


def test_update_batch_equals_single_updates():
    """Several related geometries updated together (rs_update_moved_nodes_batch,
    one launch per kernel and level across them; Scheme A of the paper's
    optimization experiments): each context is bitwise the context updated on
    its own, and equal to a fresh factorization of its new geometry."""
    from paper_2001_11619_amd import update_moved_nodes_batch

    base = random_holes_geometry(23, 6.0, 768, [192] * 5)
    single, batch, moves, news = [], [], [], []
    for i in range(4):
        rng = np.random.Generator(np.random.PCG64(100 + i))
        g2, moved = move_hole(base, 1 + i, rng, radius=6.0)
        a = _solver(base, leaf_size=32).factor()
        b = _solver(base, leaf_size=32).factor()
        mv = _moved_args(g2, moved) + (g2.hole_xy,)
        a.update_moved_nodes(*mv[:5], hole_xy=mv[5])
        single.append(a)
        batch.append(b)
        moves.append(mv)
        news.append(g2)
    update_moved_nodes_batch(batch, moves)
    root = tuple(single[0].boxes()["geom"][0])
    for i in range(4):
        f = boundary_data(news[i], exterior_forces_for_geometry(news[i], 2, seed=i))
        xs = single[i].solve(f)
        xb = batch[i].solve(f)
        assert np.array_equal(xs, xb)
        assert batch[i].stats()["boxes_recomputed"] == single[i].stats()["boxes_recomputed"]
        g = news[i]
        g.root = np.array(root)
        fresh = _solver(g, leaf_size=32, root=root).factor()
        assert np.array_equal(fresh.solve(f), xb)
        # and against the oracle's own update of the same move (Section 2.8)
        orc = RSFactorization(base, RSParams(leaf_size=32, pivot="key20")).factor()
        rec = orc.update(g, moves[i][0])
        assert sum(orc.fac[b].I.size > 0 for b in rec) == batch[i].stats()["boxes_recomputed"]
        em, eb = _elem(xb, orc.solve(f), g.n_dofs)
        assert em < 1e-10 and eb < 1e-10, (em, eb)


def test_update_batch_rejects_bad_input_atomically():
    """An invalid move in one context of the batch changes no context."""
    from paper_2001_11619_amd import RSError, update_moved_nodes_batch

    g = random_holes_geometry(22, 6.0, 512, [128] * 3)
    ss = [_solver(g, leaf_size=32).factor() for _ in range(2)]
    f = boundary_data(g, exterior_forces_for_geometry(g, 1, seed=1))
    x0 = [s.solve(f) for s in ss]
    good = (np.array([3], np.int32), g.xy[3:4] * 1.001, g.normal[3:4], g.weight[3:4], g.curvature[3:4])
    bad = (np.array([3], np.int32), np.array([[100.0, 0.0]]), g.normal[3:4], g.weight[3:4], g.curvature[3:4])
    with pytest.raises(RSError) as e:
        update_moved_nodes_batch(ss, [good, bad])
    assert e.value.name == "RS_ERR_OUT_OF_ROOT"
    for s, x in zip(ss, x0):
        assert np.array_equal(s.solve(f), x)
