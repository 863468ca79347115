"""Pin of the oracle's updating rule (Section 2.8): with the root square kept,
recompressing only the marked boxes gives exactly the factorization a fresh
factorization of the moved geometry gives (the paper reports this equality
for its experiments), while recompressing far fewer boxes than all."""

import numpy as np

from oracle.rs import RSFactorization, RSParams
from workloads import boundary_data, exterior_forces_for_geometry, move_hole, random_holes_geometry


def test_update_equals_refactor():
    g = random_holes_geometry(21, 6.0, 1024, [256] * 6)
    g.root = None
    prm = RSParams(tol=1e-10, leaf_size=32)
    rs = RSFactorization(g, prm).factor()
    root = rs.root
    rng = np.random.Generator(np.random.PCG64(5))
    g2, moved = move_hole(g, 1, rng, radius=6.0)
    g2.root = np.array(root)
    f = boundary_data(g2, exterior_forces_for_geometry(g2, 2, seed=3))
    rec = rs.update(g2, moved)
    x_up = rs.solve(f)
    fresh = RSFactorization(g2, prm, root=root).factor()
    x_new = fresh.solve(f)
    assert np.array_equal(x_up, x_new)
    nb = sum(1 for b in fresh.boxes[1:] if fresh.fac[b.id].I.size)
    assert 0 < len(rec) < 0.5 * nb
    # ranks and skeletons of every box agree with the fresh factorization
    for b in fresh.boxes[1:]:
        assert np.array_equal(rs.fac[b.id].S, fresh.fac[b.id].S)


def test_update_without_motion_recomputes_nothing():
    g = random_holes_geometry(22, 6.0, 512, [128] * 3)
    prm = RSParams(tol=1e-10, leaf_size=32)
    rs = RSFactorization(g, prm).factor()
    g.root = np.array(rs.root)
    rec = rs.update(g, np.zeros(0, dtype=np.int64))
    assert len(rec) == 0


def _fresh_equal(rs, g2, prm, root, nrhs=2):
    f = boundary_data(g2, exterior_forces_for_geometry(g2, nrhs, seed=3))
    g2.root = np.array(root)
    fresh = RSFactorization(g2, prm, root=root).factor()
    assert np.array_equal(rs.solve(f), fresh.solve(f))
    for b in fresh.boxes[1:]:
        assert np.array_equal(rs.fac[b.id].S, fresh.fac[b.id].S)
    return fresh


def test_hole_insertion_and_deletion_equal_refactor():
    """Section 2.8 with curves inserted and deleted (Section 4.2's experiment):
    N and p change, box membership changes near the curve, the numbering of
    later curves shifts; recompressing only the boxes whose inputs changed
    still gives exactly the fresh factorization of the new geometry, and the
    solution stays a solution of the new system."""
    from oracle import stokes
    from workloads import delete_hole, insert_hole

    g = random_holes_geometry(21, 6.0, 1024, [256] * 4)
    prm = RSParams(tol=1e-10, leaf_size=32)
    rs = RSFactorization(g, prm).factor()
    root = rs.root
    g.root = np.array(root)
    rng = np.random.Generator(np.random.PCG64(8))
    g2, oon = insert_hole(g, rng, 256)
    assert g2.n_holes == g.n_holes + 1 and g2.n_nodes == g.n_nodes + 256
    rec = rs.update_geometry(g2, oon)
    fresh = _fresh_equal(rs, g2, prm, root)
    nb = sum(1 for b in fresh.boxes[1:] if fresh.fac[b.id].I.size)
    assert 0 < len(rec) < 0.6 * nb
    # delete a hole in the middle of the numbering (later nodes shift down)
    g3, oon = delete_hole(g2, 2)
    assert g3.n_holes == g2.n_holes - 1 and g3.n_nodes == g2.n_nodes - 256
    rec = rs.update_geometry(g3, oon)
    _fresh_equal(rs, g3, prm, root)
    assert 0 < len(rec) < 0.6 * nb
    f = boundary_data(g3, exterior_forces_for_geometry(g3, 1, seed=4))
    r = stokes.apply_system(g3, rs.solve(f)) - np.vstack([f, np.zeros((3 * g3.n_holes, 1))])
    assert np.linalg.norm(r) / np.linalg.norm(f) < 1e-8


def test_update_geometry_rejects_reordered_or_changed_nodes():
    import pytest

    from workloads import delete_hole

    g = random_holes_geometry(22, 6.0, 512, [128] * 3)
    rs = RSFactorization(g, RSParams(tol=1e-10, leaf_size=32)).factor()
    g.root = np.array(rs.root)
    g2, oon = delete_hole(g, 1)
    bad = oon.copy()
    bad[[10, 11]] = bad[[11, 10]]
    with pytest.raises(ValueError):
        rs.update_geometry(g2, bad)
    g2.xy = g2.xy.copy()
    g2.xy[5] += 1e-3
    with pytest.raises(ValueError):
        rs.update_geometry(g2, oon)
