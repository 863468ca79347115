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
