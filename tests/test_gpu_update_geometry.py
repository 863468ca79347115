"""GPU updating after curves are inserted or deleted (rs_update_geometry).

Section 2.8's claim carried to the experiment of Section 4.2 (holes added to
and removed from the domain): with the root square kept, recompressing only
the boxes whose compression inputs changed gives exactly the factorization a
fresh factorization of the new boundary gives.  Checked bitwise against a
fresh GPU factorization with the same root, element by element (densities
and border unknowns separately, 1e-10) against the oracle's own update of the
same insertion and deletion, and for the refusal of inputs that break the
node correspondence (the context is then unchanged)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle.rs import RSFactorization, RSParams
from workloads import boundary_data, delete_hole, exterior_forces_for_geometry, insert_hole, random_holes_geometry


def _solver(g, **kw):
    import torch

    assert torch.cuda.is_available()
    from paper_2001_11619_amd import RSSolver

    return RSSolver.from_geometry(g, **kw)


def _elem(x, xo, n2):
    em = np.max(np.abs(x[:n2] - xo[:n2]).max(axis=0) / np.abs(xo[:n2]).max(axis=0))
    eb = np.max(np.abs(x[n2:] - xo[n2:]).max(axis=0) / np.abs(xo[n2:]).max(axis=0))
    return float(em), float(eb)


def _update(s, g, oon):
    return s.update_geometry(g.xy, g.normal, g.weight, g.curvature, g.curve_id, oon, hole_xy=g.hole_xy)


@pytest.mark.parametrize("precision", [0, 1])
def test_insert_then_delete_equals_fresh_factorization(precision):
    g = random_holes_geometry(21, 6.0, 1024, [256] * 4)
    kw = dict(leaf_size=32, tol=1e-10 if precision == 0 else 1e-7, precision=precision)
    s = _solver(g, **kw).factor()
    root = tuple(s.boxes()["geom"][0])
    g.root = np.array(root)
    orc = RSFactorization(g, RSParams(leaf_size=32, tol=kw["tol"], pivot="key20")).factor()
    rng = np.random.Generator(np.random.PCG64(8))
    g2, oon2 = insert_hole(g, rng, 256)
    g3, oon3 = delete_hole(g2, 2)
    for gn, oon in ((g2, oon2), (g3, oon3)):
        _update(s, gn, oon)
        st = s.stats()
        gn.root = np.array(root)
        fresh = _solver(gn, root=root, **kw).factor()
        f = boundary_data(gn, exterior_forces_for_geometry(gn, 3, seed=4))
        x = s.solve(f)
        assert np.array_equal(x, fresh.solve(f))
        nb = int(np.sum(fresh.boxes()["n"][1:] > 0))
        assert 0 < st["boxes_recomputed"] < 0.6 * nb
        assert st["n_nodes"] == gn.n_nodes and st["n_holes"] == gn.n_holes
        rec = orc.update_geometry(gn, oon)
        assert sum(orc.fac[b].I.size > 0 for b in rec) == st["boxes_recomputed"]
        if precision == 0:
            em, eb = _elem(x, orc.solve(f), gn.n_dofs)
            assert em < 1e-10 and eb < 1e-10, (em, eb)
        fresh.close()


def test_update_geometry_rejects_bad_correspondence():
    from paper_2001_11619_amd import RSError

    g = random_holes_geometry(22, 6.0, 512, [128] * 3)
    s = _solver(g, leaf_size=32).factor()
    root = tuple(s.boxes()["geom"][0])
    g.root = np.array(root)
    f = boundary_data(g, exterior_forces_for_geometry(g, 1, seed=1))
    x0 = s.solve(f)
    g2, oon = delete_hole(g, 1)
    bad = oon.copy()
    bad[[10, 11]] = bad[[11, 10]]
    with pytest.raises(RSError) as e:
        _update(s, g2, bad)
    assert e.value.name == "RS_ERR_ARG"
    moved = g2.xy.copy()
    moved[5] += 1e-3
    with pytest.raises(RSError) as e:
        s.update_geometry(moved, g2.normal, g2.weight, g2.curvature, g2.curve_id, oon, hole_xy=g2.hole_xy)
    assert e.value.name == "RS_ERR_ARG"
    # the context still holds its factorization of the old boundary
    assert np.array_equal(s.solve(f), x0)
