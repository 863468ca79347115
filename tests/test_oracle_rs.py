"""Pins of the oracle's recursive skeletonization (Sections 2.2-2.7, 3.2).

* Agreement with the dense LU of the augmented system to O(eps) and a
  residual that tracks the ID tolerance (the paper's accuracy study,
  Section 4.1).
* Brute force on tiny inputs: the factors assembled into explicit matrices
  U and V make U A V block diagonal (eq. ddef) and V X_D^{-1} U solves the
  system (eq. kinv).  A dropped term or a wrong sweep order in U, V or the
  row sweep for Psi^T V fails this at O(1).
* Tree invariants of Section 2.3.
"""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import stokes
from oracle.rs import RSFactorization, RSParams
from oracle.tree import build_tree
from workloads import (boundary_data, exterior_forces_for_geometry, single_ellipse,
                       workload_small, build_geometry, Curve)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_tree_partition_and_leaf_bound():
    g = workload_small(seed=11, n_outer=256, n_holes=3, nodes_per_hole=96, radius=3.0)
    boxes = build_tree(g.xy, 16)
    leaves = [b for b in boxes if b.is_leaf]
    allnodes = np.sort(np.concatenate([b.nodes for b in leaves]))
    assert np.array_equal(allnodes, np.arange(g.n_nodes))
    for b in leaves:
        assert 1 <= b.nodes.size <= 16
    for b in boxes:
        h = b.side / 2
        p = g.xy[b.nodes]
        assert np.all(p[:, 0] >= b.cx - h) and np.all(p[:, 0] < b.cx + h)
        assert np.all(p[:, 1] >= b.cy - h) and np.all(p[:, 1] < b.cy + h)
        if b.children:
            assert np.array_equal(np.sort(np.concatenate([boxes[c].nodes for c in b.children])), b.nodes)
            for c in b.children:
                assert boxes[c].level == b.level + 1


@pytest.mark.parametrize("tol", [1e-6, 1e-8, 1e-10])
def test_rs_tracks_tolerance_multiply_connected(tol):
    g = workload_small(seed=11, n_outer=256, n_holes=2, nodes_per_hole=128, radius=3.0)
    f = boundary_data(g, exterior_forces_for_geometry(g, 2, seed=5))
    xd = stokes.dense_solve(g, f)
    rs = RSFactorization(g, RSParams(tol=tol, leaf_size=32)).factor()
    xr = rs.solve(f)
    res = stokes.apply_system(g, xr) - np.vstack([f, np.zeros((3 * g.n_holes, f.shape[1]))])
    rres = np.linalg.norm(res) / np.linalg.norm(f)
    assert rres < 30 * tol
    assert _rel(xr, xd) < 100 * tol
    # compression actually happens
    assert sum(fb.r for fb in rs.fac.values()) > 0.5 * g.n_dofs


def test_rs_simply_connected_ellipse():
    g = single_ellipse(1024, 1.0, 0.6)
    f = boundary_data(g, exterior_forces_for_geometry(g, 1, seed=1))
    xd = stokes.dense_solve(g, f)
    rs = RSFactorization(g, RSParams(tol=1e-10, leaf_size=64)).factor()
    assert rs.L >= 3
    assert _rel(rs.solve(f), xd) < 1e-8


def _dense_U_V(rs):
    n = rs.geom.n_dofs
    U = rs.apply_U(np.eye(n))
    V = rs.apply_V(np.eye(n))
    return U, V


def test_brute_force_block_diagonal_tiny():
    g = build_geometry([Curve(40, 1.0, 0.8, 0.2, 0.0, 0.0, False),
                        Curve(20, 0.25, 0.2, 0.5, 0.3, 0.1, True)])
    rs = RSFactorization(g, RSParams(tol=1e-14, leaf_size=4)).factor()
    n = g.n_dofs
    A = stokes.operator_entries(g, np.arange(n), np.arange(n), -0.5)
    U, V = _dense_U_V(rs)
    X = U @ A @ V
    # expected X_D: X_RR of every box on its R block and X_SS of the root on I0
    XD = np.zeros_like(X)
    for fb in rs.fac.values():
        if fb.r:
            R = fb.R
            lu, piv = fb.lu
            Lm = np.tril(lu, -1) + np.eye(fb.r)
            Um = np.triu(lu)
            Pm = np.eye(fb.r)
            for i, p in enumerate(piv):
                Pm[[i, p]] = Pm[[p, i]]
            XD[np.ix_(R, R)] = Pm.T @ Lm @ Um
    XD[np.ix_(rs.I0, rs.I0)] = rs.X0
    scale = np.abs(A).max()
    assert np.abs(X - XD).max() < 1e-9 * scale
    # row sweep equals the explicit product Psi^T V
    Pt = stokes.psi_t_matrix(g)
    assert np.abs(rs.apply_Vt_rows(Pt) - Pt @ V).max() < 1e-12 * np.abs(Pt).max() * np.abs(V).max()
    # and the full solve equals the dense solve
    f = boundary_data(g, exterior_forces_for_geometry(g, 1, seed=3))
    assert _rel(rs.solve(f), stokes.dense_solve(g, f)) < 1e-9


def test_level_parallel_compresses():
    """Compression keeps most unknowns redundant at the leaves (Section 2.7)."""
    g = single_ellipse(1024, 1.0, 0.6)
    rs = RSFactorization(g, RSParams(tol=1e-10, leaf_size=64)).factor()
    assert rs.I0.size < 0.25 * g.n_dofs
