"""Pins of the Laplace Neumann oracle (Section 4.4.1) against facts the
mathematics fixes, independent of the oracle's own formulas:

* on a circle the adjoint double layer has a closed form (every entry
  w_j / (4 pi R)), so the discrete -I/2 - D annihilates constants exactly;
* the range of -I/2 - D is orthogonal to constants (w^T (-I/2 - D) = 0) and
  its null space is one-dimensional, which the rank-one completion N removes;
* for f = 1 the completion fixes sum_j w_j mu_j = 1;
* exact harmonic fields (point sources outside the domain plus a linear
  field) are reproduced up to one constant at spectral accuracy, and their
  x-derivative too; a dropped or sign-flipped curvature term, or the wrong
  sign of the identity, fails this by many orders of magnitude;
* the eq. (neumanndata) flux integrates to zero on the workload (its two
  holes have the same size and discretisation).
"""

import numpy as np
import pytest

from oracle import laplace as L
from workloads import Geometry, starfish_geometry, starfish_nodes


def _circle(n, R):
    xy, nrm, w, kap = starfish_nodes(n, R, 0.0, 1, 0.0, 0.0, 0.0, False)
    return Geometry(xy=xy, normal=nrm, weight=w, curvature=kap, curve_id=np.zeros(n, np.int32),
                    hole_xy=np.zeros((0, 2)), curves=[])


def test_circle_closed_form():
    R = 1.7
    g = _circle(96, R)
    A = L.operator_matrix(g, lam=0.0) - g.weight[None, :]       # -D alone
    expect = np.broadcast_to(g.weight[None, :] / (4 * np.pi * R), A.shape)
    assert np.allclose(A, expect, rtol=1e-12, atol=0)
    B = A - 0.5 * np.eye(g.n_nodes)
    assert np.abs(B @ np.ones(g.n_nodes)).max() < 1e-13


def test_range_and_null_space():
    g = starfish_geometry(900)
    A = L.operator_matrix(g)
    B = A - g.weight[None, :]                                    # -I/2 - D
    assert np.abs(g.weight @ B).max() < 1e-12
    sv = np.linalg.svd(B, compute_uv=False)
    assert sv[-1] < 1e-12 and sv[-2] > 1e-2
    assert np.linalg.cond(A) < 1e3


def test_completion_scale():
    g = starfish_geometry(900)
    mu = L.solve(g, np.ones(g.n_nodes))
    assert abs(g.weight @ mu - 1.0) < 1e-12


def _harmonic(g):
    srcs = np.array([[1.6, 0.3], [-0.2, 1.7], g.hole_xy[0], g.hole_xy[1]])
    q = np.array([0.7, -0.4, 1.1, -0.5])
    a = np.array([0.3, -0.8])

    def grad(x):
        r = x[:, None, :] - srcs[None]
        r2 = (r * r).sum(-1)
        return (q[None, :, None] * r / r2[..., None]).sum(1) + a

    def u(x):
        r = x[:, None, :] - srcs[None]
        return (q[None] * 0.5 * np.log((r * r).sum(-1))).sum(1) + x @ a

    return u, grad


@pytest.mark.parametrize("n", [1200, 2400])
def test_exact_harmonic_solution(n):
    g = starfish_geometry(n)
    u, grad = _harmonic(g)
    f = -(grad(g.xy) * g.normal).sum(1)                          # flux along the inward normal
    assert abs(g.weight @ f) < 1e-12
    mu = L.solve(g, f)
    T = np.array([[0.0, 0.3], [0.2, -0.4], [-0.6, 0.1], [0.35, 0.45]])
    d = L.single_layer(g, mu, T) - u(T)
    assert d.max() - d.min() < 1e-12
    assert np.abs(L.single_layer_dx(g, mu, T) - grad(T)[:, 0]).max() < 1e-12
    assert abs(g.weight @ mu) < 1e-12                           # compatible data: N mu = 0


def test_dx_against_differences():
    g = starfish_geometry(600)
    mu = L.solve(g, L.neumann_data(g.curve_id))
    T = np.array([[0.0, 0.0], [0.1, -0.3]])
    h = 1e-4
    e = np.array([h, 0.0])
    fd = (L.single_layer(g, mu, T + e) - L.single_layer(g, mu, T - e)) / (2 * h)
    assert np.allclose(L.single_layer_dx(g, mu, T), fd, rtol=1e-6, atol=1e-9)


def test_neumann_data_compatible():
    g = starfish_geometry(16384)
    f = L.neumann_data(g.curve_id)
    assert np.count_nonzero(f == 1) == np.count_nonzero(f == -1) == (16384 - np.count_nonzero(f == 0)) // 2
    assert abs(g.weight @ f) < 1e-13
