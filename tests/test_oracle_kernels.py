"""Pins of the oracle's kernels against identities the mathematics fixes.

* Gauss identity (from the jump relation eq. (jump)): with normals pointing
  out of the fluid, the double layer applied to a constant density gives
  -e/2 at every node, on the outer curve and on every hole.  A wrong sign,
  a wrong self term (curvature limit), a wrong weight or a transposed block
  each break it at the 1e-2 level while the right kernel meets it to ~1e-13.
* Null space eq. (null-space): rigid motions on one hole are annihilated by
  -I/2 + D + N, and N annihilates them on its own.
* The self block equals the limit of the off-diagonal kernel along the curve.
"""

import numpy as np
import pytest

from oracle import stokes
from workloads import build_geometry, Curve, workload_small, single_ellipse


def _geoms():
    return [
        single_ellipse(256, 1.0, 0.6),
        workload_small(seed=11, n_outer=256, n_holes=2, nodes_per_hole=128, radius=3.0),
        build_geometry([Curve(300, 2.0, 1.5, 0.3, 0.1, -0.2, False),
                        Curve(160, 0.4, 0.25, 1.1, 0.5, 0.3, True)]),
    ]


@pytest.mark.parametrize("gi", range(3))
@pytest.mark.parametrize("comp", [0, 1])
def test_gauss_identity(gi, comp):
    g = _geoms()[gi]
    n = g.n_dofs
    dofs = np.arange(n)
    D = stokes.operator_entries(g, dofs, dofs, 0.0)
    e = np.zeros(n)
    e[comp::2] = 1.0
    # N e = n_i * sum_j w_j n_j . e = 0 to quadrature accuracy, so D+N works too.
    assert np.abs(D @ e + 0.5 * e).max() < 1e-11


def test_gauss_identity_detects_wrong_self_term():
    g = _geoms()[1]
    n = g.n_dofs
    dofs = np.arange(n)
    D = stokes.operator_entries(g, dofs, dofs, 0.0)
    # remove the curvature self term: the identity must fail visibly
    Sblk = stokes.double_layer_self_block(g.normal, g.weight, g.curvature)
    D2 = D.copy()
    for j in range(g.n_nodes):
        D2[2 * j:2 * j + 2, 2 * j:2 * j + 2] -= Sblk[j]
    e = np.zeros(n)
    e[0::2] = 1.0
    assert np.abs(D2 @ e + 0.5 * e).max() > 1e-4


@pytest.mark.parametrize("gi", [1, 2])
def test_rigid_motion_null_space(gi):
    g = _geoms()[gi]
    n = g.n_dofs
    dofs = np.arange(n)
    K = stokes.operator_entries(g, dofs, dofs, -0.5)
    P = stokes.psi_t_matrix(g)
    for h in range(g.n_holes):
        idx = np.nonzero(g.curve_id == h + 1)[0]
        for c in range(3):
            psi = np.zeros(n)
            if c == 0:
                psi[2 * idx] = 1.0
            elif c == 1:
                psi[2 * idx + 1] = 1.0
            else:
                psi[2 * idx] = -g.xy[idx, 1]
                psi[2 * idx + 1] = g.xy[idx, 0]
            assert np.abs(K @ psi).max() < 1e-11
            # the Psi^T row of this mode is the weighted mode itself
            assert np.allclose(P[3 * h + c], np.repeat(g.weight, 2) * psi)


def test_rank_one_completion():
    """lam I + D + N minus an independently built D is exactly n_i w_j n_j^T,
    and that term annihilates rigid motions on a hole (eq. null-spaceop)."""
    g = _geoms()[1]
    n = g.n_dofs
    dofs = np.arange(n)
    full = stokes.operator_entries(g, dofs, dofs, 0.0)
    N = g.n_nodes
    D = np.zeros((n, n))
    for i in range(N):
        for j in range(N):
            if i == j:
                t = np.array([-g.normal[i, 1], g.normal[i, 0]])
                D[2 * i:2 * i + 2, 2 * i:2 * i + 2] = -g.weight[i] * g.curvature[i] / (2 * np.pi) * np.outer(t, t)
            else:
                r = g.xy[i] - g.xy[j]
                r2 = r @ r
                D[2 * i:2 * i + 2, 2 * j:2 * j + 2] = (g.weight[j] / np.pi) * (r @ g.normal[j]) / r2 ** 2 * np.outer(r, r)
    wn = (g.weight[:, None] * g.normal).reshape(-1)
    nn = g.normal.reshape(-1)
    assert np.abs(full - D - np.outer(nn, wn)).max() < 1e-13
    idx = np.nonzero(g.curve_id == 1)[0]
    psi = np.zeros(n)
    psi[2 * idx] = -g.xy[idx, 1]
    psi[2 * idx + 1] = g.xy[idx, 0]
    assert abs(wn @ psi) < 1e-12


def test_self_block_is_curve_limit():
    # ellipse: compare the curvature limit with the smooth kernel at a very
    # close neighbour on a finely discretised curve
    g = single_ellipse(200000, 1.0, 0.6)
    j = 12345
    tx = g.xy[j:j + 1]
    blk = stokes.double_layer_blocks(tx, g.xy[j + 1:j + 2], g.normal[j + 1:j + 2], np.ones(1))[0, 0]
    lim = stokes.double_layer_self_block(g.normal[j:j + 1], np.ones(1), g.curvature[j:j + 1])[0]
    assert np.abs(blk - lim).max() < 1e-4 * np.abs(lim).max() + 1e-6


def test_curvature_sign_convention():
    g = workload_small(seed=11, n_outer=64, n_holes=2, nodes_per_hole=64, radius=3.0)
    assert np.all(g.curvature[g.curve_id == 0] > 0)
    assert np.all(g.curvature[g.curve_id > 0] < 0)
    # outer circle: curvature 1/R, normal outward
    o = g.curve_id == 0
    assert np.allclose(g.curvature[o], 1.0 / 3.0)
    assert np.allclose(np.einsum("ij,ij->i", g.xy[o], g.normal[o]), 3.0)
