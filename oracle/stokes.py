"""Kernels and the dense augmented Stokes system (paper Section 3.1).

TEST INFRASTRUCTURE ONLY (see the package header).

Unknown layout: degree of freedom 2j is the x-component of the density at
node j, 2j+1 its y-component; the 3p augmented unknowns follow, per hole h
(1-based) in the order (alpha_h1, alpha_h2, beta_h).

Pins (tests/test_oracle_kernels.py, tests/test_oracle_dense.py):
  * Gauss identity of the double layer (consequence of the jump relation
    eq. (jump)): D e = -e/2 at every node of a multiply-connected boundary.
  * Null space eq. (null-space): (-I/2 + D + N) psi = 0 for rigid motions.
  * Exterior point-force solutions: the solved density reproduces the exact
    interior velocity, and alpha / beta equal the force / torque enclosed by
    each hole (the force and torque statements of Section 3.1).
  * Couette flow between concentric circles (the analytic test of Section 4.1).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

INV_PI = 1.0 / np.pi
INV_4PI = 1.0 / (4.0 * np.pi)


def double_layer_blocks(tx, sy, sn, sw):
    """Stresslet double-layer 2x2 blocks, eq. (stokesbie):

        K(x, y) = (1/pi) * ((x - y) . n_y) / |x - y|^4 * (x - y)(x - y)^T * w_y

    tx (Mt, 2) targets, sy (Ms, 2) sources with normals sn and weights sw.
    Returns (Mt, Ms, 2, 2).  Coincident target/source pairs are not allowed.
    """
    r = tx[:, None, :] - sy[None, :, :]
    r2 = np.einsum("ijk,ijk->ij", r, r)
    rn = np.einsum("ijk,jk->ij", r, sn)
    coef = INV_PI * sw[None, :] * rn / (r2 * r2)
    return coef[:, :, None, None] * r[:, :, :, None] * r[:, :, None, :]


def double_layer_self_block(normal, weight, curvature):
    """Diagonal block of the discretised double layer at a node.

    The smooth kernel tends to -(kappa / (2 pi)) t t^T as y -> x along the
    curve, with t the unit tangent and kappa the signed curvature (positive
    where the curve bends away from n).  Times the node weight.
    """
    t = np.stack([-normal[:, 1], normal[:, 0]], axis=1)
    c = -(weight * curvature) / (2.0 * np.pi)
    return c[:, None, None] * t[:, :, None] * t[:, None, :]


def stokeslet_blocks(tx, sy, sw):
    """Stokeslet 2x2 blocks (1/(4 pi)) (ln(1/|r|) I + r r^T / |r|^2) * w_y, r = x - y."""
    r = tx[:, None, :] - sy[None, :, :]
    r2 = np.einsum("ijk,ijk->ij", r, r)
    eye = np.eye(2)[None, None, :, :]
    return INV_4PI * sw[None, :, None, None] * (
        -0.5 * np.log(r2)[:, :, None, None] * eye + r[:, :, :, None] * r[:, :, None, :] / r2[:, :, None, None]
    )


def rotlet_columns(tx, c):
    """Rotlet velocity at tx (M, 2) for a unit torque at c: r_perp / (4 pi |r|^2), r_perp = (-r2, r1)."""
    r = tx - c[None, :]
    r2 = np.einsum("ij,ij->i", r, r)
    return INV_4PI * np.stack([-r[:, 1], r[:, 0]], axis=1) / r2[:, None]


def _pick(blocks, rdofs, cdofs, rnode_pos, cnode_pos):
    return blocks[rnode_pos[:, None], cnode_pos[None, :], (rdofs % 2)[:, None], (cdofs % 2)[None, :]]


def operator_entries(geom, rdofs, cdofs, lam):
    """Entries of lam*I + D + N restricted to rows rdofs and columns cdofs.

    D off-diagonal blocks use the stresslet formula; diagonal node blocks use
    the curvature limit; N_ij = w_j n_i n_j^T over all node pairs (eq. null-spaceop).
    """
    rdofs = np.asarray(rdofs, dtype=np.int64)
    cdofs = np.asarray(cdofs, dtype=np.int64)
    rn_u, rpos = np.unique(rdofs // 2, return_inverse=True)
    cn_u, cpos = np.unique(cdofs // 2, return_inverse=True)
    xy, nr, w, kap = geom.xy, geom.normal, geom.weight, geom.curvature
    same = rn_u[:, None] == cn_u[None, :]
    tx = xy[rn_u]
    sy = xy[cn_u]
    with np.errstate(divide="ignore", invalid="ignore"):
        blk = double_layer_blocks(tx, sy, nr[cn_u], w[cn_u])
    if same.any():
        ii, jj = np.nonzero(same)
        blk[ii, jj] = double_layer_self_block(nr[cn_u[jj]], w[cn_u[jj]], kap[cn_u[jj]])
    wn = w[cn_u][:, None] * nr[cn_u]                       # (Mc, 2): w_j n_j
    blk = blk + nr[rn_u][:, None, :, None] * wn[None, :, None, :]
    out = _pick(blk, rdofs, cdofs, rpos, cpos)
    out = out + lam * (rdofs[:, None] == cdofs[None, :])
    return out


def h_matrix(geom):
    """H = [S R] of eq. (forwardeq): (2N, 3p) Stokeslet (2 columns) and rotlet (1 column) per hole."""
    N, p = geom.n_nodes, geom.n_holes
    H = np.zeros((2 * N, 3 * p))
    for h in range(p):
        c = geom.hole_xy[h]
        S = stokeslet_blocks(geom.xy, c[None, :], np.ones(1))[:, 0]   # (N, 2, 2)
        H[:, 3 * h + 0] = S[:, :, 0].reshape(-1)
        H[:, 3 * h + 1] = S[:, :, 1].reshape(-1)
        H[:, 3 * h + 2] = rotlet_columns(geom.xy, c).reshape(-1)
    return H


def psi_t_matrix(geom):
    """Psi^T of eq. (backwardeq): quadrature of the rigid motions e1, e2, x^perp on each hole.

    x^perp = (-x2, x1), taken about the origin as printed.
    """
    N, p = geom.n_nodes, geom.n_holes
    P = np.zeros((3 * p, 2 * N))
    for h in range(p):
        idx = np.nonzero(geom.curve_id == h + 1)[0]
        w = geom.weight[idx]
        P[3 * h + 0, 2 * idx] = w
        P[3 * h + 1, 2 * idx + 1] = w
        P[3 * h + 2, 2 * idx] = -w * geom.xy[idx, 1]
        P[3 * h + 2, 2 * idx + 1] = w * geom.xy[idx, 0]
    return P


def dense_system(geom, lam=-0.5):
    """The full augmented matrix [[lam I + D + N, H], [Psi^T, -I]] of eq. (backwardeq)."""
    n = geom.n_dofs
    p3 = 3 * geom.n_holes
    dofs = np.arange(n)
    A = np.empty((n + p3, n + p3))
    A[:n, :n] = operator_entries(geom, dofs, dofs, lam)
    if p3:
        A[:n, n:] = h_matrix(geom)
        A[n:, :n] = psi_t_matrix(geom)
        A[n:, n:] = -np.eye(p3)
    return A


def dense_solve(geom, f, lam=-0.5):
    """Exact discrete solution [mu; lambda] by LU with partial pivoting (LAPACK getrf/getrs)."""
    A = dense_system(geom, lam)
    f = np.asarray(f, dtype=np.float64)
    one = f.ndim == 1
    F = f.reshape(f.shape[0], -1)
    rhs = np.zeros((A.shape[0], F.shape[1]))
    rhs[: F.shape[0]] = F
    x = sla.lu_solve(sla.lu_factor(A), rhs)
    return x[:, 0] if one else x


def apply_system(geom, x, lam=-0.5, block=32, threads=None):
    """[f; 0] = A [mu; lambda] by on-the-fly evaluation (no dense matrix kept).

    Written out from the definitions: for every target node i,
      (D mu)_i = sum_{j != i} (w_j / pi) (r . n_j) / |r|^4 r (r . mu_j),  r = x_i - x_j
                 - (w_i kappa_i / (2 pi)) t_i (t_i . mu_i)          (curvature limit)
      (N mu)_i = n_i sum_j w_j (n_j . mu_j)                         (eq. null-spaceop)
    plus lam mu_i, H lambda, and the rows Psi^T mu - lambda.  The pair sums are
    taken for `block` target nodes at a time as products of the 2x2 kernel
    components (c r_a r_b, an (Mt, N) matrix each) with the density components,
    on `threads` host threads (NumPy releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    import os

    n = geom.n_dofs
    N = geom.n_nodes
    p3 = 3 * geom.n_holes
    xy, nr, w, kap = geom.xy, geom.normal, geom.weight, geom.curvature
    X = np.asarray(x, dtype=np.float64).reshape(n + p3, -1)
    out = np.zeros_like(X)
    mux = np.ascontiguousarray(X[0:n:2])
    muy = np.ascontiguousarray(X[1:n:2])
    yx = np.zeros_like(mux)
    yy = np.zeros_like(muy)

    def rows(t0):
        t1 = min(N, t0 + block)
        i = np.arange(t0, t1)
        rx = xy[i, 0][:, None] - xy[None, :, 0]
        ry = xy[i, 1][:, None] - xy[None, :, 1]
        r2 = rx * rx + ry * ry
        with np.errstate(divide="ignore", invalid="ignore"):
            c = (INV_PI * w[None, :]) * (rx * nr[None, :, 0] + ry * nr[None, :, 1]) / (r2 * r2)
        c[np.arange(i.size), i] = 0.0                  # the diagonal is the limit, below
        kxy = c * rx * ry
        yx[i] = (c * rx * rx) @ mux + kxy @ muy
        yy[i] = kxy @ mux + (c * ry * ry) @ muy

    nt = threads or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(rows, range(0, N, block)))
    tx, ty = -nr[:, 1], nr[:, 0]
    cs = -(w * kap) / (2.0 * np.pi)
    tmu = tx[:, None] * mux + ty[:, None] * muy
    yx += cs[:, None] * tx[:, None] * tmu
    yy += cs[:, None] * ty[:, None] * tmu
    s = (w * nr[:, 0])[:, None] * mux + (w * nr[:, 1])[:, None] * muy
    tot = s.sum(axis=0)[None, :]
    yx += nr[:, 0][:, None] * tot + lam * mux
    yy += nr[:, 1][:, None] * tot + lam * muy
    out[0:n:2] = yx
    out[1:n:2] = yy
    if p3:
        out[:n] += h_matrix(geom) @ X[n:]
        out[n:] = psi_t_matrix(geom) @ X[:n] - X[n:]
    return out


def evaluate_interior(geom, x, targets):
    """u = D mu + H lambda at off-boundary targets (eq. forwardeq); returns (M, 2) per column."""
    n = geom.n_dofs
    p = geom.n_holes
    X = np.asarray(x, dtype=np.float64).reshape(n + 3 * p, -1)
    blk = double_layer_blocks(targets, geom.xy, geom.normal, geom.weight)  # (M, N, 2, 2)
    M = targets.shape[0]
    Dm = blk.transpose(0, 2, 1, 3).reshape(2 * M, n)
    U = Dm @ X[:n]
    for h in range(p):
        c = geom.hole_xy[h]
        S = stokeslet_blocks(targets, c[None, :], np.ones(1))[:, 0]
        R = rotlet_columns(targets, c)
        U += S[:, :, 0].reshape(-1, 1) * X[n + 3 * h][None, :]
        U += S[:, :, 1].reshape(-1, 1) * X[n + 3 * h + 1][None, :]
        U += R.reshape(-1, 1) * X[n + 3 * h + 2][None, :]
    return U.reshape(M, 2, -1)
