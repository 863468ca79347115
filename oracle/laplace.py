"""The Laplace Neumann formulation of the paper's Section 4.4.1 (heat flux on
the boundary of a multiply-connected domain), written out densely.

TEST INFRASTRUCTURE ONLY (see the package header).

Section 4.4.1 replaces the Stokes pair of Section 3.1 by
  * the representation u = S mu, S the Laplace single layer with kernel
    -(1/(2 pi)) log|x - y|;
  * the boundary equation f = (-I/2 - D + N) mu, D the adjoint double layer
    with kernel -(1/(2 pi)) ((x - y) . n(x)) / |x - y|^2 (the normal at the
    target), and no augmentation (the operator is full rank).
N is the rank-one completion N mu = integral of mu over the whole boundary
(read: the section does not restate N; this is the standard choice that
removes the one-dimensional null space of -I/2 - D, see the pins).  n is the
unit normal pointing out of the domain (the convention of Section 3.1), so
-I/2 - D is the interior limit of -d(S mu)/dn and f is the flux of u along
the normal pointing into the domain.

Discretisation: the trapezoid (Nystrom) rule at the nodes with weights w;
the diagonal of D is the smooth kernel's limit along the curve,
-(1/(2 pi)) kappa / 2 times the weight, kappa the signed curvature (positive
where the curve bends away from n).

Pins (tests/test_oracle_laplace.py):
  * Circle closed form: on a circle of radius R every entry of -D, the
    diagonal included, is w_j / (4 pi R), so (-I/2 - D) 1 = 0.
  * Range / null space: w^T (-I/2 - D) = 0 to quadrature accuracy on a
    multiply-connected boundary (the range is orthogonal to constants), the
    discrete -I/2 - D has one tiny singular value, and -I/2 - D + N is well
    conditioned.
  * Scale of N: for f = 1, sum_j w_j mu_j = 1.
  * Exact harmonic solutions: for u = sum_k q_k log|x - s_k| + a . x with
    the s_k outside the domain and f its inward flux, S mu reproduces u at
    interior points up to one constant, to spectral accuracy.
  * The x-derivative of S mu against central differences of S mu.
"""

from __future__ import annotations

import numpy as np

INV_2PI = 1.0 / (2.0 * np.pi)


def minus_adjoint_dl(tx, tn, sy, sw):
    """-D between distinct points, Section 4.4.1:

        (1/(2 pi)) ((x - y) . n(x)) / |x - y|^2 * w_y

    tx (Mt, 2) targets with normals tn, sy (Ms, 2) sources with weights sw.
    Returns (Mt, Ms); coincident pairs are not allowed."""
    r = tx[:, None, :] - sy[None, :, :]
    r2 = np.einsum("ijk,ijk->ij", r, r)
    rn = np.einsum("ijk,ik->ij", r, tn)
    return INV_2PI * rn / r2 * sw[None, :]


def minus_adjoint_dl_self(weight, curvature):
    """Diagonal of -D: (x - y) . n(x) / |x - y|^2 tends to kappa / 2 as y -> x
    along the curve, so the entry is kappa w / (4 pi)."""
    return curvature * weight * (INV_2PI / 2.0)


def operator_matrix(g, lam: float = -0.5):
    """Dense lam I - D + N (N x N), the operator of Section 4.4.1 with lam = -1/2."""
    return operator_rows(g, np.arange(g.n_nodes), lam)


def operator_rows(g, rows, lam: float = -0.5):
    """Rows `rows` of lam I - D + N (all of them for the dense operator, a
    sample for checks at sizes where the dense matrix does not fit)."""
    rows = np.asarray(rows)
    out = np.empty((rows.size, g.n_nodes))
    for k0 in range(0, rows.size, 512):            # row blocks bound the temporaries
        rb = rows[k0:k0 + 512]
        blk = out[k0:k0 + rb.size]
        # the diagonal's pairs are coincident: give them a harmless offset,
        # then overwrite them with the curvature limit
        r = g.xy[rb][:, None, :] - g.xy[None, :, :]
        r[np.arange(rb.size), rb] = 1.0
        r2 = np.einsum("ijk,ijk->ij", r, r)
        rn = np.einsum("ijk,ik->ij", r, g.normal[rb])
        blk[:] = INV_2PI * rn / r2 * g.weight[None, :]
        blk[np.arange(rb.size), rb] = minus_adjoint_dl_self(g.weight[rb], g.curvature[rb]) + lam
        blk += g.weight[None, :]                  # N: every row integrates mu
    return out


def solve(g, f, lam: float = -0.5):
    """mu = (lam I - D + N)^-1 f by a dense LU solve; f (N,) or (N, ncols)."""
    return np.linalg.solve(operator_matrix(g, lam), f)


def single_layer(g, mu, targets):
    """u = S mu at targets off the boundary: -(1/(2 pi)) sum_j log|x - y_j| w_j mu_j."""
    T = np.asarray(targets, dtype=np.float64).reshape(-1, 2)
    r = T[:, None, :] - g.xy[None, :, :]
    lg = 0.5 * np.log(np.einsum("ijk,ijk->ij", r, r))
    return -INV_2PI * (lg * g.weight[None, :]) @ mu


def single_layer_dx(g, mu, targets):
    """d(S mu)/dx at targets: -(1/(2 pi)) sum_j (x - y_j)_1 / |x - y_j|^2 w_j mu_j."""
    T = np.asarray(targets, dtype=np.float64).reshape(-1, 2)
    r = T[:, None, :] - g.xy[None, :, :]
    r2 = np.einsum("ijk,ijk->ij", r, r)
    return -INV_2PI * (r[:, :, 0] / r2 * g.weight[None, :]) @ mu


def neumann_data(curve_id):
    """The flux data of Section 4.4.1's eq. (neumanndata): 0 on the outer
    curve, +1 on the first hole, -1 on the second."""
    c = np.asarray(curve_id)
    return np.where(c == 1, 1.0, np.where(c == 2, -1.0, 0.0))
