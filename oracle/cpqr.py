"""Householder QR with column pivoting and the interpolative decomposition.

TEST INFRASTRUCTURE ONLY (see the package header).

Section 2.2 (eq. lowrank): a column-pivoted QR of a block splits its columns
into skeleton S and redundant R with M_R ~= M_S T, T = R11^{-1} R12, to a
tolerance eps.  Readings taken where the paper is silent:
  * pivot = remaining column of largest 2-norm, the norms recomputed from
    the trailing block at every step; an exact tie goes to the column that
    came first in the block's original order.  This is the default rule
    (`pivot="max"`), the plain column pivoting the paper names;
  * an optional rule (`pivot="key20"`) compares the squared norms on their
    leading 20 mantissa bits only (the low 32 bits of the float64 pattern
    cleared, a relative quantum of 2^-20), the first column winning among
    the columns tied at that precision.  Mirror-symmetric node pairs give
    columns whose norms agree up to rounding, and two implementations that
    sum in different orders pick different, equally valid, skeletons for
    them; the coarser comparison makes such choices reproducible.  Any
    choice within a factor 1 + 2^-20 of the largest norm keeps the
    rank-revealing property of the pivoting;
  * the tolerance is relative: step j counts toward the rank k while
    |R_jj| > eps |R_11|.

Pinned by tests/test_oracle_cpqr.py: same permutation and |R| as LAPACK
dgeqp3 on random matrices (default rule), the tie rules of both options,
exact rank on products of rank-k factors, and the ID residual bound.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def pivot_key(sq_norms: np.ndarray) -> np.ndarray:
    """Squared norms truncated to their leading 20 mantissa bits (the value
    the pivot rule compares; non-negative inputs, so truncation is monotone)."""
    bits = np.ascontiguousarray(sq_norms, dtype=np.float64).view(np.uint64)
    return (bits & np.uint64(0xFFFFFFFF00000000)).view(np.float64)


PIVOT_RULES = ("max", "key20")


class PivotedQR:
    """Pivoted Householder QR of a copy of M, one step at a time.

    pivot: "max" (largest remaining norm, exact ties to the first column) or
    "key20" (norms compared on their leading 20 mantissa bits)."""

    def __init__(self, M: np.ndarray, pivot: str = "max"):
        if pivot not in PIVOT_RULES:
            raise ValueError("pivot rule %r not in %r" % (pivot, PIVOT_RULES))
        self.A = np.array(M, dtype=np.float64, copy=True)
        self.m, self.n = self.A.shape
        self.perm = np.arange(self.n)
        self.steps = 0
        self.pivot = pivot

    @property
    def max_steps(self) -> int:
        return min(self.m, self.n)

    def step(self) -> float:
        """Take one pivoted Householder step; return |R_jj|."""
        j = self.steps
        A = self.A
        sub = A[j:, j:]
        norms = np.einsum("ij,ij->j", sub, sub)
        if self.pivot == "key20":
            norms = pivot_key(norms)
        mx = norms.max()
        cand = np.nonzero(norms == mx)[0]
        p = j + cand[np.argmin(self.perm[j + cand])]
        if p != j:
            A[:, [j, p]] = A[:, [p, j]]
            self.perm[[j, p]] = self.perm[[p, j]]
        x = A[j:, j]
        alpha = x[0]
        xnorm = np.linalg.norm(x[1:])
        if xnorm != 0.0:
            beta = -np.copysign(np.hypot(alpha, xnorm), alpha)
            v = x / (alpha - beta)
            v[0] = 1.0
            tau = (beta - alpha) / beta
            if j + 1 < self.n:
                w = v @ A[j:, j + 1:]
                A[j:, j + 1:] -= tau * np.outer(v, w)
            A[j, j] = beta
            A[j + 1:, j] = 0.0
        self.steps += 1
        return abs(A[j, j])

    def advance_to(self, k: int):
        while self.steps < min(k, self.max_steps):
            self.step()

    def rank(self, tol: float) -> int:
        """Number of steps with |R_jj| > tol * |R_11| (steps taken on demand)."""
        if self.max_steps == 0:
            return 0
        if self.steps == 0:
            self.step()
        r11 = abs(self.A[0, 0])
        if r11 == 0.0:
            return 0
        k = 0
        while True:
            if k >= self.steps:
                if self.steps >= self.max_steps:
                    return k
                self.step()
            if abs(self.A[k, k]) > tol * r11:
                k += 1
            else:
                return k

    def interpolation(self, k: int) -> np.ndarray:
        """T = R11^{-1} R12 for the first k pivots (k x (n - k))."""
        self.advance_to(k)
        if k == 0:
            return np.zeros((0, self.n))
        R11 = np.triu(self.A[:k, :k])
        R12 = self.A[:k, k:]
        return sla.solve_triangular(R11, R12, lower=False)

    def r_factor(self) -> np.ndarray:
        s = self.steps
        return np.triu(self.A[:s, :])
