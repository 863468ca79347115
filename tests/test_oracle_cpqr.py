"""Pins of the oracle's pivoted QR / interpolative decomposition (Section 2.2).

* On matrices whose column norms are distinct at every step, the pivot
  order and |R| equal LAPACK dgeqp3's (scipy.linalg.qr(pivoting=True)).
* ID accuracy: ||M_R - M_S T||_2 <= sqrt(k (n - k) + 1) |R_{k+1,k+1}| ... up
  to the factor of the strong rank-revealing bound, checked with margin.
* Exact rank: a product of rank-k factors gives rank k at tolerance 1e-10.
* Tie rules: the default rule ("max") takes the largest norm and only an
  exact tie goes to the first column; the optional "key20" rule also ties
  norms equal to 2^-20 relative.  Both rules give the same ranks and IDs of
  the same accuracy on generic matrices.
"""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle.cpqr import PivotedQR


@pytest.mark.parametrize("shape", [(40, 12), (200, 64), (30, 50)])
def test_matches_lapack_geqp3(shape):
    rng = np.random.Generator(np.random.PCG64(7))
    m, n = shape
    M = rng.standard_normal((m, n)) * np.logspace(0, -3, n)[None, :]
    q = PivotedQR(M)
    q.advance_to(min(m, n))
    _, R, P = sla.qr(M, pivoting=True, mode="economic")
    assert np.array_equal(q.perm, P)
    Ro = q.r_factor()
    kk = min(m, n)
    assert np.allclose(np.abs(Ro[:kk]), np.abs(R[:kk]), rtol=1e-10, atol=1e-13)


def test_rank_and_id_bound():
    rng = np.random.Generator(np.random.PCG64(3))
    m, n, k = 300, 80, 23
    M = rng.standard_normal((m, k)) @ rng.standard_normal((k, n))
    M += 1e-13 * rng.standard_normal((m, n))
    q = PivotedQR(M)
    kk = q.rank(1e-10)
    assert kk == k
    T = q.interpolation(kk)
    S, Rr = q.perm[:kk], q.perm[kk:]
    err = np.linalg.norm(M[:, Rr] - M[:, S] @ T, 2)
    q.advance_to(kk + 1)
    rkk = abs(q.A[kk, kk])
    assert err <= np.sqrt(kk * (n - kk) + 1) * rkk * 10 + 1e-14
    assert err < 1e-10 * np.linalg.norm(M, 2)


def test_tie_break_prefers_first_column():
    M = np.array([[1.0, 0.0, 1.0], [0.0, 1.0, 0.0]])
    q = PivotedQR(M)
    q.step()
    assert q.perm[0] == 0


def test_plain_rule_takes_largest_norm_by_ulps():
    """Default rule: a norm larger by a few ulps wins; only exact ties go to
    the first column."""
    M = np.array([[1.0, 0.0, 1.0 + 4e-16], [0.0, 1.0, 0.0], [0.0, 0.0, 0.0]])
    q = PivotedQR(M)
    q.step()
    assert q.perm[0] == 2
    M2 = np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 0.0]])
    q2 = PivotedQR(M2)
    q2.step()
    assert q2.perm[0] == 0


def test_key20_near_tie_goes_to_first_column():
    """key20 rule: norms that agree to 2^-20 count as tied and the earlier
    column wins even when the later one is larger by a few ulps."""
    M = np.array([[1.0, 0.0, 1.0 + 4e-16], [0.0, 1.0, 0.0], [0.0, 0.0, 0.0]])
    q = PivotedQR(M, pivot="key20")
    q.step()
    assert q.perm[0] == 0
    # a genuine difference (1e-5 relative) is not a tie
    M2 = np.array([[1.0, 0.0, 1.0 + 1e-5], [0.0, 1.0, 0.0]])
    q2 = PivotedQR(M2, pivot="key20")
    q2.step()
    assert q2.perm[0] == 2


def test_rules_agree_on_generic_matrices():
    """On matrices without near-ties the two rules take the same pivots."""
    rng = np.random.Generator(np.random.PCG64(21))
    M = rng.standard_normal((120, 40)) * np.logspace(0, -6, 40)[None, :]
    a, b = PivotedQR(M), PivotedQR(M, pivot="key20")
    assert a.rank(1e-4) == b.rank(1e-4)
    a.advance_to(40)
    b.advance_to(40)
    assert np.array_equal(a.perm, b.perm)


def test_unknown_rule_rejected():
    with pytest.raises(ValueError):
        PivotedQR(np.eye(3), pivot="nearest")


def test_pivot_key_is_truncation():
    from oracle.cpqr import pivot_key

    x = np.array([1.0, 1.0 + 2.0 ** -21, 1.0 + 2.0 ** -19, 3.5, 0.0])
    k = pivot_key(x)
    assert k[0] == k[1] == 1.0           # below the 2^-20 quantum: tied
    assert k[2] == 1.0 + 2.0 ** -19      # representable in 20 bits: kept
    assert k[3] == 3.5 and k[4] == 0.0
    assert np.all(k <= x)


def test_zero_matrix_rank_zero():
    q = PivotedQR(np.zeros((5, 3)))
    assert q.rank(1e-10) == 0
