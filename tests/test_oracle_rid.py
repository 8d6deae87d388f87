"""Pins of the interpolative and CUR decomposition oracle (Sec. 6).

* The column pivots equal greedy column selection written out here (at each
  step the column with the largest norm after projecting out the chosen
  ones), on small inputs.
* Exact rank k: A = C Z and A = C U R to rounding, and Z holds the identity
  at the chosen columns.
* The randomized ID picks the same columns as the deterministic one when B
  = Q^T A keeps all of A's information (rank(A) <= l): B's columns have the
  same norms and inner products as A's (Q has orthonormal columns), so
  greedy pivoting takes the same path.
"""
import numpy as np
import pytest

from oracle import rid as orid
from synth import matrices as syn


def greedy_columns(A, k):
    """Greedy column selection by largest residual norm (Gram-Schmidt form of
    column-pivoted QR)."""
    R = np.array(A, dtype=np.float64)
    chosen = []
    for _ in range(k):
        norms = np.sum(R * R, axis=0)
        norms[chosen] = -1.0
        j = int(np.argmax(norms))
        chosen.append(j)
        u = R[:, j] / np.linalg.norm(R[:, j])
        R = R - np.outer(u, u @ R)
    return np.array(chosen)


@pytest.mark.parametrize("m,n,k,seed", [(12, 20, 5, 1), (40, 30, 8, 2), (25, 60, 10, 3)])
def test_pivots_are_greedy_column_selection(m, n, k, seed):
    A = np.random.default_rng(seed).standard_normal((m, n))
    _, _, P = orid.cpqr(A)
    assert np.array_equal(P[:k], greedy_columns(A, k))


def test_exact_rank_id_and_cur_reproduce_the_matrix():
    rng = np.random.default_rng(4)
    m, n, k = 120, 90, 7
    A = rng.standard_normal((m, k)) @ rng.standard_normal((k, n))
    C, Z, J = orid.interp_decomp(A, k)
    np.testing.assert_allclose(Z[:, J], np.eye(k), atol=1e-14)
    np.testing.assert_allclose(C @ Z, A, atol=1e-10 * np.abs(A).max())
    Cr, Zr, Jr = orid.rid(A, k, p=5, q=1, seed=3)
    np.testing.assert_allclose(Cr @ Zr, A, atol=1e-9 * np.abs(A).max())
    cur = orid.rcur(A, k, p=5, q=1, seed=3)
    np.testing.assert_allclose(cur["C"] @ cur["U"] @ cur["R"], A, atol=1e-8 * np.abs(A).max())
    assert len(set(cur["I"].tolist())) == k and len(set(cur["J"].tolist())) == k
    np.testing.assert_array_equal(cur["R"], A[cur["I"]])


def test_randomized_id_picks_the_deterministic_columns():
    m, n, k, r = 400, 150, 12, 20
    A = syn.planted(m, n, np.exp(-np.arange(r) / 4.0), 5)       # rank 20 <= l = 22
    _, _, J = orid.interp_decomp(A, k)
    _, _, Jr = orid.rid(A, k, p=10, q=0, seed=6)
    assert np.array_equal(J, Jr)


def test_id_error_is_close_to_the_optimum():
    """Approximation quality (Sec. 6.3): on a planted spectrum the ID error
    stays within a modest factor of the rank-k optimum sigma_{k+1}."""
    m, n, k = 300, 200, 10
    sig = np.exp(-np.arange(n) / 5.0)
    A = syn.planted(m, n, sig, 7)
    C, Z, J = orid.rid(A, k, p=10, q=2, seed=8)
    err = np.linalg.norm(A - C @ Z, 2)
    assert sig[k] <= err <= 20 * sig[k]
