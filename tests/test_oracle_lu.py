"""Pins of the oracle's normalized power iterations (Alg. normalized_iter).

* The LU factor matches Gaussian elimination with partial pivoting written
  out here element by element (brute force on small inputs): same pivot
  rows, same factors.
* L spans the column space of the factored matrix, so the rSVD with LU
  normalisation equals the one with subspace iterations (QR) up to rounding
  on well-conditioned inputs, and the direct power scheme of Alg.
  poweriter_direct for a small q.
"""
import numpy as np
import pytest

from oracle import rsvd as orc
from synth import matrices as syn


def gepp(Y):
    """Textbook Gaussian elimination with partial pivoting on a copy of Y
    (m x l, m >= l): returns (L m x l with rows in Y's order, U, piv)."""
    Y = np.array(Y, dtype=np.float64)
    m, l = Y.shape
    order = list(range(m))
    W = Y.copy()
    for j in range(l):
        cand = [abs(W[order[i], j]) for i in range(j, m)]
        p = j + int(np.argmax(cand))
        order[j], order[p] = order[p], order[j]
        piv = W[order[j], j]
        for i in range(j + 1, m):
            r = order[i]
            f = W[r, j] / piv
            W[r, j] = f
            for c in range(j + 1, l):
                W[r, c] -= f * W[order[j], c]
    L = np.zeros((m, l))
    U = np.zeros((l, l))
    for i in range(m):
        r = order[i]
        if i < l:
            L[r, :i] = W[r, :i]
            L[r, i] = 1.0
            U[i, i:] = W[r, i:]
        else:
            L[r, :] = W[r, :l]
    return L, U, np.array(order[:l])


@pytest.mark.parametrize("m,l,seed", [(12, 5, 1), (30, 7, 2), (9, 9, 3), (40, 3, 4)])
def test_lu_factor_matches_textbook_gepp(m, l, seed):
    Y = np.random.default_rng(seed).standard_normal((m, l))
    L, U, piv = orc.lu_factor(Y)
    Lb, Ub, pivb = gepp(Y)
    assert np.array_equal(piv, pivb)
    np.testing.assert_allclose(L, Lb, atol=1e-13)
    np.testing.assert_allclose(U, Ub, atol=1e-13)
    np.testing.assert_allclose(L @ U, Y, atol=1e-13)
    assert np.all(np.abs(L) <= 1.0 + 1e-15)
    np.testing.assert_allclose(L[piv], np.tril(L[piv]), atol=0)
    np.testing.assert_allclose(np.diag(L[piv]), 1.0, atol=0)


@pytest.mark.parametrize("q", [1, 2, 3])
def test_lu_iterations_match_subspace_iterations(q):
    m, n, k, p = 600, 300, 10, 10
    A = syn.planted(m, n, syn.spectrum("exp", n, tau=15.0), 21)
    Uq, sq, Vq = orc.rsvd(A, k, p=p, q=q, seed=5)
    Ul, sl, Vl = orc.rsvd(A, k, p=p, q=q, seed=5, scheme="lu")
    np.testing.assert_allclose(sl, sq, rtol=1e-10)
    np.testing.assert_allclose(Ul, Uq, atol=1e-8)
    np.testing.assert_allclose(Vl, Vq, atol=1e-8)


def test_lu_iterations_span_the_direct_power_scheme():
    """q = 1 on a well-conditioned matrix: the normalised sketch spans
    (A A^T) A Omega, the direct scheme's sketch."""
    A = syn.planted(200, 120, np.linspace(2.0, 1.0, 120), 22)
    Om = np.random.default_rng(23).standard_normal((120, 12))
    Y1 = orc.norm_iterations(A, A @ Om, 1)
    Y2 = orc.power_iterations(A, A @ Om, 1)
    Q1, _ = np.linalg.qr(Y1)
    Q2, _ = np.linalg.qr(Y2)
    s = np.linalg.svd(Q1.T @ Q2, compute_uv=False)
    np.testing.assert_allclose(s, 1.0, atol=1e-12)
