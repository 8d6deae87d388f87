"""FP64 oracle of the randomized robust PCA (TEST INFRASTRUCTURE ONLY).

Follows Alg. rpca (Sec. 5.2, the inexact augmented Lagrange multiplier
method of Eq. IALM with the randomized SVD of Alg. RSVDalgorithm as its
workhorse): A = L + S with L low rank and S sparse.

    k = 2; mu = 1.25 / ||A||_2; Z = A / J(A); S = 0
    repeat
        U, s, V = rsvd(A - S + Z / mu, k, p, q)
        l = #{s_i > 1/mu};  k = next target rank
        L = U[:, :l] diag(s[:l] - 1/mu) V[:, :l]^T
        S = shrink(A - L + Z / mu, lambda / mu)
        Z = Z + mu (A - L - S)
        mu = min(rho mu, mu_max)
    until ||A - L - S||_F / ||A||_F < tol or maxiter iterations

Readings where the paper defers to Lin, Chen & Ma (2010, "The augmented
Lagrange multiplier method for exact recovery of corrupted low-rank
matrices", arXiv:1009.5055, the inexact ALM algorithm), each listed in the
design notes:

* mu's start: the listing prints 1.25 ||A||_2, which would make 1/mu, the
  singular-value threshold, tiny; the inexact ALM starts from
  mu = 1.25 / ||A||_2, read here.
* dual_norm(A) = J(A) = max(||A||_2, ||A||_max / lambda), the dual of the
  combined norm of the Lagrangian, so that Z starts feasible.
* mu grows by rho = 1.6 per iteration (the inexact ALM's choice), capped at
  mu_max = 1e7 mu_0.
* predict_rank: l = the number of singular values above the threshold 1/mu;
  the next target rank is l + 1 when l < k, else l + round(0.05 min(m, n)),
  clamped to [1, k_max].
* The stopping test is the relative residual of the constraint A = L + S.
* lambda defaults to max(m, n)^-1/2 (Sec. 5.4).
* ||A||_2 is taken from the randomized SVD itself (rank 1, same p, q), the
  estimate the method has at hand; the exact value is the same to its
  accuracy on the inputs used here.
"""
import math

import numpy as np

from . import rsvd as orc


def shrink(X, tau):
    """Soft thresholding, the proximal map of tau ||.||_1: sign(x) max(|x| - tau, 0)."""
    return np.sign(X) * np.maximum(np.abs(X) - tau, 0.0)


def next_rank(l, k, m, n, k_max):
    """Target rank for the next iteration from the number l of singular
    values above the threshold (the inexact ALM's rank prediction)."""
    if l < k:
        k = l + 1
    else:
        k = l + int(round(0.05 * min(m, n)))
    return int(min(max(k, 1), k_max))


def rrpca(A, lam=None, maxiter=50, tol=1e-5, p=10, q=2, seed=0, rho=1.6, k_max=None):
    """Alg. rpca.  Returns dict(L, S, iterations, rank (the last l), residual)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    lam = 1.0 / math.sqrt(max(m, n)) if lam is None else float(lam)
    if k_max is None:
        k_max = min(m, n) - 1
    k_max = min(k_max, min(m, n) - 1)
    _, s1, _ = orc.rsvd(A, 1, p=p, q=q, seed=seed)
    norm2 = float(s1[0])
    normF = float(np.linalg.norm(A))
    mu = 1.25 / norm2
    mu_max = mu * 1e7
    J = max(norm2, float(np.max(np.abs(A))) / lam)
    Z = A / J
    S = np.zeros_like(A)
    L = np.zeros_like(A)
    k = 2
    it, l, res = 0, 0, float("inf")
    for it in range(1, maxiter + 1):
        U, s, V = orc.rsvd(A - S + Z / mu, k, p=p, q=q, seed=seed)
        l = int(np.sum(s > 1.0 / mu))
        k = next_rank(l, k, m, n, k_max)
        L = (U[:, :l] * (s[:l] - 1.0 / mu)[None, :]) @ V[:, :l].T
        S = shrink(A - L + Z / mu, lam / mu)
        R = A - L - S
        Z = Z + mu * R
        mu = min(rho * mu, mu_max)
        res = float(np.linalg.norm(R)) / normF
        if res < tol:
            break
    return dict(L=L, S=S, iterations=it, rank=l, residual=res, Z=Z, lam=lam)
