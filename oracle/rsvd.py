"""FP64 oracle of the randomized SVD and PCA (TEST INFRASTRUCTURE ONLY).

Follows Erichson et al., arXiv:1608.02148, step by step:

* Alg. rqb (Sec. 3.3): l = k + p; Omega = n x l test matrix; Y = A Omega;
  Y = sub_iterations(A, Y, q); Q = qr(Y); B = Q^T A.
* Alg. subspace_iter (Sec. 2.2, "Power iteration scheme"): q times
  Q = qr(Y); Q = qr(A^T Q); Y = A Q.
* Alg. RSVDalgorithm (Sec. 3.3): [U~, S, V] = svd(B); U = Q U~; keep the
  first k columns / values.
* Alg. RPCAalgorithm (Sec. 4.2): run the randomized SVD on the column-centred
  data; eigenvalues S^2 / (m - 1); principal components U S; rotation V.

Readings where the paper is silent (each listed in the design notes):

* QR: thin Householder QR (LAPACK via numpy) with the signs fixed so that
  R has a non-negative diagonal.
* k + p larger than min(m, n): l is clamped to min(m, n).
* Omega is always n x l, whatever the aspect ratio (Alg. rqb).
* Sign of singular vector pairs: (u_i, v_i) is flipped together so that the
  entry of v_i with the largest magnitude is positive (lowest index on ties).
* rPCA divides by m - 1 whether or not the data were centred; x = U S.
"""
import math

import numpy as np

from . import philox


def check_args(m, n, k, p, q):
    """Argument rules of the rsvd interface (Sec. 3.6): 1 <= k < min(m, n)."""
    if m < 1 or n < 1:
        raise ValueError("m and n must be positive")
    if k < 1 or k >= min(m, n):
        raise ValueError("k must satisfy 1 <= k < min(m, n)")
    if p < 0 or q < 0:
        raise ValueError("p and q must be non-negative")


def sketch_width(m, n, k, p):
    """l = k + p (Alg. rqb), clamped to min(m, n)."""
    return min(k + p, min(m, n))


def hqr(Y):
    """Economic QR (the paper's ``qr``), Q with R_ii >= 0.  Returns (Q, R)."""
    Q, R = np.linalg.qr(Y, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def sub_iterations(A, Y, q):
    """Alg. subspace_iter: q subspace iterations, re-orthonormalised each half."""
    for _ in range(q):
        Q, _ = hqr(Y)
        Q, _ = hqr(A.T @ Q)
        Y = A @ Q
    return Y


def power_iterations(A, Y, q):
    """Alg. poweriter_direct: the direct power scheme, no re-orthonormalisation.

    Kept only as an independent cross-check of sub_iterations (the paper advises
    against it in practice because of round-off).
    """
    for _ in range(q):
        Y = A.T @ Y
        Y = A @ Y
    return Y


def rqb(A, k, p=10, q=2, seed=0, stream_id=0, sdist="normal"):
    """Alg. rqb: randomized QB decomposition.  Returns (Q, B, Omega)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    check_args(m, n, k, p, q)
    l = sketch_width(m, n, k, p)
    omega = philox.test_matrix(n, l, seed, stream_id, sdist)
    Y = A @ omega
    Y = sub_iterations(A, Y, q)
    Q, _ = hqr(Y)
    B = Q.T @ A
    return Q, B, omega


def sign_rule(U, V):
    """Flip each pair (u_i, v_i) so that max-|.| entry of v_i is positive."""
    idx = np.argmax(np.abs(V), axis=0)
    s = np.sign(V[idx, np.arange(V.shape[1])])
    s[s == 0] = 1.0
    return U * s[None, :], V * s[None, :]


def rsvd(A, k, p=10, q=2, seed=0, stream_id=0, sdist="normal", full=False):
    """Alg. RSVDalgorithm.  Returns (U m x k, s k, V n x k), V not transposed.

    With ``full=True`` also returns a dict holding Q, B, Omega and the
    untruncated factors for diagnostics.
    """
    Q, B, omega = rqb(A, k, p, q, seed, stream_id, sdist)
    Ut, s, Vt = np.linalg.svd(B, full_matrices=False)
    U = Q @ Ut
    V = Vt.T
    U, V = sign_rule(U, V)
    Uk, sk, Vk = U[:, :k].copy(), s[:k].copy(), V[:, :k].copy()
    if full:
        return Uk, sk, Vk, dict(Q=Q, B=B, omega=omega, U=U, s=s, V=V)
    return Uk, sk, Vk


def rpca(A, k, p=10, q=2, center=True, seed=0, stream_id=0, sdist="normal"):
    """Alg. RPCAalgorithm with explicit centring (Sec. 4.2 and 4.4).

    Returns a dict with rotation (n x k), eigvals, sdev, x (m x k), center.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    mu = A.mean(axis=0) if center else np.zeros(n)
    X = A - mu[None, :]
    U, s, V = rsvd(X, k, p, q, seed, stream_id, sdist)
    eigvals = s ** 2 / (m - 1)
    return dict(rotation=V, eigvals=eigvals, sdev=np.sqrt(eigvals),
                x=U * s[None, :], center=mu, s=s, U=U)


# --------------------------------------------------------------- diagnostics

def eckart_young(svals, k):
    """Optimal rank-k errors (Sec. 3.2): (sigma_{k+1}, sqrt(sum_{j>k} sigma_j^2))."""
    svals = np.asarray(svals, dtype=np.float64)
    spec = svals[k] if k < len(svals) else 0.0
    return spec, math.sqrt(float(np.sum(svals[k:] ** 2)))


def expected_error_factor(m, n, k, p, q):
    """Bracket of Eq. rsvd_expected_error (Sec. 3.4), valid for p >= 2.

    E||A - A_k||_2 <= factor * sigma_{k+1}(A).
    """
    if p < 2:
        raise ValueError("the bound assumes p >= 2")
    inner = (1.0 + math.sqrt(k / (p - 1))
             + math.e * math.sqrt(k + p) / p * math.sqrt(min(m, n) - k))
    return inner ** (1.0 / (2 * q + 1))


def lowrank_residual(A, U, s, V, ord="fro"):
    """||A - U diag(s) V^T|| in the Frobenius ("fro") or spectral (2) norm."""
    R = np.asarray(A, dtype=np.float64) - (U * s[None, :]) @ V.T
    return float(np.linalg.norm(R, ord))


def projection_residual(A, Q, ord="fro"):
    """||A - Q Q^T A|| (Eq. AQQA)."""
    A = np.asarray(A, dtype=np.float64)
    R = A - Q @ (Q.T @ A)
    return float(np.linalg.norm(R, ord))
