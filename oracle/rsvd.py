"""FP64 oracle of the randomized SVD and PCA (TEST INFRASTRUCTURE ONLY).

Follows Erichson et al., arXiv:1608.02148, step by step:

* Alg. rqb (Sec. 3.3): l = k + p; Omega = n x l test matrix; Y = A Omega;
  Y = sub_iterations(A, Y, q); Q = qr(Y); B = Q^T A.
* Alg. subspace_iter (Sec. 2.2, "Power iteration scheme"): q times
  Q = qr(Y); Q = qr(A^T Q); Y = A Q.
* Alg. normalized_iter (Sec. 2.2): the same with the pivoted LU factor L in
  place of Q (L = lu(Y); L = lu(A^T L); Y = A L).
* Alg. RSVDalgorithm (Sec. 3.3): [U~, S, V] = svd(B); U = Q U~; keep the
  first k columns / values.
* Alg. RPCAalgorithm (Sec. 4.2): run the randomized SVD on the column-centred
  data; eigenvalues S^2 / (m - 1); principal components U S; rotation V.

Readings where the paper is silent (each listed in the design notes):

* QR: thin Householder QR (LAPACK via numpy) with the signs fixed so that
  R has a non-negative diagonal.
* Pivoted LU: partial row pivoting (LAPACK via scipy); L is the row-permuted
  unit lower trapezoidal factor, Y = L U (the two-output form of lu).
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


def lu_factor(Y):
    """Pivoted LU of the paper's normalized power iterations: partial (row)
    pivoting, Y = L U with L the row-permuted unit lower trapezoidal factor
    (m x l) and U upper triangular (l x l).  Returns (L, U, piv), piv[i] the
    row of Y chosen at step i (so L[piv] is unit lower triangular)."""
    import scipy.linalg
    P, Lt, U = scipy.linalg.lu(Y)              # Y = P Lt U
    piv = np.argmax(P[:, :Y.shape[1]], axis=0)  # step i takes row piv[i] of Y
    return P @ Lt, U, piv


def norm_iterations(A, Y, q):
    """Alg. normalized_iter: q power iterations normalised by pivoted LU
    (Rokhlin, Szlam & Tygert 2009): L = lu(Y); L = lu(A^T L); Y = A L.
    L spans the same space as the matrix it factors, so the result matches
    Alg. subspace_iter in exact arithmetic."""
    for _ in range(q):
        L, _, _ = lu_factor(Y)
        L, _, _ = lu_factor(A.T @ L)
        Y = A @ L
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


def rqb(A, k, p=10, q=2, seed=0, stream_id=0, sdist="normal", scheme="qr"):
    """Alg. rqb: randomized QB decomposition.  Returns (Q, B, Omega).

    scheme: "qr" (Alg. subspace_iter) or "lu" (Alg. normalized_iter)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    check_args(m, n, k, p, q)
    l = sketch_width(m, n, k, p)
    omega = philox.test_matrix(n, l, seed, stream_id, sdist)
    Y = A @ omega
    Y = norm_iterations(A, Y, q) if scheme == "lu" else sub_iterations(A, Y, q)
    Q, _ = hqr(Y)
    B = Q.T @ A
    return Q, B, omega


def sign_rule(U, V):
    """Flip each pair (u_i, v_i) so that max-|.| entry of v_i is positive."""
    idx = np.argmax(np.abs(V), axis=0)
    s = np.sign(V[idx, np.arange(V.shape[1])])
    s[s == 0] = 1.0
    return U * s[None, :], V * s[None, :]


def rsvd(A, k, p=10, q=2, seed=0, stream_id=0, sdist="normal", full=False, scheme="qr"):
    """Alg. RSVDalgorithm.  Returns (U m x k, s k, V n x k), V not transposed.

    With ``full=True`` also returns a dict holding Q, B, Omega and the
    untruncated factors for diagnostics.  scheme: normalisation of the power
    iterations ("qr" subspace iterations, "lu" normalized iterations).
    """
    Q, B, omega = rqb(A, k, p, q, seed, stream_id, sdist, scheme)
    Ut, s, Vt = np.linalg.svd(B, full_matrices=False)
    U = Q @ Ut
    V = Vt.T
    U, V = sign_rule(U, V)
    Uk, sk, Vk = U[:, :k].copy(), s[:k].copy(), V[:, :k].copy()
    if full:
        return Uk, sk, Vk, dict(Q=Q, B=B, omega=omega, U=U, s=s, V=V)
    return Uk, sk, Vk


def column_scales(A, c):
    """Column scalings of Sec. 4.3's scale option: the root mean square of
    each column about c (the column means when centring, else zero) with the
    m - 1 divisor, i.e. the column standard deviation when centring.  A zero
    scale (a constant column) is replaced by 1: the column then stays zero
    after centring instead of dividing by zero."""
    A = np.asarray(A, dtype=np.float64)
    d = A - c[None, :]
    s = np.sqrt(np.sum(d * d, axis=0) / (A.shape[0] - 1))
    zero = s == 0
    s[zero] = 1.0
    return s, zero


def rpca(A, k, p=10, q=2, center=True, seed=0, stream_id=0, sdist="normal", scale=False):
    """Alg. RPCAalgorithm with explicit centring and scaling (Sec. 4.2 and 4.3).

    The data are X = (A - 1 mu^T) D^-1 with mu the column means (center) and
    D the column scalings (scale, see column_scales; identity otherwise),
    formed explicitly.  Returns a dict with rotation (n x k), eigvals = s^2 /
    (m - 1), sdev, x = U S (m x k), center, scale (ones when not scaling),
    loadings = rotation diag(sdev) and x_white = x diag(1 / sdev) (the
    whitened components, Sec. 4.1; zero where sdev = 0), and total_var, the
    sum of the column variances of X (the trace of its covariance, so that
    eigvals / total_var are the explained proportions of Sec. 4.1).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    mu = A.mean(axis=0) if center else np.zeros(n)
    if scale:
        sc, zero = column_scales(A, mu)
    else:
        sc, zero = np.ones(n), np.zeros(n, dtype=bool)
    X = (A - mu[None, :]) / sc[None, :]
    U, s, V = rsvd(X, k, p, q, seed, stream_id, sdist)
    eigvals = s ** 2 / (m - 1)
    sdev = np.sqrt(eigvals)
    x = U * s[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        x_white = np.where(sdev[None, :] > 0, x / sdev[None, :], 0.0)
    return dict(rotation=V, eigvals=eigvals, sdev=sdev, x=x, center=mu, s=s, U=U, scale=sc,
                zero_scale=zero, loadings=V * sdev[None, :], x_white=x_white,
                total_var=float(np.sum(X * X)) / (m - 1))


def rpca_predict(model, A_new):
    """Principal components of new rows (the predict step of Sec. 4.4): the rows are
    centred and scaled with the model's centre and scalings, then rotated:
    ((A_new - 1 center^T) D^-1) rotation."""
    A_new = np.asarray(A_new, dtype=np.float64)
    X = (A_new - model["center"][None, :]) / model["scale"][None, :]
    return X @ model["rotation"]


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
