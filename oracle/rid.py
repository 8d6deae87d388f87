"""FP64 oracle of the randomized interpolative and CUR decompositions (TEST
INFRASTRUCTURE ONLY).

Follows Sec. 6 of the paper:

* Alg. id (column ID): column-pivoted QR A P = Q S; T = pinv(S[:k, :k])
  S[:k, k:]; Z[:, P] = [I_k, T]; J = P[:k]; C = A[:, J].  Then A ~ C Z.
* Alg. rid: [Q, B] = rqb(A, k, p, q); the ID of B gives Z and J; C = A[:, J]
  (the ID is computed on B, as the paper advocates).
* Alg. rcur: C, Z, J = rid(A, k, p, q); the column-pivoted QR of C^T picks the
  row indices I = P[:k]; R = A[I, :]; U = Z pinv(R).  Then A ~ C U R.

Readings (listed in the design notes): the listing of Alg. rid calls
rqb(A, k, q, p) with p and q swapped and returns "V" for Z; read as
rqb(A, k, p, q) returning Z.  The pivoted QR is Businger-Golub column
pivoting (the largest remaining column norm at each step, LAPACK's geqp3 via
scipy); pinv is the SVD-based pseudoinverse (numpy).
"""
import numpy as np
import scipy.linalg

from . import rsvd as orc


def cpqr(A):
    """Column-pivoted QR A[:, P] = Q S.  Returns (Q, S, P)."""
    Q, S, P = scipy.linalg.qr(np.asarray(A, dtype=np.float64), mode="economic", pivoting=True)
    return Q, S, P


def interp_decomp(A, k):
    """Alg. id: (C m x k, Z k x n, J k) with A ~ C Z and Z[:, J] = I."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    _, S, P = cpqr(A)
    T = np.linalg.pinv(S[:k, :k]) @ S[:k, k:]
    Z = np.zeros((k, n))
    Z[:, P] = np.hstack([np.eye(k), T])
    J = P[:k].copy()
    return A[:, J].copy(), Z, J


def rid(A, k, p=10, q=0, seed=0, stream_id=0, sdist="normal"):
    """Alg. rid: randomized column ID.  Returns (C, Z, J)."""
    A = np.asarray(A, dtype=np.float64)
    _, B, _ = orc.rqb(A, k, p, q, seed, stream_id, sdist)
    _, Z, J = interp_decomp(B, k)
    return A[:, J].copy(), Z, J


def rcur(A, k, p=10, q=0, seed=0, stream_id=0, sdist="normal"):
    """Alg. rcur: randomized CUR.  Returns dict(C, U, R, J (columns), I (rows))."""
    A = np.asarray(A, dtype=np.float64)
    C, Z, J = rid(A, k, p, q, seed, stream_id, sdist)
    _, _, P = cpqr(C.T)
    I = P[:k].copy()
    R = A[I, :].copy()
    U = Z @ np.linalg.pinv(R)
    return dict(C=C, U=U, R=R, J=J, I=I, Z=Z)
