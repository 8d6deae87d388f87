"""FP64 oracle of the learned choice of (q, p) (TEST INFRASTRUCTURE ONLY).

The paper leaves q and p to the user: p = 10 and q = 2 are its defaults
(Sec. 3.6), more power iterations help when the spectrum decays slowly
(Sec. 2.2).  The selector reads the spectrum of a cheap q = 0 sketch and
picks the cheapest pair that reaches the accuracy target:

* Sketch: l0 = max(2k, k + 20), clamped to min(m, n) and to 128;
  Y0 = A Omega[:, :l0] with the solve's own test matrix (Alg. rqb,
  same seed and stream, so Omega[:, :l] of the later solve is a prefix).
* Features (131): the singular values of Y0 divided by the largest, in
  descending order, zero-padded to 128; then log2(m)/12, log2(n)/12,
  log2(k)/12.
* Classes: c = 3 q + j for q in 0..4 and p = (5, 10, 20)[j].
* Cost of a pair: (2q + 2)(k + p), the passes over A times the sketch width;
  ties go to the lower class index.
* Label: the cheapest pair whose excess error
      ||A - U_k S_k V_k^T||_2 / sigma_{k+1}(A) - 1
  is at most 1 %; class 14 = (4, 20), flagged unreachable, if none is.
"""
import math

import numpy as np

from . import philox
from . import rsvd as orc

P_CHOICES = (5, 10, 20)
Q_MAX = 4
N_CLASSES = (Q_MAX + 1) * len(P_CHOICES)
N_SIGMA = 128


def class_pair(c):
    """(q, p) of class c."""
    return c // len(P_CHOICES), P_CHOICES[c % len(P_CHOICES)]


def pair_class(q, p):
    return q * len(P_CHOICES) + P_CHOICES.index(p)


def pair_cost(k, q, p):
    return (2 * q + 2) * (k + p)


def classes_by_cost(k):
    """All classes, cheapest first (ties: lower class index first)."""
    return sorted(range(N_CLASSES), key=lambda c: (pair_cost(k, *class_pair(c)), c))


def sketch_width0(m, n, k):
    return min(max(2 * k, k + 20), m, n, N_SIGMA)


def sketch(A, k, seed=0, stream_id=0, sdist="normal"):
    """Y0 = A Omega[:, :l0] (Alg. rqb at q = 0)."""
    m, n = A.shape
    l0 = sketch_width0(m, n, k)
    Om = philox.test_matrix(n, l0, seed, stream_id, sdist)
    return A @ Om


def features(A, k, seed=0, stream_id=0, sdist="normal"):
    """The 131 selector inputs of matrix A (see the module notes)."""
    m, n = A.shape
    Y0 = sketch(np.asarray(A, dtype=np.float64), k, seed, stream_id, sdist)
    s = np.linalg.svd(Y0, compute_uv=False)
    f = np.zeros(N_SIGMA + 3)
    if s[0] > 0:
        f[:len(s)] = s / s[0]
    f[N_SIGMA:] = [math.log2(m) / 12.0, math.log2(n) / 12.0, math.log2(k) / 12.0]
    return f


def excess_error(A, k, q, p, seed=0, stream_id=0, sigma_next=None):
    """||A - U S V^T||_2 / sigma_{k+1} - 1 of the randomized SVD with (q, p)."""
    if sigma_next is None:
        sigma_next = np.linalg.svd(A, compute_uv=False)[k]
    U, s, V = orc.rsvd(A, k, p=p, q=q, seed=seed, stream_id=stream_id)
    r = np.linalg.norm(A - (U * s[None, :]) @ V.T, 2)
    return r / sigma_next - 1.0


def label(A, k, seed=0, stream_id=0, sigma_next=None, tol=0.01):
    """(class, reachable): the cheapest pair with excess error <= tol."""
    if sigma_next is None:
        sigma_next = np.linalg.svd(A, compute_uv=False)[k]
    for c in classes_by_cost(k):
        q, p = class_pair(c)
        if excess_error(A, k, q, p, seed, stream_id, sigma_next) <= tol:
            return c, True
    return N_CLASSES - 1, False


def posterior_estimate(A, U, s, V, r=10, seed=0, stream_id=0):
    """A-posteriori bound of ||A - U S V^T||_2 from r Gaussian probes:
    10 sqrt(2/pi) max_i ||(A - U S V^T) w_i||, which holds with probability
    at least 1 - 10^-r (Halko, Martinsson & Tropp, SIAM Review 53, 2011,
    Sec. 4.3, Eq. 4.3).  The probes are the Gaussian test matrix n x r of the
    given seed and stream."""
    W = philox.test_matrix(A.shape[1], r, seed, stream_id)
    R = A @ W - (U * s[None, :]) @ (V.T @ W)
    return 10.0 * math.sqrt(2.0 / math.pi) * float(np.max(np.linalg.norm(R, axis=0)))
