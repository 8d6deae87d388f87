"""Planted-spectrum test matrices A = U diag(sigma) V^T (+ noise).

U and V are Haar-distributed: the Q factor of a seeded Gaussian matrix with
its columns multiplied by sign(R_ii) (Mezzadri, "How to generate random
matrices from the classical compact groups", 2007).

Workload recipes (sizes, spectra and seeds):

* harmonic_2000x1000: 2000 x 1000 float64, sigma_i = 1/i (all 1000 values);
      k=20, p=10, q=2.
* tall_exp_100000x5000: 100000 x 5000 float32, sigma_i = exp(-i/50) for
      i <= 1000 plus a Gaussian noise floor of 1e-6 sigma_1 (entries N(0,1) *
      1e-6 sigma_1 / sqrt(m)); k=100, p=20, q=2.  For PCA a column offset
      mu_j ~ N(0,1) * sigma_1 / sqrt(m) is added.
* poly_bf16_200000x20000: 200000 x 20000 bfloat16, sigma_i = i^-1.5 for
      i <= 4096, computed in float64 and rounded to bfloat16 (the rounded
      matrix is the instance).
* ragged_4096: 4096 ragged float32 matrices: m ~ U{256..4096},
      n ~ U{64..1024}, k ~ U{8..min(64, min(m,n)-10)}, sigma_i = i^-alpha,
      alpha ~ U[0.5, 3].
* paper-shaped: the rank-200 product of two Gaussian matrices used for the
  paper's timing study (Sec. 3.8).
"""
import math

import numpy as np

CONFIGS = {
    "harmonic_2000x1000": dict(m=2000, n=1000, k=20, p=10, q=2, dtype="f64", gen_seed=1608, omega_seed=2148),
    "tall_exp_100000x5000": dict(m=100000, n=5000, k=100, p=20, q=2, dtype="f32", gen_seed=5000, omega_seed=2148),
    "poly_bf16_200000x20000": dict(m=200000, n=20000, k=200, p=20, q=2, dtype="bf16", gen_seed=20000, omega_seed=2148),
    "ragged_4096": dict(batch=4096, p=10, q=2, dtype="f32", gen_seed=4096, omega_seed=2148),
}


def spectrum(kind, count, **kw):
    """Planted singular values sigma_1 >= sigma_2 >= ... (float64)."""
    i = np.arange(1, count + 1, dtype=np.float64)
    if kind == "inverse":          # sigma_i = 1 / i
        return 1.0 / i
    if kind == "poly":             # sigma_i = i^-alpha
        return i ** (-float(kw["alpha"]))
    if kind == "exp":              # sigma_i = exp(-i / tau)
        return np.exp(-i / float(kw["tau"]))
    raise ValueError(kind)


def haar(rng, m, r):
    """m x r matrix with orthonormal columns, Haar distributed (r <= m)."""
    g = rng.standard_normal((m, r))
    q, rr = np.linalg.qr(g, mode="reduced")
    s = np.sign(np.diag(rr))
    s[s == 0] = 1.0
    return q * s[None, :]


def planted(m, n, sigma, seed, noise=0.0):
    """A = U diag(sigma) V^T + noise * G (float64, numpy)."""
    rng = np.random.default_rng(seed)
    r = len(sigma)
    U = haar(rng, m, r)
    V = haar(rng, n, r)
    A = (U * np.asarray(sigma)[None, :]) @ V.T
    if noise:
        A += noise * rng.standard_normal((m, n))
    return A


def planted_torch(m, n, sigma, seed, noise=0.0, device="cuda", out_dtype=None,
                  chunk_rows=16384):
    """Same recipe as ``planted`` on a torch device, returned in ``out_dtype``.

    Generated in float64 and rounded once to ``out_dtype`` (round to nearest
    even), in row chunks so that only the rounded matrix is held in full.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    r = len(sigma)
    f64 = torch.float64

    def _haar(rows):
        x = torch.randn(rows, r, generator=g, device=device, dtype=f64)
        q, rr = torch.linalg.qr(x, mode="reduced")
        s = torch.sign(torch.diagonal(rr))
        s[s == 0] = 1.0
        return q * s[None, :]

    U = _haar(m)
    V = _haar(n)
    sig = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    US = U * sig[None, :]
    del U
    out_dtype = out_dtype or f64
    A = torch.empty(m, n, dtype=out_dtype, device=device)
    Vt = V.t().contiguous()
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        blk = US[r0:r1] @ Vt
        if noise:
            blk += noise * torch.randn(r1 - r0, n, generator=g, device=device, dtype=f64)
        A[r0:r1] = blk.to(out_dtype)
    return A


def harmonic_2000x1000():
    """The 2000 x 1000 float64 instance with sigma_i = 1/i."""
    c = CONFIGS["harmonic_2000x1000"]
    sig = spectrum("inverse", min(c["m"], c["n"]))
    return planted(c["m"], c["n"], sig, c["gen_seed"])


def tall_exp_sigma():
    return spectrum("exp", 1000, tau=50.0)


def tall_exp_matrix(device="cuda", m=None, n=None):
    """The 100000 x 5000 exponential-spectrum instance (float32 torch tensor on
    ``device``), optionally resized."""
    import torch
    c = CONFIGS["tall_exp_100000x5000"]
    m = m or c["m"]
    n = n or c["n"]
    sig = tall_exp_sigma()[: min(m, n, 1000)]
    noise = 1e-6 * sig[0] / math.sqrt(m)
    return planted_torch(m, n, sig, c["gen_seed"], noise=noise, device=device,
                         out_dtype=torch.float32)


def tall_exp_offsets(n, m, seed=5001):
    """Column offsets mu_j ~ N(0,1) * sigma_1 / sqrt(m) for the PCA variant."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) * (tall_exp_sigma()[0] / math.sqrt(m))


def poly_bf16_torch(device="cuda", m=200000, n=20000, rank=4096, seed=20000, chunk_rows=8192,
                   dtype=None):
    """A matrix of the 200000 x 20000 bf16 workload's shape and spectrum (sigma_i = i^-1.5, i <= rank),
    rounded once to ``dtype`` (default bfloat16).  The orthonormal factors
    are polar factors of Gaussian blocks, computed with matrix products only
    (Newton-Schulz iteration X <- X (3 I - X^T X) / 2 from the block scaled
    below its largest singular value; the polar factor of a Gaussian block is
    Haar distributed).  Formed in float64 row chunks."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    dtype = dtype or torch.bfloat16

    def _orth(rows):
        X = torch.randn(rows, rank, generator=g, device=device, dtype=f64)
        X /= math.sqrt(rows) + math.sqrt(rank) + 10.0          # sigma_max(G) bound (Gaussian block)
        eye = torch.eye(rank, dtype=f64, device=device)
        for _ in range(10):
            X = X @ (1.5 * eye - 0.5 * (X.t() @ X))
        return X

    sig = torch.as_tensor(spectrum("poly", rank, alpha=1.5), device=device)
    Vt = _orth(n).t().contiguous()
    US = _orth(m)
    US *= sig[None, :]
    A = torch.empty(m, n, dtype=dtype, device=device)
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        A[r0:r1] = (US[r0:r1] @ Vt).to(dtype)
    return A


def ragged_shapes(batch=4096, seed=4096, m_range=(256, 4096), n_range=(64, 1024),
              k_max=64):
    """Ragged shapes and decay exponents of the 4096-matrix batch (numpy arrays)."""
    rng = np.random.default_rng(seed)
    m = rng.integers(m_range[0], m_range[1] + 1, size=batch)
    n = rng.integers(n_range[0], n_range[1] + 1, size=batch)
    kmax = np.minimum(k_max, np.minimum(m, n) - 10)
    k = np.array([rng.integers(8, km + 1) for km in kmax])
    alpha = rng.uniform(0.5, 3.0, size=batch)
    return m, n, k, alpha


def ragged_batch(batch=4096, seed=4096, **shape_kw):
    """Ragged batch: list of (A float64 numpy, k, alpha).  CPU; small batches."""
    m, n, k, alpha = ragged_shapes(batch, seed, **shape_kw)
    out = []
    for b in range(batch):
        r = int(min(m[b], n[b]))
        sig = spectrum("poly", r, alpha=alpha[b])
        A = planted(int(m[b]), int(n[b]), sig, seed * 100003 + b)
        out.append((A, int(k[b]), float(alpha[b])))
    return out


def _haar_torch(rows, r, g, device, max_iter=80):
    """rows x r Haar-distributed orthonormal columns on a torch device: the
    polar factor of a Gaussian block (orthogonally invariant, hence Haar),
    by the Newton-Schulz iteration X <- X (3 I - X^T X) / 2 from the block
    scaled below its largest singular value (matrix products only).  Near-
    square blocks converge slowly (their smallest singular value is small),
    so the iteration runs until X^T X = I to 1e-13 or max_iter steps, then
    falls back to Householder QR (sign-fixed) for the rare block that has not
    converged."""
    import torch
    X = torch.randn(rows, r, generator=g, device=device, dtype=torch.float64)
    G0 = X
    X = X / (math.sqrt(rows) + math.sqrt(r) + 10.0)
    eye = torch.eye(r, dtype=torch.float64, device=device)
    for it in range(max_iter):
        XtX = X.t() @ X
        if it % 8 == 7 and float((XtX - eye).abs().max()) < 1e-13:
            return X
        X = X @ (1.5 * eye - 0.5 * XtX)
    if float((X.t() @ X - eye).abs().max()) < 1e-13:
        return X
    q, rr = torch.linalg.qr(G0, mode="reduced")
    sgn = torch.sign(torch.diagonal(rr))
    sgn[sgn == 0] = 1.0
    return q * sgn[None, :]


def ragged_torch(device="cuda", batch=4096, seed=4096, out_dtype=None, **shape_kw):
    """The 4096-matrix ragged batch on a torch device: A_b = U_b diag(i^-alpha_b) V_b^T with Haar
    U_b, V_b over all min(m_b, n_b) values, rounded once to ``out_dtype``
    (default float32) into one ragged buffer.

    Returns dict(buffer, A (list of row-major views), m, n, k, alpha).
    """
    import torch
    out_dtype = out_dtype or torch.float32
    m, n, k, alpha = ragged_shapes(batch, seed, **shape_kw)
    sizes = (m.astype(np.int64) * n.astype(np.int64))
    offs = np.concatenate([[0], np.cumsum(sizes)])
    buf = torch.empty(int(offs[-1]), dtype=out_dtype, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    views = []
    for b in range(batch):
        mb, nb = int(m[b]), int(n[b])
        r = min(mb, nb)
        sig = torch.arange(1, r + 1, device=device, dtype=torch.float64) ** (-float(alpha[b]))
        U = _haar_torch(mb, r, g, device)
        V = _haar_torch(nb, r, g, device)
        view = buf[int(offs[b]):int(offs[b + 1])].view(mb, nb)
        view.copy_((U * sig[None, :]) @ V.t())
        views.append(view)
    return dict(buffer=buf, A=views, m=m, n=n, k=k, alpha=alpha)


def paper_lowrank_product(m, n, rank=200, seed=1135):
    """Rank-``rank`` product of two Gaussian matrices (float64)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, rank)) @ rng.standard_normal((rank, n))
