"""Matrices for training and evaluating the learned (q, p) selector.

Recipe (the shape distribution of the 4096-matrix batch workload):

* m ~ U{256..4096}, n ~ U{64..1024}, k ~ U{8..min(64, min(m, n) - 10)}
  (optionally with smaller bounds for quick checks).
* Spectrum over all r = min(m, n) values, half of the matrices each:
  polynomial f(i) = i^-alpha, alpha ~ U[0.5, 3], or exponential
  f(i) = exp(-(i - 1) / tau), tau ~ logU[2, 200]; f(1) = 1.  Then a spectral
  floor: sigma_i = f(i) + nu with nu ~ logU[1e-8, 1e-2], so every singular
  value of the planted matrix is known exactly.
* Singular vectors (factors="householder", the default): U = H(a1) H(a2)
  and V = H(b1) H(b2) with Householder
  reflections H(x) = I - 2 x x^T about Gaussian unit vectors, so A =
  U[:, :r] diag(sigma) V[:, :r]^T is dense and has exactly the planted
  singular values.  A Gaussian test matrix only sees the spectrum (V^T Omega
  has the same distribution as Omega), so the randomized SVD's error
  statistics are those of Haar-distributed factors, at a fraction of the
  generation cost.  The reflection vectors are kept so that an evaluation can
  apply U^T exactly.  These factors are close to the identity (a rank-two
  change each), so A is nearly diagonal and its f32 rounding is relative to
  each singular value; factors="haar" draws dense Haar factors instead
  (polar factors of Gaussian blocks), whose rounding error spreads over all
  entries as in the 4096-matrix batch workload.
* A is formed in float64 and rounded once to the storage type.

Splits use separate seeds: train 5101, validation 5102, test 5103.
"""
import math

import numpy as np

SPLIT_SEEDS = {"train": 5101, "val": 5102, "test": 5103}


def shapes(count, seed, m_range=(256, 4096), n_range=(64, 1024), k_max=64):
    """Shapes, spectrum kind / parameter and floor of `count` matrices."""
    rng = np.random.default_rng(seed)
    m = rng.integers(m_range[0], m_range[1] + 1, size=count)
    n = rng.integers(n_range[0], n_range[1] + 1, size=count)
    kmax = np.minimum(k_max, np.minimum(m, n) - 10)
    k = np.array([rng.integers(8, km + 1) for km in kmax])
    poly = rng.random(count) < 0.5
    alpha = rng.uniform(0.5, 3.0, size=count)
    tau = np.exp(rng.uniform(math.log(2.0), math.log(200.0), size=count))
    nu = np.exp(rng.uniform(math.log(1e-8), math.log(1e-2), size=count))
    return dict(m=m, n=n, k=k, poly=poly, alpha=alpha, tau=tau, nu=nu)


def spectrum_of(spec, b):
    """Planted singular values of matrix b (float64 numpy, length min(m, n))."""
    r = int(min(spec["m"][b], spec["n"][b]))
    i = np.arange(1, r + 1, dtype=np.float64)
    f = i ** (-spec["alpha"][b]) if spec["poly"][b] else np.exp(-(i - 1.0) / spec["tau"][b])
    return f + spec["nu"][b]


def build_range(count, split, lo, hi, device="cuda", out_dtype=None, factors="householder", **shape_kw):
    """Matrices lo..hi-1 of a split of `count` matrices (the shapes and
    spectra of shapes(count, seed)), generated with their own torch generator
    seeded from (split seed, lo): a large split is built shard by shard with
    a fixed shard layout.  Returns the same dict as build() for that range."""
    seed = SPLIT_SEEDS[split] if isinstance(split, str) else int(split)
    full = shapes(count, seed, **shape_kw)
    spec = {key: val[lo:hi] for key, val in full.items()}
    return _form(spec, seed * 1000003 + lo, device, out_dtype, factors)


def build(count, split="train", device="cuda", out_dtype=None, factors="householder", **shape_kw):
    """The split's matrices in one ragged buffer on ``device``.

    Returns dict(buffer, A (list of row-major views), spec (shapes()), sigma
    (list of float64 numpy spectra), hh (list of (a1, a2) float64 tensors)).
    """
    seed = SPLIT_SEEDS[split] if isinstance(split, str) else int(split)
    return _form(shapes(count, seed, **shape_kw), seed, device, out_dtype, factors)


def _form(spec, seed, device, out_dtype, factors="householder"):
    """Planted matrices for the shapes and spectra in spec (see build()).

    factors = "householder": U = H(a1) H(a2), V = H(b1) H(b2) (hh holds the
    reflection vectors); "haar": dense Haar factors (polar factors of
    Gaussian blocks, synth.matrices._haar_torch), hh = None."""
    import torch
    out_dtype = out_dtype or torch.float32
    count = len(spec["m"])
    m, n = spec["m"].astype(np.int64), spec["n"].astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(m * n)])
    buf = torch.empty(int(offs[-1]), dtype=out_dtype, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    f64 = torch.float64

    def unit(size):
        x = torch.randn(size, generator=g, device=device, dtype=f64)
        return x / x.norm()

    views, sigmas, hh = [], [], []
    for b in range(count):
        mb, nb = int(m[b]), int(n[b])
        sig = spectrum_of(spec, b)
        r = len(sig)
        if factors == "haar":
            from . import matrices as mat
            U = mat._haar_torch(mb, r, g, device)
            V = mat._haar_torch(nb, r, g, device)
            view = buf[int(offs[b]):int(offs[b + 1])].view(mb, nb)
            view.copy_((U * torch.as_tensor(sig, device=device)[None, :]) @ V.t())
            views.append(view)
            sigmas.append(sig)
            continue
        a1, a2, b1, b2 = unit(mb), unit(mb), unit(nb), unit(nb)
        A = torch.zeros(mb, nb, dtype=f64, device=device)
        A[torch.arange(r, device=device), torch.arange(r, device=device)] = torch.as_tensor(sig, device=device)
        A -= 2.0 * torch.outer(a2, a2 @ A)          # H(a2) D
        A -= 2.0 * torch.outer(a1, a1 @ A)          # H(a1) H(a2) D
        A -= 2.0 * torch.outer(A @ b2, b2)          # ... H(b2)
        A -= 2.0 * torch.outer(A @ b1, b1)          # ... H(b2) H(b1) = (H(b1) H(b2))^T
        view = buf[int(offs[b]):int(offs[b + 1])].view(mb, nb)
        view.copy_(A)
        views.append(view)
        sigmas.append(sig)
        hh.append((a1, a2))
    return dict(buffer=buf, A=views, spec=spec, sigma=sigmas, hh=hh if factors != "haar" else None)
