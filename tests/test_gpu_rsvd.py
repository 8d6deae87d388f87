"""End-to-end parity of the HIP randomized SVD / PCA against the FP64 oracle.

Tolerances (derived from the arithmetic; see the design notes):
* f64 path: singular values elementwise |ds_i| / s_i <= 1e-10 for i <= k.
* f32 / bf16-stored path (f32 arithmetic): normwise |ds_i| <= 1e-4 s_1, and
  elementwise 1e-4 where s_i >= 1e-3 s_1.
* Singular vectors: the sign rule is the same on both sides, so vectors are
  compared entrywise where the singular value gap is large, and by the cosine
  of the angle between corresponding vectors otherwise.
"""
import math

import numpy as np
import pytest
import torch

from oracle import rsvd as orc
from synth import matrices as syn

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _np(t):
    return None if t is None else t.detach().cpu().to(torch.float64).numpy()


def _check_sigma(s_gpu, s_ora, dtype):
    if dtype == torch.float64:
        np.testing.assert_allclose(s_gpu, s_ora, rtol=1e-10, atol=0)
    else:
        s1 = s_ora[0]
        assert np.max(np.abs(s_gpu - s_ora)) <= 1e-4 * s1
        big = s_ora >= 1e-3 * s1
        np.testing.assert_allclose(s_gpu[big], s_ora[big], rtol=1e-4)


def _gap_ok(s, i, rel=1e-3):
    lo = abs(s[i] - s[i + 1]) if i + 1 < len(s) else s[i]
    hi = abs(s[i - 1] - s[i]) if i > 0 else s[i]
    return min(lo, hi) > rel * s[0]


def _check_vectors(U, V, Uo, Vo, s, tol):
    k = len(s)
    for i in range(k):
        if not _gap_ok(s, i):
            continue
        cu = abs(float(U[:, i] @ Uo[:, i]))
        cv = abs(float(V[:, i] @ Vo[:, i]))
        assert cu > 1 - tol and cv > 1 - tol, (i, cu, cv)
        # same sign convention on both sides
        assert float(V[:, i] @ Vo[:, i]) > 0


def run_both(A_np, k, p, q, seed, dtype, sdist="normal", stream_id=0):
    from paper_1608_02148_amd import api
    Ag = torch.tensor(A_np, dtype=dtype, device=DEV)
    A_inst = Ag.detach().cpu().to(torch.float64).numpy()          # the stored instance
    U, S, V = api.rsvd(Ag, k, p=p, q=q, seed=seed, stream_id=stream_id, sdist=sdist)
    torch.cuda.synchronize()
    Uo, so, Vo = orc.rsvd(A_inst, k, p=p, q=q, seed=seed, stream_id=stream_id, sdist=sdist)
    return A_inst, (_np(U), _np(S), _np(V)), (Uo, so, Vo)


def test_c1_fp64_parity():
    """2000 x 1000 f64, sigma_i = 1/i, k=20, p=10, q=2, Omega seed 2148."""
    c = syn.CONFIGS["harmonic_2000x1000"]
    A = syn.harmonic_2000x1000()
    A_inst, (U, s, V), (Uo, so, Vo) = run_both(A, c["k"], c["p"], c["q"], c["omega_seed"], torch.float64)
    _check_sigma(s, so, torch.float64)
    np.testing.assert_allclose(U, Uo, atol=1e-9)
    np.testing.assert_allclose(V, Vo, atol=1e-9)
    np.testing.assert_allclose(U.T @ U, np.eye(c["k"]), atol=1e-13)
    np.testing.assert_allclose(V.T @ V, np.eye(c["k"]), atol=1e-13)
    r_gpu = orc.lowrank_residual(A_inst, U, s, V)
    r_ora = orc.lowrank_residual(A_inst, Uo, so, Vo)
    assert r_gpu == pytest.approx(r_ora, rel=1e-10)


@pytest.mark.parametrize("m,n,k,p,q,seed", [
    (333, 257, 7, 5, 1, 11),      # ragged tiles
    (257, 333, 7, 5, 1, 12),      # wide: Omega stays n x l
    (1000, 100, 90, 20, 1, 13),   # l clamped to min(m, n)
    (500, 120, 10, 10, 0, 14),    # no power iterations
    (800, 300, 20, 0, 2, 15),     # no oversampling
    (4000, 700, 100, 28, 3, 16),  # l = 128, the largest tile
    (64, 40, 1, 2, 2, 17),        # k = 1
    (3000, 600, 85, 10, 2, 18),   # l = 95: square 96 tiles for the l x l products
    (2500, 400, 40, 5, 1, 19),    # l = 45: square 48 tiles
    (2500, 700, 66, 10, 1, 20),   # l = 76: square 80 tiles
])
def test_fp64_shapes(m, n, k, p, q, seed):
    sig = syn.spectrum("poly", min(m, n), alpha=1.0)
    A = syn.planted(m, n, sig, seed)
    A_inst, (U, s, V), (Uo, so, Vo) = run_both(A, k, p, q, seed, torch.float64)
    _check_sigma(s, so, torch.float64)
    _check_vectors(U, V, Uo, Vo, so, 1e-9)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("m,n,k,p,q", [(3000, 500, 20, 10, 2), (777, 1030, 50, 14, 1), (5000, 2000, 100, 20, 2)])
def test_fp32_arithmetic_paths(dtype, m, n, k, p, q):
    sig = syn.spectrum("exp", min(m, n), tau=20.0)
    A = syn.planted(m, n, sig, m + n)
    A_inst, (U, s, V), (Uo, so, Vo) = run_both(A, k, p, q, 2148, dtype)
    _check_sigma(s, so, torch.float32)
    _check_vectors(U, V, Uo, Vo, so, 1e-5)


@pytest.mark.parametrize("sdist", ["unif", "rademacher"])
def test_other_test_matrices(sdist):
    sig = syn.spectrum("poly", 300, alpha=1.5)
    A = syn.planted(900, 300, sig, 21)
    A_inst, (U, s, V), (Uo, so, Vo) = run_both(A, 15, 10, 2, 99, torch.float64, sdist=sdist, stream_id=4)
    _check_sigma(s, so, torch.float64)


def test_determinism_bitwise():
    from paper_1608_02148_amd import api
    A = torch.tensor(syn.planted(3000, 800, syn.spectrum("poly", 800, alpha=0.7), 3), dtype=torch.float32,
                     device=DEV)
    r1 = api.rsvd(A, 40, p=10, q=2, seed=7)
    r2 = api.rsvd(A, 40, p=10, q=2, seed=7)
    for a, b in zip(r1, r2):
        assert torch.equal(a, b)


def test_power_of_two_scaling_exact():
    from paper_1608_02148_amd import api
    A = torch.tensor(syn.planted(1200, 300, syn.spectrum("poly", 300, alpha=1.0), 4), device=DEV)
    U1, s1, V1 = api.rsvd(A, 12, seed=3)
    U2, s2, V2 = api.rsvd(A * 8.0, 12, seed=3)
    assert torch.equal(s2, s1 * 8.0)
    assert torch.equal(U1, U2) and torch.equal(V1, V2)


def test_rpca_matches_explicit_centring():
    from paper_1608_02148_amd import api
    m, n, k = 3000, 400, 12
    A = syn.planted(m, n, syn.spectrum("exp", n, tau=15.0), 31)
    mu = np.random.default_rng(5).standard_normal(n) * 0.05
    X = A + mu[None, :]
    Xg = torch.tensor(X, device=DEV)
    res = api.rpca(Xg, k, p=10, q=2, seed=8)
    ora = orc.rpca(X, k, p=10, q=2, seed=8)
    np.testing.assert_allclose(_np(res["center"]), ora["center"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(_np(res["eigvals"]), ora["eigvals"], rtol=1e-10)
    np.testing.assert_allclose(_np(res["sdev"]), ora["sdev"], rtol=1e-10)
    np.testing.assert_allclose(_np(res["rotation"]), ora["rotation"], atol=1e-9)
    np.testing.assert_allclose(_np(res["x"]), ora["x"], atol=1e-9)


@pytest.mark.parametrize("precision", ["plain", "bf16_mixed"])
def test_rpca_bf16_storage_matches_explicit_centring(precision):
    """bf16-stored data with column offsets: implicit centring subtracts the
    f64 means from the stored values.  In the mixed mode the early (bf16)
    passes round A - mu to bf16, while the last sketch and the projection
    stage A - mu as bf16 hi + lo terms, so the result keeps the split
    arithmetic's near-f32 accuracy.  Against the oracle on the stored instance
    with explicit centring: sqrt(eigvals) normwise 1e-4 of the largest, and in
    the mixed mode the leading half also 1e-4 relative (the bound the
    uncentred mixed mode meets)."""
    from paper_1608_02148_amd import api
    m, n, k = 2500, 333, 10
    A = syn.planted(m, n, syn.spectrum("exp", n, tau=12.0), 77)
    mu = np.random.default_rng(6).standard_normal(n) * 0.05
    Xg = torch.tensor(A + mu[None, :], dtype=torch.bfloat16, device=DEV)
    X = _np(Xg)
    res = api.rpca(Xg, k, p=10, q=2, seed=3, precision=precision)
    ora = orc.rpca(X, k, p=10, q=2, seed=3)
    np.testing.assert_allclose(_np(res["center"]), ora["center"], rtol=1e-6, atol=1e-7)
    sd, sdo = np.sqrt(_np(res["eigvals"])), np.sqrt(ora["eigvals"])
    assert np.max(np.abs(sd - sdo)) <= 1e-4 * sdo[0]
    if precision == "bf16_mixed":
        np.testing.assert_allclose(sd[: k // 2], sdo[: k // 2], rtol=1e-4)


def test_rpca_fp32_without_centring():
    from paper_1608_02148_amd import api
    A = syn.planted(2000, 300, syn.spectrum("exp", 300, tau=10.0), 41)
    Ag = torch.tensor(A, dtype=torch.float32, device=DEV)
    res = api.rpca(Ag, 10, center=False, retx=False, p=10, q=2, seed=1)
    ora = orc.rpca(_np(Ag), 10, p=10, q=2, center=False, seed=1)
    assert res["x"] is None
    s1 = math.sqrt(ora["eigvals"][0])
    assert np.max(np.abs(np.sqrt(_np(res["eigvals"])) - np.sqrt(ora["eigvals"]))) <= 1e-4 * s1 * 1.0001
    assert np.all(_np(res["center"]) == 0)


def test_zero_matrix_is_flagged_not_nan():
    from paper_1608_02148_amd import api
    A = torch.zeros(500, 200, dtype=torch.float64, device=DEV)
    info = api.new_info(DEV)
    U, S, V = api.rsvd(A, 5, info=info)
    st, host = api.sync_info(info)
    assert torch.all(S == 0)
    assert torch.all(torch.isfinite(U)) and torch.all(torch.isfinite(V))
    assert host.flags & 2 and st == -5
    assert host.l == 15 and host.q == 2 and host.p == 10


def test_nan_input_is_flagged():
    from paper_1608_02148_amd import api
    A = torch.randn(400, 100, dtype=torch.float32, device=DEV)
    A[17, 3] = float("nan")
    info = api.new_info(DEV)
    api.rsvd(A, 5, info=info)
    st, host = api.sync_info(info)
    assert host.flags & 4 and st == -4


def test_rank_deficient_input():
    from paper_1608_02148_amd import api
    r = 6
    A = syn.planted(1000, 300, np.linspace(3, 1, r), 51)
    U, S, V = api.rsvd(torch.tensor(A, device=DEV), 10, p=10, q=2, seed=2)
    s = _np(S)
    np.testing.assert_allclose(s[:r], np.linspace(3, 1, r), rtol=1e-10)
    assert np.all(s[r:] < 1e-12)
    assert np.all(np.isfinite(_np(U))) and np.all(np.isfinite(_np(V)))


def test_invalid_arguments_raise():
    from paper_1608_02148_amd import api, lib
    A = torch.zeros(50, 20, device=DEV)
    with pytest.raises(lib.RsvdError):
        api.rsvd(A, 20)
    with pytest.raises(lib.RsvdError):
        api.rsvd(A, 0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("m,n,k,p,q", [(6000, 800, 40, 10, 2), (3000, 1200, 60, 20, 1)])
def test_bf16_mixed_mode(dtype, m, n, k, p, q):
    """Mixed mode: bf16 early passes, f32-accurate last sketch and projection.

    Checked against the FP64 oracle on the same stored instance: leading
    singular values (well separated from the tail) to 1e-4 relative, all k
    values normwise to 2e-3 sigma_1, and the rank-k residual within 1% of the
    oracle's.
    """
    from paper_1608_02148_amd import api
    sig = syn.spectrum("exp", min(m, n), tau=20.0)
    A = syn.planted(m, n, sig, m + 7 * n)
    Ag = torch.tensor(A, dtype=dtype, device=DEV)
    A_inst = _np(Ag)
    U, S, V = api.rsvd(Ag, k, p=p, q=q, seed=5, precision="bf16_mixed")
    Uo, so, Vo = orc.rsvd(A_inst, k, p=p, q=q, seed=5)
    s = _np(S)
    np.testing.assert_allclose(s[: k // 2], so[: k // 2], rtol=1e-4)
    assert np.max(np.abs(s - so)) <= 2e-3 * so[0]
    r_gpu = orc.lowrank_residual(A_inst, _np(U), s, _np(V))
    r_ora = orc.lowrank_residual(A_inst, Uo, so, Vo)
    assert r_gpu <= 1.01 * r_ora


def test_bf16_mixed_rejected_for_f64():
    from paper_1608_02148_amd import api, lib
    A = torch.zeros(100, 50, dtype=torch.float64, device=DEV)
    with pytest.raises(lib.RsvdError):
        api.rsvd(A, 5, precision="bf16_mixed")


# Shapes whose A X products split their n-reduction (three chunks for
# 20000 x 4096 and four for 12000 x 4100 on a 256-CU device), the form the
# 100000 x 5000 and 200000 x 20000 workloads run.
@pytest.mark.parametrize("dtype,precision", [(torch.float32, "plain"), (torch.float32, "bf16_mixed"),
                                             (torch.float64, "plain")])
def test_split_k_solve_parity(dtype, precision):
    from paper_1608_02148_amd import api
    m, n, k, p, q = 20000, 4096, 100, 20, 2
    sig = np.exp(-np.arange(1, 601) / 50.0)
    A = syn.planted(m, n, sig, 4096, noise=1e-6 / math.sqrt(m))
    Ag = torch.tensor(A, dtype=dtype, device=DEV)
    A_inst = _np(Ag)
    U, S, V = api.rsvd(Ag, k, p=p, q=q, seed=2148, precision=precision)
    Uo, so, Vo = orc.rsvd(A_inst, k, p=p, q=q, seed=2148)
    U, s, V = _np(U), _np(S), _np(V)
    if dtype == torch.float64:
        _check_sigma(s, so, torch.float64)
        _check_vectors(U, V, Uo, Vo, so, 1e-9)
    elif precision == "plain":
        _check_sigma(s, so, torch.float32)
        _check_vectors(U, V, Uo, Vo, so, 1e-5)
    else:
        np.testing.assert_allclose(s[: k // 2], so[: k // 2], rtol=1e-4)
        assert np.max(np.abs(s - so)) <= 2e-3 * so[0]
        r_gpu = orc.lowrank_residual(A_inst, U, s, V)
        r_ora = orc.lowrank_residual(A_inst, Uo, so, Vo)
        assert r_gpu <= 1.01 * r_ora


@pytest.mark.parametrize("precision", ["plain", "bf16_mixed"])
def test_split_k_wide_sketch_bf16_storage(precision):
    """bf16-stored 12000 x 4100, k = 200, p = 20 (l = 220: two column tiles,
    blocked Cholesky, block Jacobi) with a four-way split of A X."""
    from paper_1608_02148_amd import api
    m, n, k, p, q = 12000, 4100, 200, 20, 1
    A = syn.planted(m, n, syn.spectrum("poly", 1000, alpha=1.5), 220)
    Ag = torch.tensor(A, dtype=torch.bfloat16, device=DEV)
    A_inst = _np(Ag)
    U, S, V = api.rsvd(Ag, k, p=p, q=q, seed=2148, precision=precision)
    Uo, so, Vo = orc.rsvd(A_inst, k, p=p, q=q, seed=2148)
    U, s, V = _np(U), _np(S), _np(V)
    if precision == "plain":
        _check_sigma(s, so, torch.float32)
        _check_vectors(U, V, Uo, Vo, so, 1e-4)
    else:
        np.testing.assert_allclose(s[: k // 2], so[: k // 2], rtol=1e-4)
        assert np.max(np.abs(s - so)) <= 2e-3 * so[0]
    r_gpu = orc.lowrank_residual(A_inst, U, s, V)
    r_ora = orc.lowrank_residual(A_inst, Uo, so, Vo)
    assert r_gpu <= 1.01 * r_ora
