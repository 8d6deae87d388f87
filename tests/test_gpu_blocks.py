"""Kernel-level parity of the HIP building blocks against the oracle (GPU).

Exact-arithmetic inputs (small integers) make every product exact in f64, f32
and bf16 whatever the summation order, so those comparisons are bitwise.
"""
import numpy as np
import pytest
import torch

from oracle import philox as oph
from oracle import rsvd as orc

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _np(t):
    t = t.detach().cpu()
    return (t.to(torch.float64) if t.dtype == torch.bfloat16 else t).numpy()


@pytest.mark.parametrize("n,groups,seed,sid", [(1000, 8, 2148, 0), (257, 33, 2**40 + 12345, 7),
                                               (5, 1, 0, 2**32 - 1)])
def test_philox_words_bit_exact(gpu_lib, n, groups, seed, sid):
    from paper_1608_02148_amd import api
    got = _np(api.philox_words(n, groups, seed, sid)).astype(np.int64) & 0xFFFFFFFF
    want = oph.raw_words(n, 4 * groups, seed, sid).astype(np.int64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("sdist", ["normal", "unif", "rademacher"])
def test_test_matrix_matches_oracle(gpu_lib, sdist):
    from paper_1608_02148_amd import api
    n, l = 3001, 37
    want = oph.test_matrix(n, l, 2148, 3, sdist)
    got64 = _np(api.test_matrix(n, l, 2148, 3, sdist, torch.float64))
    got32 = _np(api.test_matrix(n, l, 2148, 3, sdist, torch.float32))
    if sdist == "rademacher":
        assert np.array_equal(got64, want) and np.array_equal(got32, want)
    else:
        np.testing.assert_allclose(got64, want, rtol=0, atol=2e-14)
        np.testing.assert_allclose(got32, want, rtol=0, atol=3e-6)


def _int_matrix(rng, shape, lo=-8, hi=8):
    return rng.integers(lo, hi + 1, size=shape).astype(np.float64)


DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("m,K,c", [(300, 257, 5), (129, 64, 30), (1000, 515, 64), (517, 1000, 100),
                                   (64, 33, 128), (1, 7, 3), (700, 333, 220)])
def test_gemm_nn_exact_integers(gpu_lib, dt, m, K, c):
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(m * 7 + K + c)
    A = _int_matrix(rng, (m, K))
    X = _int_matrix(rng, (K, c), -4, 4)
    xdt = torch.float64 if dt == "f64" else torch.float32
    Ag = torch.tensor(A, dtype=DT[dt], device=DEV)
    Xg = torch.tensor(X, dtype=xdt, device=DEV)
    Y = _np(api.gemm_nn(Ag, Xg))
    assert np.array_equal(Y, A @ X)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("m,n,c", [(300, 257, 5), (5000, 129, 30), (20000, 300, 100), (77, 1000, 64),
                                   (3, 5, 2), (3000, 250, 256)])
def test_gemm_tn_exact_integers(gpu_lib, dt, m, n, c):
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(m + 3 * n + c)
    A = _int_matrix(rng, (m, n), -4, 4)
    Q = _int_matrix(rng, (m, c), -3, 3)
    xdt = torch.float64 if dt == "f64" else torch.float32
    Z = _np(api.gemm_tn(torch.tensor(A, dtype=DT[dt], device=DEV), torch.tensor(Q, dtype=xdt, device=DEV)))
    assert np.array_equal(Z, A.T @ Q)


def test_gemm_random_f64_accuracy_and_strided_input(gpu_lib):
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(5)
    A = rng.standard_normal((700, 333))
    big = np.zeros((700, 340))
    big[:, :333] = A
    Ag = torch.tensor(big, device=DEV)[:, :333]          # lda = 340 > n
    X = rng.standard_normal((333, 40))
    Y = _np(api.gemm_nn(Ag, torch.tensor(X, device=DEV)))
    np.testing.assert_allclose(Y, A @ X, rtol=0, atol=1e-12 * np.abs(A).max() * np.abs(X).max() * 333)
    Q = rng.standard_normal((700, 40))
    Z = _np(api.gemm_tn(Ag, torch.tensor(Q, device=DEV)))
    np.testing.assert_allclose(Z, A.T @ Q, rtol=0, atol=1e-12 * 700 * 4)


@pytest.mark.parametrize("dt,tol", [("f64", 1e-13), ("f32", 2e-6)])
@pytest.mark.parametrize("m,c", [(5000, 30), (1000, 128), (33, 17), (20000, 100), (3000, 73), (4000, 96), (777, 65),
                                 (2000, 81)])
def test_orthonormalize_matches_householder(gpu_lib, dt, tol, m, c):
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(m + c)
    Y = rng.standard_normal((m, c)) @ np.diag(np.logspace(0, -3, c))
    Yd = DT[dt]
    Yg = torch.tensor(Y, dtype=Yd, device=DEV)
    Yin = _np(Yg).astype(np.float64)
    Qg, Rg, flags = api.orthonormalize(Yg)
    Q, R = _np(Qg).astype(np.float64), _np(Rg)
    np.testing.assert_allclose(Q.T @ Q, np.eye(c), atol=tol * 10)
    assert np.allclose(np.tril(R, -1), 0) and np.all(np.diag(R) > 0)
    np.testing.assert_allclose(Q @ R, Yin, atol=tol * np.abs(Yin).max() * 10)
    Qh, Rh = orc.hqr(Yin)
    np.testing.assert_allclose(R, Rh, rtol=0, atol=(3e-5 if dt == "f32" else 1e-11) * np.abs(Rh).max())


def test_orthonormalize_rank_deficient_uses_shift(gpu_lib):
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(1)
    base = rng.standard_normal((4000, 10))
    Y = np.concatenate([base, base[:, :5] * 2.0, base[:, :5] + 1e-14 * rng.standard_normal((4000, 5))], axis=1)
    Qg, Rg, flags = api.orthonormalize(torch.tensor(Y, device=DEV))
    Q = _np(Qg)
    assert np.all(np.isfinite(Q)) and np.all(np.isfinite(_np(Rg)))
    assert int(_np(flags)[0]) & 1          # shifted Cholesky was needed
    # the range of Y is contained in the range of Q
    resid = Y - Q @ (Q.T @ Y)
    assert np.abs(resid).max() < 1e-10


@pytest.mark.parametrize("c", [1, 2, 7, 30, 64, 89, 100, 128])
def test_small_svd_matches_lapack(gpu_lib, c):
    """W orthonormal and s to LAPACK accuracy; J_i = R^T w_i / s_i is accurate
    to about u s_1 / s_i, so J is checked column by column on that scale.

    Random triangular R are exponentially ill-conditioned, and some of these
    have singular values below the rounding level c u s_1.  There no SVD
    method has relative accuracy (its backward error is u |R|), so s_i only
    has to lie within the absolute bound, and J_i, which divides by s_i, is
    checked only for s_i above that level."""
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(c)
    R = np.triu(rng.standard_normal((c, c)))
    R[np.diag_indices(c)] = np.abs(R[np.diag_indices(c)]) + 0.1
    s, W, J, flags = api.small_svd(torch.tensor(R, device=DEV))
    s, W, J = _np(s), _np(W), _np(J)
    Ue, se, Vte = np.linalg.svd(R)
    np.testing.assert_allclose(s, se, rtol=1e-12, atol=1e-14 * se[0])
    np.testing.assert_allclose(W.T @ W, np.eye(c), atol=1e-12)
    assert int(_np(flags)[0]) & 8 == 0
    floor = 10 * c * 2.0 ** -53 * se[0]
    for i in range(c):
        if se[i] <= floor:
            continue
        tol = 1e-13 * se[0] / se[i] * c
        sep = min([abs(se[i] - se[j]) for j in range(c) if j != i] + [se[0]]) / se[0]
        np.testing.assert_allclose(R @ J[:, i], W[:, i] * s[i], atol=tol * se[0])
        if sep > 1e-6:           # well separated: the vectors are unique up to sign
            np.testing.assert_allclose(abs(J[:, i] @ Vte[i]), 1.0, atol=tol / sep)
            np.testing.assert_allclose(abs(W[:, i] @ Ue[:, i]), 1.0, atol=1e-12 / sep)


@pytest.mark.parametrize("arith", ["bf16", "split"])
@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("m,K,c", [(300, 257, 5), (517, 1000, 100), (64, 33, 128), (2000, 640, 30),
                                   (700, 520, 200), (260, 300, 256)])
def test_bf16_products_exact_integers(gpu_lib, arith, dt, m, K, c):
    """Integers of magnitude <= 8 are exact in bf16, so both bf16 modes are exact."""
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(m + K + c)
    A = _int_matrix(rng, (m, K))
    X = _int_matrix(rng, (K, c), -4, 4)
    Y = _np(api.gemm_nn(torch.tensor(A, dtype=DT[dt], device=DEV), torch.tensor(X, dtype=torch.float32,
                                                                                 device=DEV), arith))
    assert np.array_equal(Y, A @ X)
    Q = _int_matrix(rng, (m, c), -3, 3)
    Z = _np(api.gemm_tn(torch.tensor(A, dtype=DT[dt], device=DEV), torch.tensor(Q, dtype=torch.float32,
                                                                                device=DEV), arith))
    assert np.array_equal(Z, A.T @ Q)


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_split_bf16_is_f32_accurate(gpu_lib, dt):
    """Split products: the dropped A_lo X_lo term bounds the error near 2^-18 of
    |A||X| per product (a few times plain f32); plain bf16 products are ~2^-9."""
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(7)
    m, K, c = 3000, 700, 64
    Ag = torch.tensor(rng.standard_normal((m, K)), dtype=DT[dt], device=DEV)
    A = _np(Ag).astype(np.float64)
    Xg = torch.tensor(rng.standard_normal((K, c)), dtype=torch.float32, device=DEV)
    X = _np(Xg).astype(np.float64)
    ref = A @ X
    scale = np.abs(A).max() * np.abs(X).max() * np.sqrt(K)
    err_split = np.abs(_np(api.gemm_nn(Ag, Xg, "split")) - ref).max() / scale
    err_bf16 = np.abs(_np(api.gemm_nn(Ag, Xg, "bf16")) - ref).max() / scale
    err_f32 = np.abs(_np(api.gemm_nn(Ag, Xg)) - ref).max() / scale
    assert err_split < 2e-6 and err_split < 10 * max(err_f32, 1e-7)
    assert err_bf16 > 30 * err_split
    Qg = torch.tensor(rng.standard_normal((m, c)), dtype=torch.float32, device=DEV)
    refz = A.T @ _np(Qg).astype(np.float64)
    sz = np.abs(A).max() * np.sqrt(m) * 4
    assert np.abs(_np(api.gemm_tn(Ag, Qg, "split")) - refz).max() / sz < 1e-6


@pytest.mark.parametrize("c", [30, 100])
@pytest.mark.parametrize("shift", [-600, 600])
def test_small_svd_is_exactly_scale_invariant(gpu_lib, c, shift):
    """The Jacobi works on 2^-e R with 2^(e-1) <= max |R_ij| < 2^e, an exact
    scaling, so R 2^shift gives the singular values of R times 2^shift bit for
    bit and the same W -- also where the squared column norms of R 2^shift
    would overflow (shift = 600) or underflow (shift = -600) in f64."""
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(c + 7)
    R = np.triu(rng.standard_normal((c, c)))
    R[np.diag_indices(c)] = np.abs(R[np.diag_indices(c)]) + 0.5
    s0, W0, _, f0 = api.small_svd(torch.tensor(R, device=DEV))
    s1, W1, _, f1 = api.small_svd(torch.tensor(np.ldexp(R, shift), device=DEV))
    assert torch.equal(s1, torch.ldexp(s0, torch.tensor(shift, device=DEV)))
    assert torch.equal(W1, W0)
    assert int(_np(f1)[0]) & 8 == 0
    se = np.linalg.svd(R, compute_uv=False)     # (ill-conditioned R: absolute floor as above)
    np.testing.assert_allclose(np.ldexp(_np(s1), -shift), se, rtol=1e-12, atol=1e-14 * se[0])


@pytest.mark.parametrize("dt,arith", [("f64", "storage"), ("f32", "storage"), ("bf16", "storage"),
                                      ("f32", "bf16"), ("f32", "split"), ("bf16", "split")])
@pytest.mark.parametrize("m,K,c,splits", [(2000, 4100, 100, 3), (777, 3001, 220, 4), (129, 2048, 30, 2),
                                          (300, 257, 64, 4)])
def test_gemm_nn_split_k_exact_integers(gpu_lib, dt, arith, m, K, c, splits):
    """A X with its K-reduction split into partial blocks (the form rsvd_run
    takes when the row tiles alone leave most of the device idle), summed in
    chunk order: on small integers every partial sum is exact, so the result
    equals A X bit for bit whatever the split; at (300, 257) the chunks are
    rounded up to the tile's K-step, so the last ones reach past K (partly
    or wholly) and must contribute zeros."""
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(m + K + c + splits)
    A = _int_matrix(rng, (m, K), -4, 4)
    X = _int_matrix(rng, (K, c), -4, 4)
    xdt = torch.float64 if dt == "f64" else torch.float32
    Ag = torch.tensor(A, dtype=DT[dt], device=DEV)
    Xg = torch.tensor(X, dtype=xdt, device=DEV)
    Y = _np(api.gemm_nn(Ag, Xg, arith, splits=splits))
    assert np.array_equal(Y, A @ X)


@pytest.mark.parametrize("splits", [0, 2, 3, 4])
def test_gemm_nn_split_k_random_f64(gpu_lib, splits):
    """Random f64 operands: each split (and the split rsvd_run picks, 0) agrees
    with the exact product to the rounding of a K-term dot product."""
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(11 + splits)
    m, K, c = 20000, 4096, 120
    A = rng.standard_normal((m, K))
    X = rng.standard_normal((K, c))
    Y = _np(api.gemm_nn(torch.tensor(A, device=DEV), torch.tensor(X, device=DEV), splits=splits))
    ref = A @ X
    np.testing.assert_allclose(Y, ref, rtol=0, atol=K * 2.0 ** -52 * np.sqrt(K) * 4)
