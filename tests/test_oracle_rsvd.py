"""Pins for the FP64 rSVD / rPCA oracle (CPU only).

Each test ties the oracle to something other than itself: closed forms
(planted spectra, the Eckart-Young optimum, exact low-rank recovery), library
special cases (l = min(m, n) reduces to the full SVD), invariants (interlacing,
the Frobenius identity, scale and translation equivariance), a 50-digit brute
force on a tiny input, and the paper's expected-error bound tested in
expectation over seeds.
"""
import math

import numpy as np
import pytest

from oracle import rsvd as orc
from synth import matrices as syn

U64 = np.finfo(np.float64).eps


def _planted(m, n, sig, seed=0):
    return syn.planted(m, n, sig, seed)


def test_check_args_rejects_bad_rank():
    A = np.ones((10, 6))
    for k in (0, 6, 7):
        with pytest.raises(ValueError):
            orc.rsvd(A, k)
    with pytest.raises(ValueError):
        orc.rsvd(A, 2, p=-1)
    with pytest.raises(ValueError):
        orc.rsvd(A, 2, q=-1)


def test_hqr_is_a_qr_with_nonnegative_diagonal():
    Y = np.random.default_rng(0).standard_normal((50, 12))
    Q, R = orc.hqr(Y)
    np.testing.assert_allclose(Q.T @ Q, np.eye(12), atol=1e-14)
    np.testing.assert_allclose(Q @ R, Y, atol=1e-13)
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)


def test_exact_rank_is_recovered_without_power_iterations():
    """rank(A) <= l: range(A Omega) = range(A), so the result is exact (Sec. 2.1)."""
    sig = np.array([5.0, 3.0, 2.0, 1.5, 1.0, 0.7, 0.4, 0.1])
    A = _planted(80, 50, sig, seed=3)
    U, s, V, full = orc.rsvd(A, 6, p=4, q=0, seed=11, full=True)
    np.testing.assert_allclose(s, sig[:6], rtol=1e-12)
    assert orc.projection_residual(A, full["Q"]) < 1e-12
    np.testing.assert_allclose(U.T @ U, np.eye(6), atol=1e-13)
    np.testing.assert_allclose(V.T @ V, np.eye(6), atol=1e-13)
    np.testing.assert_allclose(A @ V, U * s, atol=1e-12)


@pytest.mark.parametrize("m,n", [(60, 40), (40, 60)])
def test_full_width_sketch_equals_the_full_svd(m, n):
    """l = min(m, n): Q spans the whole range, so the result is svd(A)."""
    A = np.random.default_rng(4).standard_normal((m, n))
    k = min(m, n) - 5
    U, s, V = orc.rsvd(A, k, p=20, q=1, seed=2)
    Ue, se, Vte = np.linalg.svd(A, full_matrices=False)
    np.testing.assert_allclose(s, se[:k], rtol=1e-12)
    np.testing.assert_allclose(np.abs(np.sum(U * Ue[:, :k], axis=0)), 1.0, atol=1e-9)
    np.testing.assert_allclose(np.abs(np.sum(V * Vte.T[:, :k], axis=0)), 1.0, atol=1e-9)


def test_interlacing_frobenius_identity_and_eckart_young():
    sig = syn.spectrum("poly", 200, alpha=0.8)
    A = _planted(400, 200, sig, seed=5)
    k, p = 20, 10
    U, s, V, full = orc.rsvd(A, k, p=p, q=1, seed=7, full=True)
    # interlacing: Q orthonormal, so sigma_i(Q^T A) <= sigma_i(A)
    assert np.all(full["s"] <= sig[: k + p] * (1 + 64 * U64))
    # ||A - U_k S_k V_k^T||_F^2 = ||A||_F^2 - sum s_i^2
    lhs = orc.lowrank_residual(A, U, s, V) ** 2
    rhs = np.sum(A * A) - np.sum(s * s)
    assert lhs == pytest.approx(rhs, rel=1e-10)
    # Eckart-Young lower bounds (Sec. 3.2), spectral and Frobenius
    assert orc.lowrank_residual(A, U, s, V, 2) >= sig[k] * (1 - 1e-12)
    assert orc.lowrank_residual(A, U, s, V) >= orc.eckart_young(sig, k)[1] * (1 - 1e-12)
    assert orc.projection_residual(A, full["Q"], 2) >= sig[k + p] * (1 - 1e-12)


def test_singular_vectors_satisfy_the_svd_relations():
    sig = syn.spectrum("exp", 120, tau=10.0)
    A = _planted(300, 120, sig, seed=6)
    U, s, V, full = orc.rsvd(A, 10, p=10, q=2, seed=1, full=True)
    B = full["B"]
    Q = full["Q"]
    # B = U~ S V^T with U = Q U~  =>  Q^T U S = B V and A^T U = V S up to the projection
    np.testing.assert_allclose(Q.T @ U * s, B @ V, atol=1e-13)
    np.testing.assert_allclose(A.T @ U, V * s, atol=1e-12)


def test_sign_rule():
    A = np.random.default_rng(8).standard_normal((70, 30))
    _, _, V = orc.rsvd(A, 5, seed=3)
    idx = np.argmax(np.abs(V), axis=0)
    assert np.all(V[idx, np.arange(5)] > 0)


def test_power_of_two_scaling_is_exact():
    A = np.random.default_rng(9).standard_normal((90, 40))
    U1, s1, V1 = orc.rsvd(A, 8, seed=4)
    U2, s2, V2 = orc.rsvd(A * 2.0 ** 7, 8, seed=4)
    np.testing.assert_allclose(s2, s1 * 2.0 ** 7, rtol=1e-14)
    np.testing.assert_allclose(U2, U1, atol=1e-13)
    np.testing.assert_allclose(V2, V1, atol=1e-13)


def test_subspace_iteration_spans_the_direct_power_subspace():
    """Alg. subspace_iter and Alg. poweriter_direct span range((A A^T)^q A Omega)."""
    sig = np.linspace(2.0, 1.0, 30)
    A = _planted(100, 30, sig, seed=10)
    from oracle import philox
    om = philox.test_matrix(30, 8, seed=12)
    Y1 = orc.sub_iterations(A, A @ om, 2)
    Y2 = orc.power_iterations(A, A @ om, 2)
    Q1, _ = orc.hqr(Y1)
    Q2, _ = orc.hqr(Y2)
    cosines = np.linalg.svd(Q1.T @ Q2, compute_uv=False)
    np.testing.assert_allclose(cosines, 1.0, atol=1e-10)


def test_tiny_input_against_50_digit_svd():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    rng = np.random.default_rng(13)
    A = rng.integers(-9, 10, size=(8, 6)).astype(np.float64)
    U, s, V = orc.rsvd(A, 5, p=3, q=1, seed=5)      # l = 6 = min(m, n)
    exact = mp.svd_r(mp.matrix(A.tolist()), compute_uv=False)
    exact = sorted([float(x) for x in exact], reverse=True)
    np.testing.assert_allclose(s, exact[:5], rtol=1e-13)


def _mean_spectral_error(A, k, p, q, seeds):
    errs = []
    for sd in seeds:
        U, s, V = orc.rsvd(A, k, p=p, q=q, seed=sd)
        errs.append(orc.lowrank_residual(A, U, s, V, 2))
    return float(np.mean(errs))


@pytest.mark.parametrize("q", [0, 1, 2])
def test_expected_error_bound_holds_in_mean(q):
    """Eq. rsvd_expected_error (Sec. 3.4), in expectation over 32 test matrices."""
    m, n, k, p = 200, 120, 10, 5
    sig = syn.spectrum("poly", 120, alpha=0.5)          # slow decay
    A = _planted(m, n, sig, seed=14)
    mean_err = _mean_spectral_error(A, k, p, q, range(32))
    bound = orc.expected_error_factor(m, n, k, p, q) * sig[k]
    assert sig[k] <= mean_err <= bound


def test_power_iterations_reduce_the_error():
    """The bound shrinks with q; a loop that does nothing would not."""
    m, n, k, p = 200, 120, 10, 5
    sig = syn.spectrum("poly", 120, alpha=0.5)
    A = _planted(m, n, sig, seed=14)
    e0 = _mean_spectral_error(A, k, p, 0, range(8))
    e2 = _mean_spectral_error(A, k, p, 2, range(8))
    assert e2 < e0 and e2 < 1.1 * sig[k]


def test_c1_planted_reference_values():
    A = syn.harmonic_2000x1000()
    sig = 1.0 / np.arange(1, 1001)
    s_full = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(s_full, sig, rtol=1e-11)
    assert math.sqrt(np.sum(A * A)) == pytest.approx(1.2822, abs=1e-4)
    spec, frob = orc.eckart_young(sig, 20)
    assert spec == pytest.approx(0.0476, abs=1e-4) and frob == pytest.approx(0.2186, abs=1e-4)
    U, s, V, full = orc.rsvd(A, 20, p=10, q=2, seed=2148, full=True)
    assert np.all(s <= sig[:20] * (1 + 1e-13))
    np.testing.assert_allclose(s[:10], sig[:10], rtol=2e-3)
    assert orc.projection_residual(A, full["Q"]) >= orc.eckart_young(sig, 30)[1] * (1 - 1e-12)


def test_rpca_translation_invariance_and_definitions():
    rng = np.random.default_rng(15)
    A = _planted(150, 60, syn.spectrum("exp", 60, tau=8.0), seed=16)
    shift = rng.standard_normal(60) * 3.0
    r1 = orc.rpca(A, 6, p=10, q=2, seed=3)
    r2 = orc.rpca(A + shift[None, :], 6, p=10, q=2, seed=3)
    np.testing.assert_allclose(r2["eigvals"], r1["eigvals"], rtol=1e-10)
    np.testing.assert_allclose(r2["rotation"], r1["rotation"], atol=1e-9)
    np.testing.assert_allclose(r2["x"], r1["x"], atol=1e-9)
    np.testing.assert_allclose(r2["center"] - r1["center"], shift, atol=1e-12)
    assert np.all(r1["eigvals"] == r1["s"] ** 2 / 149)
    np.testing.assert_allclose(r1["sdev"] ** 2, r1["eigvals"], rtol=1e-15)


def test_rpca_full_width_equals_covariance_eigendecomposition():
    rng = np.random.default_rng(17)
    A = rng.standard_normal((80, 12)) @ np.diag(np.linspace(3, 0.5, 12)) + 2.0
    res = orc.rpca(A, 10, p=5, q=0, seed=1)                  # l = 12 = n
    X = A - A.mean(axis=0)
    w, W = np.linalg.eigh(X.T @ X / 79)
    w, W = w[::-1], W[:, ::-1]
    np.testing.assert_allclose(res["eigvals"], w[:10], rtol=1e-11)
    np.testing.assert_allclose(np.abs(np.sum(res["rotation"] * W[:, :10], axis=0)), 1.0, atol=1e-9)
    np.testing.assert_allclose(res["x"], X @ res["rotation"], atol=1e-10)


@pytest.mark.parametrize("m,n,k,p,q,want", [
    (2000, 1000, 20, 10, 2, 2.18),        # 2000 x 1000, k = 20, p = 10, q = 2
    (100000, 5000, 100, 20, 2, 2.55),     # 100000 x 5000, k = 100, p = 20, q = 2
    (200000, 20000, 200, 20, 1, 6.60),    # 200000 x 20000, k = 200, p = 20, q = 1..3
    (200000, 20000, 200, 20, 2, 3.10),
    (200000, 20000, 200, 20, 3, 2.25),
])
def test_expected_error_factor_values(m, n, k, p, q, want):
    """Eq. rsvd_expected_error evaluated independently (by hand, to two
    decimals) at the benchmark workloads' sizes."""
    assert orc.expected_error_factor(m, n, k, p, q) == pytest.approx(want, abs=0.005)


def test_expected_error_factor_closed_form():
    """k = 1, p = 2, min(m, n) = 10, q = 0: the bracket is
    1 + sqrt(1/1) + e sqrt(3) / 2 * sqrt(9) = 2 + 1.5 e sqrt(3) = 9.06230...;
    with q the bracket's (2q+1)-th root: q = 1 gives 2.08487...."""
    assert orc.expected_error_factor(10, 12, 1, 2, 0) == pytest.approx(9.06230, abs=1e-5)
    assert orc.expected_error_factor(12, 10, 1, 2, 1) == pytest.approx(9.06230 ** (1 / 3), abs=1e-5)
    assert orc.expected_error_factor(12, 10, 1, 2, 1) == pytest.approx(2.08487, abs=1e-5)
