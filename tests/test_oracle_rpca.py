"""Pins of the oracle's PCA extras (Sec. 4.1 and 4.3): correlation PCA
(scale), loadings, whitened components, total variance and predict.

Each is pinned against something other than the oracle's own formulas:
* at l = min(m, n) the randomized PCA is exact, so eigvals and rotation equal
  the eigen-decomposition of numpy's covariance / correlation matrix (library
  routines on the data, not on the oracle's intermediate values);
* the loadings factor the covariance (squared column sums = eigenvalues,
  squared row sums = the variables' variances once k covers the rank);
* whitened components are uncorrelated with unit variance;
* predict on the training rows returns the training components;
* scaling a column by any positive factor leaves correlation PCA unchanged;
* a constant column drops out of correlation PCA (flagged, no division by 0).
"""
import numpy as np
import pytest

from oracle import rsvd as orc


def _data(m, n, seed, offset=3.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) @ np.diag(np.linspace(3.0, 0.2, n)) @ rng.standard_normal((n, n)) * 0.3
    return A + offset * rng.standard_normal(n)[None, :]


def _match_vectors(V, W):
    for i in range(V.shape[1]):
        assert abs(abs(float(V[:, i] @ W[:, i])) - 1.0) < 1e-9, i


@pytest.mark.parametrize("scale", [False, True])
def test_full_width_pca_equals_eigendecomposition(scale):
    m, n, k = 300, 12, 11
    A = _data(m, n, 1)
    res = orc.rpca(A, k, p=5, q=1, scale=scale, seed=3)       # l = min(m, n) = 12
    C = np.corrcoef(A, rowvar=False) if scale else np.cov(A, rowvar=False)
    w, E = np.linalg.eigh(C)
    w, E = w[::-1], E[:, ::-1]
    np.testing.assert_allclose(res["eigvals"], w[:k], rtol=1e-10)
    _match_vectors(res["rotation"], E[:, :k])
    np.testing.assert_allclose(res["total_var"], np.trace(C), rtol=1e-12)
    if scale:
        np.testing.assert_allclose(res["scale"], A.std(axis=0, ddof=1), rtol=1e-13)
        assert res["total_var"] == pytest.approx(n, rel=1e-12)


def test_loadings_factor_the_covariance():
    rng = np.random.default_rng(2)
    m, n, r, k = 400, 8, 5, 6
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n)) + rng.standard_normal(n)[None, :]
    res = orc.rpca(A, k, p=2, q=2, seed=4)                     # centred rank 5 <= k
    L = res["loadings"]
    np.testing.assert_allclose(np.sum(L * L, axis=0), res["eigvals"], rtol=1e-12)
    np.testing.assert_allclose(np.sum(L * L, axis=1), A.var(axis=0, ddof=1), rtol=1e-9)
    np.testing.assert_allclose(L @ L.T, np.cov(A, rowvar=False), atol=1e-10 * np.abs(A).max() ** 2)


def test_whitened_components_have_unit_covariance():
    A = _data(500, 20, 5)
    res = orc.rpca(A, 6, p=10, q=2, seed=6)
    Z = res["x_white"]
    np.testing.assert_allclose(Z.mean(axis=0), 0.0, atol=1e-12)
    np.testing.assert_allclose(Z.T @ Z / (A.shape[0] - 1), np.eye(6), atol=1e-10)


@pytest.mark.parametrize("scale", [False, True])
def test_predict_on_training_rows_returns_the_components(scale):
    A = _data(200, 15, 7)
    res = orc.rpca(A, 14, p=5, q=1, scale=scale, seed=8)      # l = min(m, n): exact decomposition
    np.testing.assert_allclose(orc.rpca_predict(res, A), res["x"], atol=1e-10 * np.abs(res["x"]).max())
    # rows that are the training mean map to zero
    assert np.abs(orc.rpca_predict(res, res["center"][None, :])).max() < 1e-12


def test_correlation_pca_is_invariant_to_column_units():
    A = _data(600, 30, 9)
    c = np.exp(np.random.default_rng(10).uniform(-5, 5, size=30))
    r1 = orc.rpca(A, 5, p=10, q=2, scale=True, seed=11)
    r2 = orc.rpca(A * c[None, :], 5, p=10, q=2, scale=True, seed=11)
    np.testing.assert_allclose(r2["eigvals"], r1["eigvals"], rtol=1e-10)
    np.testing.assert_allclose(r2["rotation"], r1["rotation"], atol=1e-9)
    np.testing.assert_allclose(r2["x"], r1["x"], atol=1e-9 * np.abs(r1["x"]).max())


def test_constant_column_drops_out_of_correlation_pca():
    A = _data(300, 10, 12)
    B = np.concatenate([A[:, :4], np.full((300, 1), 2.5), A[:, 4:]], axis=1)
    r1 = orc.rpca(A, 9, p=3, q=1, scale=True, seed=13)          # l = 10 = n: exact
    r2 = orc.rpca(B, 9, p=3, q=1, scale=True, seed=13)          # l = 11 = n: exact
    assert r2["zero_scale"][4] and r2["scale"][4] == 1.0 and not np.any(r2["zero_scale"][np.arange(11) != 4])
    np.testing.assert_allclose(r2["eigvals"], r1["eigvals"], rtol=1e-10)
    np.testing.assert_allclose(r2["rotation"][4], 0.0, atol=1e-12)
    assert r2["total_var"] == pytest.approx(10.0, rel=1e-12)
