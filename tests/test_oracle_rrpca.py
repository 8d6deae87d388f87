"""Pins of the robust PCA oracle (Alg. rpca, Sec. 5).

* The paper's synthetic study (Sec. 5.5): a 300 x 300 rank-5 product of
  Gaussian factors plus a sparse component with about 20 % entries uniform in
  [-500, 500]; robust PCA recovers both (the low-rank part to 1e-3, the
  rank exactly).
* Optimality of the convex problem min ||L||_* + lambda ||S||_1 s.t.
  A = L + S: the objective at the result is no larger than at the planted
  pair (which is feasible), and the final multiplier Z satisfies the dual
  conditions |Z_ij| <= lambda (equality on the support of S) and
  ||Z||_2 <= 1 up to the stopping tolerance.
* No corruption: S stays (near) zero and L equals A.
* shrink is the proximal map of tau |x| (checked by brute force).
"""
import numpy as np
import pytest

from oracle import rrpca as rr


def _paper_example(seed, m=300, n=300, k=5, frac=0.2):
    rng = np.random.default_rng(seed)
    L0 = rng.standard_normal((m, k)) @ rng.standard_normal((k, n))
    S0 = rng.uniform(-500, 500, (m, n)) * (rng.random((m, n)) < frac)
    return L0, S0


def _nuclear(X):
    return float(np.linalg.svd(X, compute_uv=False).sum())


@pytest.mark.parametrize("seed", [1, 2])
def test_recovers_the_papers_synthetic_example(seed):
    L0, S0 = _paper_example(seed)
    r = rr.rrpca(L0 + S0)
    assert r["rank"] == 5 and r["residual"] < 1e-5 and r["iterations"] < 50
    assert np.linalg.norm(r["L"] - L0) / np.linalg.norm(L0) < 1e-3
    assert np.linalg.norm(r["S"] - S0) / np.linalg.norm(S0) < 1e-4


def test_result_is_optimal_for_the_convex_problem():
    L0, S0 = _paper_example(3)
    r = rr.rrpca(L0 + S0, tol=1e-7, maxiter=100)
    lam, Z = r["lam"], r["Z"]
    obj = _nuclear(r["L"]) + lam * np.abs(r["S"]).sum()
    obj0 = _nuclear(L0) + lam * np.abs(S0).sum()
    assert obj <= obj0 * (1 + 1e-6)
    assert np.abs(Z).max() <= lam * (1 + 1e-9)
    on = np.abs(r["S"]) > 0
    np.testing.assert_allclose(np.abs(Z[on]), lam, rtol=1e-6)
    assert np.linalg.norm(Z, 2) <= 1.01


def test_uncorrupted_low_rank_input_gives_no_sparse_part():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((200, 4)) @ rng.standard_normal((4, 150))
    r = rr.rrpca(A)
    assert np.abs(r["S"]).max() <= 1e-3 * np.abs(A).max()
    assert np.linalg.norm(r["L"] - A) / np.linalg.norm(A) < 1e-4


def test_shrink_is_the_l1_proximal_map():
    grid = np.linspace(-5, 5, 200001)
    for v in (-3.0, -0.4, 0.0, 0.2, 1.7):
        for tau in (0.0, 0.5, 2.0):
            best = grid[np.argmin(0.5 * (grid - v) ** 2 + tau * np.abs(grid))]
            assert abs(rr.shrink(np.array([v]), tau)[0] - best) <= 1e-4
