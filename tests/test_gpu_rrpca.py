"""Robust PCA (Alg. rpca) on the GPU against the FP64 oracle.

The iteration takes integer decisions (the predicted rank: how many singular
values exceed 1/mu) from f64 singular values on both sides, so in f64 the two
runs follow the same path: same iteration count and ranks, L and S to
rounding.  In f32 the path may differ by an iteration at the stopping
threshold; the recovery of the planted low-rank and sparse parts is
compared instead (Sec. 5.5's synthetic study)."""
import numpy as np
import pytest
import torch

from oracle import rrpca as rr

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _np(t):
    return t.detach().cpu().to(torch.float64).numpy()


def _example(seed, m=300, n=300, k=5, frac=0.2):
    rng = np.random.default_rng(seed)
    L0 = rng.standard_normal((m, k)) @ rng.standard_normal((k, n))
    S0 = rng.uniform(-500, 500, (m, n)) * (rng.random((m, n)) < frac)
    return L0, S0


@pytest.mark.parametrize("m,n,k,seed", [(300, 300, 5, 1), (500, 260, 8, 2), (257, 700, 3, 3)])
def test_rrpca_f64_follows_the_oracle(m, n, k, seed):
    from paper_1608_02148_amd import api
    L0, S0 = _example(seed, m, n, k)
    A = L0 + S0
    res = api.rrpca(torch.tensor(A, device=DEV), seed=5)
    ora = rr.rrpca(A, seed=5, k_max=min(min(m, n) - 1, 246))
    assert res["iterations"] == ora["iterations"] and res["rank"] == ora["rank"]
    assert res["lam"] == pytest.approx(ora["lam"], rel=1e-15)
    np.testing.assert_allclose(_np(res["L"]), ora["L"], rtol=0, atol=1e-8 * np.abs(ora["L"]).max())
    np.testing.assert_allclose(_np(res["S"]), ora["S"], rtol=0, atol=1e-8 * np.abs(ora["S"]).max())
    assert res["residual"] == pytest.approx(ora["residual"], rel=1e-6)


def test_rrpca_f32_recovers_the_planted_parts():
    from paper_1608_02148_amd import api
    L0, S0 = _example(4, 600, 400, 6)
    res = api.rrpca(torch.tensor(L0 + S0, dtype=torch.float32, device=DEV), seed=2)
    assert res["rank"] == 6 and res["residual"] < 1e-5
    assert np.linalg.norm(_np(res["L"]) - L0) / np.linalg.norm(L0) < 1e-3
    assert np.linalg.norm(_np(res["S"]) - S0) / np.linalg.norm(S0) < 1e-4


def test_rrpca_rejects_bad_options():
    from paper_1608_02148_amd import api, lib
    A = torch.zeros(50, 40, device=DEV)
    with pytest.raises(lib.RsvdError):
        api.rrpca(A, maxiter=0)
    with pytest.raises(lib.RsvdError):
        api.rrpca(A.to(torch.bfloat16))
