"""Normalized power iterations (Alg. normalized_iter): the pivoted LU
normalisation on the GPU and the randomized SVD that uses it, against the
FP64 oracle.

* Up to 256 rows the tournament has a single block, so the pivots are those
  of partial pivoting: pivot rows equal the oracle's exactly, L and U to
  rounding.
* Taller bases: the tournament may pick other pivot rows, which is still a
  pivoted LU: L U = Y, L[piv] unit lower triangular, U upper triangular, and
  L spans the columns of Y.
* End to end: L spans what Q would, so the rSVD with either normalisation
  matches the oracle (which runs partial pivoting) to the usual tolerances.
"""
import numpy as np
import pytest
import torch

from oracle import rsvd as orc
from synth import matrices as syn

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _np(t):
    return t.detach().cpu().to(torch.float64).numpy()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
@pytest.mark.parametrize("m,c", [(256, 128), (200, 30), (64, 64), (129, 7)])
def test_single_block_equals_partial_pivoting(dtype, tol, m, c):
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(m + c)
    Yg = torch.tensor(rng.standard_normal((m, c)), dtype=dtype, device=DEV)
    Y = _np(Yg)
    Lg, U, piv, flags = api.lu_normalize(Yg.clone())
    Lo, Uo, pivo = orc.lu_factor(Y)
    assert np.array_equal(_np(piv).astype(int), pivo)
    assert int(_np(flags)[0]) & 3 == 0
    np.testing.assert_allclose(_np(U), Uo, rtol=0, atol=tol * np.abs(Uo).max() * c)
    np.testing.assert_allclose(_np(Lg), Lo, rtol=0, atol=tol * c)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11), (torch.float32, 3e-5)])
@pytest.mark.parametrize("m,c", [(257, 40), (5000, 120), (20000, 128), (1000, 16), (777, 100)])
def test_tournament_lu_is_a_pivoted_lu(dtype, tol, m, c):
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(3 * m + c)
    Yg = torch.tensor(rng.standard_normal((m, c)) @ np.diag(np.logspace(0, -2, c)), dtype=dtype, device=DEV)
    Y = _np(Yg)
    Lg, Ug, pivg, flags = api.lu_normalize(Yg.clone())
    L, U, piv = _np(Lg), _np(Ug), _np(pivg).astype(int)
    assert int(_np(flags)[0]) & 3 == 0
    assert len(set(piv.tolist())) == c and piv.min() >= 0 and piv.max() < m
    assert np.all(U == np.triu(U))
    Lp = L[piv]
    np.testing.assert_allclose(np.triu(Lp, 1), 0.0, atol=tol * 10)
    np.testing.assert_allclose(np.diag(Lp), 1.0, atol=tol * 10)
    np.testing.assert_allclose(L @ U, Y, rtol=0, atol=tol * np.abs(Y).max() * c)
    Q, _ = np.linalg.qr(L)
    resid = Y - Q @ (Q.T @ Y)
    assert np.abs(resid).max() <= tol * np.abs(Y).max() * c
    print(f"m={m} c={c}: max |L| = {np.abs(L).max():.3g}")


def test_rank_deficient_basis_is_flagged_and_finite():
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(9)
    base = rng.standard_normal((3000, 10))
    Y = np.concatenate([base, base[:, :4] * 3.0], axis=1)
    Lg, U, piv, flags = api.lu_normalize(torch.tensor(Y, device=DEV))
    assert int(_np(flags)[0]) & 2
    assert np.all(np.isfinite(_np(Lg))) and np.all(np.isfinite(_np(U)))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,n,k,p,q", [(3000, 600, 20, 10, 2), (777, 1030, 50, 14, 1), (20000, 4096, 100, 20, 2),
                                       (500, 120, 10, 10, 3)])
def test_rsvd_with_lu_iterations_matches_oracle(dtype, m, n, k, p, q):
    from paper_1608_02148_amd import api
    sig = syn.spectrum("exp", min(m, n), tau=20.0) if m * n < 5e7 else np.exp(-np.arange(1, 601) / 50.0)
    A = syn.planted(m, n, sig, m + n + 5)
    Ag = torch.tensor(A, dtype=dtype, device=DEV)
    A_inst = _np(Ag)
    U, S, V = api.rsvd(Ag, k, p=p, q=q, seed=7, scheme="lu")
    Uo, so, Vo = orc.rsvd(A_inst, k, p=p, q=q, seed=7, scheme="lu")
    s = _np(S)
    if dtype == torch.float64:
        np.testing.assert_allclose(s, so, rtol=1e-10)
        tol = 1e-9
    else:
        assert np.max(np.abs(s - so)) <= 1e-4 * so[0]
        tol = 1e-4
    Un, Vn = _np(U), _np(V)
    for i in range(k):
        gap = min(abs(so[i] - so[i + 1]) if i + 1 < k else so[i], abs(so[i - 1] - so[i]) if i else so[i])
        if gap > 1e-3 * so[0]:
            assert abs(float(Un[:, i] @ Uo[:, i])) > 1 - tol and abs(float(Vn[:, i] @ Vo[:, i])) > 1 - tol


def test_lu_scheme_rejected_for_wide_sketches():
    from paper_1608_02148_amd import api, lib
    A = torch.zeros(2000, 1000, device=DEV)
    with pytest.raises(lib.RsvdError):
        api.rsvd(A, 150, p=10, scheme="lu")
