"""Interpolative and CUR decompositions (Alg. rid, Alg. rcur) on the GPU
against the FP64 oracle.

The column and row choices are index decisions taken from f64 column norms on
both sides (the device recomputes the remaining norms at every step, LAPACK
updates them), so in f64 they agree exactly on inputs without near-ties; C and
R are gathered entries of A (bit-exact); Z and U agree to rounding.  In f32
the pivots may differ where two norms are within f32 rounding of each other:
there the index sets are checked for validity and the approximation error
against the oracle's."""
import numpy as np
import pytest
import torch

from oracle import rid as orid
from synth import matrices as syn

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _np(t):
    return t.detach().cpu().to(torch.float64).numpy()


def _mat(m, n, seed, decay=8.0):
    return syn.planted(m, n, syn.spectrum("exp", min(m, n), tau=decay), seed)


@pytest.mark.parametrize("m,n,k,p,q", [(2000, 1000, 20, 10, 1), (500, 3000, 30, 10, 0), (20000, 4096, 100, 20, 0),
                                       (300, 250, 1, 5, 2), (1200, 700, 90, 30, 1)])
def test_rid_f64_matches_oracle(m, n, k, p, q):
    from paper_1608_02148_amd import api
    A = _mat(m, n, m + n + k)
    res = api.rid(torch.tensor(A, device=DEV), k, p=p, q=q, seed=3)
    C, Z, J = orid.rid(A, k, p=p, q=q, seed=3)
    assert np.array_equal(_np(res["J"]).astype(int), J)
    assert np.array_equal(_np(res["C"]), C)
    np.testing.assert_allclose(_np(res["Z"]), Z, rtol=0, atol=1e-9 * max(1.0, np.abs(Z).max()))


def test_rid_indices_only_and_f32():
    from paper_1608_02148_amd import api
    m, n, k = 3000, 900, 25
    A = _mat(m, n, 5)
    Ag = torch.tensor(A, dtype=torch.float32, device=DEV)
    Ai = _np(Ag)
    J_only = _np(api.rid(Ag, k, seed=4, idx_only=True)["J"]).astype(int)
    res = api.rid(Ag, k, seed=4)
    J = _np(res["J"]).astype(int)
    assert np.array_equal(J, J_only) and len(set(J.tolist())) == k and J.min() >= 0 and J.max() < n
    assert np.array_equal(_np(res["C"]), Ai[:, J])
    Co, Zo, Jo = orid.rid(Ai, k, seed=4)
    err = np.linalg.norm(Ai - _np(res["C"]) @ _np(res["Z"]))
    err_o = np.linalg.norm(Ai - Co @ Zo)
    assert err <= 1.05 * err_o + 1e-6 * np.linalg.norm(Ai)
    np.testing.assert_allclose(_np(res["Z"])[:, J], np.eye(k), atol=0)


@pytest.mark.parametrize("m,n,k,p,q", [(1500, 800, 15, 10, 1), (600, 2000, 40, 10, 0), (9000, 3000, 64, 16, 1)])
def test_rcur_f64_matches_oracle(m, n, k, p, q):
    from paper_1608_02148_amd import api
    A = _mat(m, n, 2 * m + n)
    res = api.rcur(torch.tensor(A, device=DEV), k, p=p, q=q, seed=6)
    ora = orid.rcur(A, k, p=p, q=q, seed=6)
    assert np.array_equal(_np(res["J"]).astype(int), ora["J"])
    assert np.array_equal(_np(res["I"]).astype(int), ora["I"])
    assert np.array_equal(_np(res["C"]), ora["C"]) and np.array_equal(_np(res["R"]), ora["R"])
    U, Uo = _np(res["U"]), ora["U"]
    np.testing.assert_allclose(U, Uo, rtol=0, atol=1e-8 * np.abs(Uo).max())


def test_exact_rank_cur_reproduces_the_matrix():
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(8)
    A = rng.standard_normal((700, 9)) @ rng.standard_normal((9, 500))
    res = api.rcur(torch.tensor(A, device=DEV), 9, p=5, q=1, seed=1)
    approx = _np(res["C"]) @ _np(res["U"]) @ _np(res["R"])
    np.testing.assert_allclose(approx, A, atol=1e-9 * np.abs(A).max())


def test_bf16_storage_gathers_exact_entries():
    from paper_1608_02148_amd import api
    Ag = torch.tensor(_mat(800, 400, 9), dtype=torch.bfloat16, device=DEV)
    res = api.rcur(Ag, 12, seed=2)
    Ai = _np(Ag)
    J, I = _np(res["J"]).astype(int), _np(res["I"]).astype(int)
    assert np.array_equal(_np(res["C"]), Ai[:, J]) and np.array_equal(_np(res["R"]), Ai[I])
