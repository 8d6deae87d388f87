"""Sketch widths above 128 (single solves, up to RSVD_MAX_L_SINGLE = 256):
blocked Cholesky on 128-blocks and the Jacobi with its matrix in global
memory, against the FP64 oracle.

Tolerances as for the narrow path: f64 singular values elementwise 1e-10
relative; f32 arithmetic normwise 1e-4 sigma_1 (elementwise 1e-4 where
sigma_i >= 1e-3 sigma_1); mixed mode normwise 2e-3 sigma_1.  Vectors: cosine
with the oracle's where the gap to the neighbours exceeds 1e-3 sigma_1.
Orthonormality of the f64 factors: U's columns come from J_i = R_b^T w_i /
sigma_i, accurate to about l u sigma_1 / sigma_i, so U^T U = I is checked to
4 l u sigma_1 / sigma_k (1e-11 at sigma_1 / sigma_k = 236, l = 256; the narrow
path's 2000 x 1000 f64 test, l = 30 and sigma_1 / sigma_k = 20, is the same bound).
"""
import numpy as np
import pytest
import torch

from oracle import learned as orl
from oracle import rsvd as orc
from synth import matrices as syn

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _np(t):
    return None if t is None else t.detach().cpu().to(torch.float64).numpy()


def _gap_ok(s, i, rel=1e-3):
    lo = abs(s[i] - s[i + 1]) if i + 1 < len(s) else s[i]
    hi = abs(s[i - 1] - s[i]) if i > 0 else s[i]
    return min(lo, hi) > rel * s[0]


@pytest.mark.parametrize("m,n,k,p,q", [(2500, 1200, 200, 20, 1), (2000, 600, 236, 20, 1), (700, 1500, 140, 5, 2)])
def test_wide_sketch_f64_matches_oracle(m, n, k, p, q):
    from paper_1608_02148_amd import api
    A = syn.planted(m, n, syn.spectrum("inverse", min(m, n)), m + n)
    Ag = torch.tensor(A, device=DEV)
    info = api.new_info(DEV)
    U, S, V = api.rsvd(Ag, k, p=p, q=q, seed=11, info=info)
    st, rec = api.sync_info(info)
    assert st == 0 and rec.l == min(k + p, m, n)
    # the block sweeps (one launch, grid barriers between rounds) converged:
    # no sweep-limit / barrier time-out flag, and bits 24..31 count the sweeps
    assert not (rec.flags & 8) and 2 <= (rec.flags >> 24) <= 30, hex(rec.flags)
    Uo, so, Vo = orc.rsvd(A, k, p=p, q=q, seed=11)
    U, s, V = _np(U), _np(S), _np(V)
    np.testing.assert_allclose(s, so, rtol=1e-10)
    l = min(k + p, m, n)
    tol = 4 * l * 2.0 ** -53 * so[0] / so[-1]
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=tol)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=tol)
    for i in range(k):
        if _gap_ok(so, i):
            assert abs(U[:, i] @ Uo[:, i]) > 1 - 1e-8 and V[:, i] @ Vo[:, i] > 1 - 1e-8, i


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_wide_sketch_f32_arithmetic(dtype):
    from paper_1608_02148_amd import api
    m, n, k, p, q = 3000, 1500, 150, 30, 2
    A = syn.planted(m, n, syn.spectrum("exp", min(m, n), tau=60.0), 91)
    Ag = torch.tensor(A, dtype=dtype, device=DEV)
    A_inst = _np(Ag)
    U, S, V = api.rsvd(Ag, k, p=p, q=q, seed=4)
    _, so, _ = orc.rsvd(A_inst, k, p=p, q=q, seed=4)
    s = _np(S)
    assert np.max(np.abs(s - so)) <= 1e-4 * so[0]
    big = so >= 1e-3 * so[0]
    np.testing.assert_allclose(s[big], so[big], rtol=1e-4)
    np.testing.assert_allclose(_np(V).T @ _np(V), np.eye(k), atol=1e-5)


def test_wide_sketch_bf16_mixed():
    """The 200000 x 20000 bf16 workload's shape of problem at small size: bf16 storage, k = 200, p = 20."""
    from paper_1608_02148_amd import api
    m, n, k, p, q = 6000, 1000, 200, 20, 2
    A = syn.planted(m, n, syn.spectrum("poly", min(m, n), alpha=1.5), 5)
    Ag = torch.tensor(A, dtype=torch.bfloat16, device=DEV)
    A_inst = _np(Ag)
    U, S, V = api.rsvd(Ag, k, p=p, q=q, seed=7, precision="bf16_mixed")
    Uo, so, Vo = orc.rsvd(A_inst, k, p=p, q=q, seed=7)
    s = _np(S)
    assert np.max(np.abs(s - so)) <= 2e-3 * so[0]
    r_gpu = orc.lowrank_residual(A_inst, _np(U), s, _np(V))
    r_ora = orc.lowrank_residual(A_inst, Uo, so, Vo)
    assert r_gpu <= 1.01 * r_ora


def test_wide_rpca_and_estimate():
    from paper_1608_02148_amd import api
    m, n, k = 2000, 800, 150
    A = syn.planted(m, n, syn.spectrum("exp", n, tau=40.0), 13) + 0.3
    Ag = torch.tensor(A, device=DEV)
    info = api.new_info(DEV)
    res = api.rpca(Ag, k, p=10, q=1, seed=2, info=info, probes=6)
    st, rec = api.sync_info(info)
    assert st == 0
    ora = orc.rpca(A, k, p=10, q=1, seed=2)
    np.testing.assert_allclose(_np(res["eigvals"]), ora["eigvals"], rtol=1e-10)
    Xc = A - A.mean(axis=0)[None, :]
    ref = orl.posterior_estimate(Xc, _np(res["x"]), np.ones(k), _np(res["rotation"]), r=6, seed=2,
                                 stream_id=0x80000000)
    assert rec.est_err == pytest.approx(ref, rel=1e-9)


def test_wide_rank_deficient_input_is_finite():
    """Exact rank 140 < l = 170: the second Cholesky block sees a singular
    Schur complement; the shifted factorisation keeps everything finite and the
    trailing singular values vanish."""
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(3)
    A = rng.standard_normal((1500, 140)) @ rng.standard_normal((140, 900))
    Ag = torch.tensor(A, device=DEV)
    info = api.new_info(DEV)
    U, S, V = api.rsvd(Ag, 150, p=20, q=1, seed=1, info=info)
    api.sync_info(info)
    s = _np(S)
    se = np.linalg.svd(A, compute_uv=False)
    assert np.all(np.isfinite(s)) and np.all(np.isfinite(_np(U))) and np.all(np.isfinite(_np(V)))
    np.testing.assert_allclose(s[:140], se[:140], rtol=1e-8)
    assert np.all(s[140:] <= 1e-8 * se[0])


def test_widths_above_the_single_solve_limit_are_rejected():
    from paper_1608_02148_amd import api, lib
    Ag = torch.zeros(1000, 600, device=DEV)
    with pytest.raises(lib.RsvdError):
        api.rsvd(Ag, 240, p=20)          # l = 260 > 256


@pytest.mark.parametrize("dtype,k", [(torch.float32, 120), (torch.float32, 200), (torch.float64, 140)])
def test_wide_solves_are_deterministic(dtype, k):
    """Two solves of one matrix agree bitwise (with two column tiles the
    orthonormalisation's product does not overwrite its own input)."""
    from paper_1608_02148_amd import api
    A = syn.planted(6000, 900, syn.spectrum("poly", 900, alpha=1.0), 17)
    Ag = torch.tensor(A, dtype=dtype, device=DEV)
    outs = [api.rsvd(Ag, k, p=20, q=1, seed=5) for _ in range(3)]
    for U, S, V in outs[1:]:
        assert torch.equal(S, outs[0][1]) and torch.equal(U, outs[0][0]) and torch.equal(V, outs[0][2])
