"""Ragged batches (rsvd_batch_* through the C ABI) against the FP64 oracle.

Each matrix b of a batch is solved with Omega stream b, so the oracle call for
it is orc.rsvd(A_b, k_b, p, q, seed, stream_id=b).  Tolerances as for single
solves: f64 singular values 1e-10 relative; f32 normwise 1e-4 sigma_1 and
1e-4 relative where sigma_i >= 1e-3 sigma_1.
"""
import numpy as np
import pytest
import torch

from oracle import rsvd as orc
from synth import matrices as syn

pytestmark = pytest.mark.gpu
DEV = "cuda"

# Shapes spanning the three tile groups (l <= 32, <= 64, <= 128), wide and
# tall matrices, ragged tiles, q = 0 style small n, and l clamped by min(m, n).
SHAPES = [
    (333, 257, 7), (257, 333, 9), (1000, 100, 50), (64, 40, 1), (800, 300, 20),
    (4000, 700, 100), (1200, 64, 30), (300, 1024, 40), (2049, 515, 63), (520, 260, 22),
    (256, 64, 8), (700, 1300, 118),
]


def _np(t):
    return t.detach().cpu().to(torch.float64).numpy()


def _mats(dtype, shapes=SHAPES, seed0=100):
    out = []
    for b, (m, n, k) in enumerate(shapes):
        sig = syn.spectrum("poly", min(m, n), alpha=0.5 + (b % 5) * 0.5)
        out.append(torch.tensor(syn.planted(m, n, sig, seed0 + b), dtype=dtype, device=DEV))
    return out


def _check(bt, As, ks, p, q, seed, dtype, vec_tol):
    torch.cuda.synchronize()
    for b, (A, k) in enumerate(zip(As, ks)):
        A_inst = _np(A)
        Uo, so, Vo = orc.rsvd(A_inst, k, p=p, q=q, seed=seed, stream_id=b)
        s = _np(bt.S[b])
        if dtype == torch.float64:
            np.testing.assert_allclose(s, so, rtol=1e-10, atol=0, err_msg=f"matrix {b}")
        else:
            assert np.max(np.abs(s - so)) <= 1e-4 * so[0], b
            big = so >= 1e-3 * so[0]
            np.testing.assert_allclose(s[big], so[big], rtol=1e-4, err_msg=f"matrix {b}")
        U, V = _np(bt.U[b]), _np(bt.V[b])
        for i in range(k):
            gap = min(abs(so[i] - so[i + 1]) if i + 1 < len(so) else so[i],
                      abs(so[i - 1] - so[i]) if i > 0 else so[i])
            if gap <= 1e-3 * so[0]:
                continue
            assert float(V[:, i] @ Vo[:, i]) > 1 - vec_tol, (b, i)
            assert float(U[:, i] @ Uo[:, i]) > 1 - vec_tol, (b, i)


@pytest.mark.parametrize("graph", [True, False])
def test_batch_fp64_matches_oracle(graph):
    from paper_1608_02148_amd import api
    As = _mats(torch.float64)
    ks = [k for _, _, k in SHAPES]
    bt = api.Batch(As, ks, p=10, q=2, seed=77, graph=graph)
    bt.run()
    _check(bt, As, ks, 10, 2, 77, torch.float64, 1e-9)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_batch_fp32_matches_oracle(dtype):
    from paper_1608_02148_amd import api
    As = _mats(dtype, seed0=300)
    ks = [k for _, _, k in SHAPES]
    bt = api.Batch(As, ks, p=10, q=1, seed=5)
    bt.run()
    _check(bt, As, ks, 10, 1, 5, torch.float32, 1e-5)


def test_batch_matches_single_solves():
    """Same steps as rsvd_run: f64 results agree to the f64 tolerance."""
    from paper_1608_02148_amd import api
    As = _mats(torch.float64, seed0=500)
    ks = [k for _, _, k in SHAPES]
    bt = api.Batch(As, ks, p=8, q=2, seed=3)
    bt.run()
    torch.cuda.synchronize()
    for b, (A, k) in enumerate(zip(As, ks)):
        U, S, V = api.rsvd(A, k, p=8, q=2, seed=3, stream_id=b)
        torch.testing.assert_close(bt.S[b], S, rtol=1e-10, atol=0)


def test_graph_replays_are_identical_and_rerun_after_input_change():
    from paper_1608_02148_amd import api
    As = _mats(torch.float32, seed0=700)
    ks = [k for _, _, k in SHAPES]
    bt = api.Batch(As, ks, p=10, q=2, seed=9, graph=True)
    eager = api.Batch(As, ks, p=10, q=2, seed=9, graph=False)
    eager.run()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (eager.s_flat, eager.u_flat, eager.v_flat)]
    for rep in range(3):
        bt.run()
        torch.cuda.synchronize()
        for got, want in zip((bt.s_flat, bt.u_flat, bt.v_flat), ref):
            assert torch.equal(got, want), rep
        # unrelated eager work between replays
        junk = torch.randn(1000, 1000, device=DEV) @ torch.randn(1000, 1000, device=DEV)
        del junk
    # the graph reads A at replay time: scaling A by 2 scales S by 2 exactly
    for A in As:
        A.mul_(2.0)
    bt.run()
    torch.cuda.synchronize()
    assert torch.equal(bt.s_flat, 2.0 * ref[0])


def test_batch_infos_and_stamps():
    from paper_1608_02148_amd import api
    As = _mats(torch.float64, shapes=SHAPES[:6], seed0=900)
    As[2].zero_()                                   # a zero matrix is flagged, not NaN
    ks = [k for _, _, k in SHAPES[:6]]
    bt = api.Batch(As, ks, p=10, q=2, seed=1, stamps=True, infos=True)
    bt.run()
    infos = bt.infos()
    for b, inf in enumerate(infos):
        m, n, k = SHAPES[b]
        assert inf.l == min(k + 10, m, n) and inf.q == 2
    assert infos[2].flags & 2
    assert torch.all(bt.S[2] == 0)
    st, hz = bt.stamps()
    assert hz > 0
    assert np.all(st[:, 1] > st[:, 0]) and np.all(st[:, 0] > 0)


def test_batch_bf16_mixed():
    from paper_1608_02148_amd import api
    shapes = [(3000, 800, 40), (2000, 600, 20), (1500, 1000, 60)]
    As = []
    for b, (m, n, k) in enumerate(shapes):
        sig = syn.spectrum("exp", min(m, n), tau=20.0)
        As.append(torch.tensor(syn.planted(m, n, sig, 40 + b), dtype=torch.float32, device=DEV))
    ks = [k for _, _, k in shapes]
    bt = api.Batch(As, ks, p=10, q=2, seed=5, precision="bf16_mixed")
    bt.run()
    torch.cuda.synchronize()
    for b, (A, k) in enumerate(zip(As, ks)):
        A_inst = _np(A)
        Uo, so, Vo = orc.rsvd(A_inst, k, p=10, q=2, seed=5, stream_id=b)
        s = _np(bt.S[b])
        np.testing.assert_allclose(s[: k // 2], so[: k // 2], rtol=1e-4)
        r_gpu = orc.lowrank_residual(A_inst, _np(bt.U[b]), s, _np(bt.V[b]))
        r_ora = orc.lowrank_residual(A_inst, Uo, so, Vo)
        assert r_gpu <= 1.01 * r_ora


def test_batch_invalid_arguments():
    from paper_1608_02148_amd import api, lib
    A = torch.zeros(50, 20, device=DEV)
    B = torch.zeros(50, 20, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        api.Batch([A, B], [5, 5])
    with pytest.raises(lib.RsvdError):
        api.Batch([A, A], [5, 20])          # k >= min(m, n)
    big = torch.zeros(400, 300, device=DEV)
    with pytest.raises(lib.RsvdError):
        api.Batch([big], [125])            # l = 135 > the largest sketch width


def test_c4_full_batch_sampled_against_oracle():
    """The full 4096-matrix ragged batch in the benchmark's launch configuration
    (f32, p=10, q=2, one captured graph); a sample of solves is checked against
    the oracle on the stored instances."""
    from paper_1608_02148_amd import api
    c = syn.CONFIGS["ragged_4096"]
    data = syn.ragged_torch(device=DEV, batch=c["batch"], seed=c["gen_seed"])
    ks = [int(x) for x in data["k"]]
    bt = api.Batch(data["A"], ks, p=c["p"], q=c["q"], seed=c["omega_seed"], graph=True)
    bt.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    order = np.argsort(data["m"] * data["n"])
    sample = set(rng.choice(c["batch"], 4, replace=False).tolist()) | {int(order[0]), int(order[-1])}
    for b in sorted(sample):
        A_inst = _np(data["A"][b])
        k = ks[b]
        Uo, so, Vo = orc.rsvd(A_inst, k, p=c["p"], q=c["q"], seed=c["omega_seed"], stream_id=b)
        s = _np(bt.S[b])
        assert np.max(np.abs(s - so)) <= 1e-4 * so[0], b
        big = so >= 1e-3 * so[0]
        np.testing.assert_allclose(s[big], so[big], rtol=1e-4, err_msg=f"matrix {b}")
    assert torch.all(torch.isfinite(bt.s_flat))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_chunked_batch_equals_unchunked(dtype):
    """RSVD_BATCH_CHUNKED only changes which launches a solve shares (each
    size class split into chunks run one after another): every member's steps
    and kernels are the same, so the outputs are bit for bit those of the
    unchunked batch, and each member's device-clock span is recorded."""
    from paper_1608_02148_amd import api
    shapes = SHAPES * 6                        # several members per size class
    As = _mats(dtype, shapes, 700)
    ks = [k for _, _, k in shapes]
    ref = api.Batch(As, ks, p=10, q=2, seed=3)
    ref.run()
    ch = api.Batch(As, ks, p=10, q=2, seed=3, chunked=True, stamps=True)
    ch.run()
    torch.cuda.synchronize()
    assert torch.equal(ref.s_flat, ch.s_flat) and torch.equal(ref.u_flat, ch.u_flat)
    assert torch.equal(ref.v_flat, ch.v_flat)
    st, hz = ch.stamps()
    assert np.all(st[:, 1] > st[:, 0])
    ref.close()
    ch.close()
