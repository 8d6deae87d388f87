"""Learned batches (rsvd_batch_create_learned): sketch features, network and
choice of q on the device, then each solve from its own q = 0 sketch.

* theta = None: every matrix runs the fallback q = 3; singular values match
  the FP64 oracle's rsvd with (q, p) = (3, p) and the matrix's Omega stream
  (f64: elementwise 1e-10).
* With a network: the chosen q equals the rule applied on the host to the
  network's probabilities on the same features (fewest iterations whose
  classes hold mass >= tau, sums in the same order in float64), and every
  solve matches the oracle's rsvd at (q_b, p) (f32: normwise 1e-4 sigma_1 and
  elementwise 1e-4 where sigma_i >= 1e-3 sigma_1; bf16 mixed mode: normwise
  2e-3 sigma_1).
"""
import numpy as np
import pytest
import torch

from oracle import rsvd as orc
from synth import matrices as syn

pytestmark = pytest.mark.gpu
DEV = "cuda"

SHAPES = [(333, 257, 7), (257, 333, 9), (1000, 100, 50), (800, 300, 20), (4000, 700, 64), (300, 64, 30),
          (1200, 500, 12), (520, 260, 22), (129, 65, 40)]


def _np(t):
    return t.detach().cpu().to(torch.float64).numpy()


def _mats(dtype, seed0):
    out = []
    for b, (m, n, k) in enumerate(SHAPES):
        kind = "poly" if b % 2 else "exp"
        sig = syn.spectrum(kind, min(m, n), alpha=0.5 + 0.3 * b) if kind == "poly" else \
            syn.spectrum("exp", min(m, n), tau=3.0 + 8 * b)
        out.append(torch.tensor(syn.planted(m, n, sig, seed0 + b), dtype=dtype, device=DEV))
    return out


def q_rule(prob, tau, p_solve=20):
    """Host statement of the device rule (float64 sums in class order): the
    fewest q whose pairs (q' <= q, p' <= p_solve) hold mass >= tau, else 4."""
    out = []
    for pb in prob:
        if tau <= 0:
            out.append(int(np.argmax(pb)) // 3)
            continue
        cum, pick = 0.0, 4
        for q in range(5):
            for j, pp in enumerate((5, 10, 20)):
                if pp <= p_solve:
                    cum += float(pb[3 * q + j])
            if cum >= tau:
                pick = q
                break
        out.append(pick)
    return np.array(out)


def _check_f32(s, so):
    s1 = so[0]
    assert np.max(np.abs(s - so)) <= 1e-4 * s1
    big = so >= 1e-3 * s1
    np.testing.assert_allclose(s[big], so[big], rtol=1e-4)


def test_fallback_q3_matches_oracle_f64():
    from paper_1608_02148_amd import api
    As = _mats(torch.float64, 200)
    ks = [k for *_, k in SHAPES]
    bt = api.Batch(As, ks, p=20, seed=12, learned=True, theta=None, infos=True, stamps=True)
    bt.run()
    q = bt.choices()
    assert (q == 3).all()
    infos = bt.infos()
    st, hz = bt.stamps()
    for b, (A, k) in enumerate(zip(As, ks)):
        m, n, _ = SHAPES[b]
        _, so, _ = orc.rsvd(_np(A), k, p=20, q=3, seed=12, stream_id=b)
        np.testing.assert_allclose(_np(bt.S[b]), so, rtol=1e-10, err_msg=f"matrix {b}")
        assert infos[b].q == 3 and infos[b].l == min(k + 20, m, n)
        assert st[b, 1] > st[b, 0] > 0
    bt.close()


@pytest.mark.parametrize("tau,p", [(0.0, 20), (0.5, 20), (0.8, 20), (0.95, 20), (0.8, 10), (0.5, 5)])
def test_network_choice_and_solves_f32(tau, p):
    """The device's choice of q equals the host rule for the solves'
    oversampling p (pairs needing more oversampling than p do not count as
    covered), and each solve equals the oracle's with that (q, p)."""
    from paper_1608_02148_amd import api
    from paper_1608_02148_amd import learned as L
    theta, _ = L.load_checkpoint(device=DEV)
    As = _mats(torch.float32, 300)
    ks = [k for *_, k in SHAPES]
    bt = api.Batch(As, ks, p=p, seed=5, learned=True, theta=theta, tau=tau, infos=True)
    bt.run()
    q = bt.choices()
    # the same features as an RSVD_BATCH_FEATURES batch under the same seed
    fb = api.Batch(As, ks, seed=5, features=True)
    fb.run()
    prob, _ = api.mlp_forward(theta, fb.features)
    np.testing.assert_array_equal(q, q_rule(prob.cpu().numpy(), tau, p))
    infos = bt.infos()
    for b, (A, k) in enumerate(zip(As, ks)):
        assert infos[b].q == q[b]
        _, so, _ = orc.rsvd(_np(A), k, p=p, q=int(q[b]), seed=5, stream_id=b)
        _check_f32(_np(bt.S[b]), so)
    bt.close()
    fb.close()


def test_learned_batch_replays_bitwise_and_matches_own_qp_batch():
    """Two graph replays give identical bits; the solves equal an explicit
    per-matrix (q, p) batch with the chosen q to f32 accuracy."""
    from paper_1608_02148_amd import api
    from paper_1608_02148_amd import learned as L
    theta, _ = L.load_checkpoint(device=DEV)
    As = _mats(torch.float32, 400)
    ks = [k for *_, k in SHAPES]
    bt = api.Batch(As, ks, p=10, seed=9, learned=True, theta=theta, tau=0.8)
    bt.run()
    s1 = bt.s_flat.clone()
    u1 = bt.u_flat.clone()
    bt.run()
    torch.cuda.synchronize()
    assert torch.equal(s1, bt.s_flat) and torch.equal(u1, bt.u_flat)
    q = bt.choices()
    ref = api.Batch(As, ks, seed=9, qs=[int(x) for x in q], ps=[10] * len(ks))
    ref.run()
    torch.cuda.synchronize()
    for b in range(len(ks)):
        s, so = _np(bt.S[b]), _np(ref.S[b])
        assert np.max(np.abs(s - so)) <= 1e-4 * so[0], b
    bt.close()
    ref.close()


def test_bf16_mixed_learned_batch():
    from paper_1608_02148_amd import api
    from paper_1608_02148_amd import learned as L
    theta, _ = L.load_checkpoint(device=DEV)
    As = _mats(torch.float32, 500)
    ks = [k for *_, k in SHAPES]
    bt = api.Batch(As, ks, p=20, seed=7, learned=True, theta=theta, precision="bf16_mixed")
    bt.run()
    q = bt.choices()
    for b, (A, k) in enumerate(zip(As, ks)):
        _, so, _ = orc.rsvd(_np(A), k, p=20, q=int(q[b]), seed=7, stream_id=b)
        assert np.max(np.abs(_np(bt.S[b]) - so)) <= 2e-3 * so[0], b
    bt.close()
