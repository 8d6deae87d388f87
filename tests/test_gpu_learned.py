"""Learned (q, p) path on the GPU against the FP64 oracle.

* Sketch features (RSVD_BATCH_FEATURES) against oracle.learned.features on
  the stored instances.  Features are f32 outputs (values in [0, 1], rounded
  once to f32, error <= 2^-24): from f64 arithmetic within 1e-7, from f32
  arithmetic within 2e-5 (absolute: entries are singular values relative to
  the largest).
* Per-matrix (q, p) batches solve each matrix as rsvd_run does with that pair.
* rsvd_select picks the argmax class of the network on those features.
"""
import numpy as np
import pytest
import torch

from oracle import learned as lrn
from oracle import mlp as om
from oracle import rsvd as orc
from synth import matrices as syn

pytestmark = pytest.mark.gpu
DEV = "cuda"

SHAPES = [(333, 257, 7), (257, 333, 9), (1000, 100, 50), (800, 300, 20), (4000, 700, 64), (300, 64, 30),
          (1200, 500, 12), (520, 260, 22)]


def _np(t):
    return t.detach().cpu().to(torch.float64).numpy()


def _mats(dtype, seed0):
    out = []
    for b, (m, n, k) in enumerate(SHAPES):
        kind = "poly" if b % 2 else "exp"
        sig = syn.spectrum(kind, min(m, n), alpha=0.5 + 0.4 * b) if kind == "poly" else \
            syn.spectrum("exp", min(m, n), tau=3.0 + 10 * b)
        out.append(torch.tensor(syn.planted(m, n, sig, seed0 + b), dtype=dtype, device=DEV))
    return out


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-7), (torch.float32, 2e-5)])
def test_features_match_oracle(dtype, tol):
    from paper_1608_02148_amd import api
    As = _mats(dtype, 10)
    ks = [k for _, _, k in SHAPES]
    bt = api.Batch(As, ks, seed=31, features=True)
    bt.run()
    torch.cuda.synchronize()
    F = _np(bt.features)
    for b, (A, k) in enumerate(zip(As, ks)):
        f = lrn.features(_np(A), k, seed=31, stream_id=b)
        np.testing.assert_allclose(F[b], f, rtol=0, atol=tol, err_msg=f"matrix {b}")


def test_own_qp_batch_matches_single_solves():
    from paper_1608_02148_amd import api
    As = _mats(torch.float64, 40)
    ks = [k for _, _, k in SHAPES]
    qs = [b % 5 for b in range(len(SHAPES))]
    ps = [(5, 10, 20)[b % 3] for b in range(len(SHAPES))]
    bt = api.Batch(As, ks, seed=3, qs=qs, ps=ps)
    bt.run()
    torch.cuda.synchronize()
    for b, (A, k) in enumerate(zip(As, ks)):
        Uo, so, Vo = orc.rsvd(_np(A), k, p=ps[b], q=qs[b], seed=3, stream_id=b)
        np.testing.assert_allclose(_np(bt.S[b]), so, rtol=1e-10, err_msg=f"matrix {b}")


def test_select_picks_network_argmax():
    from paper_1608_02148_amd import api
    As = _mats(torch.float32, 70)
    ks = [k for _, _, k in SHAPES]
    theta = (np.random.default_rng(5).standard_normal(om.N_PARAMS) * 0.3).astype(np.float32)
    qs, ps, feats = api.select(As, ks, torch.tensor(theta, device=DEV), seed=17)
    F = _np(feats)
    z = om.forward(theta.astype(np.float64), F)["z"]
    for b in range(len(SHAPES)):
        top = np.sort(z[b])[::-1]
        if top[0] - top[1] < 1e-3:
            continue                      # a near tie may go either way in f32
        c = int(np.argmax(z[b]))
        assert (qs[b], ps[b]) == lrn.class_pair(c), b
    # the features it used are the sketch features
    for b, (A, k) in enumerate(zip(As, ks)):
        np.testing.assert_allclose(F[b], lrn.features(_np(A), k, seed=17, stream_id=b), rtol=0, atol=2e-5)


def test_select_decision_rule_matches_host_rule():
    from paper_1608_02148_amd import api
    from paper_1608_02148_amd import learned as L
    As = _mats(torch.float32, 90)
    ks = [k for _, _, k in SHAPES]
    theta, _ = L.load_checkpoint(device=DEV)
    for tau in (0.5, 0.8, 0.95):
        qs, ps, feats = api.select(As, ks, theta, seed=4, tau=tau)
        prob, _ = api.mlp_forward(theta, feats)
        pick = L.decide(prob.cpu().numpy(), ks, tau)
        assert [(int(q), int(p)) for q, p in zip(qs, ps)] == [L.CLASS_PAIRS[c] for c in pick]
