"""Selector-network kernels (through the C ABI) against the FP64 oracle.

Tolerances: forward probabilities 1e-5 relative (f32 sums of <= 131 terms);
gradients within 1e-4 of the largest oracle gradient entry of the same layer
(f32 accumulation over the batch); one Adam step within 1e-6 relative.
"""
import numpy as np
import pytest
import torch

from oracle import mlp as om

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _np(t):
    return t.detach().cpu().to(torch.float64).numpy()


def _data(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, om.N_IN)).astype(np.float32)
    X[:, :128] = np.abs(X[:, :128]) * 0.5
    y = rng.integers(0, om.N_OUT, size=B).astype(np.int32)
    return X, y


def _theta(seed):
    return (np.random.default_rng(seed).standard_normal(om.N_PARAMS) * 0.2).astype(np.float32)


def test_init_is_he_uniform_and_deterministic():
    from paper_1608_02148_amd import api
    t1 = _np(api.mlp_init(seed=11))
    t2 = _np(api.mlp_init(seed=11))
    assert np.array_equal(t1, t2)
    P = om.unpack(t1)
    for name, fan in (("W1", 131), ("W2", 64), ("W3", 64)):
        a = np.sqrt(6.0 / fan)
        assert np.all(np.abs(P[name]) <= a) and np.std(P[name]) > 0.4 * a
    for name in ("b1", "b2", "b3"):
        assert np.all(P[name] == 0)


@pytest.mark.parametrize("B", [1, 37, 512])
def test_forward_matches_oracle(B):
    from paper_1608_02148_amd import api
    X, _ = _data(B, 1)
    th = _theta(2)
    prob, cls = api.mlp_forward(torch.tensor(th, device=DEV), torch.tensor(X, device=DEV))
    f = om.forward(th.astype(np.float64), X.astype(np.float64))
    np.testing.assert_allclose(_np(prob), f["prob"], rtol=1e-5, atol=1e-7)
    agree = np.mean(_np(cls).astype(int) == np.argmax(f["z"], axis=1))
    assert agree >= 0.99


@pytest.mark.parametrize("B", [5, 256, 3000])
def test_gradients_match_oracle(B):
    from paper_1608_02148_amd import api
    X, y = _data(B, 3)
    th = _theta(4)
    tr = api.MlpTrainer(torch.tensor(th, device=DEV))
    loss = tr.step(torch.tensor(X, device=DEV), torch.tensor(y, device=DEV), update=False)
    lo, go = om.loss_and_grad(th.astype(np.float64), X.astype(np.float64), y)
    assert float(loss) == pytest.approx(lo, rel=1e-5)
    g = _np(tr.grad)
    off = 0
    for name, shape in om.SHAPES:
        size = int(np.prod(shape))
        a, b = g[off:off + size], go[off:off + size]
        assert np.max(np.abs(a - b)) <= 1e-4 * np.max(np.abs(b)), name
        off += size
    # the parameters are untouched by a gradient-only step
    assert np.array_equal(_np(tr.theta).astype(np.float32), th)


def test_adam_steps_match_oracle():
    from paper_1608_02148_amd import api
    X, y = _data(64, 5)
    th = _theta(6)
    tr = api.MlpTrainer(torch.tensor(th, device=DEV), lr=1e-3)
    t, m, v = th.astype(np.float64), np.zeros(om.N_PARAMS), np.zeros(om.N_PARAMS)
    for step in range(1, 4):
        tr.step(torch.tensor(X, device=DEV), torch.tensor(y, device=DEV))
        _, g = om.loss_and_grad(t, X.astype(np.float64), y)
        # the oracle step uses the GPU's gradient so only the update is compared
        g_gpu = _np(tr.grad)
        t, m, v = om.adam_step(t, g_gpu, m, v, step, 1e-3)
        np.testing.assert_allclose(_np(tr.theta), t, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(g_gpu, g, atol=1e-4 * np.max(np.abs(g)))


def test_training_learns_a_separable_rule():
    """A rule the network can represent: class = 3 * floor(5 x0) + (x1 > 0)."""
    from paper_1608_02148_amd import api
    rng = np.random.default_rng(7)
    B = 2048
    X = np.zeros((B, om.N_IN), dtype=np.float32)
    X[:, 0] = rng.uniform(0, 0.999, B)
    X[:, 1] = rng.standard_normal(B)
    X[:, 2:] = rng.uniform(0, 0.1, (B, om.N_IN - 2))
    y = (3 * np.floor(5 * X[:, 0]) + (X[:, 1] > 0)).astype(np.int32)
    Xg, yg = torch.tensor(X, device=DEV), torch.tensor(y, device=DEV)
    tr = api.MlpTrainer(api.mlp_init(seed=1), lr=3e-3)
    first = float(tr.step(Xg, yg))
    for _ in range(600):
        tr.step(Xg, yg)
    last = float(tr.step(Xg, yg))
    _, cls = api.mlp_forward(tr.theta, Xg)
    acc = float(np.mean(_np(cls).astype(int) == y))
    assert last < 0.3 * first and acc > 0.9, (first, last, acc)


def test_mlp_load_round_trip(gpu_lib, tmp_path):
    """A checkpoint written from device vectors reads back bit for bit through
    rsvd_mlp_load (theta and both Adam moments)."""
    import struct
    from paper_1608_02148_amd import learned as L
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    vecs = [torch.randn(13583, generator=g, device="cuda") for _ in range(3)]
    path = tmp_path / "ck.bin"
    hdr = b"RSVDMLP1" + struct.pack("<IIIQQ", 1, 13583, 9, 4, 123) + b"\x01" * 8
    path.write_bytes(hdr + b"\0" * (64 - len(hdr)) + b"".join(v.cpu().numpy().astype("<f4").tobytes()
                                                              for v in vecs))
    (theta, m, v), info = L.load_checkpoint(str(path), device="cuda", adam=True)
    torch.cuda.synchronize()
    assert torch.equal(theta, vecs[0]) and torch.equal(m, vecs[1]) and torch.equal(v, vecs[2])
    assert info["step"] == 9 and info["n_train"] == 123 and info["seed"] == 4
