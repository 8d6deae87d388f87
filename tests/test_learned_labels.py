"""Host-side checks of the learned-(q, p) label machinery (CPU tensors).

* The generator plants exactly the stated spectrum (numpy SVD of the stored
  float64 instance) and keeps the reflection vectors of its left factor.
* The exact residual norm ||(I - U U^T) A||_2 computed from the planted
  factors and a Krylov iteration equals numpy's 2-norm of the residual.
* Labels pick the cheapest class under the stated cost order.
"""
import numpy as np
import torch

from oracle import learned as lrn
from oracle import rsvd as orc
from paper_1608_02148_amd import learned as L
from synth import learned_data as ld


def _small(count=6, split=77):
    return ld.build(count, split, device="cpu", out_dtype=torch.float64, m_range=(60, 200), n_range=(40, 120),
                    k_max=20)


def test_generator_plants_the_spectrum():
    data = _small()
    for b, A in enumerate(data["A"]):
        s = np.linalg.svd(A.numpy(), compute_uv=False)
        np.testing.assert_allclose(s, data["sigma"][b], rtol=1e-12, atol=1e-15 * s[0])
        a1, a2 = data["hh"][b]
        assert abs(float(a1.norm()) - 1) < 1e-14 and abs(float(a2.norm()) - 1) < 1e-14


def test_spectra_follow_the_recipe():
    spec = ld.shapes(2000, 5)
    assert 0.4 < spec["poly"].mean() < 0.6
    assert spec["nu"].min() >= 1e-8 and spec["nu"].max() <= 1e-2
    assert spec["tau"].min() >= 2 and spec["tau"].max() <= 200
    assert np.all(spec["k"] >= 8) and np.all(spec["k"] <= np.minimum(64, np.minimum(spec["m"], spec["n"]) - 10))
    s = ld.spectrum_of(spec, 0)
    assert s[0] == 1 + spec["nu"][0] and np.all(np.diff(s) <= 0)


def test_exact_residual_norm_matches_numpy():
    data = _small(8, 78)
    Us, want = [], []
    for b, A in enumerate(data["A"]):
        k = int(data["spec"]["k"][b])
        U, s, V = orc.rsvd(A.numpy(), k, p=5, q=b % 3, seed=1, stream_id=b)
        Us.append(torch.tensor(U))
        want.append(np.linalg.norm(A.numpy() - U @ (U.T @ A.numpy()), 2))
    got = L.residual_norms(data, Us, list(range(len(Us))), bucket=3)
    np.testing.assert_allclose(got, want, rtol=1e-9)


def test_labels_follow_cost_order():
    ks = [10, 30]
    tab = np.full((2, 15), 0.5)
    tab[0, lrn.pair_class(1, 5)] = 0.005       # cost 4 * 15 = 60
    tab[0, lrn.pair_class(0, 20)] = 0.009      # cost 2 * 30 = 60: same cost, lower class wins
    lab, ok = L.labels_from_table(tab, ks)
    assert ok[0] and lab[0] == lrn.pair_class(0, 20)
    assert not ok[1] and lab[1] == 14
    assert L.CLASS_PAIRS == [lrn.class_pair(c) for c in range(15)]
    for k in (8, 20, 64):
        assert L.classes_by_cost(k) == lrn.classes_by_cost(k)


def test_missing_or_corrupt_weights_fall_back_to_fixed_q(tmp_path):
    assert L.load_or_fallback(str(tmp_path / "absent.bin")) is None
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"RSVDMLP1" + b"\0" * 100)
    assert L.load_or_fallback(str(bad)) is None
    qs, ps = L.choose(None, [torch.zeros(300, 200)], [10])
    assert qs.tolist() == [3] and ps.tolist() == [10]


def test_committed_checkpoint_header():
    import struct
    raw = open(L.DEFAULT_CHECKPOINT, "rb").read()
    assert raw[:8] == L.MAGIC and len(raw) == 64 + 3 * 4 * 13583
    ver, npar, step, seed, ntrain = struct.unpack("<IIIQQ", raw[8:36])
    assert ver == 1 and npar == 13583 and step > 0 and ntrain > 0
    theta = np.frombuffer(raw, dtype="<f4", offset=64)[:npar]
    assert np.all(np.isfinite(theta))


def test_decision_rule():
    prob = np.zeros((2, 15))
    prob[0, lrn.pair_class(1, 10)] = 1.0          # certain: (1, 10)
    prob[1, lrn.pair_class(0, 5)] = 0.5           # split between (0, 5) and (2, 20)
    prob[1, lrn.pair_class(2, 20)] = 0.5
    pick = L.decide(prob, [20, 20], tau=0.8)
    assert pick[0] == lrn.pair_class(1, 10)
    # (2, 20) dominates both (0, 5) and itself: cumulative 1.0 >= 0.8, and no
    # cheaper class dominates both
    assert pick[1] == lrn.pair_class(2, 20)
    assert L.decide(prob, [20, 20], tau=0.4)[1] == lrn.pair_class(0, 5)


def test_dense_haar_data_and_their_residual_norms():
    """factors="haar": the planted spectrum is exact (numpy SVD of the stored
    f64 instance) and the residual norm computed from the stored matrices
    equals numpy's 2-norm."""
    data = ld.build(6, 79, device="cpu", out_dtype=torch.float64, m_range=(60, 200), n_range=(40, 120), k_max=20,
                    factors="haar")
    assert data["hh"] is None
    Us, want = [], []
    for b, A in enumerate(data["A"]):
        s = np.linalg.svd(A.numpy(), compute_uv=False)
        np.testing.assert_allclose(s, data["sigma"][b], rtol=1e-10, atol=1e-14 * s[0])
        k = int(data["spec"]["k"][b])
        U, _, _ = orc.rsvd(A.numpy(), k, p=5, q=b % 3, seed=2, stream_id=b)
        Us.append(torch.tensor(U))
        want.append(np.linalg.norm(A.numpy() - U @ (U.T @ A.numpy()), 2))
    np.testing.assert_allclose(L.residual_norms(data, Us, list(range(6))), want, rtol=1e-9)


def test_sharded_build_is_deterministic_and_matches_the_recipe():
    a = ld.build_range(40, "val", 8, 16, device="cpu", out_dtype=torch.float64, m_range=(60, 120),
                       n_range=(40, 80), k_max=20)
    b = ld.build_range(40, "val", 8, 16, device="cpu", out_dtype=torch.float64, m_range=(60, 120),
                       n_range=(40, 80), k_max=20)
    full = ld.shapes(40, ld.SPLIT_SEEDS["val"], m_range=(60, 120), n_range=(40, 80), k_max=20)
    assert np.array_equal(a["spec"]["m"], full["m"][8:16]) and np.array_equal(a["spec"]["k"], full["k"][8:16])
    for x, y in zip(a["A"], b["A"]):
        assert torch.equal(x, y)
