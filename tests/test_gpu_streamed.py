"""Parity of the streamed-A products (A read straight into the matrix cores,
X staged in LDS) at the sizes where the library takes them: m K >= 2^24,
64 < c <= 224, 16-byte aligned rows of A (TN also needs n % 4 == 0).

* Small integers make every product exact in f32, bf16 and split bf16
  whatever the summation order, so those comparisons are bitwise: they cover
  ragged row tiles (m not a multiple of 256), a ragged last chunk of the
  reduction (K not a multiple of the 32 / 64-element chunk), split reductions
  with their partial blocks, both column classes (c <= 128 and c <= 224), TN
  strips whose last columns fall past n, and the last-round pieces (tail
  dealing) after whole rounds and on their own.
* Random operands bound the rounding: f32 arithmetic and split bf16 within a
  few f32 roundings of a K-term dot product, bf16 within bf16 rounding.
* Full solves at streamed sizes (f32 and bf16 storage, plain and mixed, with
  and without centring) match the oracle.
"""
import numpy as np
import pytest
import torch

from oracle import rsvd as orc

pytestmark = pytest.mark.gpu

DEV = "cuda"
DT = {"f32": torch.float32, "bf16": torch.bfloat16}


def _np(t):
    t = t.detach().cpu()
    return (t.to(torch.float64) if t.dtype == torch.bfloat16 else t).numpy()


def _ints(rng, shape, lo, hi):
    return rng.integers(lo, hi + 1, size=shape).astype(np.float64)


@pytest.mark.parametrize("dt,arith", [("f32", "storage"), ("bf16", "storage"), ("f32", "bf16"),
                                      ("f32", "split"), ("bf16", "bf16"), ("bf16", "split")])
@pytest.mark.parametrize("m,K,c,splits", [(8229, 2051, 100, 1), (8229, 2051, 220, 1), (16500, 1030, 128, 3),
                                          (4100, 4131, 65, 2), (40000, 1024, 224, 0)])
def test_streamed_nn_exact_integers(gpu_lib, dt, arith, m, K, c, splits):
    from paper_1608_02148_amd import api
    print(f"streamed NN {dt} {arith} m={m} K={K} c={c} splits={splits}", flush=True)
    rng = np.random.default_rng(m + K + c + splits)
    A = _ints(rng, (m, K), -8, 8)
    X = _ints(rng, (K, c), -4, 4)
    Ag = torch.tensor(A, dtype=DT[dt], device=DEV)
    Xg = torch.tensor(X, dtype=torch.float32, device=DEV)
    Y = _np(api.gemm_nn(Ag, Xg, arith, splits=splits))
    assert np.array_equal(Y, A @ X)


@pytest.mark.parametrize("dt,arith", [("f32", "storage"), ("f32", "bf16"), ("bf16", "storage"), ("bf16", "bf16")])
@pytest.mark.parametrize("m,K,c", [(76837, 1100, 100), (76837, 1100, 220)])
def test_streamed_nn_whole_rounds_and_tail(gpu_lib, dt, arith, m, K, c):
    """f32 A (and bf16 A at 100 columns): 301 tiles of 256 rows, one whole
    round of 256 workgroups (placed by hardware block index) and 45 tiles
    dealt in pieces to a second round, whose slots TailFixBody sums.  bf16 A
    at 220 columns runs 128-row tiles, two workgroups per CU: 601 tiles, one
    round of 512 and 89 dealt.  Bitwise on small integers."""
    from paper_1608_02148_amd import api
    print(f"streamed NN tail {dt} {arith} m={m} K={K} c={c}", flush=True)
    rng = np.random.default_rng(m + c)
    A = _ints(rng, (m, K), -8, 8)
    X = _ints(rng, (K, c), -4, 4)
    Y = _np(api.gemm_nn(torch.tensor(A, dtype=DT[dt], device=DEV), torch.tensor(X, dtype=torch.float32, device=DEV),
                        arith, splits=1))
    assert np.array_equal(Y, A @ X)


@pytest.mark.parametrize("dt,arith", [("f32", "storage"), ("bf16", "bf16"), ("bf16", "split")])
def test_streamed_tn_split_rounds_and_tail(gpu_lib, dt, arith):
    """A^T Q at 50000 x 5120: 20 column tiles x 13 splits = 260 pairs, one
    whole round and 4 pairs dealt in 64 pieces each; bitwise on integers."""
    from paper_1608_02148_amd import api
    m, n, c = 50000, 5120, 120
    print(f"streamed TN tail {dt} {arith} m={m} n={n} c={c}", flush=True)
    rng = np.random.default_rng(5120)
    A = _ints(rng, (m, n), -4, 4)
    Q = _ints(rng, (m, c), -3, 3)
    Z = _np(api.gemm_tn(torch.tensor(A, dtype=DT[dt], device=DEV),
                        torch.tensor(Q, dtype=torch.float32, device=DEV), arith))
    assert np.array_equal(Z, A.T @ Q)


@pytest.mark.parametrize("dt,arith", [("f32", "storage"), ("bf16", "storage"), ("f32", "bf16"),
                                      ("f32", "split"), ("bf16", "bf16"), ("bf16", "split")])
@pytest.mark.parametrize("m,n,c", [(8200, 2052, 100), (8203, 2300, 220), (40011, 1000, 128), (5000, 4100, 77)])
def test_streamed_tn_exact_integers(gpu_lib, dt, arith, m, n, c):
    from paper_1608_02148_amd import api
    print(f"streamed TN {dt} {arith} m={m} n={n} c={c}", flush=True)
    rng = np.random.default_rng(m + 3 * n + c)
    A = _ints(rng, (m, n), -4, 4)
    Q = _ints(rng, (m, c), -3, 3)
    Z = _np(api.gemm_tn(torch.tensor(A, dtype=DT[dt], device=DEV),
                        torch.tensor(Q, dtype=torch.float32, device=DEV), arith))
    assert np.array_equal(Z, A.T @ Q)


@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("c", [120, 220])
def test_streamed_random_rounding(gpu_lib, dt, c):
    """Errors per entry, relative to sqrt(K) |a|_max |x|_max: f32 and split
    bf16 near f32 rounding, plain bf16 near bf16 rounding (and well above the
    split's)."""
    from paper_1608_02148_amd import api
    print(f"streamed random {dt} c={c}", flush=True)
    rng = np.random.default_rng(c)
    m, K = 12000, 2000
    Ag = torch.tensor(rng.standard_normal((m, K)), dtype=DT[dt], device=DEV)
    A = _np(Ag)
    Xg = torch.tensor(rng.standard_normal((K, c)), dtype=torch.float32, device=DEV)
    X = _np(Xg).astype(np.float64)
    scale = np.abs(A).max() * np.abs(X).max() * np.sqrt(K)
    ref = A @ X
    err = {a: np.abs(_np(api.gemm_nn(Ag, Xg, a)) - ref).max() / scale for a in ("storage", "split", "bf16")}
    assert err["storage"] < 1e-6 and err["split"] < 2e-6 and 1e-4 < err["bf16"] < 1e-2
    Qg = torch.tensor(rng.standard_normal((m, c)), dtype=torch.float32, device=DEV)
    refz = A.T @ _np(Qg).astype(np.float64)
    sz = np.abs(A).max() * np.abs(_np(Qg)).max() * np.sqrt(m)
    errz = {a: np.abs(_np(api.gemm_tn(Ag, Qg, a)) - refz).max() / sz for a in ("storage", "split", "bf16")}
    assert errz["storage"] < 1e-6 and errz["split"] < 2e-6 and 1e-4 < errz["bf16"] < 1e-2


def _planted(m, n, seed, decay=50.0):
    rng = np.random.default_rng(seed)
    r = min(m, n)
    U, _ = np.linalg.qr(rng.standard_normal((m, 300)))
    V, _ = np.linalg.qr(rng.standard_normal((n, 300)))
    s = np.exp(-np.arange(300) / decay)
    return (U * s) @ V.T + 1e-6 * rng.standard_normal((m, n)) / np.sqrt(r)


@pytest.mark.parametrize("dt,precision", [("f32", "plain"), ("f32", "bf16_mixed"), ("bf16", "plain"),
                                          ("bf16", "bf16_mixed")])
def test_streamed_solve_matches_oracle(gpu_lib, dt, precision):
    """rsvd at a streamed size (8192 x 2560, l = 120) against the f64 oracle on
    the same stored data: sigma to 1e-4 relative (the f32 bar), and the
    subspaces of the leading vectors (well separated) to 1e-3."""
    from paper_1608_02148_amd import api
    print(f"streamed solve {dt} {precision}", flush=True)
    m, n, k = 8192, 2560, 100
    A = _planted(m, n, 3)
    Ag = torch.tensor(A, dtype=DT[dt], device=DEV)
    As = _np(Ag)
    U, s, V = api.rsvd(Ag, k, p=20, q=2, seed=5, precision=precision)
    Uo, so, Vo = orc.rsvd(As, k, p=20, q=2, seed=5)
    np.testing.assert_allclose(_np(s), so, rtol=1e-4, atol=1e-4 * so[0] * 1e-2)
    top = 20
    c = np.abs(np.sum(_np(U)[:, :top] * Uo[:, :top], axis=0))
    assert c.min() > 1 - 1e-3


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_streamed_pca_matches_oracle(gpu_lib, dt):
    """rPCA (implicit centring: the column means are subtracted while A
    streams into the matrix cores) at 8192 x 2560 with offsets of 10x the
    centred signal, against the oracle's explicit centring."""
    from paper_1608_02148_amd import api
    print(f"streamed pca {dt}", flush=True)
    m, n, k = 8192, 2560, 100
    rng = np.random.default_rng(8)
    A = _planted(m, n, 4) + 10.0 * rng.standard_normal(n)[None, :] / np.sqrt(m)
    Ag = torch.tensor(A, dtype=DT[dt], device=DEV)
    As = _np(Ag)
    out = api.rpca(Ag, k, p=20, q=2, seed=9)
    want = orc.rpca(As, k, p=20, q=2, seed=9)
    ev = _np(out["eigvals"])
    np.testing.assert_allclose(ev, want["eigvals"], rtol=1e-3, atol=1e-4 * want["eigvals"][0])
