"""Pins for the oracle's counter-based test matrices (CPU only).

The round structure, key schedule and double-width multiply are shared by the
32- and 64-bit Philox variants, and the 64-bit variant is checked word for
word against numpy's own Philox-4x64-10 bit generator (an implementation the
oracle does not share).  The 32-bit multipliers and Weyl constants are the
published ones (Salmon et al., SC'11); they are pinned by bijectivity and
statistical tests.  Box-Muller is pinned by closed-form values and by the
moments / Kolmogorov-Smirnov distance of its output.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import philox

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _numpy_philox_block(key, counter):
    """First 4 raw outputs of numpy's Philox: the block of ``counter + 1``."""
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(counter, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("key,counter", [
    ((5, 7), (1, 2, 3, 4)),
    ((0, 0), (0, 0, 0, 0)),
    ((2**64 - 1, 2**64 - 1), (2**64 - 3, 2**64 - 1, 2**64 - 1, 2**64 - 1)),
    ((0x0123456789ABCDEF, 0xFEDCBA9876543210), (2**63, 17, 2**40 + 3, 99)),
])
def test_round_structure_matches_numpy_philox4x64(key, counter):
    want = _numpy_philox_block(key, counter)
    c = list(counter)
    c[0] = (c[0] + 1) % 2**64          # numpy advances the counter first
    got = philox.philox4([np.uint64(x) for x in c], [np.uint64(x) for x in key], width=64)
    assert [int(v) for v in got] == want


@pytest.mark.parametrize("width", [32, 64])
def test_mulhilo_exact_against_python_integers(width):
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2**width, size=2000, dtype=np.uint64, endpoint=False) if width == 32 \
        else rng.integers(0, 2**63, size=2000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = np.uint64(philox.PHILOX_CONSTANTS[width][0])
    hi, lo = philox._mulhilo(b, a, width)
    for x, h, l_ in zip(a[:200], hi[:200], lo[:200]):
        full = int(b) * int(x)
        assert int(h) == full >> width and int(l_) == full & ((1 << width) - 1)


def test_philox4x32_is_a_bijection_on_counters():
    n = 1 << 16
    ctr = np.arange(n, dtype=np.uint64)
    x = philox.philox4((ctr, 0, 0, 0), (123, 456), width=32)
    packed = (x[0] << np.uint64(32)) | x[1]
    assert len(np.unique(packed)) == n


def test_philox4x32_words_are_uniform():
    w = philox.raw_words(4096, 64, seed=2148)
    assert w.max() < 2**32
    top = (w >> np.uint64(24)).ravel()
    counts = np.bincount(top.astype(np.int64), minlength=256)
    chi2 = stats.chisquare(counts)
    assert chi2.pvalue > 1e-4
    u = philox.uniforms(w).ravel()
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    # every bit is balanced
    for bit in (0, 7, 15, 31):
        frac = float(np.mean((w >> np.uint64(bit)) & np.uint64(1)))
        assert abs(frac - 0.5) < 4.0 * 0.5 / math.sqrt(w.size)


def test_key_and_stream_change_the_stream():
    a = philox.raw_words(64, 16, seed=1)
    b = philox.raw_words(64, 16, seed=2)
    c = philox.raw_words(64, 16, seed=1, stream_id=1)
    d = philox.raw_words(64, 16, seed=1 + (1 << 32))
    for other in (b, c, d):
        assert np.mean(a == other) < 1e-3


def test_uniform_map_is_exact_and_in_unit_interval():
    w = np.array([0, 1, 2**31, 2**32 - 1], dtype=np.uint64)
    u = philox.uniforms(w)
    assert u[0] == 2.0 ** -32 and u[-1] == 1.0 and u[2] == 0.5 + 2.0 ** -32


def test_box_muller_closed_forms():
    u0 = np.array([math.exp(-0.5)] * 3 + [1.0])
    u1 = np.array([0.25, 0.5, 1.0, 0.3])
    z0, z1 = philox.box_muller(u0, u1)
    np.testing.assert_allclose(z0[:3], [0.0, -1.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(z1[:3], [1.0, 0.0, 0.0], atol=1e-15)
    assert z0[3] == 0.0 and z1[3] == 0.0          # u0 = 1 gives radius 0


def test_gaussian_test_matrix_statistics():
    om = philox.test_matrix(20000, 40, seed=2148)
    assert om.shape == (20000, 40)
    x = om.ravel()
    n = x.size
    assert abs(x.mean()) < 4.0 / math.sqrt(n)
    assert abs(x.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    c = np.corrcoef(om.T)
    off = c[~np.eye(40, dtype=bool)]
    assert np.max(np.abs(off)) < 5.0 / math.sqrt(20000)


def test_gaussian_layout_uses_word_t_of_group_c():
    om = philox.test_matrix(5, 10, seed=77, stream_id=3)
    for j, col in [(0, 0), (4, 9), (2, 5)]:
        c, t = divmod(col, 4)
        x = philox.philox4((np.uint64(j), np.uint64(c), np.uint64(3), np.uint64(0)),
                           (np.uint64(77), np.uint64(0)), width=32)
        u = [(int(v) + 1) * 2.0 ** -32 for v in x]
        pair = (u[0], u[1]) if t < 2 else (u[2], u[3])
        r = math.sqrt(-2.0 * math.log(pair[0]))
        want = r * (math.cos(2 * math.pi * pair[1]) if t % 2 == 0 else math.sin(2 * math.pi * pair[1]))
        assert om[j, col] == pytest.approx(want, rel=1e-15, abs=1e-15)


def test_uniform_and_rademacher_test_matrices():
    u = philox.test_matrix(20000, 16, seed=5, sdist="unif").ravel()
    assert u.min() > -1.0 and u.max() <= 1.0
    assert abs(u.mean()) < 4.0 * math.sqrt(1.0 / 3.0 / u.size)
    assert abs(u.var() - 1.0 / 3.0) < 0.01
    r = philox.test_matrix(20000, 16, seed=5, sdist="rademacher").ravel()
    assert set(np.unique(r)) == {-1.0, 1.0}
    assert abs(r.mean()) < 4.0 / math.sqrt(r.size)


def test_truncation_keeps_leading_columns():
    a = philox.test_matrix(7, 13, seed=9)
    b = philox.test_matrix(7, 16, seed=9)
    np.testing.assert_array_equal(a, b[:, :13])
