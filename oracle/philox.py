"""Counter-based random test matrices for the oracle (TEST INFRASTRUCTURE ONLY).

The paper's default test matrix has i.i.d. standard normal entries (Sec. 2.3,
"Random test matrices"; Alg. rqb draws it with ``rnorm(n, l)``); uniform
U(-1,1) and Rademacher entries are the two alternatives of the same section.
R's own random stream cannot be reproduced, so the entries here come from a
counter-based generator that any implementation can evaluate independently:

* Philox-4xW-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11).  Four W-bit counter words, two key words, ten
  rounds.  Each round multiplies counter words 0 and 2 by fixed odd
  multipliers, takes the high and low halves of the double-width products,
  and mixes them as (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0); the key is
  advanced by two Weyl constants between rounds.  The code below is generic in
  W so that the identical round structure can be checked against numpy's own
  Philox-4x64-10 bit generator; W = 32 is what the test matrices use.
* Box-Muller (1958) maps two uniforms u0, u1 in (0, 1] to two independent
  normals sqrt(-2 ln u0) * (cos 2 pi u1, sin 2 pi u1).

Canonical test-matrix definition (the reading this implementation fixes, the
paper being silent on the generator):

* key     = (seed mod 2^32, seed >> 32)
* counter = (j, c, stream_id, 0) for row j of Omega and column group c
* the call returns x0..x3; u_t = (x_t + 1) * 2^-32 lies in (0, 1] exactly
* normal:     Omega[j, 4c+0..3] = BoxMuller(u0,u1), BoxMuller(u2,u3)
* unif:       Omega[j, 4c+t] = 2 u_t - 1            (in (-1, 1])
* rademacher: Omega[j, 4c+t] = +1 if x_t is odd else -1
"""
import numpy as np

# Published Philox parameters (SC'11, Table 2 and Sec. 3.3): multipliers and
# Weyl key increments (golden ratio and sqrt(3) - 1 in fixed point).
PHILOX_CONSTANTS = {
    32: (0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85),
    64: (0xD2E7470EE14C6C93, 0xCA5A826395121157,
         0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B),
}

_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b, width):
    """High and low W-bit halves of the 2W-bit product a*b (uint64 arrays)."""
    if width == 32:
        prod = a * b                      # < 2^64, exact in uint64
        return prod >> _S32, prod & _M32
    # width 64: schoolbook product on 32-bit limbs, every partial < 2^64
    a0, a1 = a & _M32, a >> _S32
    b0, b1 = b & _M32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = (p00 & _M32) | ((mid & _M32) << _S32)
    return hi, lo


def philox4(counter, key, width=32, rounds=10):
    """Philox-4xW-R block function.

    counter: 4 arrays (broadcastable) of W-bit values; key: 2 such arrays.
    Returns the 4 output words as uint64 arrays holding W-bit values.
    """
    m0, m1, w0, w1 = (np.uint64(c) for c in PHILOX_CONSTANTS[width])
    mask = np.uint64((1 << width) - 1)
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & mask for c in counter)
        k0, k1 = (np.asarray(k, dtype=np.uint64) & mask for k in key)
        for r in range(rounds):
            if r:
                k0 = (k0 + w0) & mask
                k1 = (k1 + w1) & mask
            hi0, lo0 = _mulhilo(m0, x0, width)
            hi1, lo1 = _mulhilo(m1, x2, width)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def raw_words(n, l, seed, stream_id=0):
    """The four 32-bit words for every (row j, column group c) of an n x l matrix.

    Returns an (n, 4*ceil(l/4)) uint64 array W with W[j, 4c+t] = x_t(j, c).
    """
    groups = (l + 3) // 4
    j = np.arange(n, dtype=np.uint64)[:, None]
    c = np.arange(groups, dtype=np.uint64)[None, :]
    seed = int(seed)
    key = (np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF))
    sid = np.uint64(int(stream_id) & 0xFFFFFFFF)
    zero = np.uint64(0)
    x = philox4((j, c, sid, zero), key, width=32)
    out = np.empty((n, 4 * groups), dtype=np.uint64)
    for t in range(4):
        out[:, t::4] = np.broadcast_to(x[t], (n, groups))
    return out


def uniforms(words):
    """u = (x + 1) * 2^-32 in (0, 1], exact in float64."""
    return (words.astype(np.float64) + 1.0) * 2.0 ** -32


def box_muller(u0, u1):
    """Two independent N(0,1) variates from two uniforms in (0, 1]."""
    r = np.sqrt(-2.0 * np.log(u0))
    return r * np.cos(2.0 * np.pi * u1), r * np.sin(2.0 * np.pi * u1)


def test_matrix(n, l, seed, stream_id=0, sdist="normal"):
    """The n x l random test matrix Omega of Alg. rqb (float64)."""
    w = raw_words(n, l, seed, stream_id)
    if sdist == "normal":
        u = uniforms(w)
        om = np.empty_like(u)
        om[:, 0::4], om[:, 1::4] = box_muller(u[:, 0::4], u[:, 1::4])
        om[:, 2::4], om[:, 3::4] = box_muller(u[:, 2::4], u[:, 3::4])
    elif sdist == "unif":
        om = 2.0 * uniforms(w) - 1.0
    elif sdist == "rademacher":
        om = np.where((w & np.uint64(1)) == 1, 1.0, -1.0)
    else:
        raise ValueError(f"unknown sdist {sdist!r}")
    return np.ascontiguousarray(om[:, :l])
