// Counter-based test-matrix entries for Alg. rqb (Sec. 2.3).
//
// Philox-4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): per round the counter
// words 0 and 2 are multiplied by two fixed odd constants, and the high / low
// halves of the 64-bit products are mixed with the other two words and the key;
// the key advances by two Weyl increments between rounds.  Entries of Omega:
//   key = (seed lo, seed hi), counter = (row j, column group c, stream_id, 0),
//   u_t = (x_t + 1) 2^-32 in (0, 1],
//   normal:     Box-Muller on (u0, u1) and (u2, u3) -> columns 4c .. 4c+3,
//   unif:       2 u_t - 1,
//   rademacher: +1 when x_t is odd, else -1.
#pragma once

#include "common.hpp"

namespace rsvd {

struct Philox4 { uint32_t x[4]; };

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                  uint32_t c3, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
    constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += kWeyl0; k1 += kWeyl1; }
        const uint32_t hi0 = __umulhi(kMul0, c0), lo0 = kMul0 * c0;
        const uint32_t hi1 = __umulhi(kMul1, c2), lo1 = kMul1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    Philox4 out;
    out.x[0] = c0; out.x[1] = c1; out.x[2] = c2; out.x[3] = c3;
    return out;
}

// Four consecutive entries Omega[j, 4c .. 4c+3] in precision T.
template <typename T>
__device__ __forceinline__ void omega_group(uint32_t j, uint32_t c, uint64_t seed,
                                            uint32_t stream_id, int sdist, T out[4]);

template <>
__device__ __forceinline__ void omega_group<double>(uint32_t j, uint32_t c, uint64_t seed,
                                                    uint32_t stream_id, int sdist, double out[4]) {
    const Philox4 w = philox4x32_10(j, c, stream_id, 0u, static_cast<uint32_t>(seed),
                                    static_cast<uint32_t>(seed >> 32));
    if (sdist == RSVD_RADEMACHER) {
#pragma unroll
        for (int t = 0; t < 4; ++t) out[t] = (w.x[t] & 1u) ? 1.0 : -1.0;
        return;
    }
    double u[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) u[t] = (static_cast<double>(w.x[t]) + 1.0) * 0x1p-32;
    if (sdist == RSVD_UNIF) {
#pragma unroll
        for (int t = 0; t < 4; ++t) out[t] = 2.0 * u[t] - 1.0;
        return;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double r = sqrt(-2.0 * log(u[2 * h]));
        double s, co;
        sincospi(2.0 * u[2 * h + 1], &s, &co);
        out[2 * h] = r * co;
        out[2 * h + 1] = r * s;
    }
}

template <>
__device__ __forceinline__ void omega_group<float>(uint32_t j, uint32_t c, uint64_t seed,
                                                   uint32_t stream_id, int sdist, float out[4]) {
    const Philox4 w = philox4x32_10(j, c, stream_id, 0u, static_cast<uint32_t>(seed),
                                    static_cast<uint32_t>(seed >> 32));
    if (sdist == RSVD_RADEMACHER) {
#pragma unroll
        for (int t = 0; t < 4; ++t) out[t] = (w.x[t] & 1u) ? 1.0f : -1.0f;
        return;
    }
    float u[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)   // (x + 1) 2^-32 rounded once to f32
        u[t] = static_cast<float>((static_cast<double>(w.x[t]) + 1.0) * 0x1p-32);
    if (sdist == RSVD_UNIF) {
#pragma unroll
        for (int t = 0; t < 4; ++t) out[t] = 2.0f * u[t] - 1.0f;
        return;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const float r = sqrtf(-2.0f * logf(u[2 * h]));
        float s, co;
        sincospif(2.0f * u[2 * h + 1], &s, &co);
        out[2 * h] = r * co;
        out[2 * h + 1] = r * s;
    }
}

}  // namespace rsvd
