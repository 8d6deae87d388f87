// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <stddef.h>

#include <vector>

#include "../../include/rsvd_mi355x.h"

namespace rsvd {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// bf16 storage as raw 16-bit words; conversion to f32 is exact (shift by 16).
struct bf16_t { uint16_t bits; };

__device__ __forceinline__ float to_f32(bf16_t x) {
    return __uint_as_float(static_cast<uint32_t>(x.bits) << 16);
}

template <typename T> struct Conv;
template <> struct Conv<double> {
    __device__ static double to(double x) { return x; }
    __device__ static double to(float x) { return static_cast<double>(x); }
    __device__ static double to(bf16_t x) { return static_cast<double>(to_f32(x)); }
};
template <> struct Conv<float> {
    __device__ static float to(double x) { return static_cast<float>(x); }
    __device__ static float to(float x) { return x; }
    __device__ static float to(bf16_t x) { return to_f32(x); }
};

// 16x16x4 matrix-core step D += A B for f32 and f64.  Operands: A(i, k) comes
// from lane i + 16 k and B(k, j) from lane j + 16 k for both types.  Result:
// lane j + 16 g holds, in accumulator element r, D(row(g, r), j) with
//   f32: row = 4 g + r        f64: row = g + 4 r
// (the f64 layout interleaves rows across lane groups; measured on gfx950).
template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef v4f acc_t;
    __device__ __forceinline__ static int row(int g, int r) { return 4 * g + r; }
    __device__ __forceinline__ static acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    typedef v4d acc_t;
    __device__ __forceinline__ static int row(int g, int r) { return g + 4 * r; }
    __device__ __forceinline__ static acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

__host__ __device__ constexpr int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ constexpr int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// Optional launch condition: a kernel with a gate runs only if (*w & mask).
struct Gate { const uint32_t* w = nullptr; uint32_t mask = 0u; };

// Second status word of a solve in a batch group whose members have different
// q (the group runs max q iterations; each member's own are switched on here):
// bit it: iteration it runs and is not the member's last; bit 8 + it: it is the
// last; bit 16: q = 0 (the first sketch is the last); bit 17: q > 0.
enum : uint32_t { IT_LAST_SHIFT = 8, IT_Q0 = 1u << 16, IT_QPOS = 1u << 17 };

__host__ __device__ inline uint32_t iteration_word(int q, int qmax) {
    uint32_t w = q == 0 ? IT_Q0 : IT_QPOS;
    for (int it = 0; it < qmax; ++it) {
        if (it < q - 1) w |= 1u << it;
        else if (it == q - 1) w |= 1u << (IT_LAST_SHIFT + it);
    }
    return w;
}

// Status word bits kept in the workspace (a superset of RSVD_FLAG_*).
enum : uint32_t {
    ST_NEED_P2 = 1u << 16,         // pass 2 of the current orthonormalisation must run
    ST_SHIFTED = 1u << 17,         // its first pass used the shifted Cholesky
    ST_NEED_P3 = 1u << 18,         // pass 3 must run
    ST_SWEEPS_SHIFT = 24,          // bits 24..31: Jacobi sweeps of the last small SVD
};

// Per-device properties cached by the handle.
struct DeviceInfo {
    int num_cu = 256;
    int device = 0;
};

// Learned q per matrix, on stream st (defined with the selector network):
// network forward on feat (count x 131) into prob (count x 15), then q[b] =
// the fewest iterations whose pairs (q' <= q, p' <= p_solve) hold mass >= tau.
// theta null: q[b] = fallback_q and neither feat nor prob is read.
hipError_t learned_choose_q(hipStream_t st, const float* theta, int count, const float* feat, float* prob,
                            float tau, int p_solve, int fallback_q, int32_t* q);

}  // namespace rsvd

namespace rsvd {
// One recorded launch interval (optional profiling).
struct ProfRecord {
    int kind;
    hipEvent_t start, stop;
    double flops, bytes;
};
}  // namespace rsvd

struct rsvd_handle_s {
    hipStream_t stream = nullptr;
    int last_hip_error = 0;
    rsvd::DeviceInfo dev;
    bool profiling = false;
    std::vector<rsvd::ProfRecord> prof;        // recorded intervals
    std::vector<hipEvent_t> event_pool;        // reusable events
    size_t pool_used = 0;
    // f32 tall-tile variant per (mode, column class): NN 32..128, then TN
    // (rsvd_set_tile_variants; defaults measured at 100000 x 5000, l = 120)
    int variants[12] = {0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 2};
    // Side streams (default priority) and events that batches fork their
    // groups onto; created on first use, released by rsvd_destroy.
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_done;
    hipEvent_t fork = nullptr;
    // Pinned host staging for uploading batch launch tables (grown on demand;
    // uploads are synchronous, so one buffer serves every batch).
    unsigned char* staging = nullptr;
    size_t staging_bytes = 0;
};
