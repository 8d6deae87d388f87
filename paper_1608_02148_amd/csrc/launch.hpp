// Host-side launchers for the kernels (template dispatch on tile shape).
#pragma once

#include <type_traits>

#include "common.hpp"
#include "gemm.hpp"
#include "gemm_bf16.hpp"
#include "linalg.hpp"

namespace rsvd {

// Largest dynamic LDS a kernel may ask for; raised once per instantiation.
template <typename K>
inline hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

template <typename T> constexpr int gemm_bk() { return sizeof(T) == 8 ? 16 : 32; }

// Output tile width used for c output columns: 32, 64 or 128 (column tiles of
// 128 beyond that).
inline int tile_cols(int c) { return c <= 32 ? 32 : (c <= 64 ? 64 : 128); }

inline bool aligned16(const void* p, int64_t ld, size_t elem) {
    return (reinterpret_cast<uintptr_t>(p) % 16 == 0) && ((ld * static_cast<int64_t>(elem)) % 16 == 0);
}

template <typename TA, typename TX, typename TC, int MODE, int WR, int WC, int WGM, int WGN>
hipError_t launch_gemm_cfg(hipStream_t st, const GemmArgs<TA, TX, TC>& g, int S) {
    constexpr int BK = gemm_bk<TC>();
    typedef GemmTile<TA, TX, TC, MODE, WR, WC, WGM, WGN, BK> T;
    auto kern = gemm_tile_kernel<TA, TX, TC, MODE, WR, WC, WGM, WGN, BK>;
    static bool ready = false;
    if (!ready) {
        hipError_t e = allow_lds(kern, T::LDS_BYTES);
        if (e != hipSuccess) return e;
        ready = true;
    }
    dim3 grid(static_cast<unsigned>(cdiv(g.rows, T::BM)), static_cast<unsigned>(S),
              static_cast<unsigned>(cdiv(g.ncols, T::NC)));
    hipLaunchKernelGGL(kern, grid, dim3(T::NT), T::LDS_BYTES, st, g);
    return hipGetLastError();
}

// Generic product launcher.  out = A X (NN) or A^T X (TN) over the reduction
// length K; S > 1 writes S partial blocks of stride part_stride into out.
template <typename TA, typename TX, typename TC, int MODE>
hipError_t launch_gemm(hipStream_t st, const TA* A, int64_t lda, int64_t rows, int64_t K,
                       const TX* X, int64_t ldx, int ncols, TC* out, int64_t ldo, int S,
                       int64_t part_stride, const double* mu, const uint32_t* skip_flag,
                       uint32_t skip_mask) {
    constexpr int BK = gemm_bk<TC>();
    GemmArgs<TA, TX, TC> g;
    g.A = A; g.lda = lda; g.rows = rows; g.K = K;
    S = S < 1 ? 1 : S;
    g.kchunk = rup(cdiv(K, S), BK);
    g.X = X; g.ldx = ldx; g.ncols = ncols; g.out = out; g.ldo = ldo;
    g.part_stride = part_stride; g.mu = mu; g.skip_flag = skip_flag; g.skip_mask = skip_mask;
    {   // vector loads of 16 / sizeof(TC) consecutive elements of A
        const size_t vb = (16 / sizeof(TC)) * sizeof(TA);
        g.a_vec = (reinterpret_cast<uintptr_t>(A) % vb == 0) && ((lda * sizeof(TA)) % vb == 0);
    }
    g.x_vec = 0;
    // splits past the end of K find an empty range and write zero partials
    const int tc = tile_cols(ncols);
    if (tc == 32) return launch_gemm_cfg<TA, TX, TC, MODE, 2, 2, 4, 1>(st, g, S);
    if (tc == 64) return launch_gemm_cfg<TA, TX, TC, MODE, 4, 2, 2, 2>(st, g, S);
    return launch_gemm_cfg<TA, TX, TC, MODE, 4, 4, 2, 2>(st, g, S);
}


template <typename TA, int MODE, bool SPLIT, int WR, int WC, int WGM, int WGN>
hipError_t launch_bf16_cfg(hipStream_t st, const GemmArgs<TA, float, float>& g, int S) {
    constexpr int BK = SPLIT ? 32 : 64;
    typedef Bf16Tile<TA, MODE, SPLIT, WR, WC, WGM, WGN, BK> T;
    auto kern = gemm_bf16_kernel<TA, MODE, SPLIT, WR, WC, WGM, WGN, BK>;
    static bool ready = false;
    if (!ready) {
        hipError_t e = allow_lds(kern, T::LDS_BYTES);
        if (e != hipSuccess) return e;
        ready = true;
    }
    dim3 grid(static_cast<unsigned>(cdiv(g.rows, T::BM)), static_cast<unsigned>(S),
              static_cast<unsigned>(cdiv(g.ncols, T::NC)));
    hipLaunchKernelGGL(kern, grid, dim3(T::NT), T::LDS_BYTES, st, g);
    return hipGetLastError();
}

// bf16-matrix-core product (f32 in / f32 out).  split = true gives the
// f32-accurate three-term product (see gemm_bf16.hpp).
template <typename TA, int MODE>
hipError_t launch_gemm_bf16(hipStream_t st, bool split, const TA* A, int64_t lda, int64_t rows, int64_t K,
                            const float* X, int64_t ldx, int ncols, float* out, int64_t ldo, int S,
                            int64_t part_stride, const double* mu, const uint32_t* skip_flag,
                            uint32_t skip_mask) {
    GemmArgs<TA, float, float> g;
    g.A = A; g.lda = lda; g.rows = rows; g.K = K;
    S = S < 1 ? 1 : S;
    g.kchunk = rup(cdiv(K, S), 64);
    g.X = X; g.ldx = ldx; g.ncols = ncols; g.out = out; g.ldo = ldo;
    g.part_stride = part_stride; g.mu = mu; g.skip_flag = skip_flag; g.skip_mask = skip_mask;
    g.a_vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && ((lda * sizeof(TA)) % 16 == 0);
    g.x_vec = 0;
    const int tc = tile_cols(ncols);
    if (split) {
        if (tc == 32) return launch_bf16_cfg<TA, MODE, true, 2, 2, 4, 1>(st, g, S);
        if (tc == 64) return launch_bf16_cfg<TA, MODE, true, 4, 2, 2, 2>(st, g, S);
        return launch_bf16_cfg<TA, MODE, true, 4, 4, 2, 2>(st, g, S);
    }
    if (tc == 32) return launch_bf16_cfg<TA, MODE, false, 2, 2, 4, 1>(st, g, S);
    if (tc == 64) return launch_bf16_cfg<TA, MODE, false, 4, 2, 2, 2>(st, g, S);
    return launch_bf16_cfg<TA, MODE, false, 4, 4, 2, 2>(st, g, S);
}

// One product with A in the requested arithmetic: 0 = storage precision
// (f32 / f64 matrix cores), 1 = bf16, 2 = split bf16 (f32-accurate).
template <typename TA, typename TC, int MODE>
hipError_t launch_gemm_arith(hipStream_t st, int arith, const TA* A, int64_t lda, int64_t rows, int64_t K,
                             const TC* X, int64_t ldx, int ncols, TC* out, int64_t ldo, int S,
                             int64_t part_stride, const double* mu, const uint32_t* skip_flag,
                             uint32_t skip_mask) {
    if constexpr (std::is_same<TC, float>::value) {
        if (arith != 0)
            return launch_gemm_bf16<TA, MODE>(st, arith == 2, A, lda, rows, K, X, ldx, ncols, out, ldo, S,
                                              part_stride, mu, skip_flag, skip_mask);
    }
    return launch_gemm<TA, TC, TC, MODE>(st, A, lda, rows, K, X, ldx, ncols, out, ldo, S, part_stride, mu,
                                         skip_flag, skip_mask);
}

template <typename T>
hipError_t launch_reduce(hipStream_t st, const T* part, int S, int64_t part_stride, int64_t ldp,
                         int64_t rows, int ncols, T* out, int64_t ldo,
                         const uint32_t* skip_flag = nullptr, uint32_t skip_mask = 0) {
    const int64_t total = rows * ncols;
    hipLaunchKernelGGL(reduce_partials_kernel<T>, dim3(static_cast<unsigned>(cdiv(total, 256))), dim3(256),
                       0, st, part, S, part_stride, ldp, rows, ncols, out, ldo, skip_flag, skip_mask);
    return hipGetLastError();
}

}  // namespace rsvd
