// Tall-skinny products with the input matrix A on the matrix cores.
//
//   NN:  Y = A X    (A m x K row-major, X K x c)   Alg. rqb step 3 and
//                                                  Alg. subspace_iter step 4
//   TN:  Z = A^T Q  (A K x n row-major, Q K x c)   Alg. subspace_iter step 3
//                                                  and Alg. rqb step 10 (B^T)
//
// Both share one tile engine.  A workgroup owns a BM x NC block of the output
// and walks the reduction dimension in steps of BK.  The A tile is staged in
// LDS k-major (As[k][r]) in both modes -- NN transposes while staging, TN
// reads A in its natural row order -- so the matrix-core fragment reads are
// the same: lane i + 16 kk reads As[kk][i] and Xs[kk][j].  LDS is double
// buffered; the next tile's global loads are in flight while the current tile
// is multiplied, with a single barrier per step.
//
// Split-K: grid.y = S splits the reduction dimension into S contiguous chunks.
// With S > 1 every split writes its own partial block and a separate kernel
// sums the partials in split order, so results are deterministic (no atomics).
//
// Optional implicit centring: when mu != nullptr every staged element of A is
// replaced by A(i, j) - mu[j] (j = column of A), which is how the PCA path
// works on A - 1 mu^T without forming it.
#pragma once

#include "common.hpp"

namespace rsvd {

enum GemmMode { MODE_NN = 0, MODE_TN = 1 };

template <typename TA, typename TX, typename TC>
struct GemmArgs {
    const TA* A;
    int64_t lda;
    int64_t rows;        // output rows (NN: m, TN: n)
    int64_t K;           // reduction length (NN: n, TN: m)
    int64_t kchunk;      // reduction elements per split (multiple of BK)
    const TX* X;         // K x (col tiles * NC) operand
    int64_t ldx;
    int32_t ncols;       // valid output columns (all column tiles together)
    TC* out;             // rows x ncols (ldo) or S partial blocks
    int64_t ldo;
    int64_t part_stride; // elements between split partial blocks (S > 1)
    const double* mu;    // optional column means of A (implicit centring)
    const uint32_t* skip_flag;  // optional: run only if (*skip_flag & skip_mask)
    uint32_t skip_mask;
    int32_t a_vec;       // 1 when A rows are 16-byte aligned (vector loads)
    int32_t x_vec;       // 1 when X rows are 16-byte aligned
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename TA, typename TC>
__device__ __forceinline__ TC load_elem(const TA* p, const double* mu, int64_t col) {
    if (mu) return Conv<TC>::to(Conv<double>::to(*p) - mu[col]);
    return Conv<TC>::to(*p);
}

template <typename TA, typename TC, int N>
__device__ __forceinline__ void unpack16(const u32x4 raw, TC (&dst)[N]) {
    if constexpr (sizeof(TA) == 8) {
        static_assert(N == 2, "");
        dst[0] = Conv<TC>::to(__hiloint2double(raw[1], raw[0]));
        dst[1] = Conv<TC>::to(__hiloint2double(raw[3], raw[2]));
    } else if constexpr (sizeof(TA) == 4) {
        static_assert(N == 4, "");
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[e] = Conv<TC>::to(__uint_as_float(raw[e]));
    } else {
        static_assert(N == 8, "");
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            dst[2 * e] = Conv<TC>::to(__uint_as_float(raw[e] << 16));
            dst[2 * e + 1] = Conv<TC>::to(__uint_as_float(raw[e] & 0xFFFF0000u));
        }
    }
}

template <typename TA, typename TX, typename TC, int MODE, int WR, int WC, int WGM, int WGN, int BK>
struct GemmTile {
    static constexpr int BM = 16 * WR * WGM;
    static constexpr int NC = 16 * WC * WGN;
    static constexpr int NT = 64 * WGM * WGN;
    static constexpr int PAD = 64 / sizeof(TC);   // row stride = 16 mod 32 banks
    static constexpr int SA = BM + PAD;           // As row stride (elements)
    static constexpr int SX = NC + PAD;           // Xs row stride
    static constexpr int VA = 16 / sizeof(TA);    // A elements per 16-byte load
    static constexpr int VX = 16 / sizeof(TX);
    // A tile: NN reads BM rows x BK columns, TN reads BK rows x BM columns.
    static constexpr int A_TPR = (MODE == MODE_NN ? BK : BM) / VA;   // threads per A row
    static constexpr int A_RPP = NT / A_TPR;                         // A rows per pass
    static constexpr int A_ROWS = (MODE == MODE_NN ? BM : BK);        // A rows per tile
    static constexpr int A_PASSES = (A_ROWS + A_RPP - 1) / A_RPP;
    static constexpr int X_TPR = NC / VX;
    static constexpr int X_RPP = NT / X_TPR;
    static constexpr int X_PASSES = (BK + X_RPP - 1) / X_RPP;
    static_assert(NT % A_TPR == 0 && NT % X_TPR == 0, "");
    static_assert(A_ROWS % A_RPP == 0 || A_PASSES == 1, "");
    static_assert(BK % X_RPP == 0 || X_PASSES == 1, "");
    static constexpr size_t LDS_BYTES = 2ull * BK * (SA + SX) * sizeof(TC);
};

template <typename TA, typename TX, typename TC, int MODE, int WR, int WC, int WGM, int WGN, int BK>
__global__ __launch_bounds__(64 * WGM * WGN)
void gemm_tile_kernel(GemmArgs<TA, TX, TC> g) {
    typedef GemmTile<TA, TX, TC, MODE, WR, WC, WGM, WGN, BK> T;
    typedef typename Mfma<TC>::acc_t acc_t;
    if (g.skip_flag && ((*g.skip_flag & g.skip_mask) == 0u)) return;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    TC* As = reinterpret_cast<TC*>(smem_raw);            // [2][BK][SA]
    TC* Xs = As + 2 * BK * T::SA;                         // [2][BK][SX]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * T::BM;
    const int split = blockIdx.y;
    const int col0 = blockIdx.z * T::NC;
    const int64_t kbeg = static_cast<int64_t>(split) * g.kchunk;
    const int64_t kend = min(g.K, kbeg + g.kchunk);
    const TX* X = g.X + col0;

    // ---- global -> register prefetch buffers
    TC ra[T::A_PASSES][T::VA];
    TC rx[T::X_PASSES][T::VX];

    auto load_a = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < T::A_PASSES; ++p) {
            const int arow = p * T::A_RPP + tid / T::A_TPR;
            const int acol = (tid % T::A_TPR) * T::VA;
            if (arow >= T::A_ROWS) break;
            int64_t gr, gc;          // global row / column of A
            bool row_ok;
            int64_t col_lim;
            if (MODE == MODE_NN) {
                gr = r0 + arow; gc = k0 + acol; row_ok = gr < g.rows; col_lim = kend;
            } else {
                gr = k0 + arow; gc = r0 + acol; row_ok = gr < kend; col_lim = g.rows;
            }
            const TA* src = g.A + gr * g.lda + gc;
            if (row_ok && g.a_vec && gc + T::VA <= col_lim) {
                const u32x4 raw = *reinterpret_cast<const u32x4*>(src);
                unpack16<TA, TC>(raw, ra[p]);
                if (g.mu) {
#pragma unroll
                    for (int e = 0; e < T::VA; ++e)
                        ra[p][e] = Conv<TC>::to(Conv<double>::to(ra[p][e]) - g.mu[gc + e]);
                }
            } else {
#pragma unroll
                for (int e = 0; e < T::VA; ++e)
                    ra[p][e] = (row_ok && gc + e < col_lim) ? load_elem<TA, TC>(src + e, g.mu, gc + e)
                                                            : TC(0);
            }
        }
    };
    auto load_x = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < T::X_PASSES; ++p) {
            const int xr = p * T::X_RPP + tid / T::X_TPR;
            const int xc = (tid % T::X_TPR) * T::VX;
            if (xr >= BK) break;
            const int64_t gk = k0 + xr;
            const int gcol = col0 + xc;          // column of X
            const TX* src = X + gk * g.ldx + xc;
            if (gk < kend && g.x_vec && gcol + T::VX <= g.ncols) {
                const u32x4 raw = *reinterpret_cast<const u32x4*>(src);
                unpack16<TX, TC>(raw, rx[p]);
            } else {
#pragma unroll
                for (int e = 0; e < T::VX; ++e)
                    rx[p][e] = (gk < kend && gcol + e < g.ncols) ? Conv<TC>::to(src[e]) : TC(0);
            }
        }
    };
    auto store_tiles = [&](int buf) {
        TC* as = As + buf * BK * T::SA;
        TC* xs = Xs + buf * BK * T::SX;
#pragma unroll
        for (int p = 0; p < T::A_PASSES; ++p) {
            const int arow = p * T::A_RPP + tid / T::A_TPR;
            const int acol = (tid % T::A_TPR) * T::VA;
            if (arow >= T::A_ROWS) break;
#pragma unroll
            for (int e = 0; e < T::VA; ++e) {
                if (MODE == MODE_NN) as[(acol + e) * T::SA + arow] = ra[p][e];   // transpose
                else                 as[arow * T::SA + acol + e] = ra[p][e];
            }
        }
#pragma unroll
        for (int p = 0; p < T::X_PASSES; ++p) {
            const int xr = p * T::X_RPP + tid / T::X_TPR;
            const int xc = (tid % T::X_TPR) * T::VX;
            if (xr >= BK) break;
#pragma unroll
            for (int e = 0; e < T::VX; ++e) xs[xr * T::SX + xc + e] = rx[p][e];
        }
    };

    acc_t acc[WR][WC];
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
        for (int j = 0; j < WC; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    const int li = lane & 15, lk = lane >> 4;
    const int wr0 = wm * WR * 16, wc0 = wn * WC * 16;

    if (kbeg < kend) {
        load_a(kbeg);
        load_x(kbeg);
        int buf = 0;
        for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
            store_tiles(buf);
            __syncthreads();
            if (k0 + BK < kend) { load_a(k0 + BK); load_x(k0 + BK); }
            const TC* as = As + buf * BK * T::SA;
            const TC* xs = Xs + buf * BK * T::SX;
#pragma unroll
            for (int kk = 0; kk < BK / 4; ++kk) {
                TC a[WR], b[WC];
#pragma unroll
                for (int i = 0; i < WR; ++i) a[i] = as[(4 * kk + lk) * T::SA + wr0 + 16 * i + li];
#pragma unroll
                for (int j = 0; j < WC; ++j) b[j] = xs[(4 * kk + lk) * T::SX + wc0 + 16 * j + li];
#pragma unroll
                for (int i = 0; i < WR; ++i)
#pragma unroll
                    for (int j = 0; j < WC; ++j) acc[i][j] = Mfma<TC>::step(a[i], b[j], acc[i][j]);
            }
            buf ^= 1;
        }
    }

    // ---- epilogue: lane (li, lk) holds rows Mfma::row(lk, e), column li of each block
    TC* out = g.out + static_cast<int64_t>(split) * g.part_stride;
#pragma unroll
    for (int i = 0; i < WR; ++i) {
#pragma unroll
        for (int j = 0; j < WC; ++j) {
            const int c = col0 + wc0 + 16 * j + li;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t r = r0 + wr0 + 16 * i + Mfma<TC>::row(lk, e);
                if (r < g.rows && c < g.ncols) out[r * g.ldo + c] = acc[i][j][e];
            }
        }
    }
}

}  // namespace rsvd
