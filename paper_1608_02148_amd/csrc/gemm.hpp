// Tall-skinny products with the input matrix A on the matrix cores.
//
//   NN:  Y = A X    (A m x K row-major, X K x c)   Alg. rqb and
//                                                  Alg. subspace_iter
//   TN:  Z = A^T Q  (A K x n row-major, Q K x c)   Alg. subspace_iter
//                                                  and Alg. rqb (B^T)
//
// Both share one tile engine.  A workgroup owns a BM x NC block of the output
// and walks the reduction dimension k in steps of BK.  Lane (i, g) of a
// 16x16xKV*4 group feeds matrix-core step v with k = KV*g + v for both
// operands, so the reduction covers every k exactly once.
//   - X is staged k-contiguous, Xs[j][k]: one 16-byte LDS read gives a lane
//     its operands for KV steps.  Neighbouring lanes load neighbouring
//     columns of X, so each (scalar) global load instruction is coalesced.
//   - NN stages A k-contiguous too, As[r][k]: each thread loads KV
//     consecutive k of one row of A with one vector load and stores them with
//     one 16-byte LDS write; fragments are 16-byte LDS reads.
//   - TN stages A in its natural order, As[k][r]: each thread loads KV
//     consecutive columns of one row of A (one vector load, 16-byte LDS
//     write); a fragment is KV 4/8-byte LDS reads of 16 consecutive r.
// LDS is double buffered; the next tile's global loads are in flight while the
// current tile is multiplied, with a single barrier per step.
// X may come k-contiguous (g.xk, packed once per product), then each k-vector
// of a column is one vector load.
//
// Split-K: grid.y = S splits the reduction into S contiguous chunks.  With
// S > 1 every split writes its own partial block and a separate kernel sums the
// partials in split order, so results are deterministic (no atomics).
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
    int32_t splits;      // number of splits S (grid extent along the reduction)
    // streamed products: the (tile, split) pairs past the last whole round of
    // tail_groups workgroups are dealt to tail_groups more workgroups in equal
    // shares of chunks, which write slots of TROWS x ld_slot (see StreamBody)
    int32_t upper_only;  // square tiles of a symmetric product: skip the tiles below the diagonal
    int32_t tail_groups;
    float* tail_slots;
    int64_t ld_slot;
    const TX* X;         // K x (col tiles * NC) operand
    int64_t ldx;
    int32_t ncols;       // valid output columns (all column tiles together)
    TC* out;             // rows x ncols (ldo) or S partial blocks
    int64_t ldo;
    int64_t part_stride; // elements between split partial blocks (S > 1)
    const double* mu;    // optional column means of A (implicit centring)
    const uint32_t* skip_flag;  // optional: run only if (*skip_flag & skip_mask)
    uint32_t skip_mask;
    const uint32_t* gate;       // optional second condition: run only if (*gate & gate_mask)
    uint32_t gate_mask;
    int32_t a_vec;       // 1 when A rows allow aligned vector loads
    int32_t x_vec;       // unused (X is read with scalar loads)
    const uint16_t* xb;  // bf16 products: X packed by XPackBody, bf16 planes [column][k]
    int64_t ldxb;        // k stride of a packed column (a multiple of 8)
    int64_t xb_plane;    // elements from the hi plane to the lo plane
    const TC* xk;        // optional: X in the compute type packed [column][k] (ld ldxk, a
    int64_t ldxk;        // multiple of 16 / sizeof(TC)), read with one vector load per item
};

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// KV consecutive elements of TA starting at p (KV * sizeof(TA) bytes,
// naturally aligned), converted to TC.
template <typename TA, typename TC, int KV>
__device__ __forceinline__ void load_vec(const TA* p, TC (&dst)[KV]) {
    constexpr int BYTES = KV * sizeof(TA);
    if constexpr (BYTES == 16) {
        const u32x4 raw = *reinterpret_cast<const u32x4*>(p);
        if constexpr (sizeof(TA) == 8) {
            dst[0] = Conv<TC>::to(__hiloint2double(raw[1], raw[0]));
            dst[1] = Conv<TC>::to(__hiloint2double(raw[3], raw[2]));
        } else if constexpr (sizeof(TA) == 4) {
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[e] = Conv<TC>::to(__uint_as_float(raw[e]));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                dst[2 * e] = Conv<TC>::to(__uint_as_float(raw[e] << 16));
                dst[2 * e + 1] = Conv<TC>::to(__uint_as_float(raw[e] & 0xFFFF0000u));
            }
        }
    } else if constexpr (BYTES == 8) {
        const u32x2 raw = *reinterpret_cast<const u32x2*>(p);
        if constexpr (sizeof(TA) == 4) {
            dst[0] = Conv<TC>::to(__uint_as_float(raw[0]));
            dst[1] = Conv<TC>::to(__uint_as_float(raw[1]));
        } else {
            static_assert(sizeof(TA) == 2, "");
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                dst[2 * e] = Conv<TC>::to(__uint_as_float(raw[e] << 16));
                dst[2 * e + 1] = Conv<TC>::to(__uint_as_float(raw[e] & 0xFFFF0000u));
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < KV; ++e) dst[e] = Conv<TC>::to(p[e]);
    }
}

template <typename TA, typename TX, typename TC, int MODE, int WR, int WC, int WGM, int WGN, int BK>
struct GemmTile {
    static constexpr int BM = 16 * WR * WGM;
    static constexpr int NC = 16 * WC * WGN;
    static constexpr int NT = 64 * WGM * WGN;
    static constexpr int KV = 16 / sizeof(TC);          // k values per 16-byte LDS read
    static constexpr int KG = 4 * KV;                   // k covered by one read group
    static constexpr int SK = BK + 16 / sizeof(TC);     // LDS row stride (elements)
    static constexpr int KVECS = BK / KV;               // k-vectors per row and tile
    static constexpr int A_ITEMS = BM * KVECS;        // NN: rows x k-vectors; TN: k rows x r-vectors
    static constexpr int X_ITEMS = NC * KVECS;
    static constexpr int A_PASSES = (A_ITEMS + NT - 1) / NT;
    static constexpr int X_PASSES = (X_ITEMS + NT - 1) / NT;
    static_assert(BK % KG == 0, "BK must cover whole read groups");
    static constexpr int SR = BM + 16 / sizeof(TC);     // TN: As row stride (elements)
    static constexpr size_t A_LDS = (MODE == MODE_NN ? BM * SK : BK * SR);
    static constexpr size_t LDS_BYTES = 2ull * (A_LDS + NC * SK) * sizeof(TC);
};

// Tile (bx, by, bz) = (row tile, split, column tile) of the product g.
// XKP: X is read from the packed copy g.xk (a separate instance, so that the
// tiles without it compile exactly as before).
template <typename TA, typename TX, typename TC, int MODE, int WR, int WC, int WGM, int WGN, int BK, bool XKP = false>
__device__ __forceinline__ void gemm_tile_body(const GemmArgs<TA, TX, TC>& g, int bx, int by, int bz) {
    typedef GemmTile<TA, TX, TC, MODE, WR, WC, WGM, WGN, BK> T;
    typedef typename Mfma<TC>::acc_t acc_t;
    constexpr int KV = T::KV, SK = T::SK, KVECS = T::KVECS;
    typedef TC vec_t __attribute__((ext_vector_type(KV)));
    if (g.skip_flag && ((*g.skip_flag & g.skip_mask) == 0u)) return;
    if (g.gate && ((*g.gate & g.gate_mask) == 0u)) return;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    TC* As = reinterpret_cast<TC*>(smem_raw);            // [2][A_LDS]
    TC* Xs = As + 2 * T::A_LDS;                           // [2][NC][SK]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int64_t r0 = static_cast<int64_t>(bx) * T::BM;
    const int split = by;
    const int col0 = bz * T::NC;
    const int64_t kbeg = static_cast<int64_t>(split) * g.kchunk;
    const int64_t kend = min(g.K, kbeg + g.kchunk);

    TC ra[T::A_PASSES][KV];
    TC rx[T::X_PASSES][KV];

    // Item -> (row, k-vector) for NN, (k row, r-vector) for TN; in both the
    // vectors adjacent in global memory go to adjacent threads.
    constexpr int RVECS = T::BM / KV;
    auto a_item = [&](int it, int& r, int& kv) {
        if (MODE == MODE_NN) { r = it / KVECS; kv = it % KVECS; }
        else                 { kv = it / RVECS; r = (it % RVECS) * KV; }   // kv = k row here
    };
    auto load_a = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < T::A_PASSES; ++p) {
            const int it = p * T::NT + tid;
            if (it >= T::A_ITEMS) break;
            int r, kv;
            a_item(it, r, kv);
            const int64_t gk = k0 + kv * KV;
            const int64_t gr = r0 + r;
            if (MODE == MODE_NN) {
                const TA* src = g.A + gr * g.lda + gk;
                if (gr < g.rows && g.a_vec && gk + KV <= kend) {
                    load_vec<TA, TC, KV>(src, ra[p]);
                    if (g.mu) {
#pragma unroll
                        for (int e = 0; e < KV; ++e)
                            ra[p][e] = Conv<TC>::to(Conv<double>::to(ra[p][e]) - g.mu[gk + e]);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < KV; ++e) {
                        TC v = TC(0);
                        if (gr < g.rows && gk + e < kend)
                            v = g.mu ? Conv<TC>::to(Conv<double>::to(src[e]) - g.mu[gk + e]) : Conv<TC>::to(src[e]);
                        ra[p][e] = v;
                    }
                }
            } else {
                // TN: kv is a row of A (k), gr the first of KV columns (r).
                const int64_t ak = k0 + kv;
                const TA* src = g.A + ak * g.lda + gr;
                if (ak < kend && g.a_vec && gr + KV <= g.rows) {
                    load_vec<TA, TC, KV>(src, ra[p]);
                    if (g.mu) {
#pragma unroll
                        for (int e = 0; e < KV; ++e)
                            ra[p][e] = Conv<TC>::to(Conv<double>::to(ra[p][e]) - g.mu[gr + e]);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < KV; ++e) {
                        TC v = TC(0);
                        if (ak < kend && gr + e < g.rows)
                            v = g.mu ? Conv<TC>::to(Conv<double>::to(src[e]) - g.mu[gr + e]) : Conv<TC>::to(src[e]);
                        ra[p][e] = v;
                    }
                }
            }
        }
    };
    // X item -> (column, k-vector): columns fastest for X itself (neighbouring
    // lanes read neighbouring columns of a row), k-vectors fastest for the
    // packed copy (neighbouring lanes read consecutive 16 bytes of a column).
    auto x_item = [&](int it, int& j, int& kv) {
        if constexpr (XKP) { j = it / KVECS; kv = it % KVECS; }
        else               { j = it % T::NC; kv = it / T::NC; }
    };
    auto load_x = [&](int64_t k0) {
        if constexpr (XKP) {
#pragma unroll
            for (int p = 0; p < T::X_PASSES; ++p) {
                const int it = p * T::NT + tid;
                if (it >= T::X_ITEMS) break;
                int j, kv;
                x_item(it, j, kv);
                const int64_t gk = k0 + kv * KV;
                const int gc = col0 + j;
                const TC* src = g.xk + static_cast<int64_t>(gc) * g.ldxk + gk;
                if (gc < g.ncols && gk + KV <= kend) {
                    const vec_t v = *reinterpret_cast<const vec_t*>(src);
#pragma unroll
                    for (int e = 0; e < KV; ++e) rx[p][e] = v[e];
                } else {
#pragma unroll
                    for (int e = 0; e < KV; ++e) rx[p][e] = (gc < g.ncols && gk + e < kend) ? src[e] : TC(0);
                }
            }
            return;
        }
#pragma unroll
        for (int p = 0; p < T::X_PASSES; ++p) {
            const int it = p * T::NT + tid;
            if (it >= T::X_ITEMS) break;
            int j, kv;
            x_item(it, j, kv);
            const int64_t gk = k0 + kv * KV;
            const int gc = col0 + j;
            const bool ok = gc < g.ncols;
#pragma unroll
            for (int e = 0; e < KV; ++e)
                rx[p][e] = (ok && gk + e < kend) ? Conv<TC>::to(g.X[(gk + e) * g.ldx + gc]) : TC(0);
        }
    };
    auto store_tiles = [&](int buf) {
        TC* as = As + buf * T::A_LDS;
        TC* xs = Xs + buf * T::NC * SK;
#pragma unroll
        for (int p = 0; p < T::A_PASSES; ++p) {
            const int it = p * T::NT + tid;
            if (it >= T::A_ITEMS) break;
            int r, kv;
            a_item(it, r, kv);
            vec_t v;
#pragma unroll
            for (int e = 0; e < KV; ++e) v[e] = ra[p][e];
            if (MODE == MODE_NN) *reinterpret_cast<vec_t*>(as + r * SK + kv * KV) = v;
            else                 *reinterpret_cast<vec_t*>(as + kv * T::SR + r) = v;
        }
#pragma unroll
        for (int p = 0; p < T::X_PASSES; ++p) {
            const int it = p * T::NT + tid;
            if (it >= T::X_ITEMS) break;
            int j, kv;
            x_item(it, j, kv);
            vec_t v;
#pragma unroll
            for (int e = 0; e < KV; ++e) v[e] = rx[p][e];
            *reinterpret_cast<vec_t*>(xs + j * SK + kv * KV) = v;
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
            // 16-wave TN tiles (one workgroup per CU) issue the next tile's
            // global loads after their first group of fragment reads; measured
            // faster there, and slower for NN and for the 8-wave tiles (two
            // workgroups per CU) of batches
            constexpr int LOAD_KG = (MODE == MODE_TN && WGM * WGN >= 16 && BK > T::KG) ? T::KG : 0;
            if (LOAD_KG == 0 && k0 + BK < kend) { load_a(k0 + BK); load_x(k0 + BK); }
            const TC* as = As + buf * T::A_LDS;
            const TC* xs = Xs + buf * T::NC * SK;
#pragma unroll
            for (int kg = 0; kg < BK; kg += T::KG) {
                if (LOAD_KG != 0 && kg == LOAD_KG && k0 + BK < kend) { load_a(k0 + BK); load_x(k0 + BK); }
                vec_t a[WR], b[WC];
#pragma unroll
                for (int i = 0; i < WR; ++i) {
                    if (MODE == MODE_NN) {
                        a[i] = *reinterpret_cast<const vec_t*>(as + (wr0 + 16 * i + li) * SK + kg + KV * lk);
                    } else {
#pragma unroll
                        for (int v = 0; v < KV; ++v) a[i][v] = as[(kg + KV * lk + v) * T::SR + wr0 + 16 * i + li];
                    }
                }
#pragma unroll
                for (int j = 0; j < WC; ++j)
                    b[j] = *reinterpret_cast<const vec_t*>(xs + (wc0 + 16 * j + li) * SK + kg + KV * lk);
#pragma unroll
                for (int v = 0; v < KV; ++v)
#pragma unroll
                    for (int i = 0; i < WR; ++i)
#pragma unroll
                        for (int j = 0; j < WC; ++j) acc[i][j] = Mfma<TC>::step(a[i][v], b[j][v], acc[i][j]);
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

template <typename TA, typename TX, typename TC, int MODE, int WR, int WC, int WGM, int WGN, int BK>
__global__ __launch_bounds__(64 * WGM * WGN)
void gemm_tile_kernel(GemmArgs<TA, TX, TC> g) {
    gemm_tile_body<TA, TX, TC, MODE, WR, WC, WGM, WGN, BK>(g, blockIdx.x, blockIdx.y, blockIdx.z);
}

}  // namespace rsvd
