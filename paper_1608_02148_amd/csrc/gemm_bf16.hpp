// Tall-skinny products with A on the bf16 matrix cores (f32 accumulation).
//
// Same problem and tiling as gemm.hpp (NN: Y = A X, TN: Z = A^T Q), used by the
// mixed-precision mode:
//   - SPLIT = false: A and X are rounded to bf16 (round to nearest even, the
//     hardware pack-convert) while they are staged in LDS; one
//     v_mfma_f32_16x16x32_bf16 per 32 k.  Used for the early passes of the
//     power scheme, whose rounding errors the later iterations damp out.
//   - SPLIT = true: X = X_hi + X_lo and (for f32-stored A) A = A_hi + A_lo with
//     bf16 terms; A_hi X_hi + A_hi X_lo + A_lo X_hi is accumulated in f32.  Each
//     bf16 x bf16 product is exact in f32; the dropped A_lo X_lo term bounds
//     the error per product near 2^-18 |a||x| (a few times plain f32
//     rounding), far below bf16's 2^-9.  Used for the last sketch and for the
//     projection B^T = A^T Q.
// Both operands live in LDS k-contiguous (As[r][k], Xs[j][k]); lane (i, g) of a
// 16x16x32 step reads its 8 consecutive k with one 16-byte LDS read.  The
// 16-byte k-octets of a row are XOR-swizzled with (row / 8) so that the
// staging writes and the operand reads spread over the LDS banks.
//   - NN A: a thread loads 8 consecutive k of one row and writes one octet.
//   - TN A and X: a thread loads a 4 (k) x 8 (columns) block with four vector
//     loads (neighbouring threads take neighbouring column blocks, so the loads
//     are coalesced) and writes it transposed as eight 8-byte k-quads.
#pragma once

#include "common.hpp"
#include "gemm.hpp"

namespace rsvd {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));

// Scratch for packed X planes (see XPackBody).
struct XPack { uint16_t* p = nullptr; int64_t ld = 0; int64_t plane = 0; };

// X (K x ncols f32, ldx) -> bf16 planes P[c][k] (ld ldp): hi = bf16(x) and,
// with split, lo = bf16(x - hi) at P + plane; columns ncols..cols-1 and k in
// [K, K rounded up to 8) are zero.  One thread per (column, k-octet), the
// threads of a k-octet on consecutive columns (coalesced reads of X).
struct XPackArgs {
    const float* X; int64_t ldx; int64_t K; int ncols; int cols; uint16_t* P; int64_t ldp; int64_t plane;
    int split; const uint32_t* skip_flag; uint32_t skip_mask; Gate gate;
};
struct XPackBody {
    typedef XPackArgs Args;
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(static_cast<int64_t>(a.cols) * cdiv(a.K, 8), THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        if (a.skip_flag && ((*a.skip_flag & a.skip_mask) == 0u)) return;
        if (a.gate.w && ((*a.gate.w & a.gate.mask) == 0u)) return;
        const int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        const int c = static_cast<int>(idx % a.cols);
        const int64_t k0 = 8 * (idx / a.cols);
        if (k0 >= a.K) return;
        uint32_t hi[4], lo[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t h2 = 0, l2 = 0;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int64_t k = k0 + 2 * d + t;
                const float x = (c < a.ncols && k < a.K) ? a.X[k * a.ldx + c] : 0.0f;
                const __bf16 h = static_cast<__bf16>(x);
                const __bf16 l = static_cast<__bf16>(x - static_cast<float>(h));
                h2 |= static_cast<uint32_t>(__builtin_bit_cast(uint16_t, h)) << (16 * t);
                l2 |= static_cast<uint32_t>(__builtin_bit_cast(uint16_t, l)) << (16 * t);
            }
            hi[d] = h2; lo[d] = l2;
        }
        uint16_t* dst = a.P + static_cast<int64_t>(c) * a.ldp + k0;
        *reinterpret_cast<u32x4*>(dst) = u32x4{hi[0], hi[1], hi[2], hi[3]};
        if (a.split) *reinterpret_cast<u32x4*>(dst + a.plane) = u32x4{lo[0], lo[1], lo[2], lo[3]};
    }
};

// CENT (bf16-stored A with the column means subtracted, split arithmetic
// only): A - mu is not exact in bf16, so it is formed in f32 and staged as
// hi + lo planes like f32-stored A, instead of moving raw bf16 words.
template <typename TA, int MODE, bool SPLIT, int WR, int WC, int WGM, int WGN, int BK, bool CENT = false>
struct Bf16Tile {
    static constexpr int BM = 16 * WR * WGM;
    static constexpr int NC = 16 * WC * WGN;
    static constexpr int NT = 64 * WGM * WGN;
    static constexpr int SK = BK + 8;                // LDS row stride (bf16 elements)
    static constexpr int OCT = BK / 8;               // k-octets per row and tile
    static constexpr bool A_LO = SPLIT && (sizeof(TA) > 2 || CENT);   // bf16-stored A is exact
    static constexpr bool RAW = sizeof(TA) == 2 && !CENT;    // A staged as raw bf16 words
    static_assert(!CENT || (SPLIT && sizeof(TA) == 2), "CENT: split products of bf16-stored A");
    // NN A items: (row, octet).  TN A / X items: (k-quad, 8-column block).
    static constexpr int A_ITEMS = (MODE == MODE_NN) ? BM * OCT : (BK / 4) * (BM / 8);
    static constexpr int X_ITEMS = NC * OCT;          // (column, k-octet) of the packed X
    static constexpr int A_PASSES = (A_ITEMS + NT - 1) / NT;
    static constexpr int X_PASSES = (X_ITEMS + NT - 1) / NT;
    static constexpr int A_VALS = (MODE == MODE_NN) ? 8 : 32;   // floats per A item
    static constexpr int A_PLANES = A_LO ? 2 : 1;
    static constexpr int X_PLANES = SPLIT ? 2 : 1;
    static constexpr size_t A_LDS = static_cast<size_t>(BM) * SK;
    static constexpr size_t X_LDS = static_cast<size_t>(NC) * SK;
    static constexpr size_t STAGE = A_PLANES * A_LDS + X_PLANES * X_LDS;
    static constexpr size_t LDS_BYTES = 2ull * STAGE * sizeof(__bf16);
    static_assert(BK % 32 == 0 && (OCT & (OCT - 1)) == 0, "BK: multiple of 32, power-of-two octets");
};

// Element offset of (row r, k) in a swizzled k-contiguous plane.
template <int SK, int OCT>
__device__ __forceinline__ int swz(int r, int k) {
    return r * SK + ((((k >> 3) ^ (r >> 3)) & (OCT - 1)) << 3) + (k & 7);
}

template <typename TA>
__device__ __forceinline__ void load8(const TA* p, bool vec, int valid, float (&v)[8]) {
    if (vec && valid >= 8) {
        if constexpr (sizeof(TA) == 4) {
            float a[4], b[4];
            load_vec<TA, float, 4>(p, a);
            load_vec<TA, float, 4>(p + 4, b);
#pragma unroll
            for (int e = 0; e < 4; ++e) { v[e] = a[e]; v[4 + e] = b[e]; }
        } else {
            load_vec<TA, float, 8>(p, v);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (e < valid) ? Conv<float>::to(p[e]) : 0.0f;
    }
}

template <typename TA, int MODE, bool SPLIT, int WR, int WC, int WGM, int WGN, int BK, bool CENT = false>
__device__ __forceinline__ void gemm_bf16_body(const GemmArgs<TA, float, float>& g, int bx, int by, int bz) {
    typedef Bf16Tile<TA, MODE, SPLIT, WR, WC, WGM, WGN, BK, CENT> T;
    constexpr int SK = T::SK, OCT = T::OCT;
    if (g.skip_flag && ((*g.skip_flag & g.skip_mask) == 0u)) return;
    if (g.gate && ((*g.gate & g.gate_mask) == 0u)) return;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    __bf16* lds = reinterpret_cast<__bf16*>(smem_raw);
    auto a_plane = [&](int buf, int pl) { return lds + buf * T::STAGE + pl * T::A_LDS; };
    auto x_plane = [&](int buf, int pl) { return lds + buf * T::STAGE + T::A_PLANES * T::A_LDS + pl * T::X_LDS; };

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int64_t r0 = static_cast<int64_t>(bx) * T::BM;
    const int split = by;
    const int col0 = bz * T::NC;
    const int64_t kbeg = static_cast<int64_t>(split) * g.kchunk;
    const int64_t kend = min(g.K, kbeg + g.kchunk);

    // bf16-stored A moves as raw 16-bit words from global memory to LDS (no
    // widening and re-rounding); in the plain bf16 arithmetic the column
    // means are subtracted from those words and the difference rounded once
    // to bf16, in the split arithmetic (CENT) A - mu goes through f32.
    constexpr bool RAW = T::RAW;
    float ra[RAW ? 1 : T::A_PASSES][RAW ? 1 : T::A_VALS];
    uint32_t rb[RAW ? T::A_PASSES : 1][RAW ? T::A_VALS / 2 : 1];
    uint32_t rx[T::X_PASSES][SPLIT ? 8 : 4];
    // 8 bf16 words of A at p (vec: one 16-byte load), zero past `valid`,
    // minus mu[0..8) when mu is given (then rounded to bf16).
    auto load_raw8 = [&](const TA* p, int valid, const double* mu, uint32_t* w) {
        if (g.a_vec && valid >= 8) {
            const u32x4 v = *reinterpret_cast<const u32x4*>(p);
#pragma unroll
            for (int d = 0; d < 4; ++d) w[d] = v[d];
        } else {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const uint32_t lo = (2 * d < valid) ? *reinterpret_cast<const uint16_t*>(p + 2 * d) : 0u;
                const uint32_t hi = (2 * d + 1 < valid) ? *reinterpret_cast<const uint16_t*>(p + 2 * d + 1) : 0u;
                w[d] = lo | (hi << 16);
            }
        }
        if (mu) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                if (e >= valid) continue;
                const uint32_t bits = (w[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
                const float x = static_cast<float>(static_cast<double>(__uint_as_float(bits << 16)) - mu[e]);
                const uint32_t nb = __builtin_bit_cast(uint16_t, static_cast<__bf16>(x));
                w[e >> 1] = (e & 1) ? ((w[e >> 1] & 0x0000FFFFu) | (nb << 16)) : ((w[e >> 1] & 0xFFFF0000u) | nb);
            }
        }
    };

    auto load_a = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < T::A_PASSES; ++p) {
            const int it = p * T::NT + tid;
            if (it >= T::A_ITEMS) break;
            if constexpr (MODE == MODE_NN && RAW) {
                const int r = it / OCT, o = it % OCT;
                const int64_t gr = r0 + r, gk = k0 + 8 * o;
                const int valid = (gr < g.rows) ? static_cast<int>(max<int64_t>(0, min<int64_t>(8, kend - gk))) : 0;
                load_raw8(g.A + gr * g.lda + gk, valid, g.mu ? g.mu + gk : nullptr, rb[p]);
            } else if constexpr (MODE != MODE_NN && RAW) {
                const int cb = it % (T::BM / 8), kq = it / (T::BM / 8);
                const int64_t gc = r0 + 8 * cb;
                const int cvalid = static_cast<int>(max<int64_t>(0, min<int64_t>(8, g.rows - gc)));
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t ak = k0 + 4 * kq + q;
                    load_raw8(g.A + ak * g.lda + gc, ak < kend ? cvalid : 0, g.mu ? g.mu + gc : nullptr, rb[p] + 4 * q);
                }
            } else if constexpr (MODE == MODE_NN) {
                const int r = it / OCT, o = it % OCT;
                const int64_t gr = r0 + r, gk = k0 + 8 * o;
                const int valid = (gr < g.rows) ? static_cast<int>(max<int64_t>(0, min<int64_t>(8, kend - gk))) : 0;
                float v[8];
                load8<TA>(g.A + gr * g.lda + gk, g.a_vec, valid, v);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    float x = v[e];
                    if (g.mu && e < valid) x = static_cast<float>(static_cast<double>(x) - g.mu[gk + e]);
                    ra[p][e] = x;
                }
            } else {
                const int cb = it % (T::BM / 8), kq = it / (T::BM / 8);
                const int64_t gc = r0 + 8 * cb;          // first of 8 columns of A
                const int cvalid = static_cast<int>(max<int64_t>(0, min<int64_t>(8, g.rows - gc)));
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t ak = k0 + 4 * kq + q;
                    float v[8];
                    load8<TA>(g.A + ak * g.lda + gc, g.a_vec, ak < kend ? cvalid : 0, v);
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        float x = v[e];
                        if (g.mu && ak < kend && e < cvalid) x = static_cast<float>(static_cast<double>(x) - g.mu[gc + e]);
                        ra[p][q * 8 + e] = x;
                    }
                }
            }
        }
    };
    // Packed X: item (column j, k-octet o), eight threads per 128 contiguous
    // bytes of a column; k past the split's end reads as zero.
    auto load_x = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < T::X_PASSES; ++p) {
            const int it = p * T::NT + tid;
            if (it >= T::X_ITEMS) break;
            const int j = it / OCT, o = it % OCT;
            const int64_t gk = k0 + 8 * o;
            const int valid = static_cast<int>(max<int64_t>(0, min<int64_t>(8, kend - gk)));
            const uint16_t* src = g.xb + static_cast<int64_t>(col0 + j) * g.ldxb + gk;
#pragma unroll
            for (int pl = 0; pl < (SPLIT ? 2 : 1); ++pl) {
                const uint16_t* s = src + pl * g.xb_plane;
                if (valid == 8) {
                    const u32x4 v = *reinterpret_cast<const u32x4*>(s);
#pragma unroll
                    for (int d = 0; d < 4; ++d) rx[p][4 * pl + d] = v[d];
                } else {
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const uint32_t lo = (2 * d < valid) ? s[2 * d] : 0u;
                        const uint32_t hi = (2 * d + 1 < valid) ? s[2 * d + 1] : 0u;
                        rx[p][4 * pl + d] = lo | (hi << 16);
                    }
                }
            }
        }
    };
    // Transposed 4 (k) x 8 (rows) block: row rr+e gets k-quad kq of the tile.
    auto store_block = [&](__bf16* hi_plane, __bf16* lo_plane, bool lo_on, int rr, int kq, const float* v) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            v4bf h, lo;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float x = v[q * 8 + e];
                h[q] = static_cast<__bf16>(x);
                if (lo_on) lo[q] = static_cast<__bf16>(x - static_cast<float>(h[q]));
            }
            const int off = swz<SK, OCT>(rr + e, 4 * kq);
            *reinterpret_cast<v4bf*>(hi_plane + off) = h;
            if (lo_on) *reinterpret_cast<v4bf*>(lo_plane + off) = lo;
        }
    };
    auto store_tiles = [&](int buf) {
#pragma unroll
        for (int p = 0; p < T::A_PASSES; ++p) {
            const int it = p * T::NT + tid;
            if (it >= T::A_ITEMS) break;
            if constexpr (MODE == MODE_NN && RAW) {
                const int r = it / OCT, o = it % OCT;
                const int off = swz<SK, OCT>(r, 8 * o);
                *reinterpret_cast<u32x4*>(a_plane(buf, 0) + off) = u32x4{rb[p][0], rb[p][1], rb[p][2], rb[p][3]};
            } else if constexpr (MODE != MODE_NN && RAW) {
                // 4 (k) x 8 (rows of the tile) words: row 8 cb + e gets the
                // k-quad (w_0[e], w_1[e], w_2[e], w_3[e])
                const int cb = it % (T::BM / 8), kq = it / (T::BM / 8);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int d = e >> 1, sh = 16 * (e & 1);
                    const uint32_t v0 = (rb[p][d] >> sh) & 0xFFFFu, v1 = (rb[p][4 + d] >> sh) & 0xFFFFu;
                    const uint32_t v2 = (rb[p][8 + d] >> sh) & 0xFFFFu, v3 = (rb[p][12 + d] >> sh) & 0xFFFFu;
                    const int off = swz<SK, OCT>(8 * cb + e, 4 * kq);
                    *reinterpret_cast<u32x2*>(a_plane(buf, 0) + off) = u32x2{v0 | (v1 << 16), v2 | (v3 << 16)};
                }
            } else if constexpr (MODE == MODE_NN) {
                const int r = it / OCT, o = it % OCT;
                v8bf h, lo;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    h[e] = static_cast<__bf16>(ra[p][e]);
                    if (T::A_LO) lo[e] = static_cast<__bf16>(ra[p][e] - static_cast<float>(h[e]));
                }
                const int off = swz<SK, OCT>(r, 8 * o);
                *reinterpret_cast<v8bf*>(a_plane(buf, 0) + off) = h;
                if (T::A_LO) *reinterpret_cast<v8bf*>(a_plane(buf, 1) + off) = lo;
            } else {
                const int cb = it % (T::BM / 8), kq = it / (T::BM / 8);
                store_block(a_plane(buf, 0), a_plane(buf, T::A_LO ? 1 : 0), T::A_LO, 8 * cb, kq, ra[p]);
            }
        }
#pragma unroll
        for (int p = 0; p < T::X_PASSES; ++p) {
            const int it = p * T::NT + tid;
            if (it >= T::X_ITEMS) break;
            const int j = it / OCT, o = it % OCT;
            const int off = swz<SK, OCT>(j, 8 * o);
            *reinterpret_cast<u32x4*>(x_plane(buf, 0) + off) = u32x4{rx[p][0], rx[p][1], rx[p][2], rx[p][3]};
            if constexpr (SPLIT)
                *reinterpret_cast<u32x4*>(x_plane(buf, 1) + off) = u32x4{rx[p][4], rx[p][5], rx[p][6], rx[p][7]};
        }
    };

    v4f acc[WR][WC];
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
        for (int j = 0; j < WC; ++j) acc[i][j] = v4f{0, 0, 0, 0};

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
#pragma unroll
            for (int kg = 0; kg < BK; kg += 32) {
                v8bf ah[WR], bh[WC], al[WR], bl[WC];
#pragma unroll
                for (int i = 0; i < WR; ++i) {
                    const int off = swz<SK, OCT>(wr0 + 16 * i + li, kg + 8 * lk);
                    ah[i] = *reinterpret_cast<const v8bf*>(a_plane(buf, 0) + off);
                    if (T::A_LO) al[i] = *reinterpret_cast<const v8bf*>(a_plane(buf, 1) + off);
                }
#pragma unroll
                for (int j = 0; j < WC; ++j) {
                    const int off = swz<SK, OCT>(wc0 + 16 * j + li, kg + 8 * lk);
                    bh[j] = *reinterpret_cast<const v8bf*>(x_plane(buf, 0) + off);
                    if (SPLIT) bl[j] = *reinterpret_cast<const v8bf*>(x_plane(buf, 1) + off);
                }
#pragma unroll
                for (int i = 0; i < WR; ++i)
#pragma unroll
                    for (int j = 0; j < WC; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                        if (SPLIT) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                        if (T::A_LO) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    }
            }
            buf ^= 1;
        }
    }

    float* out = g.out + static_cast<int64_t>(split) * g.part_stride;
#pragma unroll
    for (int i = 0; i < WR; ++i) {
#pragma unroll
        for (int j = 0; j < WC; ++j) {
            const int c = col0 + wc0 + 16 * j + li;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t r = r0 + wr0 + 16 * i + 4 * lk + e;
                if (r < g.rows && c < g.ncols) out[r * g.ldo + c] = acc[i][j][e];
            }
        }
    }
}

}  // namespace rsvd
