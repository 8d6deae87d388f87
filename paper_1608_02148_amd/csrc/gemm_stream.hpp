// Streamed-A tall-skinny products: Y = A X (NN) and Z = A^T Q (TN) for large A.
//
// The large operand A is read from global memory straight into matrix-core
// operand registers, once, and never staged through LDS; only the skinny
// operand (X, or Q, packed k-contiguous per column) is staged in LDS, where
// the four waves of a workgroup (one per SIMD) share it.  Each wave owns 64
// output rows and every output column of the product (NC = 16 NCB <= 224), so
// one A fragment feeds NCB column blocks of matrix-core work and one X
// fragment feeds four row blocks: per 16-byte LDS read a wave issues four
// MFMAs.  The accumulators (up to 224 registers) live in the AGPR file; the
// next chunk of A is loaded into registers while the current one is
// multiplied (one chunk ahead), and X's next chunk is staged through
// registers into the other of two LDS buffers.  WPS = 2 runs two waves per
// SIMD instead: eight waves of 32 rows, two row blocks each, half the
// registers per wave, so that while one wave waits for a load, a barrier or
// an LDS read the other's MFMAs keep the matrix core busy; each X fragment
// then feeds two MFMAs (A^T Q: a lane then loads two columns per row of A).
// WPS = 3 splits those eight waves into two workgroups of four (128-row
// tiles, two per CU), whose barriers and X stages are independent.
//
// Lane (r, g) (r = lane & 15, g = lane >> 4) owns the k-run [k0 + LK g,
// k0 + LK (g + 1)) of each chunk of KC = 4 LK reduction elements; substep s of
// the chunk uses elements V s .. V s + V - 1 of every lane's run (V = 1 for the
// f32 16x16x4 MFMA, 8 for the bf16 16x16x32 MFMA), so lane group g always
// supplies the k-values the MFMA expects from it and A and X agree on the
// order.  (The order in which a product sums its reduction does not change
// what it computes.)
//
//   NN: lane (r, g) loads LK consecutive elements of row r0 + 16 i + r for each
//       of the wave's four row blocks i (32 or 64 contiguous bytes: whole cache
//       lines per row and chunk).
//   TN: the output rows are columns of A.  Lane (i, g) loads RB consecutive
//       columns c0 + RB i .. c0 + RB i + RB - 1 of each of its LK rows of A (16
//       lanes read 32 to 128 contiguous bytes of a row); MFMA row block e then
//       takes column c0 + RB i + e as its row i, so the wave's 16 RB output rows
//       are the columns c0 + RB (4 g + v) + e of accumulator element v of block
//       e.  For bf16 the lane transposes its LK x RB block in registers into
//       k-octets.
//
// Arithmetic (as in the LDS-staged tiles): 0 = f32 MFMA (bf16-stored A widened
// exactly), 1 = bf16 MFMA on A and X rounded to bf16, 2 = split bf16: X = X_hi
// + X_lo and, for f32-stored A or centred bf16 A (CENT), A = A_hi + A_lo, with
// A_hi X_hi + A_hi X_lo + A_lo X_hi accumulated in f32.
//
// Split reduction: workgroup (tile t, split s) sums k in [s kchunk, min(K,
// (s + 1) kchunk)) and writes partial block s (S > 1) or the result.
#pragma once

#include "common.hpp"
#include "exec.hpp"
#include "gemm.hpp"

namespace rsvd {

typedef __bf16 s8bf __attribute__((ext_vector_type(8)));

template <typename TA, int MODE, int ARITH, int NCB, int WPS = 1, bool CENT = false, bool MU = false>
struct StreamTile {
    static constexpr bool BF = ARITH != 0;
    static constexpr bool SPLIT = ARITH == 2;
    static constexpr bool A_LO = SPLIT && (sizeof(TA) == 4 || CENT);
    static constexpr int V = BF ? 8 : 1;            // values per lane per MFMA
    // k-run per lane per chunk: 16 (f32 with up to 128 columns: 64-element
    // chunks halve the per-chunk barrier and waits), else 16 for bf16 and 8
    // for f32 (the registers of two chunks of A beside 224 columns of
    // accumulators)
    static constexpr int LK = (BF || NCB <= 8) ? 16 : 8;
    static constexpr int KC = 4 * LK;               // chunk extent
    static constexpr int SUB = LK / V;              // MFMA substeps per chunk
    // layouts: WPS = 1: four waves of four row blocks (one per SIMD); 2: eight
    // waves of two (two per SIMD); 3: four waves of two in 128-row tiles, two
    // workgroups per CU
    static constexpr int RB = WPS == 1 ? 4 : 2;     // MFMA row blocks per wave
    static constexpr int WAVES = WPS == 2 ? 8 : 4;  // row strips
    static constexpr int NT = 64 * WAVES;
    static constexpr int TROWS = WAVES * 16 * RB;   // output rows per tile
    static constexpr int NC = 16 * NCB;             // output columns per tile
    static constexpr int ESZ = BF ? 2 : 4;          // staged X element bytes
    static constexpr int SX = KC + 16 / ESZ;        // LDS column stride: 16 bytes past a multiple of 128
    static constexpr int XPL = SPLIT ? 2 : 1;
    static constexpr int VPC = KC * ESZ / 16;       // 16-byte vectors per column and chunk (8)
    static constexpr int X_PASSES = (NC * VPC + NT - 1) / NT;
    static constexpr size_t PLANE = static_cast<size_t>(NC) * SX;
    static constexpr size_t STAGE = XPL * PLANE;    // elements
    static constexpr size_t LDS_BYTES = 2 * STAGE * ESZ;
    // raw A words per lane and chunk (32-bit registers)
    static constexpr int A_WORDS = RB * LK * static_cast<int>(sizeof(TA)) / 4;
    // TN: words per row of A of a lane's RB consecutive columns
    static constexpr int TW = RB * static_cast<int>(sizeof(TA)) / 4;
    static_assert((SX * ESZ) % 128 == 16, "LDS column stride");
    static_assert(!CENT || (SPLIT && sizeof(TA) == 2 && MU), "CENT: split products of centred bf16-stored A");
    static_assert(WPS >= 1 && WPS <= 3 && TROWS == (WPS == 3 ? 128 : 256), "row-strip layouts");
};

template <typename TA>
__device__ __forceinline__ float word_elem(const uint32_t* w, int e) {
    if constexpr (sizeof(TA) == 4) return __uint_as_float(w[e]);
    else return __uint_as_float(((w[e >> 1] >> (16 * (e & 1))) & 0xFFFFu) << 16);
}

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, static_cast<__bf16>(a))) |
           (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, static_cast<__bf16>(b))) << 16);
}

__device__ __forceinline__ float bf16_round(float x) {
    return static_cast<float>(static_cast<__bf16>(x));
}

// One (tile, reduction range) of the product: output rows tile * TROWS ..
// of the tile, summed over k in [kbeg, kend), written to out (row r at
// out + (r - row0) ldo).
template <typename TA, int MODE, int ARITH, int NCB, int WPS, bool CENT, bool MU>
__device__ __forceinline__ void gemm_stream_body(const GemmArgs<TA, float, float>& g, int tile, int64_t kbeg,
                                                 int64_t kend, float* out, int64_t row0, int64_t ldo) {
    typedef StreamTile<TA, MODE, ARITH, NCB, WPS, CENT, MU> T;
    constexpr int LK = T::LK, KC = T::KC, SUB = T::SUB, RB = T::RB, SX = T::SX;
    constexpr int AW = T::A_WORDS;
    if (g.skip_flag && ((*g.skip_flag & g.skip_mask) == 0u)) return;
    if (g.gate && ((*g.gate & g.gate_mask) == 0u)) return;

    // An (empty) use of an accumulation register: without one the compiler
    // gives the MFMAs their all-VGPR form, which caps the wave at 256 registers
    // and spills; with it the accumulators live in the AGPR file and the
    // operands, staging and addresses in the VGPR file (512 in all at one wave
    // per SIMD, 256 at two).
    asm volatile("" ::: "a0");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int strip = wave, cb0 = 0;                      // row strip, first column block
    const int64_t w0 = static_cast<int64_t>(tile) * T::TROWS + static_cast<int64_t>(strip) * 16 * RB;

    // ---- A: raw words of one chunk
    auto load_a = [&](int64_t k0, uint32_t (&w)[AW], bool full) {
        if constexpr (MODE == MODE_NN) {
            constexpr int WPR = LK * sizeof(TA) / 4;          // words per row block
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const int64_t r = min(w0 + 16 * i + lr, g.rows - 1);     // rows past the end: never stored
                const int64_t k = k0 + LK * lg;
                const TA* p = g.A + r * g.lda + k;
                if (full) {
#pragma unroll
                    for (int v = 0; v < WPR / 4; ++v) {
                        const u32x4 x = *reinterpret_cast<const u32x4*>(p + v * (16 / sizeof(TA)));
#pragma unroll
                        for (int d = 0; d < 4; ++d) w[i * WPR + 4 * v + d] = x[d];
                    }
                } else {
#pragma unroll
                    for (int d = 0; d < WPR; ++d) w[i * WPR + d] = 0u;
                    if constexpr (sizeof(TA) == 4) {
#pragma unroll
                        for (int e = 0; e < LK; ++e)
                            if (k + e < kend) w[i * WPR + e] = reinterpret_cast<const uint32_t*>(p)[e];
                    } else {
#pragma unroll
                        for (int e = 0; e < LK; ++e)
                            if (k + e < kend)
                                w[i * WPR + (e >> 1)] |= static_cast<uint32_t>(reinterpret_cast<const uint16_t*>(p)[e])
                                                         << (16 * (e & 1));
                    }
                }
            }
        } else {
            constexpr int WPR = T::TW;                      // words per row of RB columns (4 to 16 bytes)
            // columns past the end (whole groups of RB: rows % 4 == 0) read
            // column 0 instead and are never stored
            const int64_t c = (w0 + RB * lr < g.rows) ? w0 + RB * lr : 0;
#pragma unroll
            for (int t = 0; t < LK; ++t) {
                const int64_t k = k0 + LK * lg + t;
                const TA* p = g.A + k * g.lda + c;
                if (full || k < kend) {
                    if constexpr (WPR == 4) {
                        const u32x4 x = *reinterpret_cast<const u32x4*>(p);
#pragma unroll
                        for (int d = 0; d < 4; ++d) w[t * WPR + d] = x[d];
                    } else if constexpr (WPR == 2) {
                        const u32x2 x = *reinterpret_cast<const u32x2*>(p);
                        w[t * WPR] = x[0];
                        w[t * WPR + 1] = x[1];
                    } else {
                        w[t] = *reinterpret_cast<const uint32_t*>(p);
                    }
                } else {
#pragma unroll
                    for (int d = 0; d < WPR; ++d) w[t * WPR + d] = 0u;
                }
            }
        }
    };

    // TN with column means: this lane's four columns are fixed
    double mu_c[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (MODE == MODE_TN && MU) {
        {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t c = w0 + 4 * lr + e;
                mu_c[e] = c < g.rows ? g.mu[c] : 0.0;
            }
        }
    }

    // ---- X: one chunk of the packed columns, staged through registers
    typedef typename std::conditional<T::BF, uint16_t, float>::type XE;
    XE* xs = reinterpret_cast<XE*>(smem_raw);
    uint32_t rx[T::X_PASSES][T::XPL][4];
    auto load_x = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < T::X_PASSES; ++p) {
            const int it = p * T::NT + tid;
            const int col = it / T::VPC, v = it % T::VPC;
            const int64_t k = k0 + v * (16 / T::ESZ);
#pragma unroll
            for (int pl = 0; pl < T::XPL; ++pl) {
                u32x4 x = u32x4{0u, 0u, 0u, 0u};
                if (col < T::NC && k < kend) {
                    if constexpr (T::BF) {
                        x = *reinterpret_cast<const u32x4*>(g.xb + pl * g.xb_plane + static_cast<int64_t>(col) * g.ldxb + k);
                    } else {
                        if (col < g.ncols) x = *reinterpret_cast<const u32x4*>(g.xk + static_cast<int64_t>(col) * g.ldxk + k);
                    }
                }
#pragma unroll
                for (int d = 0; d < 4; ++d) rx[p][pl][d] = x[d];
            }
        }
    };
    auto store_x = [&](int buf) {
#pragma unroll
        for (int p = 0; p < T::X_PASSES; ++p) {
            const int it = p * T::NT + tid;
            const int col = it / T::VPC, v = it % T::VPC;
            if (col >= T::NC) continue;
#pragma unroll
            for (int pl = 0; pl < T::XPL; ++pl) {
                XE* dst = xs + buf * T::STAGE + pl * T::PLANE + col * SX + v * (16 / T::ESZ);
                *reinterpret_cast<u32x4*>(dst) = u32x4{rx[p][pl][0], rx[p][pl][1], rx[p][pl][2], rx[p][pl][3]};
            }
        }
    };

    v4f acc[RB][NCB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < NCB; ++j) acc[i][j] = v4f{0, 0, 0, 0};

    // ---- one chunk of matrix-core work from raw A words w and X stage buf.
    // The column blocks are software-pipelined by hand (the X fragment of
    // block j + 1 is read while block j's MFMAs issue) and fenced with
    // scheduling barriers, so that the scheduler does not hoist every LDS read
    // of the chunk and run out of registers.
    // (past the end of the reduction A reads as zero and stays zero)
    auto mu_nn = [&](int64_t k0, int kk, float v, bool full) -> float {     // NN: A(r, k) - mu(k) in f64
        const int64_t k = k0 + LK * lg + kk;
        return (full || k < kend) ? static_cast<float>(static_cast<double>(v) - g.mu[k]) : v;
    };
    auto mu_tn = [&](int64_t k0, int kk, int e, float v, bool full) -> float {   // TN: A(k, c) - mu(c)
        return (full || k0 + LK * lg + kk < kend) ? static_cast<float>(static_cast<double>(v) - mu_c[e]) : v;
    };
    auto compute = [&](const uint32_t (&w)[AW], int64_t k0, int buf, bool full) {
        const XE* xb = xs + buf * T::STAGE;
        if constexpr (!T::BF) {
            // f32: operand of row block i, substep t
            float a[RB][SUB];
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int t = 0; t < SUB; ++t) {
                    if constexpr (MODE == MODE_NN) {
                        const float x = word_elem<TA>(w + i * (LK * sizeof(TA) / 4), t);
                        a[i][t] = MU ? mu_nn(k0, t, x, full) : x;
                    } else {
                        const float x = word_elem<TA>(w + t * T::TW, i);
                        a[i][t] = MU ? mu_tn(k0, t, i, x, full) : x;
                    }
                }
            constexpr int BV = LK / 4;
            auto read_b = [&](int j, v4f (&b)[BV]) {
                const float* src = xb + (16 * (cb0 + j) + lr) * SX + LK * lg;
#pragma unroll
                for (int v = 0; v < BV; ++v) b[v] = *reinterpret_cast<const v4f*>(src + 4 * v);
            };
            v4f bc[BV], bn[BV];
            read_b(0, bn);
#pragma unroll
            for (int j = 0; j < NCB; ++j) {
#pragma unroll
                for (int v = 0; v < BV; ++v) bc[v] = bn[v];
                if (j + 1 < NCB) read_b(j + 1, bn);
#pragma unroll
                for (int t = 0; t < SUB; ++t)
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][t], bc[t >> 2][t & 3], acc[i][j], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            // bf16: k-octet operands (hi, and lo for A_LO) of row block i, substep s
            s8bf ah[RB][SUB], al[T::A_LO ? RB : 1][T::A_LO ? SUB : 1];
            constexpr bool RAWNN = (MODE == MODE_NN) && sizeof(TA) == 2 && !CENT;
            constexpr bool RAWTN = (MODE == MODE_TN) && sizeof(TA) == 2 && !MU;
            if constexpr (RAWNN) {
                // bf16-stored A: the words are the operands (minus the means, if any,
                // rounded once to bf16)
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int s = 0; s < SUB; ++s) {
                        u32x4 q;
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            q[d] = w[i * (LK / 2) + 4 * s + d];
                            if constexpr (MU)
                                q[d] = pack_bf16(mu_nn(k0, 8 * s + 2 * d, __uint_as_float(q[d] << 16), full),
                                                 mu_nn(k0, 8 * s + 2 * d + 1, __uint_as_float(q[d] & 0xFFFF0000u), full));
                        }
                        ah[i][s] = __builtin_bit_cast(s8bf, q);
                    }
            } else if constexpr (RAWTN) {
                // bf16-stored A, TN: transpose the lane's 16 x RB block of 16-bit
                // words into k-octets (row pairs of one column per word)
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int s = 0; s < SUB; ++s) {
                        u32x4 q;
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            const uint32_t lo = w[(8 * s + 2 * d) * T::TW + (i >> 1)];
                            const uint32_t hi = w[(8 * s + 2 * d + 1) * T::TW + (i >> 1)];
                            q[d] = (i & 1) ? ((lo >> 16) | (hi & 0xFFFF0000u)) : ((lo & 0xFFFFu) | (hi << 16));
                        }
                        ah[i][s] = __builtin_bit_cast(s8bf, q);
                    }
            } else {
                // values x(i, s, u) (row block i, substep s, element u of the octet)
                // in f32, then rounded to bf16 hi (+ lo)
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int s = 0; s < SUB; ++s) {
                        u32x4 qh, ql;
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            float x[2];
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                const int kk = 8 * s + 2 * d + h;      // position in the lane's run
                                if constexpr (MODE == MODE_NN) {
                                    const float v = word_elem<TA>(w + i * (LK * sizeof(TA) / 4), kk);
                                    x[h] = MU ? mu_nn(k0, kk, v, full) : v;
                                } else {
                                    const float v = word_elem<TA>(w + kk * T::TW, i);
                                    x[h] = MU ? mu_tn(k0, kk, i, v, full) : v;
                                }
                            }
                            qh[d] = pack_bf16(x[0], x[1]);
                            if constexpr (T::A_LO)
                                ql[d] = pack_bf16(x[0] - bf16_round(x[0]), x[1] - bf16_round(x[1]));
                        }
                        ah[i][s] = __builtin_bit_cast(s8bf, qh);
                        if constexpr (T::A_LO) al[i][s] = __builtin_bit_cast(s8bf, ql);
                    }
            }
            auto read_b = [&](int j, s8bf (&bh)[SUB], s8bf (&bl)[SUB]) {
                const uint16_t* src = xb + (16 * (cb0 + j) + lr) * SX + LK * lg;
#pragma unroll
                for (int s = 0; s < SUB; ++s) {
                    bh[s] = *reinterpret_cast<const s8bf*>(src + 8 * s);
                    if constexpr (T::SPLIT) bl[s] = *reinterpret_cast<const s8bf*>(src + T::PLANE + 8 * s);
                }
            };
            s8bf bhc[SUB], blc[SUB], bhn[SUB], bln[SUB];
            read_b(0, bhn, bln);
#pragma unroll
            for (int j = 0; j < NCB; ++j) {
#pragma unroll
                for (int s = 0; s < SUB; ++s) { bhc[s] = bhn[s]; if constexpr (T::SPLIT) blc[s] = bln[s]; }
                if (j + 1 < NCB) read_b(j + 1, bhn, bln);
#pragma unroll
                for (int s = 0; s < SUB; ++s)
#pragma unroll
                    for (int i = 0; i < RB; ++i) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i][s], bhc[s], acc[i][j], 0, 0, 0);
                        if constexpr (T::SPLIT)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i][s], blc[s], acc[i][j], 0, 0, 0);
                        if constexpr (T::A_LO)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i][s], bhc[s], acc[i][j], 0, 0, 0);
                    }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };

    if (kbeg < kend) {
        // full chunks in the loop; a ragged last chunk is loaded with masks
        const int64_t nfull = (kend - kbeg) / KC;
        const bool tail = (kend - kbeg) % KC != 0;
        uint32_t wa[AW], wb[AW];
        load_a(kbeg, wa, nfull > 0);
        load_x(kbeg);
        store_x(0);
        __syncthreads();
        int buf = 0;
        for (int64_t c = 0; c < nfull; ++c) {
            const int64_t k0 = kbeg + c * KC;
            const bool more = c + 1 < nfull || tail;
            if (more) { load_a(k0 + KC, wb, c + 1 < nfull); load_x(k0 + KC); }
            compute(wa, k0, buf, true);
            if (more) store_x(buf ^ 1);
            __syncthreads();
#pragma unroll
            for (int d = 0; d < AW; ++d) wa[d] = wb[d];
            buf ^= 1;
        }
        if (tail) compute(wa, kbeg + nfull * KC, buf, false);
    }

    // ---- epilogue
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < NCB; ++j) {
            const int c = 16 * (cb0 + j) + lr;
            if (c >= g.ncols) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t r = (MODE == MODE_NN) ? w0 + 16 * i + 4 * lg + v : w0 + RB * (4 * lg + v) + i;
                if (r < g.rows) out[(r - row0) * ldo + c] = acc[i][j][v];
            }
        }
}

// Launch body.  Workgroup b < F -> (tile b % T, split b / T), split-major,
// so that the consecutive workgroups an XCD receives (one contiguous range
// each) work on the same chunks of X in step and share them in its L2.  F is
// all T S pairs, or with tail dealing (g.tail_groups = G > 0) the pairs of
// whole rounds of G workgroups; the L = T S - F pairs left over (a partly
// filled last round) are cut into pieces, pair p into f_p = floor(G / L) or
// one more (the first G mod L pairs) pieces of about equal chunk counts, and
// the G pieces go to G more workgroups, so that the last round ends on every
// CU at about the same time.  Tail workgroup w writes its piece to slot w
// (TROWS rows of ld_slot) and TailFixBody sums the f_p slots of each pair in
// order into the pair's output block (deterministic).  (Dealing all of the
// work in equal shares instead scatters an XCD's workgroups over X, whose
// chunks then miss in L2: 10-45 % slower at C2's and C3's shapes.)
__host__ __device__ inline void tail_piece(int64_t w, int64_t leftover, int groups, int64_t& pair, int64_t& piece,
                                           int64_t& pieces) {
    const int64_t q = groups / leftover, r = groups % leftover;
    if (w < r * (q + 1)) { pair = w / (q + 1); piece = w % (q + 1); pieces = q + 1; }
    else { pair = r + (w - r * (q + 1)) / q; piece = (w - r * (q + 1)) % q; pieces = q; }
}
__host__ __device__ inline int64_t tail_first(int64_t pair, int64_t leftover, int groups) {
    const int64_t q = groups / leftover, r = groups % leftover;
    return pair < r ? pair * (q + 1) : r * (q + 1) + (pair - r) * q;
}

template <typename TA, int MODE, int ARITH, int NCB, int WPS = 1, bool CENT = false, bool MU = false>
struct StreamBody {
    typedef StreamTile<TA, MODE, ARITH, NCB, WPS, CENT, MU> T;
    typedef GemmArgs<TA, float, float> Args;
    static constexpr int THREADS = T::NT;
    static constexpr int WAVES_PER_SIMD = WPS == 3 ? 2 : 1;   // register budget of the launch
    static constexpr int TROWS = T::TROWS, KC = T::KC;
    __host__ __device__ static int tiles(const Args& g) { return static_cast<int>(cdiv(g.rows, T::TROWS)); }
    __host__ __device__ static int64_t pairs(const Args& g) { return static_cast<int64_t>(tiles(g)) * g.splits; }
    __host__ __device__ static int64_t whole(const Args& g) {
        return g.tail_groups > 0 ? (pairs(g) / g.tail_groups) * g.tail_groups : pairs(g);
    }
    static int blocks(const Args& g) {
        return static_cast<int>(whole(g) + (pairs(g) > whole(g) ? g.tail_groups : 0));
    }
    static size_t lds(const Args&) { return T::LDS_BYTES; }
    static __device__ __forceinline__ void run(const Args& g, int b) {
        const int nt = tiles(g);
        const int64_t F = whole(g);
        if (g.tail_groups > 0) {
            // the launch order decides the rounds: hardware block h < F runs
            // in the whole rounds (h % 8 is its XCD, which keeps one contiguous
            // range of pairs), h >= F in the last one (the logical order of
            // xcd_block would give some XCDs only whole pairs and the others
            // only tail pieces)
            const int64_t h = blockIdx.x;
            b = static_cast<int>((h < F && F % kXcds == 0) ? (h % kXcds) * (F / kXcds) + h / kXcds : h);
        }
        int64_t pair = b, kbeg, kend, row0 = 0, ldo = g.ldo;
        float* out;
        if (b < F) {
            kbeg = (pair / nt) * g.kchunk;
            kend = min(g.K, kbeg + g.kchunk);
            out = g.out + (pair / nt) * g.part_stride;
        } else {
            int64_t pl, piece, pieces;
            tail_piece(b - F, pairs(g) - F, g.tail_groups, pl, piece, pieces);
            pair = F + pl;
            const int64_t nch = cdiv(g.kchunk, T::KC);
            const int64_t ks = (pair / nt) * g.kchunk, ke = min(g.K, ks + g.kchunk);
            kbeg = min(ke, ks + (piece * nch / pieces) * T::KC);
            kend = min(ke, ks + ((piece + 1) * nch / pieces) * T::KC);
            out = g.tail_slots + (b - F) * T::TROWS * g.ld_slot;
            row0 = (pair % nt) * T::TROWS;
            ldo = g.ld_slot;
        }
        gemm_stream_body<TA, MODE, ARITH, NCB, WPS, CENT, MU>(g, static_cast<int>(pair % nt), kbeg, kend, out, row0,
                                                             ldo);
    }
};

// Sum of the tail slots: for each leftover pair p (tile t, split s) and each
// of its rows and columns, the slots of its pieces in order, into the pair's
// output block (out + s part_stride).
struct TailFixArgs {
    const float* slots; int64_t ld_slot; int64_t rows; int ncols; int tiles; int trows; int64_t first_pair;
    int64_t leftover; int groups; float* out; int64_t ldo; int64_t part_stride;
    const uint32_t* skip_flag; uint32_t skip_mask; Gate gate;
};
struct TailFixBody {
    typedef TailFixArgs Args;
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) {
        return static_cast<int>(cdiv(a.leftover * a.trows * cdiv(a.ncols, 4), THREADS));
    }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        if (a.skip_flag && ((*a.skip_flag & a.skip_mask) == 0u)) return;
        if (a.gate.w && ((*a.gate.w & a.gate.mask) == 0u)) return;
        const int cg = static_cast<int>(cdiv(a.ncols, 4));
        const int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (idx >= a.leftover * a.trows * cg) return;
        const int64_t pl = idx / (static_cast<int64_t>(a.trows) * cg);
        const int rr = static_cast<int>((idx / cg) % a.trows);
        const int c = 4 * static_cast<int>(idx % cg);
        const int64_t pair = a.first_pair + pl, t = pair % a.tiles, s = pair / a.tiles;
        const int64_t r = t * a.trows + rr;
        if (r >= a.rows) return;
        const int64_t w0 = tail_first(pl, a.leftover, a.groups), w1 = tail_first(pl + 1, a.leftover, a.groups);
        // one 16-byte load per slot (ld_slot is a multiple of 4 and the slots
        // start 256-byte aligned), four slots in flight, summed in slot order
        const int64_t step = static_cast<int64_t>(a.trows) * a.ld_slot;
        const float4* p = reinterpret_cast<const float4*>(a.slots + (w0 * a.trows + rr) * a.ld_slot + c);
        const int64_t st = step / 4;
        float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        int64_t w = w0;
        for (; w + 4 <= w1; w += 4, p += 4 * st) {
            const float4 v0 = p[0], v1 = p[st], v2 = p[2 * st], v3 = p[3 * st];
            acc.x += v0.x; acc.y += v0.y; acc.z += v0.z; acc.w += v0.w;
            acc.x += v1.x; acc.y += v1.y; acc.z += v1.z; acc.w += v1.w;
            acc.x += v2.x; acc.y += v2.y; acc.z += v2.z; acc.w += v2.w;
            acc.x += v3.x; acc.y += v3.y; acc.z += v3.z; acc.w += v3.w;
        }
        for (; w < w1; ++w, p += st) {
            const float4 v = p[0];
            acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
        }
        const float av[4] = {acc.x, acc.y, acc.z, acc.w};
        float* o = a.out + s * a.part_stride + r * a.ldo + c;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (c + e < a.ncols) o[e] = av[e];
    }
};

}  // namespace rsvd
