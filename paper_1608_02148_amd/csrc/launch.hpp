// Step helpers: argument records and tile-shape choice for every product of
// the solve, issued through an executor (SingleExec or BatchRecorder).
#pragma once

#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "common.hpp"
#include "exec.hpp"
#include "gemm.hpp"
#include "gemm_bf16.hpp"
#include "gemm_stream.hpp"
#include "linalg.hpp"
#include "plan.hpp"

namespace rsvd {

template <typename T> constexpr int gemm_bk() { return sizeof(T) == 8 ? 16 : 32; }


// Storage-precision product (f32 / f64 matrix cores).  Workgroup b of a
// problem covers column tile b % C, row tile (b / C) % gx, split b / (C gx).
template <typename TA, typename TX, typename TC, int MODE, int WR, int WC, int WGM, int WGN, bool XKP = false>
struct GemmBody {
    static constexpr int BK = gemm_bk<TC>();
    typedef GemmTile<TA, TX, TC, MODE, WR, WC, WGM, WGN, BK> T;
    typedef GemmArgs<TA, TX, TC> Args;
    static constexpr int THREADS = T::NT;
    static int blocks(const Args& g) {
        return static_cast<int>(cdiv(g.rows, T::BM) * g.splits * cdiv(g.ncols, T::NC));
    }
    static size_t lds(const Args&) { return T::LDS_BYTES; }
    static __device__ void run(const Args& g, int b) {
        // column tiles vary fastest: the tiles that read the same rows of A
        // run side by side (same XCD, same L2) when there are several
        const int gx = static_cast<int>(cdiv(g.rows, T::BM));
        const int nct = static_cast<int>(cdiv(g.ncols, T::NC));
        const int rest = b / nct;
        if (g.upper_only && rest % gx > b % nct) return;     // a tile below the diagonal of a symmetric product
        gemm_tile_body<TA, TX, TC, MODE, WR, WC, WGM, WGN, BK, XKP>(g, rest % gx, rest / gx, b % nct);
    }
};

// bf16 matrix-core product (f32 in / out), plain or split; CENT: split
// product of bf16-stored A with the column means subtracted.
template <typename TA, int MODE, bool SPLIT, int WR, int WC, int WGM, int WGN, bool CENT = false>
struct Bf16Body {
    static constexpr int BK = SPLIT ? 32 : 64;
    typedef Bf16Tile<TA, MODE, SPLIT, WR, WC, WGM, WGN, BK, CENT> T;
    typedef GemmArgs<TA, float, float> Args;
    static constexpr int THREADS = T::NT;
    static int blocks(const Args& g) {
        return static_cast<int>(cdiv(g.rows, T::BM) * g.splits * cdiv(g.ncols, T::NC));
    }
    static size_t lds(const Args&) { return T::LDS_BYTES; }
    static __device__ void run(const Args& g, int b) {
        const int gx = static_cast<int>(cdiv(g.rows, T::BM));
        const int nct = static_cast<int>(cdiv(g.ncols, T::NC));
        const int rest = b / nct;
        gemm_bf16_body<TA, MODE, SPLIT, WR, WC, WGM, WGN, BK, CENT>(g, rest % gx, rest / gx, b % nct);
    }
};

// Argument record of one product: out = A X (NN) or A^T X (TN) over the
// reduction length K; S > 1 writes S partial blocks of stride part_stride.
template <typename TA, typename TX, typename TC>
GemmArgs<TA, TX, TC> gemm_args(const TA* A, int64_t lda, int64_t rows, int64_t K, const TX* X, int64_t ldx,
                               int ncols, TC* out, int64_t ldo, int S, int64_t part_stride, const double* mu,
                               const uint32_t* skip_flag, uint32_t skip_mask, int kchunk_multiple,
                               size_t vec_bytes, Gate gate = {}) {
    GemmArgs<TA, TX, TC> g;
    g.A = A; g.lda = lda; g.rows = rows; g.K = K;
    S = S < 1 ? 1 : S;
    g.kchunk = rup(cdiv(K, S), kchunk_multiple);   // splits past the end of K write zero partials
    g.splits = S;
    g.upper_only = 0;
    g.tail_groups = 0; g.tail_slots = nullptr; g.ld_slot = 0;
    g.X = X; g.ldx = ldx; g.ncols = ncols; g.out = out; g.ldo = ldo;
    g.part_stride = part_stride; g.mu = mu; g.skip_flag = skip_flag; g.skip_mask = skip_mask;
    g.gate = gate.w; g.gate_mask = gate.mask;
    g.a_vec = (reinterpret_cast<uintptr_t>(A) % vec_bytes == 0) && ((lda * sizeof(TA)) % vec_bytes == 0);
    g.x_vec = 0;
    g.xb = nullptr; g.ldxb = 0; g.xb_plane = 0;
    g.xk = nullptr; g.ldxk = 0;
    return g;
}

// Output tile shapes.  Tall tiles (128 output rows per workgroup) for
// products with many output rows, NC = cls columns: 32, 64, 128 for every
// compute type plus 48, 80, 96 for f32 compute (finer classes waste fewer
// matrix-core columns when l is just above a power of two).  Square tiles
// (BM = NC = 32, 64 or 128) for products with at most that many output rows:
// Gram matrices and the l x l factors.  cls = 0 picks the tall class from
// ncols; a grouped batch step passes one class for all of its problems.
// Tall f32 tiles come in up to three variants per column class: 0 = 4 waves,
// 1 = 8 waves, 2 = 16 waves over the same 128 x NC output tile (more waves
// hide more latency, fewer keep more operands per wave); `cls` carries the
// variant in its upper 16 bits (the plan's autotuned choice).
template <typename TA, typename TX, typename TC, int MODE, bool XKP, class Ex>
hipError_t gemm_tall_f32(Ex& ex, int tc, int var, const GemmArgs<TA, TX, TC>& g) {
    switch (tc) {
        case 32:
            if (var == 1) return ex.template run<GemmBody<TA, TX, TC, MODE, 2, 1, 4, 2, XKP>>(g);
            if (var == 2) return ex.template run<GemmBody<TA, TX, TC, MODE, 1, 1, 8, 2, XKP>>(g);
            return ex.template run<GemmBody<TA, TX, TC, MODE, 2, 2, 4, 1, XKP>>(g);
        case 48:
            if (var != 0) return ex.template run<GemmBody<TA, TX, TC, MODE, 1, 3, 8, 1, XKP>>(g);
            return ex.template run<GemmBody<TA, TX, TC, MODE, 2, 3, 4, 1, XKP>>(g);
        case 64:
            if (var == 1) return ex.template run<GemmBody<TA, TX, TC, MODE, 4, 1, 2, 4, XKP>>(g);
            if (var == 2) return ex.template run<GemmBody<TA, TX, TC, MODE, 2, 1, 4, 4, XKP>>(g);
            return ex.template run<GemmBody<TA, TX, TC, MODE, 4, 2, 2, 2, XKP>>(g);
        case 80:
            if (var != 0) return ex.template run<GemmBody<TA, TX, TC, MODE, 1, 5, 8, 1, XKP>>(g);
            return ex.template run<GemmBody<TA, TX, TC, MODE, 2, 5, 4, 1, XKP>>(g);
        case 96:
            if (var == 1) return ex.template run<GemmBody<TA, TX, TC, MODE, 2, 3, 4, 2, XKP>>(g);
            if (var == 2) return ex.template run<GemmBody<TA, TX, TC, MODE, 1, 3, 8, 2, XKP>>(g);
            return ex.template run<GemmBody<TA, TX, TC, MODE, 4, 3, 2, 2, XKP>>(g);
        default:
            if (var == 1) return ex.template run<GemmBody<TA, TX, TC, MODE, 4, 2, 2, 4, XKP>>(g);
            if (var == 2) return ex.template run<GemmBody<TA, TX, TC, MODE, 2, 2, 4, 4, XKP>>(g);
            return ex.template run<GemmBody<TA, TX, TC, MODE, 4, 4, 2, 2, XKP>>(g);
    }
}

// Tall product tiles: the f32 column classes and variants, or the f64 ones.
template <typename TA, typename TX, typename TC, int MODE, bool XKP, class Ex>
hipError_t gemm_tall(Ex& ex, int tc, int var, const GemmArgs<TA, TX, TC>& g) {
    if constexpr (sizeof(TC) == 4) return gemm_tall_f32<TA, TX, TC, MODE, XKP>(ex, tc, var, g);
    if (tc == 32) return ex.template run<GemmBody<TA, TX, TC, MODE, 2, 2, 4, 1, XKP>>(g);
    if (tc == 64) return ex.template run<GemmBody<TA, TX, TC, MODE, 4, 2, 2, 2, XKP>>(g);
    return ex.template run<GemmBody<TA, TX, TC, MODE, 4, 4, 2, 2, XKP>>(g);
}

// X (K x ncols, ldx) -> XK[c][k] (ld ldk, k-contiguous) in the compute type,
// so that a product tile reads each k-vector of a column of X with one vector
// load.  One thread per (column, k-vector), consecutive threads on
// consecutive columns (coalesced reads of X).
template <typename TC>
struct XKPackBody {
    struct Args {
        const TC* X; int64_t ldx; int64_t K; int ncols; TC* XK; int64_t ldk;
        const uint32_t* skip_flag; uint32_t skip_mask; Gate gate;
    };
    static constexpr int THREADS = 256;
    static constexpr int KV = 16 / sizeof(TC);
    static int blocks(const Args& a) { return static_cast<int>(cdiv(static_cast<int64_t>(a.ncols) * cdiv(a.K, KV), THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        if (a.skip_flag && ((*a.skip_flag & a.skip_mask) == 0u)) return;
        if (a.gate.w && ((*a.gate.w & a.gate.mask) == 0u)) return;
        const int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        const int c = static_cast<int>(idx % a.ncols);
        const int64_t k0 = KV * (idx / a.ncols);
        if (k0 >= a.K) return;
        typedef TC vec_t __attribute__((ext_vector_type(KV)));
        vec_t v;
#pragma unroll
        for (int e = 0; e < KV; ++e) v[e] = (k0 + e < a.K) ? a.X[(k0 + e) * a.ldx + c] : TC(0);
        *reinterpret_cast<vec_t*>(a.XK + static_cast<int64_t>(c) * a.ldk + k0) = v;
    }
};

template <typename TA, typename TX, typename TC, int MODE, class Ex>
hipError_t gemm_plain(Ex& ex, int cls, bool square, const TA* A, int64_t lda, int64_t rows, int64_t K,
                      const TX* X, int64_t ldx, int ncols, TC* out, int64_t ldo, int S, int64_t part_stride,
                      const double* mu, const uint32_t* skip_flag, uint32_t skip_mask, Gate gate = {},
                      TC* xk = nullptr, int64_t ldxk = 0, bool upper_only = false) {
    const size_t vb = (16 / sizeof(TC)) * sizeof(TA);    // 16 / sizeof(TC) consecutive elements of A
    auto g = gemm_args<TA, TX, TC>(A, lda, rows, K, X, ldx, ncols, out, ldo, S, part_stride, mu, skip_flag,
                                   skip_mask, gemm_bk<TC>(), vb, gate);
    g.upper_only = (square && upper_only) ? 1 : 0;
    if constexpr (std::is_same<TX, TC>::value) {
        // optional k-contiguous copy of X (scratch xk, ld ldxk >= K, a multiple
        // of 16 / sizeof(TC)): one vector load per k-vector in the tiles
        if (xk && !square) {
            if (ldxk < K || ldxk % (16 / sizeof(TC)) != 0) return hipErrorInvalidValue;
            const hipError_t e = ex.template run<XKPackBody<TC>>(typename XKPackBody<TC>::Args{
                X, ldx, K, ncols, xk, ldxk, skip_flag, skip_mask, gate});
            if (e != hipSuccess) return e;
            g.xk = xk;
            g.ldxk = ldxk;
        }
    }
    if (square) {
        // square tiles: the smallest that holds max(rows, ncols), so little
        // of the f64 matrix cores' work is padding -- 32, 48, 64, 80, 96 or
        // 128 for the Gram of an f32 basis, 32 / 64 / 128 otherwise (the same
        // coarser classes the f64 solves and their batch groups use)
        const int extent = static_cast<int>(std::max<int64_t>(rows, ncols));
        int sc = tile_class(extent, sizeof(TA) == 4);
        // a single solve's small f64 products (R factors, Schur blocks, J_k:
        // reduction <= 256) spread over 32 x 32 tiles, one workgroup each,
        // instead of leaving one CU to do all of a 128 x 128 tile
        if constexpr (Ex::kSingle)
            if (sizeof(TA) == 8 && K <= 256) sc = 32;
        if (sc == 32) return ex.template run<GemmBody<TA, TX, TC, MODE, 1, 1, 2, 2>>(g);
        if (sc == 48) return ex.template run<GemmBody<TA, TX, TC, MODE, 1, 3, 3, 1>>(g);
        if (sc == 64) return ex.template run<GemmBody<TA, TX, TC, MODE, 2, 2, 2, 2>>(g);
        if (sc == 80) return ex.template run<GemmBody<TA, TX, TC, MODE, 1, 5, 5, 1>>(g);
        if (sc == 96) return ex.template run<GemmBody<TA, TX, TC, MODE, 2, 3, 3, 2>>(g);
        // 128: 16 waves (4 per SIMD hide the load-convert-stage latency that
        // one wave per SIMD left exposed; the 100000 x 120 Gram 119 -> 72 us)
        return ex.template run<GemmBody<TA, TX, TC, MODE, 2, 2, 4, 4>>(g);
    }
    const int tc = (cls & 0xFFFF) ? (cls & 0xFFFF) : tile_cols(ncols);
    if (g.xk) return gemm_tall<TA, TX, TC, MODE, true>(ex, tc, cls >> 16, g);
    return gemm_tall<TA, TX, TC, MODE, false>(ex, tc, cls >> 16, g);
}

template <typename TA, int MODE, bool SPLIT, bool CENT, class Ex>
hipError_t gemm_bf16_cls(Ex& ex, int tc, const GemmArgs<TA, float, float>& g) {
    if (tc == 32) return ex.template run<Bf16Body<TA, MODE, SPLIT, 2, 2, 4, 1, CENT>>(g);
    if (tc == 48) return ex.template run<Bf16Body<TA, MODE, SPLIT, 2, 3, 4, 1, CENT>>(g);
    if (tc == 64) return ex.template run<Bf16Body<TA, MODE, SPLIT, 4, 2, 2, 2, CENT>>(g);
    if (tc == 80) return ex.template run<Bf16Body<TA, MODE, SPLIT, 2, 5, 4, 1, CENT>>(g);
    if (tc == 96) return ex.template run<Bf16Body<TA, MODE, SPLIT, 4, 3, 2, 2, CENT>>(g);
    // 256 columns (sketches wider than 128): 16 waves of 32 x 64 (the 8-wave
    // 64 x 64 tiling was 5-7 % slower for A X at 200000 x 20000, l = 220, and
    // 16 waves of 64 x 64 over 256 rows, which halve the re-reads of the
    // packed X, took 1.3x (A X) and 1.8x (A^T Q) as long: one workgroup per
    // CU with its double-buffered 144-160 KB of LDS)
    if (tc == 256) return ex.template run<Bf16Body<TA, MODE, SPLIT, 2, 4, 4, 4, CENT>>(g);
    return ex.template run<Bf16Body<TA, MODE, SPLIT, 4, 4, 2, 2, CENT>>(g);
}

// The bf16 products read X packed once per product into bf16 planes (hi, and
// lo for the split arithmetic) laid out [column][k], so that no workgroup
// converts or transposes X itself: xp gives the scratch, ld >= K rounded up
// to 8, plane >= (column tiles x NC) x ld elements.
template <typename TA, int MODE, class Ex>
hipError_t gemm_bf16(Ex& ex, bool split, int cls, const TA* A, int64_t lda, int64_t rows, int64_t K,
                     const float* X, int64_t ldx, int ncols, float* out, int64_t ldo, int S, int64_t part_stride,
                     const double* mu, const uint32_t* skip_flag, uint32_t skip_mask, Gate gate, XPack xp) {
    auto g = gemm_args<TA, float, float>(A, lda, rows, K, X, ldx, ncols, out, ldo, S, part_stride, mu,
                                         skip_flag, skip_mask, 64, 16, gate);
    int tc = (cls & 0xFFFF) ? (cls & 0xFFFF) : tile_cols(ncols);
    if (ncols > 128) tc = 256;      // one 256-column tile: each A tile is staged once
    const int cols = static_cast<int>(cdiv(ncols, tc) * tc);
    if (!xp.p || xp.ld < rup(K, 8) || xp.ld % 8 != 0 || xp.plane < static_cast<int64_t>(cols) * xp.ld)
        return hipErrorInvalidValue;
    const hipError_t e = ex.template run<XPackBody>(XPackArgs{X, ldx, K, ncols, cols, xp.p, xp.ld, xp.plane,
                                                              split ? 1 : 0, skip_flag, skip_mask, gate});
    if (e != hipSuccess) return e;
    g.xb = xp.p; g.ldxb = xp.ld; g.xb_plane = xp.plane;
    if (split) {
        // bf16-stored A minus its column means is not exact in bf16: the
        // split product then stages it as hi + lo terms (f32-accurate)
        if constexpr (sizeof(TA) == 2)
            if (mu) return gemm_bf16_cls<TA, MODE, true, true>(ex, tc, g);
        return gemm_bf16_cls<TA, MODE, true, false>(ex, tc, g);
    }
    return gemm_bf16_cls<TA, MODE, false, false>(ex, tc, g);
}

// Streamed-A products (gemm_stream.hpp) for the large products of a single
// solve.  RSVD_PRODUCTS=staged in the environment keeps every product on the
// LDS-staged tiles (for comparisons).
inline bool streamed_products_enabled() {
    static const bool on = [] {
        const char* s = std::getenv("RSVD_PRODUCTS");
        return !(s && std::strcmp(s, "staged") == 0);
    }();
    return on;
}

// Column classes of the streamed-A kernel: 128 (65..128 columns) and 224
// (129..224).  Narrower products stay on the LDS-staged tiles (too little
// matrix-core work per loaded byte of A to hide the memory latency at one
// wave per SIMD), and so do the variants whose registers do not fit one wave
// (accumulators, two chunks of A and the staged X over 512 registers: they
// would spill).
inline int stream_cols(int ncols) { return ncols <= 128 ? 128 : 224; }

// Variants that fit their registers without spilling (a compile-time record
// of the register counts): one wave per SIMD (WPS = 1, 512 registers a wave)
// for every product, two per SIMD (WPS = 2, 256 registers a wave) for the
// products without column means.
template <typename TA, int MODE, int ARITH, int NCB, int WPS, bool CENT, bool MU>
constexpr bool stream_fits() {
    // two workgroups of 128 rows per CU: measured faster only for A X of
    // bf16-stored A at 224 columns (C3 bf16 2.69 -> 2.57 ms, f32 arithmetic
    // 13.66 -> 13.50 ms; C2 f32 A X 1.34 -> 1.39 ms, A^T Q slower as well, the
    // split arithmetic spills)
    if (WPS == 3) return !MU && !CENT && MODE == MODE_NN && NCB == 14 && sizeof(TA) == 2 && ARITH != 2;
    if (WPS == 2) {
        if (MU || CENT) return false;
        if (MODE == MODE_NN) return true;
        // A^T Q (a lane loads half as many columns per row of A): faster at
        // two waves only with f32 arithmetic on bf16-stored A (C3 13.9 -> 13.5
        // ms; f32 A at C2 1.36 -> 1.39 ms, bf16 arithmetic unchanged, the split
        // one spills at 224 columns)
        return sizeof(TA) == 2 && ARITH == 0;
    }
    if (NCB == 8) return !(MODE == MODE_TN && ARITH == 2 && sizeof(TA) == 4 && MU);
    return !MU && !CENT && (ARITH == 0 || sizeof(TA) == 2);
}

// Layout limit of the streamed kernels: RSVD_STREAM_WPS=1 keeps one wave per
// SIMD, =2 allows the eight-wave layout but not the 128-row one, otherwise
// every layout that fits (A X at C2 1.43 -> 1.35 ms, C3 bf16 2.82 -> 2.57 ms
// against one wave per SIMD).
inline int stream_wps() {
    static const int w = [] {
        const char* v = std::getenv("RSVD_STREAM_WPS");
        if (v && std::strcmp(v, "1") == 0) return 1;
        if (v && std::strcmp(v, "2") == 0) return 2;
        return 3;
    }();
    return w;
}

// The layout stream_ncb launches for these arguments.
template <typename TA, int MODE, int ARITH, bool CENT, bool MU>
int stream_lay(int ncols) {
    const int w = stream_wps();
    const bool wide = ncols > 128;
    if (w >= 3 && (wide ? stream_fits<TA, MODE, ARITH, 14, 3, CENT, MU>() : stream_fits<TA, MODE, ARITH, 8, 3, CENT, MU>()))
        return 3;
    if (w >= 2 && (wide ? stream_fits<TA, MODE, ARITH, 14, 2, CENT, MU>() : stream_fits<TA, MODE, ARITH, 8, 2, CENT, MU>()))
        return 2;
    return 1;
}

// Chunk of the reduction of the streamed kernel that stream_ncb launches.
inline int stream_kc(int arith, int ncols) { return (arith != 0 || ncols <= 128) ? 64 : 32; }
static_assert(StreamTile<float, MODE_NN, 0, 8>::KC == 64 && StreamTile<float, MODE_NN, 0, 14>::KC == 32 &&
              StreamTile<float, MODE_NN, 1, 14>::KC == 64, "stream_kc");

template <typename TA, int MODE, int ARITH, bool CENT, bool MU, class Ex>
hipError_t stream_ncb(Ex& ex, const GemmArgs<TA, float, float>& g) {
    const int lay = stream_lay<TA, MODE, ARITH, CENT, MU>(g.ncols);
    if (g.ncols <= 128) {
        if constexpr (stream_fits<TA, MODE, ARITH, 8, 3, CENT, MU>())
            if (lay == 3) return ex.template run<StreamBody<TA, MODE, ARITH, 8, 3, CENT, MU>>(g);
        if constexpr (stream_fits<TA, MODE, ARITH, 8, 2, CENT, MU>())
            if (lay == 2) return ex.template run<StreamBody<TA, MODE, ARITH, 8, 2, CENT, MU>>(g);
        if constexpr (stream_fits<TA, MODE, ARITH, 8, 1, CENT, MU>())
            return ex.template run<StreamBody<TA, MODE, ARITH, 8, 1, CENT, MU>>(g);
    } else {
        if constexpr (stream_fits<TA, MODE, ARITH, 14, 3, CENT, MU>())
            if (lay == 3) return ex.template run<StreamBody<TA, MODE, ARITH, 14, 3, CENT, MU>>(g);
        if constexpr (stream_fits<TA, MODE, ARITH, 14, 2, CENT, MU>())
            if (lay == 2) return ex.template run<StreamBody<TA, MODE, ARITH, 14, 2, CENT, MU>>(g);
        if constexpr (stream_fits<TA, MODE, ARITH, 14, 1, CENT, MU>())
            return ex.template run<StreamBody<TA, MODE, ARITH, 14, 1, CENT, MU>>(g);
    }
    return hipErrorNotSupported;
}

// Rows per tile of the kernel stream_ncb launches (the 128-row layout runs two
// workgroups per CU, so a round holds twice as many).
template <typename TA, int MODE>
int stream_trows(int arith, int ncols, bool mu) {
    constexpr bool cent = sizeof(TA) == 2;
    int lay = 1;
    if (arith == 0) lay = mu ? stream_lay<TA, MODE, 0, false, true>(ncols) : stream_lay<TA, MODE, 0, false, false>(ncols);
    else if (arith == 1) lay = mu ? stream_lay<TA, MODE, 1, false, true>(ncols) : stream_lay<TA, MODE, 1, false, false>(ncols);
    else lay = mu ? stream_lay<TA, MODE, 2, cent, true>(ncols) : stream_lay<TA, MODE, 2, false, false>(ncols);
    return lay == 3 ? 128 : 256;
}

// Whether stream_ncb would launch (checked before X is packed).
template <typename TA, int MODE>
bool stream_variant(int arith, int ncols, bool mu) {
    const bool wide = ncols > 128;
    auto fits = [&](bool ncb8, bool ncb14) { return wide ? ncb14 : ncb8; };
    if (arith == 0)
        return mu ? fits(stream_fits<TA, MODE, 0, 8, 1, false, true>(), stream_fits<TA, MODE, 0, 14, 1, false, true>())
                  : fits(stream_fits<TA, MODE, 0, 8, 1, false, false>(), stream_fits<TA, MODE, 0, 14, 1, false, false>());
    if (arith == 1)
        return mu ? fits(stream_fits<TA, MODE, 1, 8, 1, false, true>(), stream_fits<TA, MODE, 1, 14, 1, false, true>())
                  : fits(stream_fits<TA, MODE, 1, 8, 1, false, false>(), stream_fits<TA, MODE, 1, 14, 1, false, false>());
    constexpr bool cent = sizeof(TA) == 2;
    return mu ? fits(stream_fits<TA, MODE, 2, 8, 1, cent, true>(), stream_fits<TA, MODE, 2, 14, 1, cent, true>())
              : fits(stream_fits<TA, MODE, 2, 8, 1, false, false>(), stream_fits<TA, MODE, 2, 14, 1, false, false>());
}

// Scratch for the tail dealing of the streamed products (see StreamBody):
// slots for groups x 256 rows x ncols f32, and the workgroups of a round (one
// per CU).
struct StreamTail { float* p = nullptr; size_t bytes = 0; int groups = 0; };

// Returns hipErrorNotSupported (nothing launched) when the product does not
// qualify: a batch, a small or misaligned A, or no packing scratch for X.
// With tail scratch, the (tile, split) pairs of a last round that would fill
// at most half of the CUs are cut into pieces for a whole round of workgroups
// and summed into their output blocks by TailFixBody.
template <typename TA, int MODE, class Ex>
hipError_t gemm_streamed(Ex& ex, int arith, const TA* A, int64_t lda, int64_t rows, int64_t K, const float* X,
                         int64_t ldx, int ncols, float* out, int64_t ldo, int S, int64_t part_stride,
                         const double* mu, const uint32_t* skip_flag, uint32_t skip_mask, Gate gate, XPack xp,
                         float* xk, int64_t ldxk, StreamTail tail = {}) {
    if constexpr (!Ex::kSingle) {
        return hipErrorNotSupported;       // batches: many small products
    } else {
        if (!streamed_products_enabled() || !streamed_size(rows, K) || ncols <= 64 || ncols > 224)
            return hipErrorNotSupported;
        if (!stream_variant<TA, MODE>(arith, ncols, mu != nullptr)) return hipErrorNotSupported;
        // 16-byte aligned rows of A; TN reads A in groups of 4 columns (rows % 4 == 0)
        if (reinterpret_cast<uintptr_t>(A) % 16 != 0 || (lda * static_cast<int64_t>(sizeof(TA))) % 16 != 0)
            return hipErrorNotSupported;
        if (MODE == MODE_TN && rows % 4 != 0) return hipErrorNotSupported;
        const int nc = stream_cols(ncols);
        if (arith == 0) {
            if (!xk || ldxk < rup(K, 4) || ldxk % 4 != 0 || reinterpret_cast<uintptr_t>(xk) % 16 != 0)
                return hipErrorNotSupported;
        } else if (!xp.p || xp.ld < rup(K, 8) || xp.ld % 8 != 0 || xp.plane < static_cast<int64_t>(nc) * xp.ld) {
            return hipErrorNotSupported;
        }
        auto g = gemm_args<TA, float, float>(A, lda, rows, K, X, ldx, ncols, out, ldo, S, part_stride, mu, skip_flag,
                                             skip_mask, 64, 16, gate);
        hipError_t e;
        if (arith == 0) {
            e = ex.template run<XKPackBody<float>>(typename XKPackBody<float>::Args{
                X, ldx, K, ncols, xk, ldxk, skip_flag, skip_mask, gate});
            g.xk = xk;
            g.ldxk = ldxk;
        } else {
            e = ex.template run<XPackBody>(XPackArgs{X, ldx, K, ncols, nc, xp.p, xp.ld, xp.plane, arith == 2 ? 1 : 0,
                                                     skip_flag, skip_mask, gate});
            g.xb = xp.p; g.ldxb = xp.ld; g.xb_plane = xp.plane;
        }
        if (e != hipSuccess) return e;
        // tail dealing: when the pairs left over by whole rounds fill at most
        // half of a round (each then splits into two or more pieces)
        const int trows = stream_trows<TA, MODE>(arith, ncols, mu != nullptr);
        const int groups = tail.groups * (256 / trows);       // workgroups of one round
        const int64_t tiles = cdiv(rows, trows), pairs = tiles * g.splits;
        const int64_t ld_slot = rup(ncols, 4), leftover = groups > 0 ? pairs % groups : 0;
        bool dealt = false;
        if (tail.p && leftover > 0 && 2 * leftover <= groups &&
            tail.bytes >= static_cast<size_t>(groups) * trows * ld_slot * sizeof(float)) {
            g.tail_groups = groups;
            g.tail_slots = tail.p;
            g.ld_slot = ld_slot;
            dealt = true;
        }
        if (mu) {
            if (arith == 0) e = stream_ncb<TA, MODE, 0, false, true>(ex, g);
            else if (arith == 1) e = stream_ncb<TA, MODE, 1, false, true>(ex, g);
            else e = stream_ncb<TA, MODE, 2, sizeof(TA) == 2, true>(ex, g);
        } else {
            if (arith == 0) e = stream_ncb<TA, MODE, 0, false, false>(ex, g);
            else if (arith == 1) e = stream_ncb<TA, MODE, 1, false, false>(ex, g);
            else e = stream_ncb<TA, MODE, 2, false, false>(ex, g);
        }
        if (e != hipSuccess || !dealt) return e;
        return ex.template run<TailFixBody>(TailFixArgs{tail.p, ld_slot, rows, ncols, static_cast<int>(tiles), trows,
                                                        pairs - leftover, leftover, groups, out, ldo, part_stride,
                                                        skip_flag, skip_mask, gate});
    }
}

// One product with A in the requested arithmetic: 0 = storage precision
// (f32 / f64 matrix cores), 1 = bf16, 2 = split bf16 (near-f32-accurate).
// xk / ldxk (optional): scratch for the k-contiguous copy of X that the
// storage-precision tiles read (ncols x ldxk elements of TC).
template <typename TA, typename TC, int MODE, class Ex>
hipError_t gemm_step(Ex& ex, int arith, int cls, const TA* A, int64_t lda, int64_t rows, int64_t K,
                     const TC* X, int64_t ldx, int ncols, TC* out, int64_t ldo, int S, int64_t part_stride,
                     const double* mu, const uint32_t* skip_flag, uint32_t skip_mask, Gate gate = {},
                     XPack xp = {}, TC* xk = nullptr, int64_t ldxk = 0, StreamTail tail = {}) {
    if constexpr (std::is_same<TC, float>::value) {
        const hipError_t e = gemm_streamed<TA, MODE>(ex, arith, A, lda, rows, K, X, ldx, ncols, out, ldo, S,
                                                     part_stride, mu, skip_flag, skip_mask, gate, xp, xk, ldxk, tail);
        if (e != hipErrorNotSupported) return e;
        if (arith != 0)
            return gemm_bf16<TA, MODE>(ex, arith == 2, cls, A, lda, rows, K, X, ldx, ncols, out, ldo, S,
                                       part_stride, mu, skip_flag, skip_mask, gate, xp);
    }
    return gemm_plain<TA, TC, TC, MODE>(ex, cls, false, A, lda, rows, K, X, ldx, ncols, out, ldo, S, part_stride,
                                        mu, skip_flag, skip_mask, gate, xk, ldxk);
}

template <typename T, class Ex>
hipError_t reduce_step(Ex& ex, const T* part, int S, int64_t part_stride, int64_t ldp, int64_t rows, int ncols,
                       T* out, int64_t ldo, const uint32_t* skip_flag = nullptr, uint32_t skip_mask = 0,
                       Gate gate = {}) {
    typename ReduceBody<T>::Args a{part, S, part_stride, ldp, rows, ncols, out, ldo, skip_flag, skip_mask, gate};
    return ex.template run<ReduceBody<T>>(a);
}

}  // namespace rsvd
