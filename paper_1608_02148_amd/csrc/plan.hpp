// Workspace plans, argument rules and the typed solve entry points shared by
// the translation units of the library.
#pragma once

#include <algorithm>
#include <cstring>

#include "common.hpp"
#include "exec.hpp"

namespace rsvd {

// Output tile width for c output columns: 32, 64 or 128 (column tiles of 128
// beyond that); also the padded column count of the skinny work matrices.
inline int tile_cols(int c) { return c <= 32 ? 32 : (c <= 64 ? 64 : (c <= 128 ? 128 : 256)); }

// Column class of the tall product tiles for sketch width c: 32, 64, 128, and
// with fine = true (f32 compute) also 48, 80, 96.
inline int tile_class(int c, bool fine) {
    if (!fine) return std::min(tile_cols(c), 128);
    return c <= 32 ? 32 : c <= 48 ? 48 : c <= 64 ? 64 : c <= 80 ? 80 : c <= 96 ? 96 : 128;   // > 128: two tiles
}

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; }
};

inline size_t elem_size(int dtype) { return dtype == RSVD_F64 ? 8 : (dtype == RSVD_F32 ? 4 : 2); }
inline size_t comp_size(int dtype) { return dtype == RSVD_F64 ? 8 : 4; }

// Work split heuristics (deterministic for a given device and shape).
struct Splits {
    int nn;      // split of the n-reduction in A X
    int tn;      // split of the m-reduction in A^T Q
    int gram_m;  // split of the m-reduction of an m x l Gram matrix
    int gram_n;  // split of the n-reduction of an n x l Gram matrix
    int colsum;  // row split of the column-mean pass
};

// Gram matrices of a batch member: one split per 512 rows, at most 8 (the
// Cholesky sums them).
inline int batch_gram_split(int64_t rows) { return static_cast<int>(std::min<int64_t>(8, std::max<int64_t>(1, cdiv(rows, 512)))); }

// Gram matrices: one split per CU at most, at least 64 rows per split (a
// short n x l Gram then still spreads over most CUs).
inline int gram_split(int64_t rows, int num_cu) {
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(cdiv(rows, 64), num_cu)));
}

// Largest split of the n-reduction of A X (partial blocks of m x Lp each).
constexpr int kMaxNNSplit = 4;

// A^T Q: as many splits as fit the 2 resident workgroups per CU in one round
// (a partly filled second round would idle most CUs), at least 256 rows each.
// A X: split the n-reduction when the row tiles (128 rows each) leave the last
// round of resident workgroups (2 per CU) mostly empty: up to 4 splits of at
// least 1024 columns, taken only when the filled fraction of the rounds rises
// by more than 0.1 (partial blocks cost one extra write and read of m x l).
inline int nn_split(int64_t m, int64_t n, int num_cu) {
    const int64_t tiles = cdiv(m, 128), cap = 2 * static_cast<int64_t>(num_cu);
    auto filled = [&](int64_t S) {
        const int64_t t = tiles * S;
        return static_cast<double>(t) / static_cast<double>(cdiv(t, cap) * cap);
    };
    int best = 1;
    double be = filled(1);
    for (int S = 2; S <= kMaxNNSplit && n / S >= 1024; ++S)
        if (filled(S) > be + 0.1) { best = S; be = filled(S); }
    return best;
}

// Products large enough for the streamed-A kernel (rows x K elements of A).
inline bool streamed_size(int64_t rows, int64_t K) {
    return rows >= 256 && K >= 64 && rows * K >= (int64_t(1) << 24);
}

// Split of the reduction for the streamed-A products (256 output rows per
// workgroup, one workgroup per CU): the count that minimises the estimated
// time, whole rounds of workgroups plus the last one, whose L < num_cu pairs
// are dealt in floor(num_cu / L) pieces each when L <= num_cu / 2 (a whole
// round otherwise), plus one more write and read of each partial block
// (S x rows x Lp f32) relative to one read of A (rows x K f32); at most
// `max_s` splits of at least 1024 reduction elements, at most 8 rounds.
inline int stream_split(int64_t rows, int64_t K, int Lp, int num_cu, int max_s) {
    const int64_t tiles = cdiv(rows, 256);
    int best = 1;
    double best_t = 1e300;
    for (int S = 1; S <= max_s && (S == 1 || K / S >= 1024); ++S) {
        const int64_t wg = tiles * S, whole = wg / num_cu, left = wg % num_cu;
        if (S > 1 && whole > 8) break;
        double rounds = static_cast<double>(whole);
        if (left > 0) rounds += (2 * left <= num_cu) ? 1.0 / static_cast<double>(num_cu / left) : 1.0;
        const double t = rounds / S / (static_cast<double>(tiles) / num_cu) +
                         (S > 1 ? 2.0 * S * Lp / static_cast<double>(K) : 0.0);
        if (t < best_t - 1e-9) { best_t = t; best = S; }
    }
    return best;
}

// Slots of the tail dealing of the streamed products: one round's worth of
// 256-row tiles of Lp f32 columns.
inline size_t tail_slot_bytes(int num_cu, int Lp) { return static_cast<size_t>(num_cu) * 256 * Lp * sizeof(float); }

// Whether a single solve's products of sketch width l run the streamed-A
// kernel (A X: m rows, reduction n; A^T Q: n rows, n % 4 == 0, reduction m;
// A's rows must also be 16-byte aligned, which only the run checks).
inline bool stream_product(int dtype, int64_t m, int64_t n, int l, bool tn) {
    return dtype != RSVD_F64 && (tn ? streamed_size(n, m) && n % 4 == 0 : streamed_size(m, n)) && l > 64 && l <= 224;
}

// streamed: f32 / bf16 storage, where the large products of sketch width l
// take the streamed-A kernel (Lp: the padded width).
inline Splits make_splits(int64_t m, int64_t n, int num_cu, bool streamed = false, int l = 0, int Lp = 128) {
    Splits s;
    s.nn = nn_split(m, n, num_cu);
    const int64_t tn_tiles = cdiv(n, 128);
    s.tn = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((2 * num_cu) / tn_tiles, cdiv(m, 256))));
    if (streamed) {
        if (stream_product(RSVD_F32, m, n, l, false)) s.nn = stream_split(m, n, Lp, num_cu, kMaxNNSplit);
        if (stream_product(RSVD_F32, m, n, l, true)) s.tn = stream_split(n, m, Lp, num_cu, 64);
    }
    s.gram_m = gram_split(m, num_cu);
    s.gram_n = gram_split(n, num_cu);
    const int64_t cs_cols = cdiv(n, 256);
    s.colsum = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(cdiv(2 * num_cu, cs_cols), cdiv(m, 64))));
    return s;
}

struct Plan {
    int dtype = 0;
    int64_t m = 0, n = 0;
    int k = 0, p = 0, q = 0, l = 0, Lp = 0, kp = 0;
    int ncu = 0;        // compute units (the workgroups of one round of the streamed products)
    // batch members: row splits of the m x l and n x l Gram matrices, whose
    // partial sums the Cholesky adds itself (no extra step, so members with
    // different splits still issue the same steps)
    int fold_m = 1, fold_n = 1;
    int tile = 0;       // column class of the tall product tiles (tile_class of l)
    int var_nn = 0, var_tn = 0;   // tile variants of the NN / TN products (tile_variant_index)
    int qmax = 0;       // gated: power iterations issued for the whole batch group
    bool gated = false; // batch member: iterations beyond q switched off on the device
    Splits sp{};
    size_t Y = 0, Z = 0, Om = 0, part = 0, gram = 0, rinv = 0, racc = 0, sigma = 0,
           xv = 0, xu = 0, jk = 0, wks = 0, vtmp = 0, mu = 0, mupart = 0, status = 0, bytes = 0;
    // PCA column statistics: inverse scales, scales and variances (n f64 each) and the
    // total variance (one f64)
    size_t cinv = 0, cscl = 0, cvar = 0, tvar = 0;
    // LU normalisation (tournament pivoting): two candidate lists of
    // cdiv(max(m, n), 256) x l row indices and two count arrays
    size_t lucand = 0, lucnt = 0;
    // a-posteriori estimate (probes > 0): probes n x 32, A probes and U (S V^T
    // probes) m x 32, V^T probes k x 32, U scratch m x k, column partial sums
    int probes = 0, est_split = 1;
    size_t eOm = 0, eY = 0, eT = 0, eW = 0, eU = 0, epart = 0, est = 0;
    // l > 128: scratch of the blocked Cholesky (7 blocks of 128 x 128 f64) and
    // the Jacobi matrix W (l x (l rounded up to 16, plus 1), f64)
    size_t cholx = 0, wglob = 0, jrot = 0, qtmp = 0;
    // bf16 products (mixed precision): X packed into bf16 hi / lo planes of
    // Lp columns x ldxp (max(m, n) rounded up to 8) each
    size_t xpack = 0;
    int64_t ldxp = 0, xplane = 0;
    // streamed products of a single solve: slots of their tail dealing
    // (ncu x 256 x Lp f32)
    size_t tailslot = 0;
    // storage-precision products of a single solve: X copied k-contiguous,
    // Lp columns x ldxk (max(m, n) rounded up to 8) in the compute type
    size_t xk = 0;
    int64_t ldxk = 0;
};

inline int validate(int32_t dtype, int64_t m, int64_t n, int32_t k, const rsvd_params* prm,
                    int max_l = RSVD_MAX_L_SINGLE) {
    if (dtype != RSVD_F64 && dtype != RSVD_F32 && dtype != RSVD_BF16) return RSVD_ERR_UNSUPPORTED;
    if (m < 1 || n < 1 || k < 1 || k >= std::min(m, n)) return RSVD_ERR_INVALID;
    if (!prm || prm->p < 0 || prm->q < 0) return RSVD_ERR_INVALID;
    if (prm->sdist < RSVD_NORMAL || prm->sdist > RSVD_RADEMACHER) return RSVD_ERR_INVALID;
    if (prm->precision != RSVD_PREC_PLAIN && prm->precision != RSVD_PREC_BF16_MIXED) return RSVD_ERR_UNSUPPORTED;
    if (prm->precision == RSVD_PREC_BF16_MIXED && dtype == RSVD_F64) return RSVD_ERR_UNSUPPORTED;
    if (prm->probes < 0 || prm->probes > 16) return RSVD_ERR_INVALID;
    if (prm->scheme != RSVD_SCHEME_QR && prm->scheme != RSVD_SCHEME_LU) return RSVD_ERR_INVALID;
    if (m > (int64_t(1) << 32) || n > (int64_t(1) << 32)) return RSVD_ERR_UNSUPPORTED;
    const int64_t l = std::min<int64_t>(static_cast<int64_t>(k) + prm->p, std::min(m, n));
    if (l > max_l) return RSVD_ERR_UNSUPPORTED;
    if (prm->scheme == RSVD_SCHEME_LU && l > RSVD_MAX_L) return RSVD_ERR_UNSUPPORTED;
    return RSVD_OK;
}

// Index of a tall-tile class in a variant table (6 classes per mode).
inline int tile_variant_index(int cls) {
    return cls <= 32 ? 0 : cls <= 48 ? 1 : cls <= 64 ? 2 : cls <= 80 ? 3 : cls <= 96 ? 4 : 5;
}

// min_Lp: pad the column count of the bases to at least this (a sketch
// shared with a wider plan keeps that plan's leading dimension).
// batch = true: one problem of a grouped batch, whose parallelism comes from
// the batch, so no product splits its reduction (every problem then issues
// the same sequence of steps).  variants: 12 ints (NN then TN, one per tall
// class) choosing the f32 tile variant, or null for the defaults.
inline Plan make_plan(int dtype, int64_t m, int64_t n, int k, const rsvd_params* prm, int num_cu,
                      bool batch = false, const int* variants = nullptr, int min_Lp = 0) {
    Plan P;
    P.dtype = dtype; P.m = m; P.n = n; P.k = k; P.q = prm->q;
    P.l = static_cast<int>(std::min<int64_t>(static_cast<int64_t>(k) + prm->p, std::min(m, n)));
    P.p = P.l - k;
    P.Lp = std::max(tile_cols(P.l), min_Lp);
    P.kp = tile_cols(k);
    P.tile = tile_class(P.l, dtype != RSVD_F64);
    if (variants && dtype != RSVD_F64) {
        P.var_nn = variants[tile_variant_index(P.tile)];
        P.var_tn = variants[6 + tile_variant_index(P.tile)];
    }
    P.qmax = P.q;
    P.gated = batch;
    P.sp = batch ? Splits{1, 1, 1, 1, 1} : make_splits(m, n, num_cu, dtype != RSVD_F64, P.l, P.Lp);
    if (batch && P.Lp <= RSVD_MAX_L) {
        P.fold_m = batch_gram_split(m);
        P.fold_n = batch_gram_split(n);
    }
    P.ncu = num_cu;
    const size_t cs = comp_size(dtype);
    Layout L;
    P.status = L.take(kAlign);
    P.Y = L.take(static_cast<size_t>(m) * P.Lp * cs);
    P.Z = L.take(static_cast<size_t>(n) * P.Lp * cs);
    P.Om = L.take(static_cast<size_t>(n) * P.Lp * cs);
    const size_t part_tn = std::max(P.sp.tn > 1 ? static_cast<size_t>(P.sp.tn) * n * P.Lp * cs : 0,
                                    P.sp.nn > 1 ? static_cast<size_t>(P.sp.nn) * m * P.Lp * cs : 0);
    const size_t part_g = static_cast<size_t>(std::max({P.sp.gram_m, P.sp.gram_n, P.fold_m, P.fold_n})) * P.Lp *
                          P.Lp * 8;
    P.part = L.take(std::max(part_tn, part_g));
    P.gram = L.take(static_cast<size_t>(P.Lp) * P.Lp * 8);
    P.rinv = L.take(static_cast<size_t>(P.Lp) * P.Lp * cs);
    P.racc = L.take(4 * static_cast<size_t>(P.Lp) * P.Lp * 8);
    P.sigma = L.take(static_cast<size_t>(P.Lp) * 8);
    P.xv = L.take(static_cast<size_t>(P.Lp) * P.kp * cs);
    P.xu = L.take(static_cast<size_t>(P.Lp) * P.kp * cs);
    P.jk = L.take(static_cast<size_t>(P.Lp) * P.kp * 8);
    P.wks = L.take(static_cast<size_t>(P.Lp) * P.kp * 8);
    P.vtmp = L.take(static_cast<size_t>(n) * P.kp * cs);
    P.mu = L.take(static_cast<size_t>(n) * 8);
    P.mupart = L.take((2 * static_cast<size_t>(P.sp.colsum) + 1) * n * 8);
    P.cinv = L.take(static_cast<size_t>(n) * 8);
    P.cscl = L.take(static_cast<size_t>(n) * 8);
    P.cvar = L.take(static_cast<size_t>(n) * 8);
    P.tvar = L.take(8);
    if (P.l > 128) {
        P.cholx = L.take(7 * 128 * 128 * sizeof(double));
        P.wglob = L.take(static_cast<size_t>(P.l) * (rup(P.l, 16) + 1) * sizeof(double));
        P.jrot = L.take(64 * sizeof(uint32_t));
        P.qtmp = L.take(static_cast<size_t>(std::max(m, n)) * P.Lp * cs);
    }
    if (!batch && (stream_product(dtype, m, n, P.l, false) || stream_product(dtype, m, n, P.l, true)))
        P.tailslot = L.take(tail_slot_bytes(num_cu, P.Lp));
    if (prm->precision == RSVD_PREC_BF16_MIXED) {
        P.ldxp = rup(std::max(m, n), 8);
        P.xplane = static_cast<int64_t>(P.Lp) * P.ldxp;
        P.xpack = L.take(2 * static_cast<size_t>(P.xplane) * sizeof(uint16_t));
    } else if (!batch) {
        P.ldxk = rup(std::max(m, n), 8);
        P.xk = L.take(static_cast<size_t>(P.Lp) * P.ldxk * cs);
    }
    if (prm->scheme == RSVD_SCHEME_LU) {
        const size_t leaves = static_cast<size_t>(cdiv(std::max(m, n), 256));
        P.lucand = L.take(2 * leaves * P.l * sizeof(int32_t));
        P.lucnt = L.take(2 * leaves * sizeof(int32_t));
    }
    P.probes = prm->probes;
    if (P.probes > 0) {
        P.est_split = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(cdiv(m, 2048), 256)));
        P.eOm = L.take(static_cast<size_t>(n) * 32 * cs);
        P.eY = L.take(static_cast<size_t>(m) * 32 * cs);
        P.eT = L.take(static_cast<size_t>(P.kp) * 32 * cs);
        P.eW = L.take(static_cast<size_t>(m) * 32 * cs);
        P.eU = L.take(static_cast<size_t>(m) * P.kp * cs);
        P.epart = L.take(static_cast<size_t>(std::max(P.est_split, P.sp.gram_n)) * 32 * P.kp * 8);
        P.est = L.take(sizeof(double));
    }
    P.bytes = L.off;
    return P;
}

template <typename T> inline T* at(void* work, size_t off) {
    return reinterpret_cast<T*>(static_cast<unsigned char*>(work) + off);
}

#define RSVD_TRY(expr)                                   \
    do {                                                 \
        hipError_t _e = (expr);                          \
        if (_e != hipSuccess) return _e;                 \
    } while (0)

struct SolveOut {
    void* U; int64_t ldu;      // m x k or null
    void* V; int64_t ldv;      // n x k or null (then workspace)
    double* S;                 // k
    double* eigvals; double* sdev;   // PCA extras or null
    void* center_out;
    int scale_u;               // 1: U columns scaled by sigma (PCA x = U S)
    int center;
    int scale;                 // PCA: divide the centred columns by their root mean square
    void* scale_out;           // PCA: n column scales or null
    double* total_var;         // PCA: total variance of the analysed data or null
    void* loadings; int64_t ldl;     // PCA: n x k loadings or null
    void* xwhite; int64_t ldxw;      // PCA: m x k whitened components or null
    void* bt; int64_t ldbt;          // non-null: stop after B^T = A^T Q (n x l) and copy it here
    rsvd_info* info;
    uint64_t* stamps;          // optional [first step, last step] device clock
    float* features;           // non-null: stop after the sketch and write the 131 selector inputs
    int feat_k;                // target rank used in the features
    const int32_t* qsrc;       // non-null: q read on the device (gated plans, q <= qmax)
    const void* y0;            // non-null: the sketch A Omega[:, :l] already computed (ld Lp)
    int stamp_sel;             // which of the two stamps this call writes: 1 first, 2 last, 3 both
};

inline int hip_status(rsvd_handle_t h, hipError_t e) {
    if (e == hipSuccess) return RSVD_OK;
    h->last_hip_error = static_cast<int>(e);
    return RSVD_ERR_HIP;
}

// Workspace of the kernel-level building blocks (products, orthonormalisation,
// small SVD) at these sizes.
inline Plan block_plan(int32_t dtype, int64_t m, int64_t n, int32_t c, int num_cu) {
    Plan P;
    P.dtype = dtype; P.m = m; P.n = n; P.l = c; P.Lp = tile_cols(c);
    P.sp = make_splits(m, n, num_cu, dtype != RSVD_F64, c, P.Lp);
    P.ncu = num_cu;
    const size_t cs = comp_size(dtype);
    Layout L;
    P.status = L.take(kAlign);
    P.part = L.take(std::max({static_cast<size_t>(P.sp.tn) * n * P.Lp * cs,
                              static_cast<size_t>(kMaxNNSplit) * m * P.Lp * cs,
                              static_cast<size_t>(std::max(P.sp.gram_m, P.sp.gram_n)) * P.Lp * P.Lp * 8}));
    P.gram = L.take(static_cast<size_t>(P.Lp) * P.Lp * 8);
    P.rinv = L.take(static_cast<size_t>(P.Lp) * P.Lp * cs);
    P.racc = L.take(4 * static_cast<size_t>(P.Lp) * P.Lp * 8);
    P.jk = L.take(static_cast<size_t>(P.Lp) * P.Lp * 8);
    P.ldxp = rup(std::max(m, n), 8);
    P.xplane = static_cast<int64_t>(P.Lp) * P.ldxp;
    P.xpack = L.take(2 * static_cast<size_t>(P.xplane) * sizeof(uint16_t));
    P.ldxk = rup(std::max(m, n), 8);
    P.xk = L.take(static_cast<size_t>(P.Lp) * P.ldxk * cs);
    if (stream_product(dtype, m, n, c, false) || stream_product(dtype, m, n, c, true))
        P.tailslot = L.take(tail_slot_bytes(num_cu, P.Lp));
    if (c <= RSVD_MAX_L) {
        const size_t leaves = static_cast<size_t>(cdiv(std::max(m, n), 256));
        P.lucand = L.take(2 * leaves * c * sizeof(int32_t));
        P.lucnt = L.take(2 * leaves * sizeof(int32_t));
    }
    P.bytes = L.off;
    return P;
}

// Workspace of rpca_predict: the centre widened to f64 (n), the rotation
// with its rows divided by the scales, D^-1 W (n x kp in the compute type,
// zero-padded columns), and the partial blocks of a split n-reduction.
struct PredictPlan {
    int dtype = 0;
    int64_t m = 0, n = 0;
    int k = 0, kp = 0, S = 1;
    size_t mu = 0, w = 0, part = 0, bytes = 0;
};

inline PredictPlan predict_plan(int32_t dtype, int64_t m, int64_t n, int32_t k, int num_cu) {
    PredictPlan P;
    P.dtype = dtype; P.m = m; P.n = n; P.k = k; P.kp = tile_cols(k);
    P.S = nn_split(m, n, num_cu);
    const size_t cs = comp_size(dtype);
    Layout L;
    P.mu = L.take(static_cast<size_t>(n) * 8);
    P.w = L.take(static_cast<size_t>(n) * P.kp * cs);
    P.part = L.take(P.S > 1 ? static_cast<size_t>(P.S) * m * P.kp * cs : 0);
    P.bytes = L.off;
    return P;
}

// One solve of Alg. RSVDalgorithm / Alg. RPCAalgorithm for each storage type
// (f64, f32, bf16 with f32 compute): launched at once on the handle's stream,
// or recorded as one problem of a grouped batch.
#define RSVD_DECLARE_SOLVE(NAME)                                                                       \
    hipError_t solve_single_##NAME(rsvd_handle_t h, const Plan& P, const void* A, int64_t lda,         \
                                   const rsvd_params* prm, const SolveOut& o, void* work);              \
    hipError_t solve_record_##NAME(BatchRecorder& rec, const Plan& P, const void* A, int64_t lda,      \
                                   const rsvd_params* prm, uint32_t stream_id, const SolveOut& o,       \
                                   void* work);
RSVD_DECLARE_SOLVE(f64)
RSVD_DECLARE_SOLVE(f32)
RSVD_DECLARE_SOLVE(bf16)
#undef RSVD_DECLARE_SOLVE

// One single solve on the handle's stream, by storage type (defined with the
// C entry points); returns an RSVD_* status.
int dispatch(rsvd_handle_t h, int32_t dtype, const Plan& P, const void* A, int64_t lda,
             const rsvd_params* prm, const SolveOut& o, void* work);

// Principal components of new rows per storage type (rpca_predict).
#define RSVD_DECLARE_PREDICT(NAME)                                                                     \
    hipError_t predict_##NAME(rsvd_handle_t h, const PredictPlan& P, const void* A, int64_t lda,       \
                              const void* rot, int64_t ldr, const void* center, const void* scale,      \
                              void* x, int64_t ldx, void* work);
RSVD_DECLARE_PREDICT(f64)
RSVD_DECLARE_PREDICT(f32)
RSVD_DECLARE_PREDICT(bf16)
#undef RSVD_DECLARE_PREDICT

}  // namespace rsvd
