// C ABI and host orchestration of the randomized SVD / PCA hot path.
//
// One solve (Alg. RSVDalgorithm over Alg. rqb with Alg. subspace_iter):
//   Omega -> Y = A Omega -> [orth(Y); Z = A^T Y; orth(Z); Y = A Z] x q
//   -> orth(Y) -> B^T = A^T Y -> B^T = Q_b R_b -> R_b = W S J^T (Jacobi)
//   -> V = Q_b W_k -> sign rule -> U = Q J_k.
// orth() is CholeskyQR2 (shifted CholeskyQR3 when needed) in place.  Every
// step is a kernel on the handle's stream; nothing synchronises the host.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "launch.hpp"

namespace rsvd {

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
    int tn;      // split of the m-reduction in A^T Q
    int gram_m;  // split of the m-reduction of an m x l Gram matrix
    int gram_n;  // split of the n-reduction of an n x l Gram matrix
    int colsum;  // row split of the column-mean pass
};

// Gram matrices: one split per CU at most, at least 256 rows per split.
inline int gram_split(int64_t rows, int num_cu) {
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(cdiv(rows, 256), num_cu)));
}

// A^T Q: as many splits as fit the 2 resident workgroups per CU in one round
// (a partly filled second round would idle most CUs), at least 256 rows each.
inline Splits make_splits(int64_t m, int64_t n, int num_cu) {
    Splits s;
    const int64_t tn_tiles = cdiv(n, 128);
    s.tn = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((2 * num_cu) / tn_tiles, cdiv(m, 256))));
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
    int tile = 0;       // forced output tile width of every product (0: chosen per product)
    Splits sp{};
    size_t Y = 0, Z = 0, Om = 0, part = 0, gram = 0, rinv = 0, racc = 0, sigma = 0,
           xv = 0, xu = 0, jk = 0, wks = 0, vtmp = 0, mu = 0, mupart = 0, status = 0, bytes = 0;
};

inline int validate(int32_t dtype, int64_t m, int64_t n, int32_t k, const rsvd_params* prm) {
    if (dtype != RSVD_F64 && dtype != RSVD_F32 && dtype != RSVD_BF16) return RSVD_ERR_UNSUPPORTED;
    if (m < 1 || n < 1 || k < 1 || k >= std::min(m, n)) return RSVD_ERR_INVALID;
    if (!prm || prm->p < 0 || prm->q < 0) return RSVD_ERR_INVALID;
    if (prm->sdist < RSVD_NORMAL || prm->sdist > RSVD_RADEMACHER) return RSVD_ERR_INVALID;
    if (prm->precision != RSVD_PREC_PLAIN && prm->precision != RSVD_PREC_BF16_MIXED) return RSVD_ERR_UNSUPPORTED;
    if (prm->precision == RSVD_PREC_BF16_MIXED && dtype == RSVD_F64) return RSVD_ERR_UNSUPPORTED;
    if (m > (int64_t(1) << 32) || n > (int64_t(1) << 32)) return RSVD_ERR_UNSUPPORTED;
    const int64_t l = std::min<int64_t>(static_cast<int64_t>(k) + prm->p, std::min(m, n));
    if (l > RSVD_MAX_L) return RSVD_ERR_UNSUPPORTED;
    return RSVD_OK;
}

// batch = true: one problem of a grouped batch, whose parallelism comes from
// the batch, so no product splits its reduction (every problem then issues
// the same sequence of steps).
inline Plan make_plan(int dtype, int64_t m, int64_t n, int k, const rsvd_params* prm, int num_cu,
                      bool batch = false) {
    Plan P;
    P.dtype = dtype; P.m = m; P.n = n; P.k = k; P.q = prm->q;
    P.l = static_cast<int>(std::min<int64_t>(static_cast<int64_t>(k) + prm->p, std::min(m, n)));
    P.p = P.l - k;
    P.Lp = tile_cols(P.l);
    P.kp = tile_cols(k);
    P.sp = batch ? Splits{1, 1, 1, 1} : make_splits(m, n, num_cu);
    const size_t cs = comp_size(dtype);
    Layout L;
    P.status = L.take(kAlign);
    P.Y = L.take(static_cast<size_t>(m) * P.Lp * cs);
    P.Z = L.take(static_cast<size_t>(n) * P.Lp * cs);
    P.Om = L.take(static_cast<size_t>(n) * P.Lp * cs);
    const size_t part_tn = P.sp.tn > 1 ? static_cast<size_t>(P.sp.tn) * n * P.Lp * cs : 0;
    const size_t part_g = static_cast<size_t>(std::max(P.sp.gram_m, P.sp.gram_n)) * P.Lp * P.Lp * 8;
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
    P.mupart = L.take(static_cast<size_t>(P.sp.colsum) * n * 8);
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

// In-place orthonormalisation of M (rows x l, ld ldm, precision TC):
// CholeskyQR2, with a shifted first pass and a third pass when needed.
// adaptive = true (bases inside the power scheme, whose span is all that the
// next product uses) runs the second pass only when the first pass shows an
// ill-conditioned Gram matrix.
// rfac (optional, f64, 4 consecutive l x l blocks) receives R1, R2, R3 (R3 = I
// when the third pass is skipped) and, in the fourth block, R = R3 R2 R1.
template <typename TC, class Ex>
hipError_t orthonormalize(Ex& ex, int tile, TC* M, int64_t ldm, int64_t rows, int l, int Lp, int S,
                          double* part, double* gram, TC* rinv, double* rfac, uint32_t* status,
                          bool adaptive = false) {
    for (int pass = 1; pass <= 3; ++pass) {
        const bool conditional = (pass == 3) || (pass == 2 && adaptive);
        const uint32_t* skip = conditional ? status : nullptr;
        const uint32_t need = (pass == 2) ? ST_NEED_P2 : ST_NEED_P3;
        RSVD_TRY((gemm_plain<TC, TC, double, MODE_TN>(ex, tile, M, ldm, l, rows, M, ldm, l, part, Lp, S,
                                                      static_cast<int64_t>(Lp) * Lp, nullptr, skip, need)));
        if (S > 1) RSVD_TRY(reduce_step<double>(ex, part, S, static_cast<int64_t>(Lp) * Lp, Lp, l, l, gram, Lp,
                                                skip, need));
        CholArgs ca;
        ca.part = (S > 1) ? gram : part; ca.S = 1; ca.part_stride = 0; ca.ldp = Lp;
        ca.l = l; ca.mrows = rows; ca.rinv = rinv; ca.ldr = Lp;
        ca.rout = rfac ? rfac + static_cast<size_t>(pass - 1) * l * l : nullptr;
        ca.status = status; ca.pass = pass; ca.skip_unless_pending = conditional; ca.adaptive = adaptive;
        RSVD_TRY(ex.template run<CholBody<TC>>(ca));
        RSVD_TRY((gemm_plain<TC, TC, TC, MODE_NN>(ex, tile, M, ldm, rows, l, rinv, Lp, l, M, ldm, 1, 0, nullptr,
                                                  skip, need)));
    }
    if (rfac) {   // R = R3 (R2 R1); the product R2 R1 goes through the gram scratch
        const size_t ll = static_cast<size_t>(l) * l;
        RSVD_TRY((gemm_plain<double, double, double, MODE_NN>(ex, tile, rfac + ll, l, l, l, rfac, l, l, gram, l, 1,
                                                              0, nullptr, nullptr, 0)));
        RSVD_TRY((gemm_plain<double, double, double, MODE_NN>(ex, tile, rfac + 2 * ll, l, l, l, gram, l, l,
                                                              rfac + 3 * ll, l, 1, 0, nullptr, nullptr, 0)));
    }
    return hipSuccess;
}

// Optional event bracketing of the products with A (rsvd_profile_enable).
inline hipEvent_t pool_event(rsvd_handle_t h) {
    if (h->pool_used == h->event_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->event_pool.push_back(e);
    }
    return h->event_pool[h->pool_used++];
}

// h == nullptr (recorded batch steps) or profiling off: just issue the step.
template <typename F>
hipError_t timed(rsvd_handle_t h, int kind, double flops, double bytes, F&& launch) {
    if (!h || !h->profiling) return launch();
    ProfRecord r;
    r.kind = kind; r.flops = flops; r.bytes = bytes;
    r.start = pool_event(h);
    r.stop = pool_event(h);
    if (!r.start || !r.stop) return hipErrorOutOfMemory;
    RSVD_TRY(hipEventRecord(r.start, h->stream));
    RSVD_TRY(launch());
    RSVD_TRY(hipEventRecord(r.stop, h->stream));
    h->prof.push_back(r);
    return hipSuccess;
}

struct SolveOut {
    void* U; int64_t ldu;      // m x k or null
    void* V; int64_t ldv;      // n x k or null (then workspace)
    double* S;                 // k
    double* eigvals; double* sdev;   // PCA extras or null
    void* center_out;
    int scale_u;               // 1: U columns scaled by sigma (PCA x = U S)
    int center;
    rsvd_info* info;
    uint64_t* stamps;          // optional [first step, last step] device clock
};

// Every step of one solve, issued through the executor: launched at once for
// a single solve, or recorded as this problem's share of grouped batch steps.
// prof (may be null) receives the event timings of the products with A.
template <typename TA, typename TC, class Ex>
hipError_t solve_steps(Ex& ex, rsvd_handle_t prof, const Plan& P, const TA* A, int64_t lda,
                       const rsvd_params* prm, uint32_t stream_id, const SolveOut& o, void* work) {
    const int64_t m = P.m, n = P.n;
    const int l = P.l, Lp = P.Lp, k = P.k, tile = P.tile;
    uint32_t* status = at<uint32_t>(work, P.status);
    TC* Y = at<TC>(work, P.Y);
    TC* Z = at<TC>(work, P.Z);
    TC* Om = at<TC>(work, P.Om);
    TC* partc = at<TC>(work, P.part);
    double* partd = at<double>(work, P.part);
    double* gram = at<double>(work, P.gram);
    TC* rinv = at<TC>(work, P.rinv);
    double* racc = at<double>(work, P.racc);
    double* sigma = at<double>(work, P.sigma);
    TC* xv = at<TC>(work, P.xv);
    TC* xu = at<TC>(work, P.xu);
    double* jk = at<double>(work, P.jk);
    double* mu = o.center ? at<double>(work, P.mu) : nullptr;

    if (o.stamps) RSVD_TRY(ex.template run<StampBody>(StampBody::Args{o.stamps}));
    RSVD_TRY(ex.template run<ClearBody>(ClearBody::Args{status, 1}));

    if (mu) {   // column means (implicit centring, Sec. 4.2)
        const int S = P.sp.colsum;
        double* mp = at<double>(work, P.mupart);
        RSVD_TRY(ex.template run<ColsumBody<TA>>(typename ColsumBody<TA>::Args{A, lda, m, n, cdiv(m, S), S, mp}));
        RSVD_TRY(ex.template run<ColmeanBody>(ColmeanBody::Args{mp, S, m, n, mu}));
    }

    // Alg. rqb steps 2-3: Omega and the sketch Y = A Omega.
    RSVD_TRY(ex.template run<OmegaBody<TC>>(typename OmegaBody<TC>::Args{
        n, l, Lp, prm->seed, stream_id, prm->sdist, Om, static_cast<int64_t>(Lp)}));
    const double pass_flops = 2.0 * static_cast<double>(m) * n * l;
    const double a_bytes = static_cast<double>(m) * n * sizeof(TA);
    const double nn_bytes = a_bytes + (static_cast<double>(n) + m) * l * sizeof(TC);
    const double tn_bytes = a_bytes + (static_cast<double>(m) + n) * l * sizeof(TC);
    // Arithmetic of each pass: storage precision, or in the mixed mode bf16
    // for the early passes and split bf16 (f32-accurate) for the last sketch
    // and the projection (precision escalation).
    const bool mixed = prm->precision == RSVD_PREC_BF16_MIXED;
    const int early = mixed ? 1 : 0, late = mixed ? 2 : 0;
    auto ax = [&](const TC* X, int arith) -> hipError_t {     // Y (m x Lp) = A X
        return timed(prof, 0, pass_flops, nn_bytes, [&] {
            return gemm_step<TA, TC, MODE_NN>(ex, arith, tile, A, lda, m, n, X, Lp, l, Y, Lp, 1, 0, mu, nullptr,
                                              0);
        });
    };
    RSVD_TRY(ax(Om, P.q == 0 ? late : early));

    auto aty = [&](TC* dst, int arith) -> hipError_t {     // dst (n x Lp) = A^T Y
        const int S = P.sp.tn;
        if (S == 1)
            return timed(prof, 1, pass_flops, tn_bytes, [&] {
                return gemm_step<TA, TC, MODE_TN>(ex, arith, tile, A, lda, n, m, Y, Lp, l, dst, Lp, 1, 0, mu,
                                                  nullptr, 0);
            });
        RSVD_TRY(timed(prof, 1, pass_flops, tn_bytes, [&] {
            return gemm_step<TA, TC, MODE_TN>(ex, arith, tile, A, lda, n, m, Y, Lp, l, partc, Lp, S,
                                              static_cast<int64_t>(n) * Lp, mu, nullptr, 0);
        }));
        return reduce_step<TC>(ex, partc, S, static_cast<int64_t>(n) * Lp, Lp, n, l, dst, Lp);
    };

    // Alg. subspace_iter: q rounds of orth(Y); Z = orth(A^T Y); Y = A Z.
    for (int it = 0; it < P.q; ++it) {
        RSVD_TRY(orthonormalize<TC>(ex, tile, Y, Lp, m, l, Lp, P.sp.gram_m, partd, gram, rinv, nullptr, status,
                                    true));
        RSVD_TRY(aty(Z, early));
        RSVD_TRY(orthonormalize<TC>(ex, tile, Z, Lp, n, l, Lp, P.sp.gram_n, partd, gram, rinv, nullptr, status,
                                    true));
        RSVD_TRY(ax(Z, it == P.q - 1 ? late : early));
    }
    // Alg. rqb steps 9-10: Q = qr(Y); B^T = A^T Q.
    RSVD_TRY(orthonormalize<TC>(ex, tile, Y, Lp, m, l, Lp, P.sp.gram_m, partd, gram, rinv, nullptr, status));
    RSVD_TRY(aty(Z, late));
    // svd(B): B^T = Q_b R_b (Q_b overwrites Z), R_b = W S J^T by Jacobi.
    RSVD_TRY(orthonormalize<TC>(ex, tile, Z, Lp, n, l, Lp, P.sp.gram_n, partd, gram, rinv, racc, status));
    racc += 3 * static_cast<size_t>(l) * l;       // R_b = R3 R2 R1
    {
        JacobiArgs ja;
        ja.R = racc; ja.ldr = l; ja.l = l; ja.k = k;
        double* wks = at<double>(work, P.wks);
        ja.sigma = sigma; ja.xv = xv; ja.ldx = Lp; ja.xcols = P.kp; ja.wks = wks;
        ja.status = status; ja.max_sweeps = 60; ja.tol = jacobi_tol(ja.l);
        RSVD_TRY(ex.template run<JacobiBody<TC>>(ja));
        // J_k = R_b^T (W_k / sigma)
        RSVD_TRY((gemm_plain<double, double, double, MODE_TN>(ex, tile, racc, l, l, l, wks, k, k, jk, k, 1, 0,
                                                              nullptr, nullptr, 0)));
    }
    // V = Q_b W_k, sign rule, then U = Q (J_k D) with D = signs (x S for PCA).
    TC* V = o.V ? static_cast<TC*>(o.V) : at<TC>(work, P.vtmp);
    const int64_t ldv = o.V ? o.ldv : P.kp;
    RSVD_TRY((gemm_plain<TC, TC, TC, MODE_NN>(ex, tile, Z, Lp, n, l, xv, P.kp, k, V, ldv, 1, 0, nullptr, nullptr,
                                              0)));
    RSVD_TRY(ex.template run<SignLiftBody<TC>>(typename SignLiftBody<TC>::Args{
        V, ldv, n, l, k, jk, sigma, o.scale_u, xu, Lp, P.kp}));
    if (o.U)
        RSVD_TRY((gemm_plain<TC, TC, TC, MODE_NN>(ex, tile, Y, Lp, m, l, xu, P.kp, k, static_cast<TC*>(o.U), o.ldu,
                                                  1, 0, nullptr, nullptr, 0)));
    RSVD_TRY(ex.template run<FinalizeBody<TC>>(typename FinalizeBody<TC>::Args{
        sigma, k, o.S, o.eigvals, o.sdev, static_cast<double>(m - 1), mu, n, static_cast<TC*>(o.center_out),
        status, o.info, l, P.q, P.p}));
    if (o.stamps) RSVD_TRY(ex.template run<StampBody>(StampBody::Args{o.stamps + 1}));
    return hipSuccess;
}

inline int hip_status(rsvd_handle_t h, hipError_t e) {
    if (e == hipSuccess) return RSVD_OK;
    h->last_hip_error = static_cast<int>(e);
    return RSVD_ERR_HIP;
}

template <typename TA, typename TC>
int run_typed(rsvd_handle_t h, const Plan& P, const void* A, int64_t lda, const rsvd_params* prm,
              const SolveOut& o, void* work) {
    SingleExec ex{h->stream};
    return hip_status(h, solve_steps<TA, TC>(ex, h, P, static_cast<const TA*>(A), lda, prm, prm->stream_id, o,
                                             work));
}

int dispatch(rsvd_handle_t h, int32_t dtype, const Plan& P, const void* A, int64_t lda,
             const rsvd_params* prm, const SolveOut& o, void* work) {
    switch (dtype) {
        case RSVD_F64: return run_typed<double, double>(h, P, A, lda, prm, o, work);
        case RSVD_F32: return run_typed<float, float>(h, P, A, lda, prm, o, work);
        case RSVD_BF16: return run_typed<bf16_t, float>(h, P, A, lda, prm, o, work);
    }
    return RSVD_ERR_UNSUPPORTED;
}

}  // namespace rsvd

using namespace rsvd;

extern "C" {

void rsvd_default_params(rsvd_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->p = 10;
    p->q = 2;
    p->seed = 0;
    p->stream_id = 0;
    p->sdist = RSVD_NORMAL;
    p->precision = RSVD_PREC_PLAIN;
}

int rsvd_create(rsvd_handle_t* handle, void* hip_stream) {
    if (!handle) return RSVD_ERR_INVALID;
    rsvd_handle_s* h = new rsvd_handle_s();
    h->stream = static_cast<hipStream_t>(hip_stream);
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        h->dev.device = dev;
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
            h->dev.num_cu = cu;
    }
    *handle = h;
    return RSVD_OK;
}

int rsvd_destroy(rsvd_handle_t handle) {
    if (handle)
        for (hipEvent_t e : handle->event_pool) (void)hipEventDestroy(e);
    delete handle;
    return RSVD_OK;
}

int rsvd_set_stream(rsvd_handle_t handle, void* hip_stream) {
    if (!handle) return RSVD_ERR_INVALID;
    handle->stream = static_cast<hipStream_t>(hip_stream);
    return RSVD_OK;
}

int rsvd_last_hip_error(rsvd_handle_t handle) { return handle ? handle->last_hip_error : 0; }

const char* rsvd_status_string(int status) {
    switch (status) {
        case RSVD_OK: return "ok";
        case RSVD_ERR_INVALID: return "invalid argument";
        case RSVD_ERR_UNSUPPORTED: return "unsupported dtype, mode or size";
        case RSVD_ERR_HIP: return "HIP runtime error";
        case RSVD_ERR_NONFINITE: return "non-finite values reached a Gram matrix";
        case RSVD_ERR_BREAKDOWN: return "numerical breakdown after the shifted Cholesky";
    }
    return "unknown status";
}

int rsvd_workspace_size(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, int32_t k,
                        const rsvd_params* params, size_t* bytes) {
    if (!handle || !bytes) return RSVD_ERR_INVALID;
    const int v = validate(dtype, m, n, k, params);
    if (v != RSVD_OK) return v;
    *bytes = make_plan(dtype, m, n, k, params, handle->dev.num_cu).bytes;
    return RSVD_OK;
}

static int check_common(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A,
                        int64_t lda, int32_t k, const rsvd_params* params, void* work,
                        size_t work_bytes, Plan* plan) {
    if (!handle) return RSVD_ERR_INVALID;
    const int v = validate(dtype, m, n, k, params);
    if (v != RSVD_OK) return v;
    if (!A || lda < n || !work) return RSVD_ERR_INVALID;
    if (reinterpret_cast<uintptr_t>(work) % kAlign != 0) return RSVD_ERR_INVALID;
    *plan = make_plan(dtype, m, n, k, params, handle->dev.num_cu);
    if (work_bytes < plan->bytes) return RSVD_ERR_INVALID;
    return RSVD_OK;
}

int rsvd_run(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
             int32_t k, const rsvd_params* params, void* U, int64_t ldu, double* S, void* V,
             int64_t ldv, void* work, size_t work_bytes, rsvd_info* info) {
    Plan P;
    const int c = check_common(handle, dtype, m, n, A, lda, k, params, work, work_bytes, &P);
    if (c != RSVD_OK) return c;
    if (!S || (U && ldu < k) || (V && ldv < k)) return RSVD_ERR_INVALID;
    SolveOut o{};
    o.U = U; o.ldu = ldu; o.V = V; o.ldv = ldv; o.S = S;
    o.scale_u = 0; o.center = 0; o.info = info;
    return dispatch(handle, dtype, P, A, lda, params, o, work);
}

int rpca_run(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
             int32_t k, int32_t center, const rsvd_params* params, void* rotation, int64_t ldr,
             double* eigvals, double* sdev, void* x, int64_t ldx, void* center_out, void* work,
             size_t work_bytes, rsvd_info* info) {
    Plan P;
    const int c = check_common(handle, dtype, m, n, A, lda, k, params, work, work_bytes, &P);
    if (c != RSVD_OK) return c;
    if (!rotation || ldr < k || !eigvals || (x && ldx < k)) return RSVD_ERR_INVALID;
    SolveOut o{};
    o.U = x; o.ldu = ldx; o.V = rotation; o.ldv = ldr; o.S = nullptr;
    o.eigvals = eigvals; o.sdev = sdev; o.center_out = center_out;
    o.scale_u = 1; o.center = center ? 1 : 0; o.info = info;
    return dispatch(handle, dtype, P, A, lda, params, o, work);
}

int rsvd_sync_info(rsvd_handle_t handle, const rsvd_info* dinfo, rsvd_info* hinfo) {
    if (!handle || !dinfo || !hinfo) return RSVD_ERR_INVALID;
    hipError_t e = hipMemcpyAsync(hinfo, dinfo, sizeof(rsvd_info), hipMemcpyDeviceToHost, handle->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(handle->stream);
    if (e != hipSuccess) return hip_status(handle, e);
    if (hinfo->flags & RSVD_FLAG_NONFINITE) return RSVD_ERR_NONFINITE;
    if (hinfo->flags & RSVD_FLAG_DEGENERATE) return RSVD_ERR_BREAKDOWN;
    return RSVD_OK;
}

int rsvd_profile_enable(rsvd_handle_t handle, int32_t enable) {
    if (!handle) return RSVD_ERR_INVALID;
    handle->profiling = enable != 0;
    return RSVD_OK;
}

int rsvd_profile_collect(rsvd_handle_t handle, rsvd_kernel_stat* out) {
    if (!handle || !out) return RSVD_ERR_INVALID;
    for (int k = 0; k < RSVD_PROFILE_KINDS; ++k) out[k] = rsvd_kernel_stat{0, 0, 0.0, 0.0, 0.0};
    hipError_t e = hipStreamSynchronize(handle->stream);
    for (const ProfRecord& r : handle->prof) {
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (r.kind < 0 || r.kind >= RSVD_PROFILE_KINDS) continue;
        rsvd_kernel_stat& s = out[r.kind];
        s.count += 1;
        s.total_ms += ms;
        s.flops += r.flops;
        s.bytes += r.bytes;
    }
    handle->prof.clear();
    handle->pool_used = 0;
    return hip_status(handle, e);
}

// ---------------------------------------------------------- building blocks

int rsvd_philox_words(rsvd_handle_t handle, int64_t n, int32_t groups, uint64_t seed, uint32_t stream_id,
                      uint32_t* out) {
    if (!handle || n < 1 || groups < 1 || !out) return RSVD_ERR_INVALID;
    const int64_t total = n * groups;
    hipLaunchKernelGGL(philox_words_kernel, dim3(static_cast<unsigned>(cdiv(total, 256))), dim3(256), 0,
                       handle->stream, n, groups, seed, stream_id, out);
    return hip_status(handle, hipGetLastError());
}

int rsvd_test_matrix(rsvd_handle_t handle, int32_t dtype, int64_t n, int32_t l, uint64_t seed,
                     uint32_t stream_id, int32_t sdist, void* out, int64_t ldo) {
    if (!handle || n < 1 || l < 1 || !out || ldo < l) return RSVD_ERR_INVALID;
    if (sdist < RSVD_NORMAL || sdist > RSVD_RADEMACHER) return RSVD_ERR_INVALID;
    const int groups = (l + 3) / 4;
    const int64_t total = n * groups;
    (void)total;
    SingleExec ex{handle->stream};
    if (dtype == RSVD_F64)
        return hip_status(handle, ex.run<OmegaBody<double>>(OmegaBody<double>::Args{
                                      n, l, l, seed, stream_id, sdist, static_cast<double*>(out), ldo}));
    return hip_status(handle, ex.run<OmegaBody<float>>(OmegaBody<float>::Args{
                                  n, l, l, seed, stream_id, sdist, static_cast<float*>(out), ldo}));
}

static Plan block_plan(int32_t dtype, int64_t m, int64_t n, int32_t c, int num_cu) {
    rsvd_params prm;
    rsvd_default_params(&prm);
    prm.p = 0;
    Plan P;
    P.dtype = dtype; P.m = m; P.n = n; P.l = c; P.Lp = tile_cols(c);
    P.sp = make_splits(m, n, num_cu);
    const size_t cs = comp_size(dtype);
    Layout L;
    P.status = L.take(kAlign);
    P.part = L.take(std::max(static_cast<size_t>(P.sp.tn) * n * P.Lp * cs,
                             static_cast<size_t>(std::max(P.sp.gram_m, P.sp.gram_n)) * P.Lp * P.Lp * 8));
    P.gram = L.take(static_cast<size_t>(P.Lp) * P.Lp * 8);
    P.rinv = L.take(static_cast<size_t>(P.Lp) * P.Lp * cs);
    P.racc = L.take(4 * static_cast<size_t>(P.Lp) * P.Lp * 8);
    P.jk = L.take(static_cast<size_t>(P.Lp) * P.Lp * 8);
    P.bytes = L.off;
    (void)prm;
    return P;
}

int rsvd_block_workspace_size(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, int32_t c,
                              size_t* bytes) {
    if (!handle || !bytes || m < 1 || n < 1 || c < 1 || c > RSVD_MAX_L) return RSVD_ERR_INVALID;
    *bytes = block_plan(dtype, m, n, c, handle->dev.num_cu).bytes;
    return RSVD_OK;
}

}  // extern "C"

template <typename TA, typename TC>
static hipError_t gemm_nn_typed(hipStream_t st, int arith, int64_t m, int64_t K, int c, const void* A, int64_t lda,
                                const void* X, int64_t ldx, void* Y, int64_t ldy) {
    SingleExec ex{st};
    return gemm_step<TA, TC, MODE_NN>(ex, arith, 0, static_cast<const TA*>(A), lda, m, K, static_cast<const TC*>(X),
                                      ldx, c, static_cast<TC*>(Y), ldy, 1, 0, nullptr, nullptr, 0);
}

extern "C" {

int rsvd_gemm_nn(rsvd_handle_t handle, int32_t dtype, int32_t arith, int64_t m, int64_t K, int32_t c,
                 const void* A, int64_t lda, const void* X, int64_t ldx, void* Y, int64_t ldy, void* work,
                 size_t work_bytes) {
    (void)work; (void)work_bytes;
    if (!handle || m < 1 || K < 1 || c < 1 || c > RSVD_MAX_L || !A || !X || !Y) return RSVD_ERR_INVALID;
    if (lda < K || ldx < c || ldy < c || arith < 0 || arith > 2) return RSVD_ERR_INVALID;
    if (arith != 0 && dtype == RSVD_F64) return RSVD_ERR_UNSUPPORTED;
    hipError_t e;
    switch (dtype) {
        case RSVD_F64: e = gemm_nn_typed<double, double>(handle->stream, arith, m, K, c, A, lda, X, ldx, Y, ldy); break;
        case RSVD_F32: e = gemm_nn_typed<float, float>(handle->stream, arith, m, K, c, A, lda, X, ldx, Y, ldy); break;
        case RSVD_BF16: e = gemm_nn_typed<bf16_t, float>(handle->stream, arith, m, K, c, A, lda, X, ldx, Y, ldy); break;
        default: return RSVD_ERR_UNSUPPORTED;
    }
    return hip_status(handle, e);
}

}  // extern "C"

template <typename TA, typename TC>
static hipError_t gemm_tn_typed(rsvd_handle_t h, int arith, const Plan& P, int64_t m, int64_t n, int c, const void* A,
                                int64_t lda, const void* Q, int64_t ldq, void* Z, int64_t ldz, void* work) {
    SingleExec ex{h->stream};
    const int S = P.sp.tn;
    TC* part = at<TC>(work, P.part);
    if (S == 1)
        return gemm_step<TA, TC, MODE_TN>(ex, arith, 0, static_cast<const TA*>(A), lda, n, m,
                                          static_cast<const TC*>(Q), ldq, c, static_cast<TC*>(Z), ldz, 1, 0, nullptr,
                                          nullptr, 0);
    RSVD_TRY((gemm_step<TA, TC, MODE_TN>(ex, arith, 0, static_cast<const TA*>(A), lda, n, m,
                                        static_cast<const TC*>(Q), ldq, c, part, P.Lp, S,
                                        static_cast<int64_t>(n) * P.Lp, nullptr, nullptr, 0)));
    return reduce_step<TC>(ex, part, S, static_cast<int64_t>(n) * P.Lp, P.Lp, n, c, static_cast<TC*>(Z), ldz);
}

extern "C" {

int rsvd_gemm_tn(rsvd_handle_t handle, int32_t dtype, int32_t arith, int64_t m, int64_t n, int32_t c,
                 const void* A, int64_t lda, const void* Q, int64_t ldq, void* Z, int64_t ldz, void* work,
                 size_t work_bytes) {
    if (!handle || m < 1 || n < 1 || c < 1 || c > RSVD_MAX_L || !A || !Q || !Z || !work) return RSVD_ERR_INVALID;
    if (lda < n || ldq < c || ldz < c || arith < 0 || arith > 2) return RSVD_ERR_INVALID;
    if (arith != 0 && dtype == RSVD_F64) return RSVD_ERR_UNSUPPORTED;
    const Plan P = block_plan(dtype, m, n, c, handle->dev.num_cu);
    if (work_bytes < P.bytes) return RSVD_ERR_INVALID;
    hipError_t e;
    switch (dtype) {
        case RSVD_F64: e = gemm_tn_typed<double, double>(handle, arith, P, m, n, c, A, lda, Q, ldq, Z, ldz, work); break;
        case RSVD_F32: e = gemm_tn_typed<float, float>(handle, arith, P, m, n, c, A, lda, Q, ldq, Z, ldz, work); break;
        case RSVD_BF16: e = gemm_tn_typed<bf16_t, float>(handle, arith, P, m, n, c, A, lda, Q, ldq, Z, ldz, work); break;
        default: return RSVD_ERR_UNSUPPORTED;
    }
    return hip_status(handle, e);
}

int rsvd_orthonormalize(rsvd_handle_t handle, int32_t dtype, int64_t m, int32_t c, void* Y, int64_t ldy,
                        double* R, uint32_t* flags, void* work, size_t work_bytes) {
    if (!handle || m < 1 || c < 1 || c > RSVD_MAX_L || c > m || !Y || ldy < c || !R || !work)
        return RSVD_ERR_INVALID;
    if (dtype != RSVD_F64 && dtype != RSVD_F32) return RSVD_ERR_UNSUPPORTED;
    const Plan P = block_plan(dtype, m, m, c, handle->dev.num_cu);
    if (work_bytes < P.bytes) return RSVD_ERR_INVALID;
    hipStream_t st = handle->stream;
    SingleExec ex{st};
    uint32_t* status = at<uint32_t>(work, P.status);
    hipError_t e = ex.run<ClearBody>(ClearBody::Args{status, 1});
    const int S = gram_split(m, handle->dev.num_cu);
    if (e == hipSuccess) {
        if (dtype == RSVD_F64)
            e = orthonormalize<double>(ex, 0, static_cast<double*>(Y), ldy, m, c, P.Lp, S, at<double>(work, P.part),
                                       at<double>(work, P.gram), at<double>(work, P.rinv), at<double>(work, P.racc),
                                       status);
        else
            e = orthonormalize<float>(ex, 0, static_cast<float*>(Y), ldy, m, c, P.Lp, S, at<double>(work, P.part),
                                      at<double>(work, P.gram), at<float>(work, P.rinv), at<double>(work, P.racc),
                                      status);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(R, at<double>(work, P.racc) + 3 * static_cast<size_t>(c) * c,
                           static_cast<size_t>(c) * c * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && flags) e = hipMemcpyAsync(flags, status, sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    return hip_status(handle, e);
}

int rsvd_small_svd(rsvd_handle_t handle, int32_t c, const double* R, double* s, double* W, double* J,
                   uint32_t* flags, void* work, size_t work_bytes) {
    if (!handle || c < 1 || c > RSVD_MAX_L || !R || !s || !W || !J || !work) return RSVD_ERR_INVALID;
    const Plan P = block_plan(RSVD_F64, c, c, c, handle->dev.num_cu);
    if (work_bytes < P.bytes) return RSVD_ERR_INVALID;
    hipStream_t st = handle->stream;
    SingleExec ex{st};
    uint32_t* status = at<uint32_t>(work, P.status);
    hipError_t e = ex.run<ClearBody>(ClearBody::Args{status, 1});
    if (e != hipSuccess) return hip_status(handle, e);
    JacobiArgs ja;
    ja.R = R; ja.ldr = c; ja.l = c; ja.k = c;
    double* wks = at<double>(work, P.gram);
    ja.sigma = s; ja.xv = W; ja.ldx = c; ja.xcols = c; ja.wks = wks;
    ja.status = status; ja.max_sweeps = 60; ja.tol = jacobi_tol(ja.l);
    e = ex.run<JacobiBody<double>>(ja);
    if (e == hipSuccess)
        e = gemm_plain<double, double, double, MODE_TN>(ex, 0, R, c, c, c, wks, c, c, J, c, 1, 0, nullptr, nullptr, 0);
    if (e == hipSuccess && flags) e = hipMemcpyAsync(flags, status, sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    return hip_status(handle, e);
}

}  // extern "C"

// ---------------------------------------------------------------- batches
// A ragged batch runs every step of the solve as one grouped launch over all
// of its matrices (exec.hpp).  Matrices are grouped by the output tile width
// their sketch width needs (32, 64, 128 columns), each group runs its solves
// as one sequence of grouped launches, largest group tile first, and inside a
// group the matrices are ordered by descending work (m n l) so that the
// largest tiles are dispatched first.

namespace rsvd {

struct BatchGroup {
    int tile = 0;
    std::vector<int> members;
    BatchRecorder rec;
    size_t table_off = 0;
};

}  // namespace rsvd

struct rsvd_batch_s {
    rsvd_handle_t h = nullptr;
    int dtype = 0;
    int flags = 0;
    rsvd_params prm{};
    std::vector<rsvd_batch_desc> desc;
    std::vector<rsvd::Plan> plans;
    std::vector<size_t> offs;
    std::vector<rsvd::BatchGroup> groups;
    size_t stamps_off = 0, bytes = 0;
    void* work = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace rsvd {

template <typename TA, typename TC>
hipError_t record_group(rsvd_batch_s* B, BatchGroup& g, void* base) {
    g.rec.clear();
    const bool stamps = (B->flags & RSVD_BATCH_STAMPS) != 0;
    for (int i : g.members) {
        const rsvd_batch_desc& d = B->desc[i];
        SolveOut o{};
        o.U = d.U; o.ldu = d.ldu; o.V = d.V; o.ldv = d.ldv; o.S = d.S; o.info = d.info;
        o.stamps = stamps ? at<uint64_t>(base, B->stamps_off) + 2 * static_cast<size_t>(i) : nullptr;
        g.rec.begin_problem();
        RSVD_TRY((solve_steps<TA, TC>(g.rec, nullptr, B->plans[i], static_cast<const TA*>(d.A), d.lda, &B->prm,
                                      d.stream_id, o, at<unsigned char>(base, B->offs[i]))));
        if (!g.rec.complete()) return hipErrorInvalidValue;
    }
    return hipSuccess;
}

inline hipError_t record_all(rsvd_batch_s* B, void* base) {
    for (BatchGroup& g : B->groups) {
        hipError_t e = hipErrorInvalidValue;
        switch (B->dtype) {
            case RSVD_F64: e = record_group<double, double>(B, g, base); break;
            case RSVD_F32: e = record_group<float, float>(B, g, base); break;
            case RSVD_BF16: e = record_group<bf16_t, float>(B, g, base); break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

inline hipError_t launch_all(const rsvd_batch_s* B, hipStream_t st) {
    for (const BatchGroup& g : B->groups)
        RSVD_TRY(g.rec.launch(static_cast<unsigned char*>(B->work) + g.table_off, st));
    return hipSuccess;
}

inline void drop_graph(rsvd_batch_s* B) {
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
}

}  // namespace rsvd

extern "C" {

int rsvd_batch_create(rsvd_handle_t handle, int32_t dtype, int32_t count, const rsvd_batch_desc* descs,
                      const rsvd_params* params, int32_t flags, rsvd_batch_t* batch, size_t* work_bytes) {
    if (!handle || count < 1 || !descs || !params || !batch || !work_bytes) return RSVD_ERR_INVALID;
    if (flags & ~(RSVD_BATCH_GRAPH | RSVD_BATCH_STAMPS)) return RSVD_ERR_INVALID;
    const bool with_u = descs[0].U != nullptr;
    for (int32_t i = 0; i < count; ++i) {
        const rsvd_batch_desc& d = descs[i];
        const int v = validate(dtype, d.m, d.n, d.k, params);
        if (v != RSVD_OK) return v;
        if (!d.A || d.lda < d.n || !d.S) return RSVD_ERR_INVALID;
        if ((d.U != nullptr) != with_u || (d.U && d.ldu < d.k) || (d.V && d.ldv < d.k)) return RSVD_ERR_INVALID;
    }
    rsvd_batch_s* B = new rsvd_batch_s();
    B->h = handle; B->dtype = dtype; B->flags = flags; B->prm = *params;
    B->desc.assign(descs, descs + count);
    B->plans.resize(count);
    for (int32_t i = 0; i < count; ++i)
        B->plans[i] = make_plan(dtype, descs[i].m, descs[i].n, descs[i].k, params, handle->dev.num_cu, true);
    for (int tile : {128, 64, 32}) {
        BatchGroup g;
        g.tile = tile;
        for (int32_t i = 0; i < count; ++i)
            if (B->plans[i].Lp == tile) { B->plans[i].tile = tile; g.members.push_back(i); }
        if (g.members.empty()) continue;
        std::stable_sort(g.members.begin(), g.members.end(), [&](int a, int b) {
            const Plan &pa = B->plans[a], &pb = B->plans[b];
            return static_cast<double>(pa.m) * pa.n * pa.l > static_cast<double>(pb.m) * pb.n * pb.l;
        });
        B->groups.push_back(std::move(g));
    }
    // Size the step tables with a dry recording (their size does not depend
    // on the addresses recorded in them).
    void* fake = reinterpret_cast<void*>(static_cast<uintptr_t>(1) << 44);
    B->offs.assign(count, 0);
    if (record_all(B, fake) != hipSuccess) { delete B; return RSVD_ERR_UNSUPPORTED; }
    Layout L;
    for (BatchGroup& g : B->groups) g.table_off = L.take(g.rec.packed_bytes());
    B->stamps_off = L.take(2 * sizeof(uint64_t) * static_cast<size_t>(count));
    for (int32_t i = 0; i < count; ++i) B->offs[i] = L.take(B->plans[i].bytes);
    B->bytes = L.off;
    *batch = B;
    *work_bytes = B->bytes;
    return RSVD_OK;
}

int rsvd_batch_bind(rsvd_batch_t batch, void* work, size_t work_bytes) {
    if (!batch || !work || work_bytes < batch->bytes) return RSVD_ERR_INVALID;
    if (reinterpret_cast<uintptr_t>(work) % kAlign != 0) return RSVD_ERR_INVALID;
    rsvd_handle_t h = batch->h;
    drop_graph(batch);
    batch->work = nullptr;
    hipError_t e = record_all(batch, work);
    if (e != hipSuccess) return RSVD_ERR_UNSUPPORTED;
    for (BatchGroup& g : batch->groups) {
        e = g.rec.upload(static_cast<unsigned char*>(work) + g.table_off, h->stream);
        if (e == hipSuccess) e = g.rec.prepare();
        if (e != hipSuccess) return hip_status(h, e);
    }
    batch->work = work;
    if (batch->flags & RSVD_BATCH_GRAPH) {
        if (!batch->cap) {
            e = hipStreamCreateWithFlags(&batch->cap, hipStreamNonBlocking);
            if (e != hipSuccess) { batch->work = nullptr; return hip_status(h, e); }
        }
        e = hipStreamBeginCapture(batch->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t le = launch_all(batch, batch->cap);
            e = hipStreamEndCapture(batch->cap, &batch->graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&batch->exec, batch->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) { drop_graph(batch); batch->work = nullptr; return hip_status(h, e); }
    }
    return RSVD_OK;
}

int rsvd_batch_run(rsvd_batch_t batch) {
    if (!batch || !batch->work) return RSVD_ERR_INVALID;
    rsvd_handle_t h = batch->h;
    if (batch->exec) return hip_status(h, hipGraphLaunch(batch->exec, h->stream));
    return hip_status(h, launch_all(batch, h->stream));
}

int rsvd_batch_stamps(rsvd_batch_t batch, uint64_t* host, double* ticks_per_second) {
    if (!batch || !batch->work || !host || !(batch->flags & RSVD_BATCH_STAMPS)) return RSVD_ERR_INVALID;
    rsvd_handle_t h = batch->h;
    const size_t bytes = 2 * sizeof(uint64_t) * batch->desc.size();
    hipError_t e = hipMemcpyAsync(host, static_cast<unsigned char*>(batch->work) + batch->stamps_off, bytes,
                                  hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess && ticks_per_second) {
        int khz = 0;
        e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->dev.device);
        *ticks_per_second = 1e3 * khz;
    }
    return hip_status(h, e);
}

int rsvd_batch_destroy(rsvd_batch_t batch) {
    if (!batch) return RSVD_OK;
    drop_graph(batch);
    if (batch->cap) (void)hipStreamDestroy(batch->cap);
    delete batch;
    return RSVD_OK;
}

}  // extern "C"
