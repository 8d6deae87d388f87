// The steps of one solve (templates over the storage / compute types and the
// executor), compiled once per storage type in its own translation unit.
#pragma once

#include "launch.hpp"
#include "lu.hpp"
#include "plan.hpp"

namespace rsvd {

// Cholesky with inverse for 128 < l <= 256 from the one-block kernel on
// 128-blocks (all f64): R11 = chol(G11); R12 = R11^{-T} G12;
// R22 = chol(G22 - R12^T R12); R^{-1} = [R11^{-1}, -R11^{-1} R12 R22^{-1}; 0, R22^{-1}].
// x: 7 scratch blocks of 128 x 128 f64.  The second block keeps the status
// bits the first one set (shift, breakdown, further passes requested).
template <typename TC, class Ex>
hipError_t chol_blocked(Ex& ex, const CholArgs& ca, double* x) {
    const int l = ca.l, l2 = l - 128;
    const size_t B = 128 * 128;
    double *R11 = x, *I11 = x + B, *R12 = x + 2 * B, *T = x + 3 * B, *R22 = x + 4 * B, *I22 = x + 5 * B,
           *T1 = x + 6 * B;
    const uint32_t need = (ca.pass == 2) ? ST_NEED_P2 : ST_NEED_P3;
    const uint32_t* skip = ca.skip_unless_pending ? ca.status : nullptr;
    CholArgs c1 = ca;
    c1.l = 128; c1.rinv = I11; c1.ldr = 128; c1.rout = R11;
    RSVD_TRY((ex.template run<CholBody<double, CHOL_MAX_L>>(c1)));
    RSVD_TRY((gemm_plain<double, double, double, MODE_TN>(ex, 0, true, I11, 128, 128, 128, ca.part + 128, ca.ldp, l2,
                                                          R12, 128, 1, 0, nullptr, skip, need, ca.gate)));
    RSVD_TRY((gemm_plain<double, double, double, MODE_TN>(ex, 0, true, R12, 128, l2, 128, R12, 128, l2, T, 128, 1, 0,
                                                          nullptr, skip, need, ca.gate)));
    RSVD_TRY(ex.template run<SchurBody>(SchurArgs{ca.part, ca.ldp, T, l2, skip, need, ca.gate}));
    CholArgs c2 = ca;
    c2.part = T; c2.ldp = 128; c2.l = l2; c2.rinv = I22; c2.ldr = 128; c2.rout = R22; c2.keep_flags = 1;
    RSVD_TRY(run_chol<double>(ex, c2));
    RSVD_TRY((gemm_plain<double, double, double, MODE_NN>(ex, 0, true, I11, 128, 128, 128, R12, 128, l2, T1, 128, 1,
                                                          0, nullptr, skip, need, ca.gate)));
    RSVD_TRY((gemm_plain<double, double, double, MODE_NN>(ex, 0, true, T1, 128, 128, l2, I22, 128, l2, T, 128, 1, 0,
                                                          nullptr, skip, need, ca.gate)));
    return ex.template run<CholAssembleBody<TC>>(typename CholAssembleBody<TC>::Args{
        R11, I11, R12, T, R22, I22, l, static_cast<TC*>(ca.rinv), ca.ldr, ca.rout, skip, need, ca.gate});
}

// In-place orthonormalisation of M (rows x l, ld ldm, precision TC):
// CholeskyQR2, with a shifted first pass and a third pass when needed.
// adaptive = true (bases inside the power scheme, whose span is all that the
// next product uses) runs the second pass only when the first pass shows an
// ill-conditioned Gram matrix.
// rfac (optional, f64, 4 consecutive l x l blocks, ld l) receives the factors
// R1, R2, R3 of the three passes in its first three blocks and their product
// R = R3 R2 R1 (M_in = M_out R) in the fourth.  A pass that is skipped on
// the device (the second of an adaptive call, or the third) writes the
// identity as its factor (CholBody, CholAssembleBody), so the product holds
// whichever passes ran.
template <typename TC, class Ex>
hipError_t orthonormalize(Ex& ex, int tile, TC* M, int64_t ldm, int64_t rows, int l, int Lp, int S,
                          double* part, double* gram, TC* rinv, double* rfac, uint32_t* status,
                          bool adaptive = false, Gate gate = {}, double* cholx = nullptr, TC* qtmp = nullptr) {
    for (int pass = 1; pass <= 3; ++pass) {
        const bool conditional = (pass == 3) || (pass == 2 && adaptive);
        const uint32_t* skip = conditional ? status : nullptr;
        const uint32_t need = (pass == 2) ? ST_NEED_P2 : ST_NEED_P3;
        // (l > 128: the blocked Cholesky reads only the blocks on and above the
        // diagonal, so the tile below it is not formed)
        RSVD_TRY((gemm_plain<TC, TC, double, MODE_TN>(ex, 0, true, M, ldm, l, rows, M, ldm, l, part, Lp, S,
                                                      static_cast<int64_t>(Lp) * Lp, nullptr, skip, need, gate,
                                                      nullptr, 0, l > CHOL_MAX_L)));
        // (batch members: the Cholesky adds the S partial Gram matrices itself)
        const bool reduce = S > 1 && Ex::kSingle;
        if (reduce) RSVD_TRY(reduce_step<double>(ex, part, S, static_cast<int64_t>(Lp) * Lp, Lp, l, l, gram, Lp,
                                                 skip, need, gate));
        CholArgs ca;
        ca.part = reduce ? gram : part; ca.S = reduce ? 1 : S;
        ca.part_stride = static_cast<int64_t>(Lp) * Lp; ca.ldp = Lp;
        ca.l = l; ca.mrows = rows; ca.rinv = rinv; ca.ldr = Lp;
        ca.rout = rfac ? rfac + static_cast<size_t>(pass - 1) * l * l : nullptr;
        ca.status = status; ca.pass = pass; ca.skip_unless_pending = conditional; ca.adaptive = adaptive;
        ca.gate = gate;
        ca.keep_flags = 0;
        if (l > CHOL_MAX_L) {
            if (!cholx) return hipErrorInvalidValue;
            RSVD_TRY(chol_blocked<TC>(ex, ca, cholx));
        } else {
            RSVD_TRY(run_chol<TC>(ex, ca));
        }
        // Q = M R^{-1} in place: the streamed kernel takes it when the product
        // is large (one workgroup owns whole rows and writes them after its
        // last read of them; R^{-1} is packed k-contiguous into the Gram
        // scratch, free once the factor is formed).
        if constexpr (std::is_same<TC, float>::value) {
            const hipError_t e = gemm_streamed<TC, MODE_NN>(ex, 0, M, ldm, rows, l, rinv, Lp, l, M, ldm, 1, 0, nullptr,
                                                            skip, need, gate, XPack{},
                                                            reinterpret_cast<float*>(gram), Lp);
            if (e == hipSuccess) continue;
            if (e != hipErrorNotSupported) return e;
        }
        // Otherwise in place is safe while one column tile holds all l
        // columns (each workgroup reads its rows before writing them); with
        // two tiles (l > 128) one tile's writes would race the other's reads,
        // so the product goes through qtmp (rows x Lp) and is copied back.
        TC* out = M;
        int64_t ldo = ldm;
        if (l > CHOL_MAX_L) {
            if (!qtmp) return hipErrorInvalidValue;
            out = qtmp;
            ldo = Lp;
        }
        RSVD_TRY((gemm_plain<TC, TC, TC, MODE_NN>(ex, tile, false, M, ldm, rows, l, rinv, Lp, l, out, ldo, 1, 0,
                                                  nullptr, skip, need, gate)));
        if (out != M)
            RSVD_TRY(ex.template run<CopyColsBody<TC>>(typename CopyColsBody<TC>::Args{
                out, ldo, M, ldm, rows, l, skip, need, gate}));
    }
    if (rfac) {   // R = R3 (R2 R1); the product R2 R1 goes through the gram scratch
        const size_t ll = static_cast<size_t>(l) * l;
        RSVD_TRY((gemm_plain<double, double, double, MODE_NN>(ex, 0, true, rfac + ll, l, l, l, rfac, l, l, gram, l, 1,
                                                              0, nullptr, nullptr, 0)));
        RSVD_TRY((gemm_plain<double, double, double, MODE_NN>(ex, 0, true, rfac + 2 * ll, l, l, l, gram, l, l,
                                                              rfac + 3 * ll, l, 1, 0, nullptr, nullptr, 0)));
    }
    return hipSuccess;
}

// Pivoted LU normalisation of M (rows x l <= LU_MAX_L) in place, M <- L with
// M = L U (Alg. normalized_iter; tournament pivoting, see lu.hpp).  cand:
// 2 cdiv(rows, LU_ROWS) l ints, cnt: 2 cdiv(rows, LU_ROWS) ints; uinv: U^-1
// (ld Lp, compute type); uout / piv: optional U (f64, ld l) and pivot rows.
template <typename TC, class Ex>
hipError_t lu_normalize(Ex& ex, int tile, TC* M, int64_t ldm, int64_t rows, int l, int Lp, int32_t* cand,
                        int32_t* cnt, TC* uinv, uint32_t* status, double* uout = nullptr, int32_t* piv = nullptr) {
    if (l > LU_MAX_L || l > rows) return hipErrorInvalidValue;
    const int64_t leaves = cdiv(rows, LU_ROWS);
    int32_t *cin = cand, *nin = cnt, *cout = cand + leaves * l, *nout = cnt + leaves;
    typedef typename LuSelectBody<TC>::Args SelArgs;
    RSVD_TRY(ex.template run<LuSelectBody<TC>>(SelArgs{M, ldm, rows, l, nullptr, nullptr, 0, 0, cin, nin}));
    const int G = LU_ROWS / l;                       // >= 2 lists per merge
    for (int64_t count = leaves; count > 1; count = cdiv(count, G)) {
        RSVD_TRY(ex.template run<LuSelectBody<TC>>(SelArgs{M, ldm, rows, l, cin, nin, static_cast<int>(count), G,
                                                           cout, nout}));
        std::swap(cin, cout);
        std::swap(nin, nout);
    }
    RSVD_TRY(ex.template run<LuFinalBody<TC>>(typename LuFinalBody<TC>::Args{M, ldm, l, cin, uout, uinv, Lp, piv,
                                                                             status}));
    // L = M U^-1 in place (one column tile holds all l <= 128 columns)
    return gemm_plain<TC, TC, TC, MODE_NN>(ex, tile, false, M, ldm, rows, l, uinv, Lp, l, M, ldm, 1, 0, nullptr,
                                           nullptr, 0);
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

// Every step of one solve, issued through the executor: launched at once for
// a single solve, or recorded as this problem's share of grouped batch steps.
// prof (may be null) receives the event timings of the products with A.
template <typename TA, typename TC, class Ex>
hipError_t solve_steps(Ex& ex, rsvd_handle_t prof, const Plan& P, const TA* A, int64_t lda,
                       const rsvd_params* prm, uint32_t stream_id, const SolveOut& o, void* work) {
    const int64_t m = P.m, n = P.n;
    const int l = P.l, Lp = P.Lp, k = P.k;
    const int tile = P.tile | (P.var_nn << 16), tile_tn = P.tile | (P.var_tn << 16);
    uint32_t* status = at<uint32_t>(work, P.status);
    TC* Y = o.y0 ? const_cast<TC*>(static_cast<const TC*>(o.y0)) : at<TC>(work, P.Y);
    TC* Z = at<TC>(work, P.Z);
    TC* Om = at<TC>(work, P.Om);
    TC* partc = at<TC>(work, P.part);
    double* partd = at<double>(work, P.part);
    double* gram = at<double>(work, P.gram);
    const int gsm = Ex::kSingle ? P.sp.gram_m : P.fold_m, gsn = Ex::kSingle ? P.sp.gram_n : P.fold_n;
    TC* rinv = at<TC>(work, P.rinv);
    double* racc = at<double>(work, P.racc);
    double* sigma = at<double>(work, P.sigma);
    TC* xv = at<TC>(work, P.xv);
    TC* xu = at<TC>(work, P.xu);
    double* jk = at<double>(work, P.jk);
    double* mu = o.center ? at<double>(work, P.mu) : nullptr;
    double* dinv = o.scale ? at<double>(work, P.cinv) : nullptr;      // scaled PCA: D^-1
    if (dinv && P.gated) return hipErrorInvalidValue;   // (a gated step may issue a product twice)
    double* cholx = P.cholx ? at<double>(work, P.cholx) : nullptr;     // l > 128
    TC* qtmp = P.qtmp ? at<TC>(work, P.qtmp) : nullptr;                   // l > 128

    // Batch members run their group's qmax iterations with the ones beyond
    // their own q switched off by the iteration word (status[1]).
    const bool gated = P.gated;
    const int qmax = gated ? P.qmax : P.q;
    const uint32_t* itw = status + 1;
    const int stamp_sel = o.stamp_sel ? o.stamp_sel : 3;
    if (o.stamps && (stamp_sel & 1)) RSVD_TRY(ex.template run<StampBody>(StampBody::Args{o.stamps}));
    RSVD_TRY(ex.template run<ClearBody>(ClearBody::Args{status, gated ? 2 : 1, iteration_word(P.q, qmax), o.qsrc,
                                                        qmax}));

    if (mu || dinv || o.total_var) {
        // column means (implicit centring, Sec. 4.2), root mean squares
        // (scaling, Sec. 4.3) and variances, in one pass over A
        const int S = P.sp.colsum;
        double* mp = at<double>(work, P.mupart);
        double* var = o.total_var ? at<double>(work, P.cvar) : nullptr;
        RSVD_TRY(ex.template run<ColsumBody<TA>>(typename ColsumBody<TA>::Args{A, lda, m, n, cdiv(m, S), S, mp}));
        RSVD_TRY(ex.template run<ColmeanBody>(ColmeanBody::Args{mp, S, m, n, o.center, mu, dinv, var,
                                                                dinv ? at<double>(work, P.cscl) : nullptr,
                                                                status}));
        if (var) RSVD_TRY(ex.template run<TotalVarBody>(TotalVarBody::Args{var, n, at<double>(work, P.tvar)}));
    }
    // Scaled PCA works on (A - 1 mu^T) D^-1 without forming it: the skinny
    // operand of A X is scaled first (D^-1 X), the result of A^T Y after.
    auto scale_rows = [&](TC* M, int cols, int64_t ldm) -> hipError_t {
        if (!dinv) return hipSuccess;
        return ex.template run<ScaleRowsVecBody<TC>>(typename ScaleRowsVecBody<TC>::Args{M, ldm, n, cols, dinv});
    };

    // Alg. rqb: Omega and the sketch Y = A Omega (unless a wider
    // sketch under the same seed and stream already holds it in its leading
    // l columns: Omega's entries do not depend on l).
    if (!o.y0)
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
    const XPack xp{P.ldxp ? at<uint16_t>(work, P.xpack) : nullptr, P.ldxp, P.xplane};   // bf16 products
    TC* xk = P.ldxk ? at<TC>(work, P.xk) : nullptr;                                     // storage-precision products
    const StreamTail tail = (P.tailslot && !gated)                                      // streamed products
        ? StreamTail{at<float>(work, P.tailslot), tail_slot_bytes(P.ncu, Lp), P.ncu} : StreamTail{};
    auto ax = [&](const TC* X, int arith, Gate gt) -> hipError_t {     // Y (m x Lp) = A X
        const int S = P.sp.nn;
        RSVD_TRY(scale_rows(const_cast<TC*>(X), l, Lp));
        if (S == 1)
            return timed(prof, 0, pass_flops, nn_bytes, [&] {
                return gemm_step<TA, TC, MODE_NN>(ex, arith, tile, A, lda, m, n, X, Lp, l, Y, Lp, 1, 0, mu,
                                                  nullptr, 0, gt, xp, xk, P.ldxk, tail);
            });
        RSVD_TRY(timed(prof, 0, pass_flops, nn_bytes, [&] {
            return gemm_step<TA, TC, MODE_NN>(ex, arith, tile, A, lda, m, n, X, Lp, l, partc, Lp, S,
                                              static_cast<int64_t>(m) * Lp, mu, nullptr, 0, gt, xp, xk, P.ldxk, tail);
        }));
        return reduce_step<TC>(ex, partc, S, static_cast<int64_t>(m) * Lp, Lp, m, l, Y, Lp, nullptr, 0, gt);
    };
    // The last sketch of a member (after its q-th iteration) uses the late
    // arithmetic; with gates both variants are issued and the iteration word
    // picks one per member.
    auto ax_step = [&](const TC* X, bool last_if_ungated, uint32_t early_bit, uint32_t late_bit) -> hipError_t {
        if (!gated) return ax(X, last_if_ungated ? late : early, Gate{});
        if (early == late) return ax(X, early, Gate{itw, early_bit | late_bit});
        RSVD_TRY(ax(X, early, Gate{itw, early_bit}));
        return ax(X, late, Gate{itw, late_bit});
    };
    if (!o.y0) RSVD_TRY(ax_step(Om, P.q == 0, IT_QPOS, IT_Q0));

    if (o.features) {
        // Selector inputs: the singular values of the sketch, from the
        // eigenvalues of its f64 Gram matrix (one pass; the features need the
        // spectrum only, as f32 ratios to the largest).
        const int S = P.sp.gram_m;
        RSVD_TRY((gemm_plain<TC, TC, double, MODE_TN>(ex, 0, true, Y, Lp, l, m, Y, Lp, l, partd, Lp, S,
                                                      static_cast<int64_t>(Lp) * Lp, nullptr, nullptr, 0)));
        if (S > 1) RSVD_TRY(reduce_step<double>(ex, partd, S, static_cast<int64_t>(Lp) * Lp, Lp, l, l, gram, Lp));
        RSVD_TRY(run_gram_eig(ex, GramEigArgs{(S > 1) ? gram : partd, Lp, l, sigma}));
        RSVD_TRY(ex.template run<FeatureBody>(FeatureBody::Args{sigma, l, m, n, o.feat_k, o.features}));
        if (o.stamps && (stamp_sel & 2)) RSVD_TRY(ex.template run<StampBody>(StampBody::Args{o.stamps + 1}));
        return hipSuccess;
    }

    auto aty = [&](TC* dst, int arith, Gate gt) -> hipError_t {     // dst (n x Lp) = A^T Y
        const int S = P.sp.tn;
        if (S == 1) {
            RSVD_TRY(timed(prof, 1, pass_flops, tn_bytes, [&] {
                return gemm_step<TA, TC, MODE_TN>(ex, arith, tile_tn, A, lda, n, m, Y, Lp, l, dst, Lp, 1, 0, mu,
                                                  nullptr, 0, gt, xp, xk, P.ldxk, tail);
            }));
            return scale_rows(dst, l, Lp);
        }
        RSVD_TRY(timed(prof, 1, pass_flops, tn_bytes, [&] {
            return gemm_step<TA, TC, MODE_TN>(ex, arith, tile_tn, A, lda, n, m, Y, Lp, l, partc, Lp, S,
                                              static_cast<int64_t>(n) * Lp, mu, nullptr, 0, gt, xp, xk, P.ldxk, tail);
        }));
        RSVD_TRY(reduce_step<TC>(ex, partc, S, static_cast<int64_t>(n) * Lp, Lp, n, l, dst, Lp, nullptr, 0, gt));
        return scale_rows(dst, l, Lp);
    };

    // Alg. subspace_iter: q rounds of orth(Y); Z = orth(A^T Y); Y = A Z
    // (Alg. normalized_iter: the pivoted LU factor L in place of orth).
    const bool lu = prm->scheme == RSVD_SCHEME_LU;
    if (lu && (gated || l > LU_MAX_L)) return hipErrorInvalidValue;
    int32_t* lucand = lu ? at<int32_t>(work, P.lucand) : nullptr;
    int32_t* lucnt = lu ? at<int32_t>(work, P.lucnt) : nullptr;
    for (int it = 0; it < qmax; ++it) {
        const uint32_t run_bit = 1u << it, last_bit = 1u << (IT_LAST_SHIFT + it);
        const Gate act = gated ? Gate{itw, run_bit | last_bit} : Gate{};
        if (lu)
            RSVD_TRY(lu_normalize<TC>(ex, tile, Y, Lp, m, l, Lp, lucand, lucnt, rinv, status));
        else
            RSVD_TRY(orthonormalize<TC>(ex, tile, Y, Lp, m, l, Lp, gsm, partd, gram, rinv, nullptr, status,
                                        true, act, cholx, qtmp));
        RSVD_TRY(aty(Z, early, act));
        if (lu)
            RSVD_TRY(lu_normalize<TC>(ex, tile, Z, Lp, n, l, Lp, lucand, lucnt, rinv, status));
        else
            RSVD_TRY(orthonormalize<TC>(ex, tile, Z, Lp, n, l, Lp, gsn, partd, gram, rinv, nullptr, status,
                                        true, act, cholx, qtmp));
        RSVD_TRY(ax_step(Z, it == P.q - 1, run_bit, last_bit));
    }
    // Alg. rqb: Q = qr(Y); B^T = A^T Q.
    RSVD_TRY(orthonormalize<TC>(ex, tile, Y, Lp, m, l, Lp, gsm, partd, gram, rinv, nullptr, status, false,
                                Gate{}, cholx, qtmp));
    RSVD_TRY(aty(Z, late, Gate{}));
    if (o.bt) {   // the QB decomposition's B is the product (ID / CUR work on it)
        RSVD_TRY(ex.template run<CopyColsBody<TC>>(typename CopyColsBody<TC>::Args{
            Z, Lp, static_cast<TC*>(o.bt), o.ldbt, n, l, nullptr, 0, Gate{}}));
        if (o.stamps && (stamp_sel & 2)) RSVD_TRY(ex.template run<StampBody>(StampBody::Args{o.stamps + 1}));
        return hipSuccess;
    }
    // svd(B): B^T = Q_b R_b (Q_b overwrites Z), R_b = W S J^T by Jacobi.
    RSVD_TRY(orthonormalize<TC>(ex, tile, Z, Lp, n, l, Lp, gsn, partd, gram, rinv, racc, status, false,
                                Gate{}, cholx, qtmp));
    racc += 3 * static_cast<size_t>(l) * l;       // R_b = R3 R2 R1
    {
        JacobiArgs ja;
        ja.R = racc; ja.ldr = l; ja.l = l; ja.k = k;
        double* wks = at<double>(work, P.wks);
        ja.sigma = sigma; ja.xv = xv; ja.ldx = Lp; ja.xcols = P.kp; ja.wks = wks;
        // f32 outputs: pairs are rotated down to |cos| <= 1e-8, below f32
        // rounding of the vectors; the singular values' error from the
        // remaining cosines is second order (~1e-16 relative).  f64 outputs
        // go to the rounding floor l u.
        ja.status = status; ja.max_sweeps = 60;
        ja.tol = sizeof(TC) == 4 ? std::max(1e-8, jacobi_tol(ja.l)) : jacobi_tol(ja.l);
        ja.wglob = P.wglob ? at<double>(work, P.wglob) : nullptr;
        ja.rot = nullptr; ja.outer = 0;
        if (l > CHOL_MAX_L) {
            // block sweeps over W in global memory, then the one-workgroup
            // kernel only normalises, sorts and writes the outputs
            uint32_t* rot = at<uint32_t>(work, P.jrot);
            const int ldw = jacobi_ldw(l), bs = static_cast<int>(cdiv(l, JB));
            RSVD_TRY(ex.template run<JacobiPrepBody>(JacobiPrepArgs{racc, l, l, ja.wglob, ldw, rot, kJacobiRotWords}));
            RSVD_TRY(ex.template run<JacobiBlockBody>(JacobiBlockArgs{ja.wglob, ldw, l, bs, rot, ja.tol}));
            ja.rot = rot; ja.outer = kJacobiOuter;
        }
        RSVD_TRY(run_jacobi<TC>(ex, ja));
        // J_k = R_b^T (W_k / sigma)
        RSVD_TRY((gemm_plain<double, double, double, MODE_TN>(ex, 0, true, racc, l, l, l, wks, k, k, jk, k, 1, 0,
                                                              nullptr, nullptr, 0)));
    }
    // V = Q_b W_k, sign rule, then U = Q (J_k D) with D = signs (x S for PCA).
    TC* V = o.V ? static_cast<TC*>(o.V) : at<TC>(work, P.vtmp);
    const int64_t ldv = o.V ? o.ldv : P.kp;
    RSVD_TRY((gemm_plain<TC, TC, TC, MODE_NN>(ex, tile, false, Z, Lp, n, l, xv, P.kp, k, V, ldv, 1, 0, nullptr, nullptr,
                                              0)));
    RSVD_TRY(ex.template run<SignLiftBody<TC>>(typename SignLiftBody<TC>::Args{
        V, ldv, n, l, k, jk, sigma, o.scale_u, xu, Lp, P.kp}));
    // PCA: x = U S lands in the whitened output when only that is wanted
    // (scaled in place below)
    TC* xout = static_cast<TC*>(o.U ? o.U : o.xwhite);
    const int64_t ldxo = o.U ? o.ldu : o.ldxw;
    if (xout)
        RSVD_TRY((gemm_plain<TC, TC, TC, MODE_NN>(ex, tile, false, Y, Lp, m, l, xu, P.kp, k, xout, ldxo, 1, 0,
                                                  nullptr, nullptr, 0)));
    // A-posteriori bound from r Gaussian probes w (Halko, Martinsson & Tropp
    // 2011, Sec. 4.3): one more pass over A for A w, then U (S (V^T w)).
    double* est = nullptr;
    if (P.probes > 0) {
        const int r = P.probes;
        TC* eOm = at<TC>(work, P.eOm);
        TC* eY = at<TC>(work, P.eY);
        TC* eT = at<TC>(work, P.eT);
        TC* eW = at<TC>(work, P.eW);
        double* epart = at<double>(work, P.epart);
        est = at<double>(work, P.est);
        const TC* Uu = static_cast<const TC*>(o.U);
        int64_t ldu = o.ldu;
        if (!o.U) {
            RSVD_TRY((gemm_plain<TC, TC, TC, MODE_NN>(ex, tile, false, Y, Lp, m, l, xu, P.kp, k, at<TC>(work, P.eU),
                                                      P.kp, 1, 0, nullptr, nullptr, 0)));
            Uu = at<TC>(work, P.eU);
            ldu = P.kp;
        }
        RSVD_TRY(ex.template run<OmegaBody<TC>>(typename OmegaBody<TC>::Args{
            n, r, 32, prm->seed, stream_id ^ 0x80000000u, RSVD_NORMAL, eOm, 32}));
        RSVD_TRY(scale_rows(eOm, r, 32));        // (A - 1 mu^T) D^-1 w
        RSVD_TRY((gemm_step<TA, TC, MODE_NN>(ex, late, 32, A, lda, m, n, eOm, 32, r, eY, 32, 1, 0, mu, nullptr, 0,
                                             Gate{}, xp)));
        const int S = P.sp.gram_n;
        if (S == 1) {
            RSVD_TRY((gemm_plain<TC, TC, TC, MODE_TN>(ex, 32, false, V, ldv, k, n, eOm, 32, r, eT, 32, 1, 0, nullptr,
                                                      nullptr, 0)));
        } else {
            TC* tp = reinterpret_cast<TC*>(epart);
            RSVD_TRY((gemm_plain<TC, TC, TC, MODE_TN>(ex, 32, false, V, ldv, k, n, eOm, 32, r, tp, 32, S,
                                                      static_cast<int64_t>(P.kp) * 32, nullptr, nullptr, 0)));
            RSVD_TRY(reduce_step<TC>(ex, tp, S, static_cast<int64_t>(P.kp) * 32, 32, k, r, eT, 32));
        }
        if (!o.scale_u)
            RSVD_TRY(ex.template run<ScaleRowsBody<TC>>(typename ScaleRowsBody<TC>::Args{eT, 32, k, r, sigma}));
        RSVD_TRY((gemm_plain<TC, TC, TC, MODE_NN>(ex, 32, false, Uu, ldu, m, k, eT, 32, r, eW, 32, 1, 0, nullptr,
                                                  nullptr, 0)));
        RSVD_TRY(ex.template run<DiffNormBody<TC>>(typename DiffNormBody<TC>::Args{eY, eW, 32, m, r, P.est_split,
                                                                                  epart}));
        RSVD_TRY(ex.template run<EstBody>(EstBody::Args{epart, P.est_split, r, est}));
    }
    if (o.loadings || o.xwhite)
        RSVD_TRY(ex.template run<PcaOutBody<TC>>(typename PcaOutBody<TC>::Args{
            V, ldv, static_cast<TC*>(o.loadings), o.ldl, n, xout, ldxo, static_cast<TC*>(o.xwhite), o.ldxw, m, k,
            sigma, static_cast<double>(m - 1)}));
    RSVD_TRY(ex.template run<FinalizeBody<TC>>(typename FinalizeBody<TC>::Args{
        sigma, k, o.S, o.eigvals, o.sdev, static_cast<double>(m - 1), mu, n, static_cast<TC*>(o.center_out),
        status, o.info, l, P.q, P.p, est, o.qsrc, dinv ? at<double>(work, P.cscl) : nullptr,
        static_cast<TC*>(o.scale_out), o.total_var ? at<double>(work, P.tvar) : nullptr, o.total_var}));
    if (o.stamps && (stamp_sel & 2)) RSVD_TRY(ex.template run<StampBody>(StampBody::Args{o.stamps + 1}));
    return hipSuccess;
}

// x = ((A - 1 c^T) D^-1) W for new rows A (the predict step of Sec. 4.4):
// the rows of W are divided by the scales once, the centre is subtracted
// while A's tiles are staged (as in the solve), and the n-reduction is split
// like the solve's A X when the row tiles alone would leave the device idle.
template <typename TA, typename TC>
hipError_t predict_steps(rsvd_handle_t h, const PredictPlan& P, const TA* A, int64_t lda, const TC* rot,
                         int64_t ldr, const TC* center, const TC* scale, TC* x, int64_t ldx, void* work) {
    SingleExec ex{h->stream};
    double* mu = center ? at<double>(work, P.mu) : nullptr;
    TC* W = at<TC>(work, P.w);
    RSVD_TRY(ex.template run<PredictPrepBody<TC>>(typename PredictPrepBody<TC>::Args{
        rot, ldr, center, scale, P.n, P.k, P.kp, mu, W}));
    const int tc = tile_class(P.k, sizeof(TC) == 4);
    if (P.S == 1)
        return gemm_step<TA, TC, MODE_NN>(ex, 0, tc, A, lda, P.m, P.n, W, P.kp, P.k, x, ldx, 1, 0, mu, nullptr, 0);
    TC* part = at<TC>(work, P.part);
    const int64_t stride = P.m * P.kp;
    RSVD_TRY((gemm_step<TA, TC, MODE_NN>(ex, 0, tc, A, lda, P.m, P.n, W, P.kp, P.k, part, P.kp, P.S, stride, mu,
                                        nullptr, 0)));
    return reduce_step<TC>(ex, part, P.S, stride, P.kp, P.m, P.k, x, ldx);
}

#define RSVD_DEFINE_SOLVE(NAME, TA, TC)                                                                 \
    hipError_t solve_single_##NAME(rsvd_handle_t h, const Plan& P, const void* A, int64_t lda,         \
                                   const rsvd_params* prm, const SolveOut& o, void* work) {             \
        SingleExec ex{h->stream};                                                                      \
        return solve_steps<TA, TC>(ex, h, P, static_cast<const TA*>(A), lda, prm, prm->stream_id, o,   \
                                   work);                                                              \
    }                                                                                                  \
    hipError_t solve_record_##NAME(BatchRecorder& rec, const Plan& P, const void* A, int64_t lda,      \
                                   const rsvd_params* prm, uint32_t stream_id, const SolveOut& o,       \
                                   void* work) {                                                       \
        return solve_steps<TA, TC>(rec, nullptr, P, static_cast<const TA*>(A), lda, prm, stream_id, o, \
                                   work);                                                              \
    }                                                                                                  \
    hipError_t predict_##NAME(rsvd_handle_t h, const PredictPlan& P, const void* A, int64_t lda,       \
                              const void* rot, int64_t ldr, const void* center, const void* scale,      \
                              void* x, int64_t ldx, void* work) {                                       \
        return predict_steps<TA, TC>(h, P, static_cast<const TA*>(A), lda, static_cast<const TC*>(rot), ldr, \
                                     static_cast<const TC*>(center), static_cast<const TC*>(scale),     \
                                     static_cast<TC*>(x), ldx, work);                                   \
    }

}  // namespace rsvd
