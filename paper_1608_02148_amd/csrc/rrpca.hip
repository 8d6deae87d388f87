// Randomized robust PCA (Alg. rpca, Sec. 5.2): the inexact augmented
// Lagrange multiplier method of Eq. IALM with the randomized SVD as its
// workhorse, A = L + S with L low rank and S sparse.
//
// Per iteration, on the handle's stream:
//   1. U, s, V = rsvd(M, k) with M = A - S + Z / mu (the solve of rsvd_run);
//   2. the host reads s (one synchronisation), counts l = #{s_i > 1/mu} and
//      sets the next target rank (the inexact ALM's rank prediction);
//   3. one fused pass over the m x n matrices (RrpcaUpdateBody):
//      L = U_l diag(s_l - 1/mu) V_l^T formed tile by tile from U and V in LDS,
//      S = shrink(A - L + Z / mu, lambda / mu), R = A - L - S,
//      Z += mu R, M_next = A - S + Z / mu_next, and partial sums of R^2;
//   4. the partial sums reduced in a fixed order; the host reads
//      ||R||_F / ||A||_F (second synchronisation) and stops below tol.
// Start: ||A||_2 from a rank-1 randomized SVD, ||A||_max and ||A||_F from one
// reduction pass, mu = 1.25 / ||A||_2, Z = A / max(||A||_2, ||A||_max /
// lambda), S = 0.  mu grows by rho per iteration up to 1e7 times its start.
#include <cmath>
#include <vector>

#include "plan.hpp"

using namespace rsvd;

namespace {

constexpr int RT = 64;      // output tile (RT x RT elements per workgroup)
constexpr int RK = 32;      // rank chunk staged in LDS

// Partial max |a| and sum a^2 per row block of 64 rows (one workgroup each):
// part[2 b] = max, part[2 b + 1] = sum of squares (rows in order, columns
// strided by the threads, then a fixed tree).
template <typename TC>
struct NormPartBody {
    struct Args { const TC* A; int64_t lda; int64_t m; int64_t n; double* part; };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.m, 64)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        __shared__ double smax[THREADS], ssum[THREADS];
        double mx = 0.0, ss = 0.0;
        const int64_t r0 = static_cast<int64_t>(b) * 64, r1 = min(a.m, r0 + 64);
        for (int64_t r = r0; r < r1; ++r)
            for (int64_t j = threadIdx.x; j < a.n; j += THREADS) {
                const double x = static_cast<double>(a.A[r * a.lda + j]);
                mx = fmax(mx, fabs(x));
                ss += x * x;
            }
        smax[threadIdx.x] = mx;
        ssum[threadIdx.x] = ss;
        __syncthreads();
        for (int off = THREADS / 2; off > 0; off >>= 1) {
            if (static_cast<int>(threadIdx.x) < off) {
                smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
                ssum[threadIdx.x] += ssum[threadIdx.x + off];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) { a.part[2 * b] = smax[0]; a.part[2 * b + 1] = ssum[0]; }
    }
};

// out[c] = reduction over the nb pairs part[2 b + c] (c = 0: max, c = 1: sum)
// in a fixed order.  One workgroup.
struct PairReduceBody {
    struct Args { const double* part; int64_t nb; double* out; };
    static constexpr int THREADS = 256;
    static int blocks(const Args&) { return 1; }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int) {
        __shared__ double smax[THREADS], ssum[THREADS];
        double mx = 0.0, ss = 0.0;
        for (int64_t b = threadIdx.x; b < a.nb; b += THREADS) {
            mx = fmax(mx, a.part[2 * b]);
            ss += a.part[2 * b + 1];
        }
        smax[threadIdx.x] = mx;
        ssum[threadIdx.x] = ss;
        __syncthreads();
        for (int off = THREADS / 2; off > 0; off >>= 1) {
            if (static_cast<int>(threadIdx.x) < off) {
                smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
                ssum[threadIdx.x] += ssum[threadIdx.x + off];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) { a.out[0] = smax[0]; a.out[1] = ssum[0]; }
    }
};

// Z = A / J, M = A + Z / mu (S = 0), S = 0.
template <typename TC>
struct RrpcaInitBody {
    struct Args { const TC* A; int64_t lda; int64_t m; int64_t n; double invJ; double inv_mu; TC* Z; TC* M;
                  TC* S; int64_t lds; };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.m * a.n, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (idx >= a.m * a.n) return;
        const int64_t i = idx / a.n, j = idx - i * a.n;
        const double x = static_cast<double>(a.A[i * a.lda + j]);
        const double z = x * a.invJ;
        a.Z[idx] = static_cast<TC>(z);
        a.M[idx] = static_cast<TC>(x + z * a.inv_mu);
        a.S[i * a.lds + j] = TC(0);
    }
};

// Step 3 above for one RT x RT tile; part[b] = sum of R^2 over the tile
// (threads' sums combined in a fixed tree).  Each thread owns a 4 x 4 block
// of the tile; U (ld ldu) and V (ld ldv) chunks of RK ranks sit in LDS with
// the weights s_t - 1/mu folded into U.
template <typename TC>
struct RrpcaUpdateBody {
    struct Args {
        const TC* A; int64_t lda; TC* L; int64_t ldl; TC* S; int64_t lds; TC* Z; TC* M;
        const TC* U; int ldu; const TC* V; int ldv; const double* sigma; int l;
        int64_t m; int64_t n; double thr; double lam_thr; double mu; double inv_mu_next; double* part;
    };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.m, RT) * cdiv(a.n, RT)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        __shared__ TC us[RK][RT + 1], vs[RK][RT + 1];
        __shared__ double red[THREADS];
        const int64_t tiles_n = cdiv(a.n, RT);
        const int64_t i0 = (b / tiles_n) * RT, j0 = (b % tiles_n) * RT;
        const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;      // 16 x 16 threads, 4 x 4 each
        double acc[4][4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
        for (int t0 = 0; t0 < a.l; t0 += RK) {
            for (int idx = threadIdx.x; idx < RK * RT; idx += THREADS) {
                const int t = idx / RT, r = idx % RT;
                const int64_t gi = i0 + r, gj = j0 + r;
                const bool tv = t0 + t < a.l;
                const double w = tv ? a.sigma[t0 + t] - a.thr : 0.0;
                us[t][r] = static_cast<TC>((tv && gi < a.m) ? static_cast<double>(a.U[gi * a.ldu + t0 + t]) * w : 0.0);
                vs[t][r] = (tv && gj < a.n) ? a.V[gj * a.ldv + t0 + t] : TC(0);
            }
            __syncthreads();
            for (int t = 0; t < RK; ++t) {
                double uu[4], vv[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) uu[p] = static_cast<double>(us[t][ty * 4 + p]);
#pragma unroll
                for (int q = 0; q < 4; ++q) vv[q] = static_cast<double>(vs[t][tx * 4 + q]);
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[p][q] = fma(uu[p], vv[q], acc[p][q]);
            }
            __syncthreads();
        }
        double rsum = 0.0;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int64_t i = i0 + ty * 4 + p;
            if (i >= a.m) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t j = j0 + tx * 4 + q;
                if (j >= a.n) continue;
                const double x = static_cast<double>(a.A[i * a.lda + j]);
                const double Lij = static_cast<double>(static_cast<TC>(acc[p][q]));
                const int64_t e = i * a.n + j;
                const double z = static_cast<double>(a.Z[e]);
                const double y = x - Lij + z * a.thr;
                const double s = (y > a.lam_thr) ? y - a.lam_thr : (y < -a.lam_thr ? y + a.lam_thr : 0.0);
                const double sr = static_cast<double>(static_cast<TC>(s));
                const double r = x - Lij - sr;
                const double zn = static_cast<double>(static_cast<TC>(z + a.mu * r));
                a.L[i * a.ldl + j] = static_cast<TC>(Lij);
                a.S[i * a.lds + j] = static_cast<TC>(sr);
                a.Z[e] = static_cast<TC>(zn);
                a.M[e] = static_cast<TC>(x - sr + zn * a.inv_mu_next);
                rsum += r * r;
            }
        }
        red[threadIdx.x] = rsum;
        __syncthreads();
        for (int off = THREADS / 2; off > 0; off >>= 1) {
            if (static_cast<int>(threadIdx.x) < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) a.part[b] = red[0];
    }
};

// Sum of part[0 .. nb) in a fixed order into *out.  One workgroup.
struct SumReduceBody {
    struct Args { const double* part; int64_t nb; double* out; };
    static constexpr int THREADS = 256;
    static int blocks(const Args&) { return 1; }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int) {
        __shared__ double s[THREADS];
        double acc = 0.0;
        for (int64_t b = threadIdx.x; b < a.nb; b += THREADS) acc += a.part[b];
        s[threadIdx.x] = acc;
        __syncthreads();
        for (int off = THREADS / 2; off > 0; off >>= 1) {
            if (static_cast<int>(threadIdx.x) < off) s[threadIdx.x] += s[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) *a.out = s[0];
    }
};

struct RrpcaPlan {
    int64_t m = 0, n = 0;
    int k_max = 0;
    size_t Z = 0, M = 0, U = 0, V = 0, sigma = 0, part = 0, scal = 0, rs = 0, rs_bytes = 0, bytes = 0;
};

int k_max_of(int64_t m, int64_t n, const rrpca_options* o, const rsvd_params* prm) {
    int64_t km = std::min<int64_t>(std::min(m, n) - 1, RSVD_MAX_L_SINGLE - prm->p);
    if (o->k_max > 0) km = std::min<int64_t>(km, o->k_max);
    return static_cast<int>(km);
}

int rrpca_plan(rsvd_handle_t h, int32_t dtype, int64_t m, int64_t n, const rrpca_options* o,
               const rsvd_params* prm, RrpcaPlan* P) {
    if (dtype != RSVD_F64 && dtype != RSVD_F32) return RSVD_ERR_UNSUPPORTED;
    if (!o || !prm || m < 2 || n < 2 || o->maxiter < 1 || !(o->tol > 0.0) || !(o->rho >= 1.0))
        return RSVD_ERR_INVALID;
    const int km = k_max_of(m, n, o, prm);
    if (km < 1) return RSVD_ERR_INVALID;
    int v = validate(dtype, m, n, km, prm);
    if (v == RSVD_OK) v = validate(dtype, m, n, 1, prm);
    if (v != RSVD_OK) return v;
    if (prm->precision != RSVD_PREC_PLAIN) return RSVD_ERR_UNSUPPORTED;
    const size_t cs = comp_size(dtype);
    P->m = m; P->n = n; P->k_max = km;
    Layout L;
    P->Z = L.take(static_cast<size_t>(m) * n * cs);
    P->M = L.take(static_cast<size_t>(m) * n * cs);
    P->U = L.take(static_cast<size_t>(m) * km * cs);
    P->V = L.take(static_cast<size_t>(n) * km * cs);
    P->sigma = L.take(static_cast<size_t>(km) * 8);
    P->part = L.take(std::max<size_t>(2 * cdiv(m, 64), cdiv(m, RT) * cdiv(n, RT)) * 8);
    P->scal = L.take(4 * 8);
    const size_t ws = std::max(make_plan(dtype, m, n, km, prm, h->dev.num_cu, false, h->variants).bytes,
                               make_plan(dtype, m, n, 1, prm, h->dev.num_cu, false, h->variants).bytes);
    P->rs = L.take(ws);
    P->rs_bytes = ws;
    P->bytes = L.off;
    return RSVD_OK;
}

template <typename TC>
int rrpca_typed(rsvd_handle_t h, const RrpcaPlan& P, int32_t dtype, const TC* A, int64_t lda,
                const rrpca_options* o, const rsvd_params* prm, TC* Lout, int64_t ldl, TC* Sout, int64_t lds,
                void* work, rrpca_result* res) {
    const int64_t m = P.m, n = P.n;
    SingleExec ex{h->stream};
    TC* Z = at<TC>(work, P.Z);
    TC* M = at<TC>(work, P.M);
    TC* U = at<TC>(work, P.U);
    TC* V = at<TC>(work, P.V);
    double* sig = at<double>(work, P.sigma);
    double* part = at<double>(work, P.part);
    double* scal = at<double>(work, P.scal);
    void* rw = at<unsigned char>(work, P.rs);
    auto fail = [&](hipError_t e) { return hip_status(h, e); };
    auto solve = [&](const TC* X, int k, TC* u, TC* v) -> int {
        const Plan sp = make_plan(dtype, m, n, k, prm, h->dev.num_cu, false, h->variants);
        SolveOut so{};
        so.U = u; so.ldu = k; so.V = v; so.ldv = k; so.S = sig;
        return dispatch(h, dtype, sp, X, (X == A) ? lda : n, prm, so, rw);
    };
    const double lam = o->lambda > 0.0 ? o->lambda : 1.0 / std::sqrt(static_cast<double>(std::max(m, n)));
    // ||A||_2 (rank-1 randomized SVD), ||A||_max, ||A||_F
    int st = solve(A, 1, U, V);
    if (st != RSVD_OK) return st;
    const int64_t nb = cdiv(m, 64);
    hipError_t e = ex.run<NormPartBody<TC>>(typename NormPartBody<TC>::Args{A, lda, m, n, part});
    if (e == hipSuccess) e = ex.run<PairReduceBody>(PairReduceBody::Args{part, nb, scal});
    double host[3] = {0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(host, sig, sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host + 1, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(e);
    const double norm2 = host[0], amax = host[1], normF = std::sqrt(host[2]);
    if (!(normF > 0.0) || !std::isfinite(normF) || !(norm2 > 0.0)) return RSVD_ERR_INVALID;
    double mu = o->mu0_scale / norm2;
    const double mu_max = mu * 1e7;
    const double J = std::max(norm2, amax / lam);
    e = ex.run<RrpcaInitBody<TC>>(typename RrpcaInitBody<TC>::Args{A, lda, m, n, 1.0 / J, 1.0 / mu, Z, M, Sout, lds});
    if (e != hipSuccess) return fail(e);
    int k = 2 < P.k_max ? 2 : P.k_max;
    int l = 0, it = 0;
    double resid = INFINITY;
    std::vector<double> s(P.k_max);
    const int64_t ntile = cdiv(m, RT) * cdiv(n, RT);
    for (it = 1; it <= o->maxiter; ++it) {
        const int kk = k;
        st = solve(M, kk, U, V);
        if (st != RSVD_OK) return st;
        e = hipMemcpyAsync(s.data(), sig, kk * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return fail(e);
        const double thr = 1.0 / mu;
        l = 0;
        while (l < kk && s[l] > thr) ++l;
        // next target rank (the inexact ALM's rank prediction)
        int kn = (l < kk) ? l + 1 : l + static_cast<int>(std::lround(0.05 * static_cast<double>(std::min(m, n))));
        k = std::min(std::max(kn, 1), P.k_max);
        const double mu_next = std::min(o->rho * mu, mu_max);
        e = ex.run<RrpcaUpdateBody<TC>>(typename RrpcaUpdateBody<TC>::Args{
            A, lda, Lout, ldl, Sout, lds, Z, M, U, kk, V, kk, sig, l, m, n, thr, lam * thr, mu, 1.0 / mu_next,
            part});
        if (e == hipSuccess) e = ex.run<SumReduceBody>(SumReduceBody::Args{part, ntile, scal + 2});
        if (e == hipSuccess) e = hipMemcpyAsync(host, scal + 2, sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return fail(e);
        mu = mu_next;
        resid = std::sqrt(host[0]) / normF;
        if (resid < o->tol) break;
    }
    if (res) {
        res->iterations = std::min(it, o->maxiter);
        res->rank = l;
        res->k = k;
        res->reserved = 0;
        res->residual = resid;
        res->lambda = lam;
    }
    return RSVD_OK;
}

}  // namespace

extern "C" {

void rrpca_default_options(rrpca_options* o) {
    if (!o) return;
    o->lambda = 0.0;
    o->tol = 1e-5;
    o->rho = 1.6;
    o->mu0_scale = 1.25;
    o->maxiter = 50;
    o->k_max = 0;
}

int rrpca_workspace_size(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const rrpca_options* opt,
                         const rsvd_params* params, size_t* bytes) {
    if (!handle || !bytes) return RSVD_ERR_INVALID;
    RrpcaPlan P;
    const int st = rrpca_plan(handle, dtype, m, n, opt, params, &P);
    if (st != RSVD_OK) return st;
    *bytes = P.bytes;
    return RSVD_OK;
}

int rrpca_run(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
              const rrpca_options* opt, const rsvd_params* params, void* L, int64_t ldl, void* S, int64_t lds,
              void* work, size_t work_bytes, rrpca_result* result) {
    if (!handle) return RSVD_ERR_INVALID;
    RrpcaPlan P;
    const int st = rrpca_plan(handle, dtype, m, n, opt, params, &P);
    if (st != RSVD_OK) return st;
    if (!A || lda < n || !L || ldl < n || !S || lds < n || !work) return RSVD_ERR_INVALID;
    if (reinterpret_cast<uintptr_t>(work) % kAlign != 0 || work_bytes < P.bytes) return RSVD_ERR_INVALID;
    if (dtype == RSVD_F64)
        return rrpca_typed<double>(handle, P, dtype, static_cast<const double*>(A), lda, opt, params,
                                   static_cast<double*>(L), ldl, static_cast<double*>(S), lds, work, result);
    return rrpca_typed<float>(handle, P, dtype, static_cast<const float*>(A), lda, opt, params,
                              static_cast<float*>(L), ldl, static_cast<float*>(S), lds, work, result);
}

}  // extern "C"
