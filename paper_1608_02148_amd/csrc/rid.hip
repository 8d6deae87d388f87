// Randomized interpolative and CUR decompositions (Sec. 6; Alg. id, Alg. rid,
// Alg. rcur) on top of the randomized QB decomposition of Alg. rqb.
//
// rid: the solve of rsvd_run stops at B^T = A^T Q (n x l); the column ID of
// B (l x n) comes from k steps of column-pivoted QR (Businger-Golub: the
// column with the largest remaining norm, Householder reflections in the
// larfg convention), T = S11^-1 S12 by back substitution, Z[:, P] = [I, T]
// and C = A[:, J] with J = P[:k].
// rcur: the same, then k steps of column-pivoted QR of C^T choose the rows
// I, R = A[I, :], and U = Z pinv(R) = (Z Q_r) T_r^-T from the CholeskyQR
// R^T = Q_r T_r (R has full row rank k).
//
// Column-pivoted QR on the device: the matrix is held by columns in f64
// (X[pos][r] = column at position pos, row r), one thread per column.  Step
// j is two launches: CpqrApplyBody applies reflector j - 1 to every column at
// positions >= j and reduces the remaining column norms (rows j..) to one
// candidate per workgroup; CpqrPivotBody picks the largest (lowest position
// on ties), swaps it to position j and forms reflector j.  Norms are
// recomputed from the updated columns at every step (no downdating).
#include <cmath>

#include "solve.hpp"

using namespace rsvd;

namespace {

constexpr int CP_THREADS = 256;

struct CpqrArgs {
    double* X; int64_t ldx; int nr; int64_t nc; int j; double* tau; int32_t* perm; double* partv;
    int32_t* partk;
};

// X[pos][r] = src column pos (src stored with columns contiguous: src[pos * lds + r]), perm = identity.
template <typename TC>
struct CpqrInitBody {
    struct Args { const TC* src; int64_t lds; double* X; int64_t ldx; int nr; int64_t nc; int32_t* perm; };
    static constexpr int THREADS = CP_THREADS;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.nc * a.nr, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (idx >= a.nc * a.nr) return;
        const int64_t c = idx / a.nr;
        const int r = static_cast<int>(idx - c * a.nr);
        a.X[c * a.ldx + r] = static_cast<double>(a.src[c * a.lds + r]);
        if (r == 0) a.perm[c] = static_cast<int32_t>(c);
    }
};

struct CpqrApplyBody {
    typedef CpqrArgs Args;
    static constexpr int THREADS = CP_THREADS;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.nc - a.j, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        __shared__ double sv[CP_THREADS / 64];
        __shared__ int32_t sk[CP_THREADS / 64];
        const int j = a.j;
        const int64_t c = j + static_cast<int64_t>(b) * THREADS + threadIdx.x;
        double v = -1.0;
        int32_t key = INT32_MAX;
        if (c < a.nc) {
            double* x = a.X + c * a.ldx;
            if (j > 0) {           // H_{j-1} = I - tau v v^T on rows j-1.., v_{j-1} = 1
                const double* h = a.X + static_cast<int64_t>(j - 1) * a.ldx;
                const double t = a.tau[j - 1];
                if (t != 0.0) {
                    double w = x[j - 1];
                    for (int r = j; r < a.nr; ++r) w = fma(h[r], x[r], w);
                    w *= t;
                    x[j - 1] -= w;
                    for (int r = j; r < a.nr; ++r) x[r] = fma(-w, h[r], x[r]);
                }
            }
            double s = 0.0;
            for (int r = j; r < a.nr; ++r) s = fma(x[r], x[r], s);
            v = s;
            key = static_cast<int32_t>(c);
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(v, off, 64);
            const int32_t ok = __shfl_xor(key, off, 64);
            if (ov > v || (ov == v && ok < key)) { v = ov; key = ok; }
        }
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) { sv[wave] = v; sk[wave] = key; }
        __syncthreads();
        if (threadIdx.x == 0) {
            v = sv[0]; key = sk[0];
            for (int w = 1; w < THREADS / 64; ++w)
                if (sv[w] > v || (sv[w] == v && sk[w] < key)) { v = sv[w]; key = sk[w]; }
            a.partv[b] = v;
            a.partk[b] = key;
        }
    }
};

// One workgroup: the pivot of step j from the candidates, the swap, and
// reflector j from column j's rows j..nr-1 (beta = -sign(alpha) ||x||, tau =
// (beta - alpha) / beta, v = x / (alpha - beta) stored below the diagonal).
struct CpqrPivotBody {
    typedef CpqrArgs Args;
    static constexpr int THREADS = CP_THREADS;
    static int blocks(const Args&) { return 1; }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int) {
        __shared__ int64_t sp;
        __shared__ double sred[CP_THREADS];
        const int j = a.j;
        const int nb = static_cast<int>(cdiv(a.nc - j, THREADS));
        if (threadIdx.x == 0) {
            double bv = -1.0;
            int32_t bk = j;
            for (int b = 0; b < nb; ++b)
                if (a.partv[b] > bv || (a.partv[b] == bv && a.partk[b] < bk)) { bv = a.partv[b]; bk = a.partk[b]; }
            sp = bk;
        }
        __syncthreads();
        const int64_t p = sp;
        double* xj = a.X + static_cast<int64_t>(j) * a.ldx;
        if (p != j) {
            double* xp = a.X + p * a.ldx;
            for (int r = threadIdx.x; r < a.nr; r += THREADS) {
                const double t = xj[r];
                xj[r] = xp[r];
                xp[r] = t;
            }
            if (threadIdx.x == 0) {
                const int32_t t = a.perm[j];
                a.perm[j] = a.perm[p];
                a.perm[p] = t;
            }
        }
        __syncthreads();
        double s = 0.0;
        for (int r = j + 1 + threadIdx.x; r < a.nr; r += THREADS) s = fma(xj[r], xj[r], s);
        sred[threadIdx.x] = s;
        __syncthreads();
        for (int off = THREADS / 2; off > 0; off >>= 1) {
            if (static_cast<int>(threadIdx.x) < off) sred[threadIdx.x] += sred[threadIdx.x + off];
            __syncthreads();
        }
        const double sigma = sred[0];
        const double alpha = xj[j];
        double beta = alpha, tau = 0.0, scale = 0.0;
        if (sigma != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        __syncthreads();
        for (int r = j + 1 + threadIdx.x; r < a.nr; r += THREADS) xj[r] *= scale;
        if (threadIdx.x == 0) {
            xj[j] = beta;
            a.tau[j] = tau;
        }
    }
};

// T = S11^-1 S12 in place: column c >= k of X holds S12[:, c] in rows 0..k-1
// on entry and t = T[:, c - k] on exit (back substitution against the
// columns 0..k-1, S11[i][t] = X[t][i]); a zero diagonal entry gives t_i = 0.
struct IdCoefBody {
    struct Args { double* X; int64_t ldx; int k; int64_t nc; };
    static constexpr int THREADS = CP_THREADS;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.nc - a.k, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int64_t c = a.k + static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (c >= a.nc) return;
        double* x = a.X + c * a.ldx;
        for (int i = a.k - 1; i >= 0; --i) {
            double s = x[i];
            for (int t = i + 1; t < a.k; ++t) s = fma(-a.X[static_cast<int64_t>(t) * a.ldx + i], x[t], s);
            const double d = a.X[static_cast<int64_t>(i) * a.ldx + i];
            x[i] = (d != 0.0) ? s / d : 0.0;
        }
    }
};

// Z (k x nc, ldz) with Z[:, perm[pos]] = e_pos for pos < k and the
// coefficients t of X[pos] for pos >= k; J[i] = perm[i] for i < k (J may be null).
template <typename TC>
struct IdScatterBody {
    struct Args { const double* X; int64_t ldx; const int32_t* perm; int k; int64_t nc; TC* Z; int64_t ldz;
                  int32_t* J; };
    static constexpr int THREADS = CP_THREADS;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.nc * a.k, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (idx >= a.nc * a.k) return;
        const int64_t pos = idx / a.k;
        const int r = static_cast<int>(idx - pos * a.k);
        const int64_t col = a.perm[pos];
        double z;
        if (pos < a.k) {
            z = (r == pos) ? 1.0 : 0.0;
            if (a.J && r == 0) a.J[pos] = static_cast<int32_t>(col);
        } else {
            z = a.X[pos * a.ldx + r];
        }
        if (a.Z) a.Z[static_cast<int64_t>(r) * a.ldz + col] = static_cast<TC>(z);
    }
};

// out[i][c] = A[i][idx[c]] (columns, transpose = 0) or out[c][j] = A[idx[c]][j]
// (rows) or its transpose out[j][c] = A[idx[c]][j] (transpose = 1).
template <typename TA, typename TC>
struct GatherBody {
    struct Args { const TA* A; int64_t lda; const int32_t* idx; int k; int64_t len; int rows; int transpose;
                  TC* out; int64_t ldo; };
    static constexpr int THREADS = CP_THREADS;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.len * a.k, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int64_t e = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (e >= a.len * a.k) return;
        const int64_t i = e / a.k;                  // position along the kept dimension
        const int c = static_cast<int>(e - i * a.k);
        const int64_t s = a.idx[c];
        if (!a.rows) {
            a.out[i * a.ldo + c] = static_cast<TC>(Conv<double>::to(a.A[i * a.lda + s]));
        } else {
            const TC v = static_cast<TC>(Conv<double>::to(a.A[s * a.lda + i]));
            if (a.transpose) a.out[i * a.ldo + c] = v;
            else a.out[static_cast<int64_t>(c) * a.ldo + i] = v;
        }
    }
};

// U = W T^-T row by row: for each row w of W (k x k, ldw), u solves T u = w
// (T upper triangular k x k, f64, ld k; zero diagonal: u_i = 0).
template <typename TC>
struct TriSolveRowsBody {
    struct Args { const TC* W; int64_t ldw; const double* T; int k; TC* U; int64_t ldu; };
    static constexpr int THREADS = 64;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.k, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int row = b * THREADS + threadIdx.x;
        if (row >= a.k) return;
        TC* u = a.U + static_cast<int64_t>(row) * a.ldu;
        const TC* w = a.W + static_cast<int64_t>(row) * a.ldw;
        for (int i = a.k - 1; i >= 0; --i) {
            double s = static_cast<double>(w[i]);
            for (int t = i + 1; t < a.k; ++t) s = fma(-a.T[i * a.k + t], static_cast<double>(u[t]), s);
            const double d = a.T[i * a.k + i];
            u[i] = static_cast<TC>(d != 0.0 ? s / d : 0.0);
        }
    }
};

struct IdPlan {
    Plan sp;                  // the QB solve
    int64_t m = 0, n = 0;
    int k = 0, l = 0, Lpk = 0;
    size_t solve = 0, bt = 0, X = 0, perm = 0, tau = 0, partv = 0, partk = 0, Z = 0, RT = 0, W = 0, opart = 0,
           gram = 0, rinv = 0, racc = 0, status = 0, bytes = 0;
};

int id_plan(rsvd_handle_t h, int32_t dtype, int64_t m, int64_t n, int32_t k, const rsvd_params* prm, bool cur,
            IdPlan* P) {
    const int v = validate(dtype, m, n, k, prm);
    if (v != RSVD_OK) return v;
    if (prm->precision != RSVD_PREC_PLAIN) return RSVD_ERR_UNSUPPORTED;
    if (cur && k > RSVD_MAX_L) return RSVD_ERR_UNSUPPORTED;
    P->sp = make_plan(dtype, m, n, k, prm, h->dev.num_cu, false, h->variants);
    P->m = m; P->n = n; P->k = k; P->l = P->sp.l; P->Lpk = tile_cols(k);
    const size_t cs = comp_size(dtype);
    Layout L;
    P->solve = L.take(P->sp.bytes);
    P->bt = L.take(static_cast<size_t>(n) * P->l * cs);
    const size_t xcount = std::max(static_cast<size_t>(n) * P->l, cur ? static_cast<size_t>(m) * k : 0);
    P->X = L.take(xcount * sizeof(double));
    P->perm = L.take(static_cast<size_t>(std::max(m, n)) * sizeof(int32_t));
    P->tau = L.take(static_cast<size_t>(std::max(P->l, k)) * sizeof(double));
    const size_t nb = static_cast<size_t>(cdiv(std::max(m, n), CP_THREADS));
    P->partv = L.take(nb * sizeof(double));
    P->partk = L.take(nb * sizeof(int32_t));
    P->Z = L.take(static_cast<size_t>(k) * n * cs);
    if (cur) {
        const int S = gram_split(n, h->dev.num_cu);
        P->RT = L.take(static_cast<size_t>(n) * P->Lpk * cs);
        P->W = L.take(static_cast<size_t>(k) * P->Lpk * cs);
        P->opart = L.take(static_cast<size_t>(S) * P->Lpk * P->Lpk * 8);
        P->gram = L.take(static_cast<size_t>(P->Lpk) * P->Lpk * 8);
        P->rinv = L.take(static_cast<size_t>(P->Lpk) * P->Lpk * cs);
        P->racc = L.take(4 * static_cast<size_t>(k) * k * 8);
        P->status = L.take(kAlign);
    }
    P->bytes = L.off;
    return RSVD_OK;
}

// k steps of column-pivoted QR of the nr x nc matrix held by columns in X.
hipError_t cpqr_steps(SingleExec& ex, double* X, int64_t ldx, int nr, int64_t nc, int k, double* tau,
                      int32_t* perm, double* partv, int32_t* partk) {
    for (int j = 0; j < k; ++j) {
        const CpqrArgs ca{X, ldx, nr, nc, j, tau, perm, partv, partk};
        RSVD_TRY(ex.run<CpqrApplyBody>(ca));
        RSVD_TRY(ex.run<CpqrPivotBody>(ca));
    }
    // reflector k - 1 on the remaining columns (S's first k rows complete)
    if (k < nc) RSVD_TRY(ex.run<CpqrApplyBody>(CpqrArgs{X, ldx, nr, nc, k, tau, perm, partv, partk}));
    return hipSuccess;
}

template <typename TA, typename TC>
hipError_t id_steps(rsvd_handle_t h, const IdPlan& P, int32_t dtype, const TA* A, int64_t lda,
                    const rsvd_params* prm, bool cur, int32_t* J, int32_t* I, TC* C, int64_t ldc, TC* Zout,
                    int64_t ldz, TC* U, int64_t ldu, TC* R, int64_t ldr, void* work, int* status) {
    SingleExec ex{h->stream};
    const int64_t m = P.m, n = P.n;
    const int k = P.k, l = P.l;
    TC* bt = at<TC>(work, P.bt);
    SolveOut so{};
    so.bt = bt;
    so.ldbt = l;
    *status = dispatch(h, dtype, P.sp, A, lda, prm, so, at<unsigned char>(work, P.solve));
    if (*status != RSVD_OK) return hipSuccess;
    double* X = at<double>(work, P.X);
    int32_t* perm = at<int32_t>(work, P.perm);
    double* tau = at<double>(work, P.tau);
    double* partv = at<double>(work, P.partv);
    int32_t* partk = at<int32_t>(work, P.partk);
    // column ID of B (l x n): B's columns are the rows of B^T
    RSVD_TRY(ex.run<CpqrInitBody<TC>>(typename CpqrInitBody<TC>::Args{bt, l, X, l, l, n, perm}));
    RSVD_TRY(cpqr_steps(ex, X, l, l, n, k, tau, perm, partv, partk));
    if (k < n) RSVD_TRY(ex.run<IdCoefBody>(IdCoefBody::Args{X, l, k, n}));
    TC* Z = cur ? at<TC>(work, P.Z) : Zout;
    const int64_t zld = cur ? n : ldz;
    RSVD_TRY(ex.run<IdScatterBody<TC>>(typename IdScatterBody<TC>::Args{X, l, perm, k, n, Z, zld, J}));
    TC* Cw = C;
    if (cur && !Cw) return hipErrorInvalidValue;
    if (Cw) RSVD_TRY((ex.run<GatherBody<TA, TC>>(typename GatherBody<TA, TC>::Args{A, lda, J, k, m, 0, 0, Cw, ldc})));
    if (!cur) return hipSuccess;
    // row selection: column-pivoted QR of C^T (k x m), C's rows are its columns
    RSVD_TRY(ex.run<CpqrInitBody<TC>>(typename CpqrInitBody<TC>::Args{Cw, ldc, X, k, k, m, perm}));
    RSVD_TRY(cpqr_steps(ex, X, k, k, m, k, tau, perm, partv, partk));
    RSVD_TRY(ex.run<IdScatterBody<TC>>(typename IdScatterBody<TC>::Args{X, k, perm, k, m, nullptr, 0, I}));
    // R = A[I, :] and R^T (n x k) for the pseudoinverse
    RSVD_TRY((ex.run<GatherBody<TA, TC>>(typename GatherBody<TA, TC>::Args{A, lda, I, k, n, 1, 0, R, ldr})));
    TC* RT = at<TC>(work, P.RT);
    RSVD_TRY((ex.run<GatherBody<TA, TC>>(typename GatherBody<TA, TC>::Args{A, lda, I, k, n, 1, 1, RT, P.Lpk})));
    // R^T = Q_r T_r (CholeskyQR2; Q_r overwrites RT, T_r = R3 R2 R1 in racc's fourth block)
    uint32_t* st = at<uint32_t>(work, P.status);
    double* racc = at<double>(work, P.racc);
    RSVD_TRY(ex.run<ClearBody>(ClearBody::Args{st, 1}));
    RSVD_TRY(orthonormalize<TC>(ex, 0, RT, P.Lpk, n, k, P.Lpk, gram_split(n, h->dev.num_cu), at<double>(work, P.opart),
                                at<double>(work, P.gram), at<TC>(work, P.rinv), racc, st));
    // W = Z Q_r (k x k), then U = W T_r^-T
    TC* W = at<TC>(work, P.W);
    RSVD_TRY((gemm_plain<TC, TC, TC, MODE_NN>(ex, 0, true, Z, n, k, n, RT, P.Lpk, k, W, P.Lpk, 1, 0, nullptr,
                                              nullptr, 0)));
    return ex.run<TriSolveRowsBody<TC>>(typename TriSolveRowsBody<TC>::Args{
        W, P.Lpk, racc + 3 * static_cast<size_t>(k) * k, k, U, ldu});
}

template <typename TA, typename TC>
int id_typed(rsvd_handle_t h, const IdPlan& P, int32_t dtype, const void* A, int64_t lda, const rsvd_params* prm,
             bool cur, int32_t* J, int32_t* I, void* C, int64_t ldc, void* Z, int64_t ldz, void* U, int64_t ldu,
             void* R, int64_t ldr, void* work) {
    int st = RSVD_OK;
    const hipError_t e = id_steps<TA, TC>(h, P, dtype, static_cast<const TA*>(A), lda, prm, cur, J, I,
                                          static_cast<TC*>(C), ldc, static_cast<TC*>(Z), ldz, static_cast<TC*>(U),
                                          ldu, static_cast<TC*>(R), ldr, work, &st);
    if (e != hipSuccess) return hip_status(h, e);
    return st;
}

int id_dispatch(rsvd_handle_t h, const IdPlan& P, int32_t dtype, const void* A, int64_t lda, const rsvd_params* prm,
                bool cur, int32_t* J, int32_t* I, void* C, int64_t ldc, void* Z, int64_t ldz, void* U, int64_t ldu,
                void* R, int64_t ldr, void* work) {
    switch (dtype) {
        case RSVD_F64: return id_typed<double, double>(h, P, dtype, A, lda, prm, cur, J, I, C, ldc, Z, ldz, U, ldu,
                                                       R, ldr, work);
        case RSVD_F32: return id_typed<float, float>(h, P, dtype, A, lda, prm, cur, J, I, C, ldc, Z, ldz, U, ldu,
                                                     R, ldr, work);
        case RSVD_BF16: return id_typed<bf16_t, float>(h, P, dtype, A, lda, prm, cur, J, I, C, ldc, Z, ldz, U,
                                                       ldu, R, ldr, work);
        default: return RSVD_ERR_UNSUPPORTED;
    }
}

}  // namespace

extern "C" {

int rid_workspace_size(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, int32_t k,
                       const rsvd_params* params, int32_t cur, size_t* bytes) {
    if (!handle || !bytes || !params) return RSVD_ERR_INVALID;
    IdPlan P;
    const int st = id_plan(handle, dtype, m, n, k, params, cur != 0, &P);
    if (st != RSVD_OK) return st;
    *bytes = P.bytes;
    return RSVD_OK;
}

int rid_run(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda, int32_t k,
            const rsvd_params* params, int32_t* J, void* C, int64_t ldc, void* Z, int64_t ldz, void* work,
            size_t work_bytes) {
    if (!handle || !params) return RSVD_ERR_INVALID;
    IdPlan P;
    const int st = id_plan(handle, dtype, m, n, k, params, false, &P);
    if (st != RSVD_OK) return st;
    if (!A || lda < n || !J || (C && ldc < k) || (Z && ldz < n) || !work) return RSVD_ERR_INVALID;
    if (reinterpret_cast<uintptr_t>(work) % kAlign != 0 || work_bytes < P.bytes) return RSVD_ERR_INVALID;
    return id_dispatch(handle, P, dtype, A, lda, params, false, J, nullptr, C, ldc, Z, ldz, nullptr, 0, nullptr, 0,
                       work);
}

int rcur_run(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda, int32_t k,
             const rsvd_params* params, int32_t* J, int32_t* I, void* C, int64_t ldc, void* U, int64_t ldu,
             void* R, int64_t ldr, void* work, size_t work_bytes) {
    if (!handle || !params) return RSVD_ERR_INVALID;
    IdPlan P;
    const int st = id_plan(handle, dtype, m, n, k, params, true, &P);
    if (st != RSVD_OK) return st;
    if (!A || lda < n || !J || !I || !C || ldc < k || !U || ldu < k || !R || ldr < n || !work)
        return RSVD_ERR_INVALID;
    if (reinterpret_cast<uintptr_t>(work) % kAlign != 0 || work_bytes < P.bytes) return RSVD_ERR_INVALID;
    return id_dispatch(handle, P, dtype, A, lda, params, true, J, I, C, ldc, nullptr, 0, U, ldu, R, ldr, work);
}

}  // extern "C"
