// Small dense kernels around the products with A:
//   - deterministic split-K reduction of partial blocks,
//   - column means of A (implicit centring for PCA, Sec. 4.2),
//   - the test matrix Omega (Alg. rqb),
//   - Cholesky of a Gram matrix and the inverse of its factor (the economic
//     QR of Alg. rqb and Alg. subspace_iter, done as
//     CholeskyQR2, with a shifted first pass when the Gram matrix is too
//     ill-conditioned, Fukaya et al., SIAM J. Sci. Comput. 42, 2020),
//   - one-sided (Hestenes) Jacobi SVD of the small triangular factor of B^T
//     (the deterministic svd(B) of Alg. RSVDalgorithm),
//   - the sign convention and the lift matrices for U = Q U~ (Eq. UQU),
//   - the final copies (singular values, PCA eigenvalues, info record).
#pragma once

#include "common.hpp"
#include "philox.hpp"

#include <algorithm>

namespace rsvd {

// Status words are cleared by a kernel rather than a memset node, so the whole
// launch sequence stays safe to capture in a HIP graph.
// p[0] = 0 and, when count = 2, p[1] = v1 (the iteration word), or with qsrc
// the word for q = *qsrc out of qmax (q chosen on the device).
struct ClearBody {
    struct Args { uint32_t* p; int count; uint32_t v1; const int32_t* qsrc; int qmax; };
    static constexpr int THREADS = 64;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.count, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int i = b * THREADS + threadIdx.x;
        if (i < a.count) a.p[i] = (i == 1) ? (a.qsrc ? iteration_word(*a.qsrc, a.qmax) : a.v1) : 0u;
    }
};

// Device clock reading (constant-rate wall clock) into *t: marks when a
// problem's first and last steps ran, for per-solve latency in batches.
struct StampBody {
    struct Args { uint64_t* t; };
    static constexpr int THREADS = 64;
    static int blocks(const Args& a) { return a.t ? 1 : 0; }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int) {
        if (threadIdx.x == 0) a.t[0] = wall_clock64();
    }
};

// ---------------------------------------------------------------- reduction
// out[r][c] = sum_s part[s][r][c] for r < rows, c < ncols (split order fixed).
// Few outputs over many splits (Gram partials: l^2 values, up to one split per
// CU) take the sliced form: a workgroup sums 64 outputs, its 4 waves each a
// quarter of the splits (s = w, w + 4, ...), and the 4 partial sums are added
// in a fixed order; otherwise one thread sums one output over all splits.
template <typename T>
struct ReduceBody {
    struct Args {
        const T* part; int S; int64_t part_stride; int64_t ldp; int64_t rows; int ncols;
        T* out; int64_t ldo; const uint32_t* skip_flag; uint32_t skip_mask;
        Gate gate;
    };
    static constexpr int THREADS = 256;
    static constexpr int SLICES = 4, PER_BLOCK = THREADS / SLICES;
    static constexpr int V = 16 / sizeof(T);                 // elements of one 16-byte access
    static bool sliced(const Args& a) { return a.S >= 8 && a.rows * a.ncols <= 65536; }
    // otherwise, with 16-byte aligned rows and blocks, a thread sums V
    // adjacent outputs with one 16-byte load per split
    __host__ __device__ static bool vec(const Args& a) {
        return a.ncols % V == 0 && a.ldp % V == 0 && a.ldo % V == 0 && a.part_stride % V == 0 &&
               reinterpret_cast<uintptr_t>(a.part) % 16 == 0 && reinterpret_cast<uintptr_t>(a.out) % 16 == 0;
    }
    static int blocks(const Args& a) {
        if (sliced(a)) return static_cast<int>(cdiv(a.rows * a.ncols, PER_BLOCK));
        return static_cast<int>(cdiv(a.rows * (vec(a) ? a.ncols / V : a.ncols), THREADS));
    }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        if (a.skip_flag && ((*a.skip_flag & a.skip_mask) == 0u)) return;
        if (a.gate.w && ((*a.gate.w & a.gate.mask) == 0u)) return;
        if (a.S >= 8 && a.rows * a.ncols <= 65536) {       // sliced (uniform per launch)
            __shared__ T red[SLICES][PER_BLOCK];
            const int e = threadIdx.x % PER_BLOCK, sl = threadIdx.x / PER_BLOCK;
            const int64_t idx = static_cast<int64_t>(b) * PER_BLOCK + e;
            const bool ok = idx < a.rows * a.ncols;
            const int64_t r = ok ? idx / a.ncols : 0;
            const int c = static_cast<int>(idx - r * a.ncols);
            T acc = T(0);
            if (ok) {
                const T* src = a.part + r * a.ldp + c;
#pragma unroll 8
                for (int k = sl; k < a.S; k += SLICES) acc += src[k * a.part_stride];
            }
            red[sl][e] = acc;
            __syncthreads();
            if (sl == 0 && ok) a.out[r * a.ldo + c] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
            return;
        }
        const int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (vec(a)) {
            typedef __attribute__((ext_vector_type(V))) T vec_t;
            const int cv = a.ncols / V;
            const int64_t r = idx / cv;
            const int c = V * static_cast<int>(idx - r * cv);
            if (r >= a.rows) return;
            const vec_t* src = reinterpret_cast<const vec_t*>(a.part + r * a.ldp + c);
            const int64_t st = a.part_stride / V;
            vec_t s = src[0];
            int k = 1;
            for (; k + 4 <= a.S; k += 4) {
                const vec_t v0 = src[k * st], v1 = src[(k + 1) * st], v2 = src[(k + 2) * st], v3 = src[(k + 3) * st];
                s += v0;
                s += v1;
                s += v2;
                s += v3;
            }
            for (; k < a.S; ++k) s += src[k * st];
            *reinterpret_cast<vec_t*>(a.out + r * a.ldo + c) = s;
            return;
        }
        const int64_t r = idx / a.ncols;
        const int c = static_cast<int>(idx - r * a.ncols);
        if (r >= a.rows) return;
        // loads four splits ahead, sums in split order
        const T* src = a.part + r * a.ldp + c;
        T s = src[0];
        int k = 1;
        for (; k + 4 <= a.S; k += 4) {
            const T v0 = src[k * a.part_stride], v1 = src[(k + 1) * a.part_stride];
            const T v2 = src[(k + 2) * a.part_stride], v3 = src[(k + 3) * a.part_stride];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; k < a.S; ++k) s += src[k * a.part_stride];
        a.out[r * a.ldo + c] = s;
    }
};

// ------------------------------------------------------- column statistics
// Column means and root mean squares (PCA centring and scaling, Sec. 4.2 and
// 4.3) in one pass over A.  Sums are shifted by the column's first entry
// a0_j (sums of d = a - a0_j), which keeps the sum of squares well
// conditioned when the offset of a column dwarfs its spread:
//   part[s][j] = sum_{i in chunk s} d_ij,  part[S + s][j] = sum d_ij^2,
//   part[2S][j] = a0_j.
// One thread per column, rows of a chunk in order (coalesced row reads).
template <typename TA>
struct ColsumBody {
    struct Args { const TA* A; int64_t lda; int64_t m; int64_t n; int64_t rows_per_split; int S; double* part; };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.n, THREADS)) * a.S; }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int cb = static_cast<int>(cdiv(a.n, THREADS));
        const int64_t j = static_cast<int64_t>(b % cb) * THREADS + threadIdx.x;
        const int s = b / cb;
        if (j >= a.n) return;
        const double a0 = Conv<double>::to(a.A[j]);
        const int64_t i0 = s * a.rows_per_split, i1 = min(a.m, i0 + a.rows_per_split);
        double acc = 0.0, acc2 = 0.0;
        for (int64_t i = i0; i < i1; ++i) {
            const double d = Conv<double>::to(a.A[i * a.lda + j]) - a0;
            acc += d;
            acc2 += d * d;
        }
        a.part[s * a.n + j] = acc;
        a.part[(a.S + s) * a.n + j] = acc2;
        if (s == 0) a.part[2 * a.S * a.n + j] = a0;
    }
};

// From the partial sums (split order): the centre c_j = a0_j + sum d / m when
// centring (mu, else 0); the mean square about it v_j = sum (a - c_j)^2 /
// (m - 1); with scaling the divisor s_j = sqrt(v_j) (1 for a constant
// column, flagged RSVD_FLAG_ZERO_SCALE in status) and inv[j] = 1 / s_j.
// var[j] = the variance of the column as the solve sees it (v_j / s_j^2).
// mu, inv, var may each be null.
struct ColmeanBody {
    struct Args {
        const double* part; int S; int64_t m; int64_t n; int center; double* mu; double* inv; double* var;
        double* sc; uint32_t* status;
    };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.n, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int64_t j = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (j >= a.n) return;
        double s1 = 0.0, s2 = 0.0;
        for (int s = 0; s < a.S; ++s) s1 += a.part[s * a.n + j];
        for (int s = 0; s < a.S; ++s) s2 += a.part[(a.S + s) * a.n + j];
        const double a0 = a.part[2 * a.S * a.n + j];
        const double md = s1 / static_cast<double>(a.m);            // mean of d
        // sum (a - c)^2 with c = a0 + md (centring) or c = 0: sum (d - e)^2 for
        // e = md or e = -a0, = s2 - 2 e s1 + m e^2
        const double e = a.center ? md : -a0;
        const double ss = fmax(0.0, s2 - 2.0 * e * s1 + static_cast<double>(a.m) * e * e);
        const double v = ss / static_cast<double>(a.m - 1);
        if (a.mu) a.mu[j] = a.center ? a0 + md : 0.0;
        double sc = 1.0;
        if (a.inv) {
            if (v > 0.0) {
                sc = sqrt(v);
            } else if (a.status) {
                atomicOr(a.status, RSVD_FLAG_ZERO_SCALE);
            }
            a.inv[j] = 1.0 / sc;
            if (a.sc) a.sc[j] = sc;
        }
        if (a.var) a.var[j] = v / (sc * sc);
    }
};

// Sum of var[0..n) in a fixed order (strided partial sums, then a tree) into
// *total: the total variance of the data the PCA sees.  One workgroup.
struct TotalVarBody {
    struct Args { const double* var; int64_t n; double* total; };
    static constexpr int THREADS = 256;
    static int blocks(const Args&) { return 1; }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int) {
        __shared__ double sh[THREADS];
        double s = 0.0;
        for (int64_t j = threadIdx.x; j < a.n; j += THREADS) s += a.var[j];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int off = THREADS / 2; off > 0; off >>= 1) {
            if (static_cast<int>(threadIdx.x) < off) sh[threadIdx.x] += sh[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) *a.total = sh[0];
    }
};

// M[j][c] *= inv[j] for j < rows, c < cols (the diagonal scaling D^-1 of
// scaled PCA applied to the skinny side of a product).
template <typename TC>
struct ScaleRowsVecBody {
    struct Args { TC* M; int64_t ld; int64_t rows; int cols; const double* inv; };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.rows * a.cols, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (idx >= a.rows * a.cols) return;
        const int64_t j = idx / a.cols;
        const int c = static_cast<int>(idx - j * a.cols);
        TC* p = a.M + j * a.ld + c;
        *p = static_cast<TC>(static_cast<double>(*p) * a.inv[j]);
    }
};

// PCA outputs from the singular values (sdev_i = sigma_i / sqrt(m - 1)):
// loadings L[j][i] = V[j][i] sdev_i (n x k) and whitened components
// W[r][i] = X[r][i] / sdev_i (m x k; 0 where sdev_i = 0).  X and W may be
// the same matrix.  Either output may be null.
template <typename TC>
struct PcaOutBody {
    struct Args {
        const TC* V; int64_t ldv; TC* L; int64_t ldl; int64_t n;
        const TC* X; int64_t ldx; TC* W; int64_t ldw; int64_t m; int k; const double* sigma; double denom;
    };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) {
        return static_cast<int>(cdiv(((a.L ? a.n : 0) + (a.W ? a.m : 0)) * a.k, THREADS));
    }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        const int64_t nl = a.L ? a.n * a.k : 0;
        if (idx < nl) {
            const int64_t j = idx / a.k;
            const int i = static_cast<int>(idx - j * a.k);
            const double sd = a.sigma[i] / sqrt(a.denom);
            a.L[j * a.ldl + i] = static_cast<TC>(static_cast<double>(a.V[j * a.ldv + i]) * sd);
            return;
        }
        idx -= nl;
        if (!a.W || idx >= a.m * a.k) return;
        const int64_t r = idx / a.k;
        const int i = static_cast<int>(idx - r * a.k);
        const double sd = a.sigma[i] / sqrt(a.denom);
        a.W[r * a.ldw + i] = static_cast<TC>(sd > 0.0 ? static_cast<double>(a.X[r * a.ldx + i]) / sd : 0.0);
    }
};

// rpca_predict's operands: mu[j] = center[j] (widened to f64) and
// W'[j][c] = rotation[j][c] / scale[j] for c < k, 0 for k <= c < kp.
// center / scale null: no centring / no scaling.
template <typename TC>
struct PredictPrepBody {
    struct Args {
        const TC* rot; int64_t ldr; const TC* center; const TC* scale; int64_t n; int k; int kp;
        double* mu; TC* W;
    };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.n * a.kp, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (idx >= a.n * a.kp) return;
        const int64_t j = idx / a.kp;
        const int c = static_cast<int>(idx - j * a.kp);
        if (c == 0 && a.center) a.mu[j] = static_cast<double>(a.center[j]);
        double w = 0.0;
        if (c < a.k) {
            w = static_cast<double>(a.rot[j * a.ldr + c]);
            if (a.scale) w /= static_cast<double>(a.scale[j]);
        }
        a.W[j * a.kp + c] = static_cast<TC>(w);
    }
};

// ------------------------------------------------------------------ Omega
// Omega[j][c] for j < n, c < ncols_out (entries c >= l written as zero).
template <typename T>
struct OmegaBody {
    struct Args { int64_t n; int l; int ncols_out; uint64_t seed; uint32_t stream_id; int sdist; T* out; int64_t ldo; };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.n * ((a.ncols_out + 3) / 4), THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int groups = (a.ncols_out + 3) / 4;
        const int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        const int64_t j = idx / groups;
        const int c = static_cast<int>(idx - j * groups);
        if (j >= a.n) return;
        T v[4];
        omega_group<T>(static_cast<uint32_t>(j), static_cast<uint32_t>(c), a.seed, a.stream_id, a.sdist, v);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int col = 4 * c + t;
            if (col < a.ncols_out) a.out[j * a.ldo + col] = (col < a.l) ? v[t] : T(0);
        }
    }
};


// ------------------------------------------------------- Cholesky + inverse
// One workgroup of 512 threads.  G = sum of the S partial Gram blocks (ldp x
// ldp, f64), of which the leading l x l block (l <= 128) is used.  Computes
// G = R^T R (R upper triangular) and writes R^{-1} (ld ldr, zero outside
// l x l) in precision TC and optionally R (f64, ld l).
//
// Register tiles: thread (tx, ty) holds rows 4ty..4ty+3 and columns
// 8tx..8tx+7 of the matrix.  Factorisation by panels of 4 rows: the owners of
// panel P turn its rows into rows of R (from the 4 x 4 diagonal block's factor
// and inverse), publish them in LDS, and one barrier later every thread below
// applies the rank-4 update.  The inverse X = R^{-1} runs over the same panels
// from the bottom.  Updates run over whole tiles, without triangle masks: row j of R is zero
// left of its diagonal and the rows of X = R^{-1} are zero left of theirs, so
// the entries above the diagonal only ever receive upper-triangle products;
// what the unmasked updates leave below the diagonal is never read (R and
// R^{-1} are written out with their lower parts zeroed).
//
// Pass policy (CholeskyQR2 with shifted CholeskyQR3 fallback):
//   pass 1: if a pivot fails (d_j <= 100 u G_jj, d_j not finite), restart on
//           G + s I with s = 11 (m l + l (l + 1)) u tr(G); that requires two
//           more passes.  In adaptive mode (a basis for the next product, not
//           the final Q) a second pass is requested only then, or when some
//           pivot ratio d_j / G_jj < 1e-6 (condition number above ~1e3);
//   pass 2: runs always (final mode) or when requested; requests a third pass
//           after a shift or when the Gram is still far from the identity
//           (some d_j < G_jj / 2);
//   pass 3: runs only when requested.
// A skipped pass still writes R = I when R is requested, so products of the
// per-pass factors stay valid.
// A pivot that still fails (a numerically zero column) gets a zero row in R
// and a zero column in R^{-1}; DEGENERATE is raised.
struct CholArgs {
    const double* part; int S; int64_t part_stride; int ldp;
    int l;
    int64_t mrows;
    void* rinv; int ldr;
    double* rout;             // optional R (ld l)
    uint32_t* status;
    int pass;                 // 1, 2 or 3
    int skip_unless_pending;  // skip unless this pass was requested (ST_NEED_P2 / P3)
    int adaptive;             // pass 1 may leave out pass 2 (see above)
    Gate gate;                // optional: the whole kernel runs only if the gate is open
    int keep_flags;           // second block of a blocked factorisation: pass 1 keeps the request bits
};

constexpr int CHOL_MAX_L = RSVD_MAX_L;
constexpr int CT_R = 4;                           // rows of the register tile per thread
// Columns of the register tile: 12 in the l <= 96 instance, else 8; either
// way a power of two of thread columns, and a 4-column panel in one lane.
template <int LM> constexpr int chol_cols() { return LM == 96 ? 12 : 8; }
// The kernel instance for l <= LM: (LM / 4) x (LM / cols) threads cover
// LM x LM, so small problems take small workgroups and more of them fit on a
// CU (the l <= 96 instance: 192 threads instead of the 512 of l <= 128).
template <int LM> constexpr int chol_threads() { return (LM / CT_R) * (LM / chol_cols<LM>()); }
static_assert(chol_threads<CHOL_MAX_L>() == 512, "tiles must cover the matrix");
static_assert(chol_threads<96>() == 192, "tiles must cover the matrix");

// Dynamic LDS of R: l rounded up to whole 4-row panels, one padding column.
inline size_t chol_r_lds(int l) {
    const size_t lp = static_cast<size_t>(CT_R) * ((l + CT_R - 1) / CT_R);
    return lp * (lp + 1) * sizeof(double);
}

template <typename TC, int LM>
__device__ __forceinline__ void chol_body(const CholArgs& a) {
    constexpr int CT_C = chol_cols<LM>();
    constexpr int CT_TX = LM / CT_C;              // thread columns (a power of two)
    constexpr int NT = chol_threads<LM>();
    const int l = a.l, tid = threadIdx.x;
    const int tx = tid % CT_TX, ty = tid / CT_TX;
    const int a0 = CT_R * ty, b0 = CT_C * tx;
    const uint32_t need_bit = (a.pass == 2) ? ST_NEED_P2 : ST_NEED_P3;
    if (a.gate.w && ((*a.gate.w & a.gate.mask) == 0u)) return;
    if (a.skip_unless_pending && ((*a.status & need_bit) == 0u)) {
        if (a.rout)
            for (int i = 0; i < CT_R; ++i)
                for (int q = 0; q < CT_C; ++q)
                    if (a0 + i < l && b0 + q < l) a.rout[(a0 + i) * l + b0 + q] = (a0 + i == b0 + q) ? 1.0 : 0.0;
        return;
    }
    // Panels of CT_R = 4 rows: the 16 threads of row group ty = P own rows
    // 4P .. 4P+3 in registers and turn them into rows of R alone (their lanes
    // lie in one wave; values move by lane shuffles), then publish them in LDS
    // and one barrier later every thread applies the rank-4 update to its
    // trailing rows.  The inverse runs the same way from the last panel up.
    __shared__ double panel[2][CT_R][LM];   // R rows (factor) / X rows (inverse)
    __shared__ double diag0[LM];
    __shared__ double xdiag[LM / CT_R][CT_R][CT_R];   // X_PP = R_PP^{-1} of each panel
    __shared__ uint32_t s_flags;
    __shared__ double s_trace;
    __shared__ int s_fail, s_dead;
    __shared__ int s_ratio;           // bit 0: some d_j < 1e-6 G_jj; bit 1: some d_j < G_jj / 2
    double g[CT_R][CT_C];
    const int npanel = (l + CT_R - 1) / CT_R;

    if (tid == 0) {
        uint32_t st = *a.status;
        if (a.pass == 1 && !a.keep_flags) st &= ~(ST_NEED_P2 | ST_NEED_P3 | ST_SHIFTED);
        s_flags = st;
    }
    auto load = [&](double shift) {
#pragma unroll
        for (int i = 0; i < CT_R; ++i)
#pragma unroll
            for (int q = 0; q < CT_C; ++q) {
                const int r = a0 + i, c = b0 + q;
                double v = 0.0;
                if (r < l && c < l) {
                    for (int s = 0; s < a.S; ++s) v += a.part[s * a.part_stride + static_cast<int64_t>(r) * a.ldp + c];
                    if (r == c) { diag0[r] = v; v += shift; }
                }
                g[i][q] = v;
            }
        __syncthreads();
    };
    // value v of lane src of this row group (16-lane segment)
    auto from_lane = [&](double v, int src) { return __shfl(v, src, CT_TX); };

    load(0.0);
    {   // trace of G: the first wave (or the whole workgroup when smaller)
        // sums strided entries, then a butterfly over its lanes
        constexpr int W = NT < 64 ? NT : 64;
        if (tid < W) {
            double tr = 0.0;
            for (int j = tid; j < l; j += W) tr += diag0[j];
#pragma unroll
            for (int off = W / 2; off > 0; off >>= 1) tr += __shfl_xor(tr, off, W);
            if (tid == 0) s_trace = tr;
        }
    }
    __syncthreads();
    const double trace = s_trace;
    const bool nonfinite = !isfinite(trace);
    const bool zero = (trace == 0.0);
    constexpr double u = 1.1102230246251565e-16;   // unit roundoff of the f64 Gram

    bool shifted = false;
    if (!nonfinite && !zero) {
        for (int attempt = 0; attempt < 2; ++attempt) {
            if (attempt == 1) {
                load(11.0 * (static_cast<double>(a.mrows) * l + static_cast<double>(l) * (l + 1)) * u * trace);
                shifted = true;
            }
            if (tid == 0) { s_fail = 0; s_dead = 0; s_ratio = 0; }
            __syncthreads();
            // the owner group of panel P turns its rows into rows of R and
            // publishes them in panel[buf]
            auto factor_panel = [&](const int P, const int buf) {
                const int j0 = CT_R * P;
                // The panel's 4 x 4 diagonal block lies in one lane (columns
                // j0..j0+3: lane j0 / 8, offset j0 % 8).  Its upper half is
                // broadcast to the group; every lane factors it (R_PP, pivot
                // rules above), inverts it (X_PP = R_PP^{-1}, zero row and
                // column for a dead pivot) and forms its own columns of the
                // panel rows as R_P = X_PP^T G_P: no step-by-step chain.
                const int dl = j0 / CT_C;
                const int off = j0 % CT_C;
                double Gd[CT_R][CT_R] = {}, Rd[CT_R][CT_R], Xd[CT_R][CT_R], dv[CT_R] = {};
                // (a static copy per offset: a select between g[t][o + v]
                // would become an indexed load from memory)
#pragma unroll
                for (int o = 0; o < CT_C; o += CT_R)
                    if (off == o) {
#pragma unroll
                        for (int t = 0; t < CT_R; ++t)
#pragma unroll
                            for (int v = 0; v < CT_R; ++v) Gd[t][v] = (v >= t) ? from_lane(g[t][o + v], dl) : 0.0;
                    }
#pragma unroll
                for (int t = 0; t < CT_R; ++t)
#pragma unroll
                    for (int v = 0; v < CT_R; ++v) {
                        Rd[t][v] = 0.0;
                        Xd[t][v] = 0.0;
                    }
                // Branch-free pivots: the diagonal of G is read ahead of the
                // chain, the square root and its reciprocal come from one
                // reciprocal square root (sqrt(d) = d / sqrt(d)), and the pivot
                // ratios d_j / G_jj are only compared with the two thresholds
                // above (1e-6 and 1/2), by multiplication.
                double d0v[CT_R];
#pragma unroll
                for (int t = 0; t < CT_R; ++t) d0v[t] = (j0 + t < l) ? diag0[j0 + t] : 1.0;
                const bool first_try = (a.pass == 1) && (attempt == 0);
                bool fail = false, dead_any = false, low = false, half = false;
#pragma unroll
                for (int t = 0; t < CT_R; ++t) {
                    // rows past l stay zero; after a failed pivot the
                    // attempt is restarted, so the rest is not needed
                    const int j = j0 + t;
                    const bool live = (j < l) & !fail;
                    double d = Gd[t][t];
#pragma unroll
                    for (int i = 0; i < t; ++i) d -= Rd[i][t] * Rd[i][t];
                    const double d0 = d0v[t];
                    const bool finite = isfinite(d);
                    const bool bad = live & first_try & (!(d > 100.0 * u * d0) | !finite);
                    fail = fail | bad;
                    const bool dead = !(d > 1e-30 * d0) | !finite | (d0 == 0.0);
                    const bool use = live & !bad & !dead;
                    const double inv_sq = use ? rsqrt(use ? d : 1.0) : 0.0;
                    const double sq = use ? d * inv_sq : 0.0;
                    dead_any = dead_any | (live & !bad & dead);
                    low = low | (use & (d < 1e-6 * d0));
                    half = half | (use & (d < 0.5 * d0));
                    Rd[t][t] = sq;
                    dv[t] = inv_sq;
#pragma unroll
                    for (int v = t + 1; v < CT_R; ++v) {
                        double w = Gd[t][v];
#pragma unroll
                        for (int i = 0; i < t; ++i) w -= Rd[i][t] * Rd[i][v];
                        Rd[t][v] = w * inv_sq;
                    }
                }
#pragma unroll
                for (int v = 0; v < CT_R; ++v) {          // R_PP X = I, column by column
                    Xd[v][v] = dv[v];
#pragma unroll
                    for (int t = v - 1; t >= 0; --t) {
                        double w = 0.0;
#pragma unroll
                        for (int i = t + 1; i <= v; ++i) w += Rd[t][i] * Xd[i][v];
                        Xd[t][v] = -dv[t] * w;
                    }
                }
#pragma unroll
                for (int q = 0; q < CT_C; ++q) {          // rows j0..j0+3 of R
                    const int c = b0 + q;
                    double gc[CT_R];
#pragma unroll
                    for (int i = 0; i < CT_R; ++i) gc[i] = g[i][q];
#pragma unroll
                    for (int t = 0; t < CT_R; ++t) {
                        double v = 0.0;
#pragma unroll
                        for (int i = 0; i <= t; ++i) v += Xd[i][t] * gc[i];
                        g[t][q] = (c < j0 + t) ? 0.0 : v;
                    }
                }
                if (tx == 0) {
                    if (fail) s_fail = 1;
                    if (dead_any) s_dead = 1;
                    s_ratio |= (low ? 1 : 0) | (half ? 2 : 0);
#pragma unroll
                    for (int t = 0; t < CT_R; ++t)
#pragma unroll
                        for (int v = 0; v < CT_R; ++v) xdiag[P][t][v] = Xd[t][v];
                }
#pragma unroll
                for (int t = 0; t < CT_R; ++t)
#pragma unroll
                    for (int q = 0; q < CT_C; ++q) panel[buf][t][b0 + q] = g[t][q];
            };
            // rows below panel P: G -= R_P^T R_P from panel[buf]
            auto update_from = [&](const int buf) {
#pragma unroll
                for (int t = 0; t < CT_R; ++t) {
                    double pc[CT_C];
#pragma unroll
                    for (int q = 0; q < CT_C; ++q) pc[q] = panel[buf][t][b0 + q];
#pragma unroll
                    for (int i = 0; i < CT_R; ++i) {
                        const double pr = panel[buf][t][a0 + i];
#pragma unroll
                        for (int q = 0; q < CT_C; ++q) g[i][q] -= pr * pc[q];
                    }
                }
            };
            // Look-ahead: while the rows below panel P apply its update, the
            // owner of panel P + 1 applies it to its own rows first and factors
            // and publishes panel P + 1 in the same phase, so a panel's serial
            // factorisation overlaps the previous panel's update.
            for (int P = -1; P < npanel; ++P) {
                if (s_fail) break;                          // uniform after the barrier
                if (P >= 0 && ty > P) update_from(P & 1);
                if (ty == P + 1 && P + 1 < npanel) factor_panel(P + 1, (P + 1) & 1);
                __syncthreads();
            }
            const bool failed = s_fail != 0;
            __syncthreads();
            if (!failed) break;
        }
    } else {
#pragma unroll
        for (int i = 0; i < CT_R; ++i)
#pragma unroll
            for (int q = 0; q < CT_C; ++q) g[i][q] = 0.0;
        for (int j = tid; j < npanel * CT_R * CT_R; j += NT) (&xdiag[0][0][0])[j] = 0.0;
    }
    if (tid == 0) {
        const bool dead_any = !nonfinite && !zero && s_dead;
        const int ratio = (!nonfinite && !zero) ? s_ratio : 0;
        uint32_t f = s_flags;
        if (nonfinite) f |= RSVD_FLAG_NONFINITE;
        if (zero || dead_any) f |= RSVD_FLAG_DEGENERATE;
        // The request bits stay set until the next orthonormalisation starts,
        // so the Gram, Cholesky and apply kernels of a pass all see them.
        if (a.pass == 1) {
            if (shifted) f |= RSVD_FLAG_CHOL_SHIFT | ST_SHIFTED | ST_NEED_P2;
            else if (a.adaptive && (ratio & 1)) f |= ST_NEED_P2;
        } else if (a.pass == 2) {
            if ((f & ST_SHIFTED) || (ratio & 2)) f |= ST_NEED_P3;
        }
        s_flags = f;
    }
    // R goes to LDS (dynamic, LP x (LP + 1) for l rounded up to LP = 4 npanel):
    // the inverse and the output read it there, so the factor's registers are
    // free for the inverse's.
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* Rs = reinterpret_cast<double*>(smem_raw);
    const int LP = CT_R * npanel, LDR = LP + 1;
#pragma unroll
    for (int i = 0; i < CT_R; ++i)
#pragma unroll
        for (int q = 0; q < CT_C; ++q)
            if (a0 + i < LP && b0 + q < LP) Rs[(a0 + i) * LDR + b0 + q] = (b0 + q >= a0 + i) ? g[i][q] : 0.0;
    __syncthreads();
    // Inverse X = R^{-1} by panels from the bottom: the panel's group forms its
    // 4 rows as X_PP B_P (X_PP kept from the factorisation), publishes them, and
    // the rows above subtract R[i][4P..4P+3] X[4P..4P+3][.] after one barrier.
    double x[CT_R][CT_C];
#pragma unroll
    for (int i = 0; i < CT_R; ++i)
#pragma unroll
        for (int q = 0; q < CT_C; ++q) x[i][q] = (a0 + i == b0 + q && a0 + i < l) ? 1.0 : 0.0;
    // the owner group of panel P forms its rows X_P = X_PP B_P (B_P: rows
    // j0..j0+3 so far) and publishes them in panel[buf]
    auto form_rows = [&](const int P, const int buf) {
#pragma unroll
        for (int q = 0; q < CT_C; ++q) {
            double bq[CT_R];
#pragma unroll
            for (int i = 0; i < CT_R; ++i) bq[i] = x[i][q];
#pragma unroll
            for (int t = 0; t < CT_R; ++t) {
                double v = 0.0;
#pragma unroll
                for (int i = t; i < CT_R; ++i) v += xdiag[P][t][i] * bq[i];
                x[t][q] = v;
            }
        }
#pragma unroll
        for (int t = 0; t < CT_R; ++t)
#pragma unroll
            for (int q = 0; q < CT_C; ++q) panel[buf][t][b0 + q] = x[t][q];
    };
    // rows above panel P: x -= R[., 4P..4P+3] X_P from panel[buf]
    auto apply_from = [&](const int P, const int buf) {
        const int j0 = CT_R * P;
#pragma unroll
        for (int t = 0; t < CT_R; ++t) {
            double xr[CT_C];
#pragma unroll
            for (int q = 0; q < CT_C; ++q) xr[q] = panel[buf][t][b0 + q];
#pragma unroll
            for (int i = 0; i < CT_R; ++i) {
                const double rij = Rs[(a0 + i) * LDR + j0 + t];
#pragma unroll
                for (int q = 0; q < CT_C; ++q) x[i][q] -= rij * xr[q];
            }
        }
    };
    // look-ahead as in the factorisation: the owner of panel P - 1 applies
    // panel P to its rows and forms its own in the same phase
    for (int P = npanel; P >= 1; --P) {
        if (P < npanel && ty < P) apply_from(P, P & 1);
        if (ty == P - 1) form_rows(P - 1, (P - 1) & 1);
        __syncthreads();
    }
    TC* rinv = static_cast<TC*>(a.rinv);
#pragma unroll
    for (int i = 0; i < CT_R; ++i) {
        const int r = a0 + i;
#pragma unroll
        for (int q = 0; q < CT_C; ++q) {
            const int c = b0 + q;
            if (r < a.ldr && c < a.ldr)
                rinv[r * a.ldr + c] = static_cast<TC>((r < l && c < l && c >= r) ? x[i][q] : 0.0);
            if (a.rout && r < l && c < l) a.rout[r * l + c] = Rs[r * LDR + c];
        }
    }
    if (tid == 0) *a.status = s_flags;
}

template <typename TC, int LM = CHOL_MAX_L>
struct CholBody {
    typedef CholArgs Args;
    static constexpr int THREADS = chol_threads<LM>();
    static int blocks(const Args&) { return 1; }
    static size_t lds(const Args& a) { return chol_r_lds(a.l); }
    static __device__ void run(const Args& a, int) { chol_body<TC, LM>(a); }
};

// Size class of the small dense kernels for an l x l problem (256: the
// Jacobi with its matrix in global memory; the Cholesky is blocked there).
inline int small_lm(int l) { return l <= 32 ? 32 : (l <= 64 ? 64 : (l <= CHOL_MAX_L ? CHOL_MAX_L : 2 * CHOL_MAX_L)); }

// ------------------------------------------------------ one-sided Jacobi SVD
// R (l x l upper triangular, f64, ld ldr) = W diag(sigma) J^T.  The columns of
// W (column-major, column c at W + c*ldw) live in LDS; l/2 disjoint column pairs
// are rotated per round (round-robin order), one 8-lane group per pair with
// the two columns held in registers during the rotation.  A
// pair is rotated when (w_a . w_b)^2 > tol^2 |w_a|^2 |w_b|^2.  J is not
// accumulated: since R^T W = J diag(sigma), the needed columns are recovered
// as J_i = R^T w_i / sigma_i, whose error relative to 1 is about
// u sigma_1 / sigma_i -- small for the k leading columns that are kept.
// Outputs (sorted by descending sigma, ties by lower index):
//   sigma[0..l), xv (ldx x xcols, TC): xv[t][i] = W[t][perm[i]] for i < k,
//   wks (f64, l x k, ld k): wks[t][i] = W[t][perm[i]] / sigma_i, from which
//   J_k = R^T wks is formed by a product kernel.
// Outer sweeps of the block Jacobi for 128 < l <= 256 (JacobiBlockBody) and
// the layout of its word array rot (sweep flags, barrier counters, failure).
constexpr int kJacobiOuter = 30;       // most outer sweeps
constexpr int kJacobiCtr = 32;         // rot[32]: barrier arrivals
constexpr int kJacobiFail = 63;        // rot[63]: a barrier wait gave up
constexpr int kJacobiRotWords = 64;
static_assert(kJacobiCtr >= kJacobiOuter && kJacobiCtr < kJacobiFail, "rot layout");
struct JacobiArgs {
    const double* R; int ldr; int l; int k;
    double* sigma;       // l
    void* xv; int ldx; int xcols;
    double* wks;         // l x k
    uint32_t* status;
    int max_sweeps;
    double tol;
    double* wglob;       // l > 128: W in global memory (l x jacobi_ldw(l) f64)
    const uint32_t* rot; // non-null: W already holds the rotated columns (block
    int outer;           // sweeps, see JacobiBlockBody); rot[s] = sweep s rotated
};

constexpr int JAC_GROUP = 16;      // lanes per column pair (one DPP row)

// Column stride of W for l > 128 (global memory, block sweeps): l rounded up
// to a multiple of 16 doubles plus one, so that the columns read by the
// groups of a wave start on different banks when staged in LDS.
__host__ __device__ inline int jacobi_ldw(int l) { return ((l + 15) / 16) * 16 + 1; }

// Rotation threshold: a rotated pair keeps |w_a . w_b| of order u sqrt(l)
// |w_a| |w_b| after rounding, so asking for less than l u would never settle.
inline double jacobi_tol(int l) { return std::max(1e-15, 2.220446049250313e-16 * l); }


// Sum over the 16 lanes of a DPP row: quad exchanges (xor 1, xor 2), then the
// half-row and row mirrors; every lane ends with the full sum.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double group_sum(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    return v;
}

// 1/sqrt(x) for x in [1/4, 8]: the hardware estimate, then two Newton steps
// y <- y (3/2 - x y^2 / 2), each squaring the relative error, so the result
// is within a few ulp of the f64 value.
__device__ __forceinline__ double rsqrt_f64(double x) {
    const double hx = 0.5 * x;
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}

// Rotation [c -s; s c] that makes two columns with |a|^2 = al, |b|^2 = be,
// a . b = ga (ga != 0) orthogonal, by the smaller of the two angles:
// tan(theta) = sgn(d) h / (|d| + r), d = be - al, h = 2 ga, r = sqrt(d^2 + h^2).
// With D = |d| + r, c = D / sqrt(D^2 + h^2) and s = sgn(d) h / sqrt(D^2 + h^2),
// so c^2 + s^2 = 1 to rounding whatever the accuracy of r (r only sets the
// angle).  d and h are first scaled by a power of two to max(|d|, |h|) in
// [1/2, 1), so that no square overflows or underflows.
__device__ __forceinline__ void jacobi_cs(double al, double be, double ga, double& c, double& s) {
    const double d = be - al, h = 2.0 * ga;
    int e;
    (void)frexp(fmax(fabs(d), fabs(h)), &e);
    const double ds = ldexp(d, -e), hs = ldexp(h, -e);
    const double q = fma(ds, ds, hs * hs);            // [1/4, 2)
    const double r = q * rsqrt_f64(q);
    const double D = fabs(ds) + r;                     // [1/2, 1 + sqrt 2)
    const double inv = rsqrt_f64(fma(D, D, hs * hs));  // argument in [1/4, 7]
    c = D * inv;
    s = (d < 0.0 ? -hs : hs) * inv;
}

// Block-cyclic ordering (l <= 128): the columns form blocks of 4, and the
// blocks are paired round-robin; per round a 16-lane group takes one block
// pair (8 columns) into registers, rotates all 16 cross pairs in 4 sub-rounds
// of 4 disjoint pairs -- in a sweep's first round also the 6 pairs inside
// each of its two blocks -- and writes the 8 columns back.  A sweep still
// visits every pair once; per rotation it moves a quarter of the LDS data of
// a pair-at-a-time ordering and takes a quarter of the barriers.
constexpr int JBS = 4;                 // columns per block
constexpr int JAC_LANES = 16;          // lanes per block pair (one DPP row)

template <int LM> constexpr int jacobi_threads() {
    return LM > CHOL_MAX_L ? 1024 : JAC_LANES * (LM / (2 * JBS));
}
// W in LDS for l <= LM: 4 * (blocks rounded up to even) columns of LM + 1
// doubles (rows l..LM-1 and the padding columns are zero).
__host__ __device__ inline int jacobi_blocks(int l) {
    const int nb = (l + JBS - 1) / JBS;
    return nb + (nb & 1);
}
template <int LM> inline size_t jacobi_block_lds_bytes(int l) {
    return static_cast<size_t>(JBS) * jacobi_blocks(l) * (LM + 1) * sizeof(double);
}

// Value of lane K of each quad (DPP quad_perm [K, K, K, K]).
template <int K>
__device__ __forceinline__ double quad_bcast(double v) {
    constexpr int CTRL = K | (K << 2) | (K << 4) | (K << 6);
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// One sub-round: rotations of the 4 disjoint register columns (I_k, J_k).
// Returns whether any pair was rotated.  Pairs below the threshold get the
// identity (c, s) = (1, 0), so the update is branch-free across the group.
// The scalar work of the 4 pairs (rotation and new squared norms) is spread
// over the lanes of each quad -- lane k of a quad computes pair k -- and
// shared by quad broadcasts.
template <int VPL, int I0, int J0, int I1, int J1, int I2, int J2, int I3, int J3>
__device__ __forceinline__ bool jacobi_sub_round(double (&x)[2 * JBS][VPL], double (&nrm)[2 * JBS], double tol2) {
    constexpr int I[4] = {I0, I1, I2, I3};
    constexpr int J[4] = {J0, J1, J2, J3};
    double ga[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < VPL; ++q) acc = fma(x[I[k]][q], x[J[k]][q], acc);
        ga[k] = acc;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) ga[k] = group_sum(ga[k]);
    bool rot[4], any = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        rot[k] = ga[k] != 0.0 && ga[k] * ga[k] > tol2 * (nrm[I[k]] * nrm[J[k]]);
        any = any || rot[k];
    }
    if (!any) return false;
    // this lane's pair: k = lane % 4, picked by an exact 0/1 blend (selects
    // between register values would be turned into an indexed load from memory)
    const int kk = threadIdx.x & 3;
    double al = 0.0, be = 0.0, g = 0.0;
    bool r = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double w = (kk == k) ? 1.0 : 0.0;
        al = fma(w, nrm[I[k]], al);
        be = fma(w, nrm[J[k]], be);
        g = fma(w, ga[k], g);
        r = r || (kk == k && rot[k]);
    }
    double cm, sm;
    jacobi_cs(al, be, r ? g : 1.0, cm, sm);
    if (!r) { cm = 1.0; sm = 0.0; }
    const double x2 = 2.0 * cm * sm * (r ? g : 0.0), cc = cm * cm, ss = sm * sm;   // |c a - s b|^2, |s a + c b|^2
    const double na = fmax(fma(cc, al, fma(ss, be, -x2)), 0.0);
    const double nb = fmax(fma(ss, al, fma(cc, be, x2)), 0.0);
    double c[4], s[4];
    c[0] = quad_bcast<0>(cm); s[0] = quad_bcast<0>(sm);
    c[1] = quad_bcast<1>(cm); s[1] = quad_bcast<1>(sm);
    c[2] = quad_bcast<2>(cm); s[2] = quad_bcast<2>(sm);
    c[3] = quad_bcast<3>(cm); s[3] = quad_bcast<3>(sm);
    nrm[I[0]] = quad_bcast<0>(na); nrm[J[0]] = quad_bcast<0>(nb);
    nrm[I[1]] = quad_bcast<1>(na); nrm[J[1]] = quad_bcast<1>(nb);
    nrm[I[2]] = quad_bcast<2>(na); nrm[J[2]] = quad_bcast<2>(nb);
    nrm[I[3]] = quad_bcast<3>(na); nrm[J[3]] = quad_bcast<3>(nb);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int q = 0; q < VPL; ++q) {
            const double xa = x[I[k]][q], xb = x[J[k]][q];
            x[I[k]][q] = fma(c[k], xa, -s[k] * xb);
            x[J[k]][q] = fma(s[k], xa, c[k] * xb);
        }
    }
    return true;
}

// Sweeps of the block-cyclic ordering over W (LDS, column c at W + c * ldw,
// ldw = LM + 1); returns the number of sweeps run.  Every thread of the
// workgroup calls it (the barriers are workgroup-wide).
template <int LM>
__device__ int jacobi_block_sweeps(double* W, int l, double tol2, int max_sweeps, int* s_rotated) {
    constexpr int VPL = LM / JAC_LANES;
    constexpr int ldw = LM + 1;
    const int tid = threadIdx.x, group = tid / JAC_LANES, gl = tid % JAC_LANES;
    const int nbp = jacobi_blocks(l), npairs = nbp / 2;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if (tid == 0) *s_rotated = 0;
        __syncthreads();
        bool rotated = false;
        for (int round = 0; round < nbp - 1; ++round) {
            if (group < npairs) {
                int ba, bb;
                if (group == 0) { ba = round; bb = nbp - 1; }
                else { ba = (round + group) % (nbp - 1); bb = (round - group + nbp - 1) % (nbp - 1); }
                double x[2 * JBS][VPL], nrm[2 * JBS];
#pragma unroll
                for (int i = 0; i < 2 * JBS; ++i) {
                    const double* wc = W + ((i < JBS ? ba : bb) * JBS + (i % JBS)) * ldw;
                    double ss = 0.0;
#pragma unroll
                    for (int q = 0; q < VPL; ++q) {
                        x[i][q] = wc[gl + JAC_LANES * q];
                        ss = fma(x[i][q], x[i][q], ss);
                    }
                    nrm[i] = ss;
                }
#pragma unroll
                for (int i = 0; i < 2 * JBS; ++i) nrm[i] = group_sum(nrm[i]);
                bool changed = false;
                if (round == 0) {   // pairs inside each block, once per sweep
                    changed |= jacobi_sub_round<VPL, 0, 1, 2, 3, 4, 5, 6, 7>(x, nrm, tol2);
                    changed |= jacobi_sub_round<VPL, 0, 2, 1, 3, 4, 6, 5, 7>(x, nrm, tol2);
                    changed |= jacobi_sub_round<VPL, 0, 3, 1, 2, 4, 7, 5, 6>(x, nrm, tol2);
                }
                changed |= jacobi_sub_round<VPL, 0, 4, 1, 5, 2, 6, 3, 7>(x, nrm, tol2);
                changed |= jacobi_sub_round<VPL, 0, 5, 1, 6, 2, 7, 3, 4>(x, nrm, tol2);
                changed |= jacobi_sub_round<VPL, 0, 6, 1, 7, 2, 4, 3, 5>(x, nrm, tol2);
                changed |= jacobi_sub_round<VPL, 0, 7, 1, 4, 2, 5, 3, 6>(x, nrm, tol2);
                if (changed) {
#pragma unroll
                    for (int i = 0; i < 2 * JBS; ++i) {
                        double* wc = W + ((i < JBS ? ba : bb) * JBS + (i % JBS)) * ldw;
#pragma unroll
                        for (int q = 0; q < VPL; ++q) wc[gl + JAC_LANES * q] = x[i][q];
                    }
                    rotated = true;
                }
            }
            __syncthreads();
        }
        if (rotated && gl == 0) *s_rotated = 1;
        __syncthreads();
        const bool again = *s_rotated != 0;
        __syncthreads();
        if (!again) break;
    }
    return sweep;
}

template <typename TC, int LM>
__device__ __forceinline__ void jacobi_body(const JacobiArgs& a) {
    constexpr int JG = JAC_LANES;
    constexpr bool BLOCKED = LM <= CHOL_MAX_L;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_rotated;
    __shared__ int s_perm[LM];
    __shared__ double s_sig[LM];
    __shared__ unsigned long long s_amax;
    const int l = a.l, tid = threadIdx.x, nt = blockDim.x;
    // column c at W + c * ldw: in LDS (block layout, l <= 128), or for l > 128
    // in global memory, where the block sweeps left it
    const int ldw = BLOCKED ? LM + 1 : jacobi_ldw(l);
    double* W = BLOCKED ? reinterpret_cast<double*>(smem_raw) : a.wglob;
    const bool finish_only = a.rot != nullptr;
    // W = 2^-e R with 2^(e-1) <= max |R_ij| < 2^e (exact), so squared norms and
    // their products stay far from overflow and underflow; sigma is scaled
    // back by 2^e at the end.
    int scale_e = 0;
    int sweep = 0;
    if (!finish_only) {
        if (tid == 0) s_amax = 0ull;
        __syncthreads();
        double amax = 0.0;
        for (int idx = tid; idx < l * l; idx += nt) {
            const int c = idx / l, r = idx - c * l;
            amax = fmax(amax, fabs(a.R[r * a.ldr + c]));
        }
        // non-negative doubles order like their bit patterns
        atomicMax(&s_amax, static_cast<unsigned long long>(__double_as_longlong(amax)));
        __syncthreads();
        const double mx = __longlong_as_double(static_cast<long long>(s_amax));
        if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &scale_e);
        const int ncols = BLOCKED ? JBS * jacobi_blocks(l) : l;
        const int nrows = BLOCKED ? LM : l;
        for (int idx = tid; idx < ncols * nrows; idx += nt) {
            const int c = idx / nrows, r = idx - c * nrows;
            W[c * ldw + r] = (r < l && c < l) ? ldexp(a.R[r * a.ldr + c], -scale_e) : 0.0;
        }
        __syncthreads();
        if constexpr (BLOCKED) {
            sweep = jacobi_block_sweeps<LM>(W, l, a.tol * a.tol, a.max_sweeps, &s_rotated);
        } else {
            sweep = a.max_sweeps;    // l > 128 is swept by JacobiBlockBody
        }
    }
    __syncthreads();
    const int group = tid / JG, gl = tid % JG;
    const int ngroups = nt / JG;
    if (tid == 0) {   // record the sweep count (bits 24..31) and the limit flag
        int limit = a.max_sweeps;
        if (finish_only) {
            sweep = 0;
            while (sweep < a.outer && a.rot[sweep]) ++sweep;
            limit = a.outer;
            if (a.rot[kJacobiFail]) sweep = limit;     // a block round was not synchronised
        }
        const uint32_t sw = static_cast<uint32_t>(min(sweep + 1, 255)) << 24;
        atomicOr(a.status, sw | (sweep >= limit ? RSVD_FLAG_JACOBI_SLOW : 0u));
    }

    // sigma_c = |W[:, c]|; normalise the columns of W.
    for (int c = group; c < l; c += ngroups) {
        double* wc = W + c * ldw;
        double ss = 0.0;
        for (int r = gl; r < l; r += JG) ss += wc[r] * wc[r];
        ss = group_sum(ss);
        const double sg = sqrt(ss);
        const double inv = (sg > 0.0) ? 1.0 / sg : 0.0;
        for (int r = gl; r < l; r += JG) wc[r] *= inv;
        if (gl == 0) s_sig[c] = ldexp(sg, scale_e);
    }
    __syncthreads();
    if (tid < l) {
        const double sv = s_sig[tid];
        int rank = 0;
        for (int d = 0; d < l; ++d) {
            const double o = s_sig[d];
            rank += (o > sv) || (o == sv && d < tid);
        }
        s_perm[rank] = tid;
    }
    __syncthreads();
    if (tid < l) a.sigma[tid] = s_sig[s_perm[tid]];
    TC* xv = static_cast<TC*>(a.xv);
    for (int idx = tid; idx < a.ldx * a.xcols; idx += nt) {
        const int t = idx / a.xcols, i = idx - t * a.xcols;
        double v = 0.0;
        if (t < l && i < a.k) v = W[s_perm[i] * ldw + t];
        xv[t * a.xcols + i] = static_cast<TC>(v);
    }
    // W_k diag(1/sigma) in f64 for J_k = R^T W_k / sigma (a product kernel
    // forms it); zero for a zero singular value.
    for (int idx = tid; idx < l * a.k; idx += nt) {
        const int t = idx / a.k, i = idx - t * a.k;
        const int c = s_perm[i];
        const double sg = s_sig[c];
        a.wks[idx] = (sg > 0.0) ? W[c * ldw + t] / sg : 0.0;
    }
}

// Instance for l <= LM: one 16-lane group per block pair of a round (LM / 8
// groups); 1024 threads for the finishing pass of l = 256.
template <typename TC, int LM = CHOL_MAX_L>
struct JacobiBody {
    typedef JacobiArgs Args;
    static constexpr int THREADS = jacobi_threads<LM>();
    static int blocks(const Args&) { return 1; }
    static size_t lds(const Args& a) { return LM > CHOL_MAX_L ? 0 : jacobi_block_lds_bytes<LM>(a.l); }
    static __device__ void run(const Args& a, int) { jacobi_body<TC, LM>(a); }
};

template <typename TC, class Ex>
hipError_t run_chol(Ex& ex, const CholArgs& a) {
    // f32 results, 64 < l <= 96: the 192-thread instance (batch groups of
    // f32 and bf16 problems never mix l <= 96 with l > 96)
    if (sizeof(TC) == 4 && a.l > 64 && a.l <= 96) return ex.template run<CholBody<TC, 96>>(a);
    switch (small_lm(a.l)) {
        case 32: return ex.template run<CholBody<TC, 32>>(a);
        case 64: return ex.template run<CholBody<TC, 64>>(a);
        case CHOL_MAX_L: return ex.template run<CholBody<TC, CHOL_MAX_L>>(a);
        default: return hipErrorInvalidValue;      // l > 128: chol_blocked
    }
}

// dst (rows x cols, ldd) = src (ld lds), under the same skip / gate conditions
// as the product that wrote src.
template <typename T>
struct CopyColsBody {
    struct Args { const T* src; int64_t lds; T* dst; int64_t ldd; int64_t rows; int cols;
                  const uint32_t* skip_flag; uint32_t skip_mask; Gate gate; };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(a.rows * a.cols, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        if (a.skip_flag && ((*a.skip_flag & a.skip_mask) == 0u)) return;
        if (a.gate.w && ((*a.gate.w & a.gate.mask) == 0u)) return;
        const int64_t idx = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (idx >= a.rows * a.cols) return;
        const int64_t r = idx / a.cols;
        const int c = static_cast<int>(idx - r * a.cols);
        a.dst[r * a.ldd + c] = a.src[r * a.lds + c];
    }
};

// Blocked factorisation pieces for 128 < l <= 256 (G = [G11 G12; G12^T G22],
// G11 128 x 128): S = G22 - R12^T R12 (T holds R12^T R12 on entry, ld 128).
struct SchurArgs { const double* G; int ldg; double* T; int l2; const uint32_t* skip_flag; uint32_t skip_mask; Gate gate; };
struct SchurBody {
    typedef SchurArgs Args;
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(static_cast<int64_t>(a.l2) * a.l2, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        if (a.skip_flag && ((*a.skip_flag & a.skip_mask) == 0u)) return;
        if (a.gate.w && ((*a.gate.w & a.gate.mask) == 0u)) return;
        const int idx = b * THREADS + threadIdx.x;
        if (idx >= a.l2 * a.l2) return;
        const int i = idx / a.l2, j = idx - i * a.l2;
        a.T[i * 128 + j] = a.G[static_cast<int64_t>(128 + i) * a.ldg + 128 + j] - a.T[i * 128 + j];
    }
};

// R^{-1} = [I11, -X12; 0, I22] (X12 = I11 R12 I22) into rinv (TC, ldr, zero
// outside l x l) and R = [R11, R12; 0, R22] into rout (f64, ld l) if given.
// A skipped pass leaves rinv and writes the identity to rout, as the
// one-block kernel does.
template <typename TC>
struct CholAssembleBody {
    struct Args {
        const double* R11; const double* I11; const double* R12; const double* X12; const double* R22;
        const double* I22; int l; TC* rinv; int ldr; double* rout; const uint32_t* skip_flag; uint32_t skip_mask;
        Gate gate;
    };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(static_cast<int64_t>(a.ldr) * a.ldr, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        if (a.gate.w && ((*a.gate.w & a.gate.mask) == 0u)) return;
        const int idx = b * THREADS + threadIdx.x;
        if (idx >= a.ldr * a.ldr) return;
        const int i = idx / a.ldr, j = idx - i * a.ldr;
        const bool skip = a.skip_flag && ((*a.skip_flag & a.skip_mask) == 0u);
        if (skip) {
            if (a.rout && i < a.l && j < a.l) a.rout[i * a.l + j] = (i == j) ? 1.0 : 0.0;
            return;
        }
        double x = 0.0, r = 0.0;
        if (i < a.l && j < a.l && j >= i) {
            if (j < 128) { x = a.I11[i * 128 + j]; r = a.R11[i * 128 + j]; }
            else if (i < 128) { x = -a.X12[i * 128 + (j - 128)]; r = a.R12[i * 128 + (j - 128)]; }
            else { x = a.I22[(i - 128) * 128 + (j - 128)]; r = a.R22[(i - 128) * (a.l - 128) + (j - 128)]; }
        }
        a.rinv[i * a.ldr + j] = static_cast<TC>(x);
        if (a.rout && i < a.l && j < a.l) a.rout[i * a.l + j] = r;
    }
};

// ---------------------------------------------- block Jacobi for 128 < l <= 256
// W (l x l, column c at W + c ldw, global memory) is split into JB = 8 column
// blocks of bs = ceil(l / 8) <= 32.  All sweeps run in one launch of JB / 2
// workgroups.  An outer sweep takes JB - 1 rounds: in round r the JB / 2
// block pairs of the round-robin schedule go to the workgroups, each of which
// loads its two blocks (<= 64 columns) into LDS, rotates every pair of those
// columns once (one-sided Jacobi, same rotation test as above), and writes
// them back.  A grid-wide barrier separates consecutive rounds and sweeps.
// rot[s] = 1 when outer sweep s rotated any pair; after the barrier that ends
// sweep s every workgroup reads rot[s] and stops when it is 0 (all read the
// same word, so all stop together), at the latest after kJacobiOuter sweeps.
// The barriers count arrivals in rot[kJacobiCtr] (the b-th barrier waits for
// b JB / 2); a wait is bounded, and one that gives up sets rot[kJacobiFail],
// which stops the sweeps (the finishing pass then reports the small SVD as
// not converged).  The JB / 2 workgroups need JB / 2 CUs at once, which any
// launch on an otherwise idle stream gets.
constexpr int JB = 8;
struct JacobiBlockArgs { double* W; int ldw; int l; int bs; uint32_t* rot; double tol; };

// Barrier of the JacobiBlockBody workgroups: after a workgroup barrier, one
// thread per workgroup arrives with an agent-scope release (which carries the
// workgroup's stores of W, ordered before it by the barrier) and waits with
// agent-scope acquires for `target` arrivals (at most 2^20 polls, none once a
// wait has given up); a second workgroup barrier then orders the other
// threads' loads after that acquire, so they see the other workgroups' stores
// (W crosses XCDs and their separate L2 caches).
__device__ __forceinline__ void jacobi_grid_sync(uint32_t* ctr, uint32_t target, uint32_t* fail) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        for (int spins = 0; __hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target; ++spins) {
            if (spins == (1 << 20) || __hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                __hip_atomic_store(fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
}
struct JacobiPrepArgs { const double* R; int ldr; int l; double* W; int ldw; uint32_t* rot; int nrot; };

// W[c][r] = R[r][c]; rot[0..nrot) = 0.
struct JacobiPrepBody {
    typedef JacobiPrepArgs Args;
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(static_cast<int64_t>(a.l) * a.l, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int idx = b * THREADS + threadIdx.x;
        if (idx < a.nrot) a.rot[idx] = 0u;
        if (idx >= a.l * a.l) return;
        const int c = idx / a.l, r = idx - c * a.l;
        a.W[c * a.ldw + r] = a.R[r * a.ldr + c];
    }
};

struct JacobiBlockBody {
    typedef JacobiBlockArgs Args;
    static constexpr int NLOC = 64;                       // two blocks of <= 32 columns
    static constexpr int THREADS = JAC_GROUP * (NLOC / 2);
    static constexpr int PER_LANE = 2 * CHOL_MAX_L / JAC_GROUP;   // rows <= 256
    static int blocks(const Args&) { return JB / 2; }
    static size_t lds(const Args& a) { return static_cast<size_t>(NLOC) * a.ldw * sizeof(double); }
    static __device__ void run(const Args& a, int p) {
        extern __shared__ __align__(16) unsigned char smem_raw[];
        double* Ws = reinterpret_cast<double*>(smem_raw);
        __shared__ int s_gcol[NLOC];
        __shared__ double s_norm[NLOC];
        __shared__ int s_rotated, s_stop;
        const int tid = threadIdx.x, l = a.l, ldw = a.ldw;
        uint32_t* const ctr = a.rot + kJacobiCtr;
        uint32_t* const fail = a.rot + kJacobiFail;
        uint32_t nbar = 0;
        for (int sweep = 0; sweep < kJacobiOuter; ++sweep) {
            if (sweep > 0) {
                // every workgroup's flag for the previous sweep is out: stop when
                // it rotated nothing (or a barrier gave up)
                jacobi_grid_sync(ctr, ++nbar * (JB / 2), fail);
                if (tid == 0) s_stop = (a.rot[sweep - 1] == 0u || *fail != 0u) ? 1 : 0;
                __syncthreads();
                if (s_stop) break;
            }
            if (tid == 0) s_rotated = 0;
            for (int bround = 0; bround < JB - 1; ++bround) {
                // the other workgroups' writes of the previous round must land first
                if (bround > 0) jacobi_grid_sync(ctr, ++nbar * (JB / 2), fail);
                int ba, bb;
                if (p == 0) { ba = bround; bb = JB - 1; }
                else { ba = (bround + p) % (JB - 1); bb = (bround - p + JB - 1) % (JB - 1); }
                const int a0 = ba * a.bs, a1 = min(l, a0 + a.bs), b0 = bb * a.bs, b1 = min(l, b0 + a.bs);
                const int na = max(0, a1 - a0), nloc = na + max(0, b1 - b0);
                if (tid < NLOC) s_gcol[tid] = (tid < na) ? a0 + tid : (tid < nloc ? b0 + tid - na : -1);
                __syncthreads();
                for (int idx = tid; idx < nloc * l; idx += THREADS) {
                    const int i = idx / l, r = idx - i * l;
                    Ws[i * ldw + r] = a.W[s_gcol[i] * ldw + r];
                }
                __syncthreads();
                const int group = tid / JAC_GROUP, gl = tid % JAC_GROUP;
                constexpr int NG = THREADS / JAC_GROUP;
                for (int c = group; c < nloc; c += NG) {
                    double ss = 0.0;
                    for (int r = gl; r < l; r += JAC_GROUP) ss += Ws[c * ldw + r] * Ws[c * ldw + r];
                    ss = group_sum(ss);
                    if (gl == 0) s_norm[c] = ss;
                }
                __syncthreads();
                const int lp = nloc + (nloc & 1), npairs = lp / 2;
                for (int round = 0; round < lp - 1; ++round) {
                    for (int q = group; q < npairs; q += NG) {
                        int ca, cb;
                        if (q == 0) { ca = round; cb = lp - 1; }
                        else { ca = (round + q) % (lp - 1); cb = (round - q + lp - 1) % (lp - 1); }
                        if (ca >= nloc || cb >= nloc) continue;
                        double* wa = Ws + ca * ldw;
                        double* wb = Ws + cb * ldw;
                        double xa[PER_LANE], xb[PER_LANE];
        #pragma unroll
                        for (int t = 0; t < PER_LANE; ++t) {
                            const int r = gl + JAC_GROUP * t;
                            xa[t] = (r < l) ? wa[r] : 0.0;
                            xb[t] = (r < l) ? wb[r] : 0.0;
                        }
                        const double al = s_norm[ca], be = s_norm[cb];
                        double ga = 0.0;
        #pragma unroll
                        for (int t = 0; t < PER_LANE; ++t) ga += xa[t] * xb[t];
                        ga = group_sum(ga);
                        if (ga != 0.0 && fabs(ga) > a.tol * sqrt(al * be)) {
                            const double zeta = (be - al) / (2.0 * ga);
                            const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                            const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
                            if (gl == 0) {
                                s_norm[ca] = fmax(al - tt * ga, 0.0);
                                s_norm[cb] = be + tt * ga;
                                s_rotated = 1;
                            }
        #pragma unroll
                            for (int t = 0; t < PER_LANE; ++t) {
                                const int r = gl + JAC_GROUP * t;
                                if (r < l) {
                                    wa[r] = c * xa[t] - sn * xb[t];
                                    wb[r] = sn * xa[t] + c * xb[t];
                                }
                            }
                        }
                    }
                    __syncthreads();
                }
                for (int idx = tid; idx < nloc * l; idx += THREADS) {
                    const int i = idx / l, r = idx - i * l;
                    a.W[s_gcol[i] * ldw + r] = Ws[i * ldw + r];
                }
            }
            __syncthreads();
            if (tid == 0 && s_rotated) a.rot[sweep] = 1u;
        }
    }
};

template <typename TC, class Ex>
hipError_t run_jacobi(Ex& ex, const JacobiArgs& a) {
    switch (small_lm(a.l)) {
        case 32: return ex.template run<JacobiBody<TC, 32>>(a);
        case 64: return ex.template run<JacobiBody<TC, 64>>(a);
        case CHOL_MAX_L: return ex.template run<JacobiBody<TC, CHOL_MAX_L>>(a);
        // l > 128: only the finishing pass after the block sweeps (JacobiBlockBody)
        default: return (a.wglob && a.rot) ? ex.template run<JacobiBody<TC, 2 * CHOL_MAX_L>>(a) : hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------- sign rule
// One workgroup per column i < k of V (n x k, ld ldv): find the entry of
// largest magnitude (lowest row on ties); if negative flip the column; then
// write the lift matrix xu[t][i] = jk[t][i] * sign * (scale ? sigma_i : 1).
template <typename TC>
struct SignLiftBody {
    struct Args {
        TC* V; int64_t ldv; int64_t n; int l; int k; const double* jk; const double* sigma;
        int scale; TC* xu; int ldxu; int xcols;
    };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return a.k; }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int i) {
        const int tid = threadIdx.x;
        __shared__ double s_val[THREADS];
        __shared__ int64_t s_idx[THREADS];
        __shared__ double s_sgn;
        double best = -1.0;
        int64_t bidx = 0;
        for (int64_t r = tid; r < a.n; r += THREADS) {
            const double v = fabs(static_cast<double>(a.V[r * a.ldv + i]));
            if (v > best) { best = v; bidx = r; }
        }
        s_val[tid] = best; s_idx[tid] = bidx;
        __syncthreads();
        for (int off = THREADS / 2; off > 0; off >>= 1) {
            if (tid < off) {
                const double ov = s_val[tid + off];
                const int64_t oi = s_idx[tid + off];
                if (ov > s_val[tid] || (ov == s_val[tid] && oi < s_idx[tid])) { s_val[tid] = ov; s_idx[tid] = oi; }
            }
            __syncthreads();
        }
        if (tid == 0) s_sgn = (static_cast<double>(a.V[s_idx[0] * a.ldv + i]) < 0.0) ? -1.0 : 1.0;
        __syncthreads();
        const double sgn = s_sgn;
        if (sgn < 0.0)
            for (int64_t r = tid; r < a.n; r += THREADS) a.V[r * a.ldv + i] = -a.V[r * a.ldv + i];
        const double f = sgn * (a.scale ? a.sigma[i] : 1.0);
        for (int t = tid; t < a.ldxu; t += THREADS)
            a.xu[t * a.xcols + i] = static_cast<TC>(t < a.l ? a.jk[t * a.k + i] * f : 0.0);
        if (i == 0)     // zero the padding columns of the lift matrix
            for (int idx = tid; idx < a.ldxu * (a.xcols - a.k); idx += THREADS) {
                const int t = idx / (a.xcols - a.k), c = a.k + idx % (a.xcols - a.k);
                a.xu[t * a.xcols + c] = TC(0);
            }
    }
};

// ------------------------------------------------------------- finalize
template <typename TC>
struct FinalizeBody {
    struct Args {
        const double* sigma; int k; double* S; double* eigvals; double* sdev; double denom;
        const double* mu; int64_t n; TC* center_out; const uint32_t* status; rsvd_info* info;
        int l; int q; int p;
        const double* est;        // a-posteriori bound or null
        const int32_t* qsrc;      // q chosen on the device, or null (q above)
        const double* scl;        // PCA column scales (null: not scaled)
        TC* scale_out;            // n scales (ones when not scaled) or null
        const double* tvar;       // total variance computed on the device, or null
        double* total_var;        // its output or null
    };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) {
        return static_cast<int>(cdiv(std::max<int64_t>(a.k, (a.center_out || a.scale_out) ? a.n : 0), THREADS));
    }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int64_t tid = static_cast<int64_t>(b) * THREADS + threadIdx.x;
        if (tid < a.k) {
            const double s = a.sigma[tid];
            if (a.S) a.S[tid] = s;
            if (a.eigvals) a.eigvals[tid] = s * s / a.denom;
            if (a.sdev) a.sdev[tid] = sqrt(s * s / a.denom);
        }
        if (a.center_out && tid < a.n) a.center_out[tid] = static_cast<TC>(a.mu ? a.mu[tid] : 0.0);
        if (a.scale_out && tid < a.n) a.scale_out[tid] = static_cast<TC>(a.scl ? a.scl[tid] : 1.0);
        if (a.total_var && tid == 0) *a.total_var = a.tvar ? *a.tvar : 0.0;
        if (a.info && tid == 0) {
            a.info->l = a.l; a.info->q = a.qsrc ? *a.qsrc : a.q; a.info->p = a.p;
            a.info->flags = *a.status & 0xFF00FFFFu;   // RSVD_FLAG_* and the sweep count
            a.info->est_err = a.est ? *a.est : 0.0;
        }
    }
};

// --------------------------------------------- a-posteriori error estimate
// T[i][c] *= sigma_i for i < k, c < r (S V^T probes from V^T probes).
template <typename TC>
struct ScaleRowsBody {
    struct Args { TC* T; int ldt; int k; int r; const double* sigma; };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return static_cast<int>(cdiv(static_cast<int64_t>(a.k) * 32, THREADS)); }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        const int idx = b * THREADS + threadIdx.x;
        const int i = idx / 32, c = idx % 32;
        if (i < a.k && c < a.r) a.T[i * a.ldt + c] = static_cast<TC>(static_cast<double>(a.T[i * a.ldt + c]) * a.sigma[i]);
    }
};

// part[b][c] = sum over rows of chunk b of (Y[i][c] - W[i][c])^2 (c < r <= 32),
// rows of a chunk in a fixed order (8 row lanes, then a fixed tree).
template <typename TC>
struct DiffNormBody {
    struct Args { const TC* Y; const TC* W; int ld; int64_t m; int r; int S; double* part; };
    static constexpr int THREADS = 256;
    static int blocks(const Args& a) { return a.S; }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int b) {
        __shared__ double acc[8][32];
        const int c = threadIdx.x % 32, j = threadIdx.x / 32;
        const int64_t rows = cdiv(a.m, a.S), r0 = static_cast<int64_t>(b) * rows, r1 = min(a.m, r0 + rows);
        double s = 0.0;
        if (c < a.r)
            for (int64_t i = r0 + j; i < r1; i += 8) {
                const double d = static_cast<double>(a.Y[i * a.ld + c]) - static_cast<double>(a.W[i * a.ld + c]);
                s += d * d;
            }
        acc[j][c] = s;
        __syncthreads();
        if (j == 0) {
            double t = 0.0;
            for (int q = 0; q < 8; ++q) t += acc[q][c];
            a.part[static_cast<int64_t>(b) * 32 + c] = t;
        }
    }
};

// est = 10 sqrt(2/pi) max_c sqrt(sum_b part[b][c]) (Halko, Martinsson &
// Tropp 2011, Sec. 4.3).
struct EstBody {
    struct Args { const double* part; int S; int r; double* est; };
    static constexpr int THREADS = 64;
    static int blocks(const Args&) { return 1; }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int) {
        __shared__ double nrm[32];
        const int c = threadIdx.x;
        if (c < 32) {
            double t = 0.0;
            if (c < a.r)
                for (int b = 0; b < a.S; ++b) t += a.part[static_cast<int64_t>(b) * 32 + c];
            nrm[c] = sqrt(t);
        }
        __syncthreads();
        if (c == 0) {
            double mx = 0.0;
            for (int q = 0; q < a.r; ++q) mx = fmax(mx, nrm[q]);
            *a.est = 10.0 * sqrt(2.0 / 3.14159265358979323846) * mx;
        }
    }
};

// ----------------------------------------------- singular values from a Gram
// sigma (descending) = sqrt(max(lambda, 0)) for the eigenvalues lambda of the
// symmetric l x l Gram matrix G = Y^T Y (f64, ld ldg; its upper triangle is
// used): Householder reduction to tridiagonal form in LDS (Golub & Van Loan,
// Matrix Computations, Sec. 8.3.1), then bisection on Sturm counts (Sec.
// 8.4.1) with eight points per eigenvalue and step.  For selector features,
// which need the spectrum only: an eigenvalue error of c l u lambda_1 moves
// sigma_i by at most sqrt(c l u) sigma_1, and by c l u sigma_1^2 / (2 sigma_i)
// when that is smaller.
struct GramEigArgs { const double* G; int ldg; int l; double* sigma; };

template <int LM>
struct GramEigBody {
    typedef GramEigArgs Args;
    static constexpr int THREADS = 8 * LM;
    static constexpr int NG = THREADS / JAC_GROUP;      // 16-lane groups
    static int blocks(const Args&) { return 1; }
    static int ldl(int l) { return l + 1; }
    static size_t lds(const Args& a) { return static_cast<size_t>(a.l) * ldl(a.l) * sizeof(double); }
    static __device__ void run(const Args& a, int) {
        extern __shared__ __align__(16) unsigned char smem_raw[];
        __shared__ double v[LM], w[LM], d[LM], e2[LM], pv[NG];
        __shared__ double s_tau;
        double* G = reinterpret_cast<double*>(smem_raw);
        const int l = a.l, ld = l + 1, tid = threadIdx.x;
        const int group = tid / JAC_GROUP, gl = tid % JAC_GROUP;
        for (int idx = tid; idx < l * l; idx += THREADS) {     // symmetric copy of the upper triangle
            const int r = idx / l, c = idx - r * l;
            G[r * ld + c] = (c >= r) ? a.G[static_cast<int64_t>(r) * a.ldg + c] : a.G[static_cast<int64_t>(c) * a.ldg + r];
        }
        __syncthreads();
        for (int j = 0; j + 2 < l; ++j) {
            const int n1 = l - j - 1, o = j + 1;               // trailing block G[o.., o..]
            if (group == 0) {                                  // reflector from column j below the diagonal
                double s = 0.0;
                for (int i = 1 + gl; i < n1; i += JAC_GROUP) {
                    const double x = G[(o + i) * ld + j];
                    s += x * x;
                }
                s = group_sum(s);
                const double x0 = G[o * ld + j];
                double tau = 0.0, beta = x0, scale = 0.0;
                if (s > 0.0) {
                    const double nrm = sqrt(x0 * x0 + s);
                    beta = -copysign(nrm, x0);
                    tau = (beta - x0) / beta;
                    scale = 1.0 / (x0 - beta);
                }
                for (int i = gl; i < n1; i += JAC_GROUP) v[i] = (i == 0) ? 1.0 : G[(o + i) * ld + j] * scale;
                if (gl == 0) { s_tau = tau; d[j] = G[j * ld + j]; e2[j] = beta * beta; }
            }
            __syncthreads();
            const double tau = s_tau;
            double acc = 0.0;                                  // p = tau G v, and the rows' p_i v_i
            for (int i = group; i < n1; i += NG) {
                const double* gr = G + (o + i) * ld + o;
                double t = 0.0;
                for (int c = gl; c < n1; c += JAC_GROUP) t += gr[c] * v[c];
                t = group_sum(t) * tau;
                if (gl == 0) w[i] = t;
                acc += t * v[i];
            }
            if (gl == 0) pv[group] = acc;
            __syncthreads();
            if (tid < 64) {                                    // K = tau / 2 p^T v; w = p - K v
                double t = 0.0;
                for (int g = tid; g < NG; g += 64) t += pv[g];
                for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
                const double K = 0.5 * tau * t;
                for (int i = tid; i < n1; i += 64) w[i] -= K * v[i];
            }
            __syncthreads();
            for (int i = group; i < n1; i += NG) {             // G -= v w^T + w v^T
                double* gr = G + (o + i) * ld + o;
                const double vi = v[i], wi = w[i];
                for (int c = gl; c < n1; c += JAC_GROUP) gr[c] -= vi * w[c] + wi * v[c];
            }
            __syncthreads();
        }
        if (tid == 0) {
            if (l >= 2) {
                d[l - 2] = G[(l - 2) * ld + (l - 2)];
                const double t = G[(l - 1) * ld + (l - 2)];
                e2[l - 2] = t * t;
            }
            d[l - 1] = G[(l - 1) * ld + (l - 1)];
        }
        __syncthreads();
        // Bisection: eight lanes per eigenvalue index i (ascending) narrow an
        // interval (lo, hi] with count(lo) <= i < count(hi), where count(x) is
        // the number of eigenvalues below x (negative pivots of T - x I).
        const int i = tid / 8, sub = tid % 8;
        double lo = 0.0, hi = 0.0, emax = 0.0;
        for (int k = 0; k < l; ++k) {
            const double r = (k > 0 ? sqrt(e2[k - 1]) : 0.0) + (k + 1 < l ? sqrt(e2[k]) : 0.0);
            lo = (k == 0) ? d[k] - r : fmin(lo, d[k] - r);
            hi = (k == 0) ? d[k] + r : fmax(hi, d[k] + r);
            if (k + 1 < l) emax = fmax(emax, e2[k]);
        }
        const double span = fmax(hi - lo, 1e-300);
        lo -= 1e-14 * span; hi += 1e-14 * span;
        const double pivmin = 1e-290 * fmax(1.0, emax);
        for (int step = 0; step < 18; ++step) {
            const double x = lo + (hi - lo) * (sub + 1) / 9.0;
            int cnt = 0;
            double q = d[0] - x;
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += q < 0.0;
            for (int k = 1; k < l; ++k) {
                q = (d[k] - x) - e2[k - 1] / q;
                if (fabs(q) < pivmin) q = -pivmin;
                cnt += q < 0.0;
            }
            // the eight counts of this eigenvalue's lanes: the new interval is
            // between the last point with count <= i and the first above it
            double nlo = lo, nhi = hi;
            for (int t = 0; t < 8; ++t) {
                const int ct = __shfl(cnt, t, 8);
                const double xt = lo + (hi - lo) * (t + 1) / 9.0;
                if (ct <= i) nlo = xt;
                else if (nhi == hi) nhi = xt;
            }
            lo = nlo; hi = nhi;
        }
        if (sub == 0 && i < l) a.sigma[l - 1 - i] = sqrt(fmax(0.5 * (lo + hi), 0.0));
    }
};

template <class Ex>
hipError_t run_gram_eig(Ex& ex, const GramEigArgs& a) {
    switch (small_lm(a.l)) {
        case 32: return ex.template run<GramEigBody<32>>(a);
        case 64: return ex.template run<GramEigBody<64>>(a);
        default: return ex.template run<GramEigBody<CHOL_MAX_L>>(a);
    }
}

// ------------------------------------------------------------- features
// Selector inputs of one matrix from the singular values sigma (descending,
// l of them) of its q = 0 sketch: sigma_i / sigma_0 zero-padded to 128, then
// log2(m)/12, log2(n)/12, log2(k)/12.
struct FeatureBody {
    struct Args { const double* sigma; int l; int64_t m; int64_t n; int k; float* out; };
    static constexpr int THREADS = 128;
    static int blocks(const Args&) { return 1; }
    static size_t lds(const Args&) { return 0; }
    static __device__ void run(const Args& a, int) {
        const int i = threadIdx.x;
        const double s0 = a.sigma[0];
        a.out[i] = (i < a.l && s0 > 0.0) ? static_cast<float>(a.sigma[i] / s0) : 0.0f;
        if (i < 3) {
            const double v = (i == 0) ? static_cast<double>(a.m) : (i == 1) ? static_cast<double>(a.n)
                                                                             : static_cast<double>(a.k);
            a.out[128 + i] = static_cast<float>(log2(v) / 12.0);
        }
    }
};

}  // namespace rsvd
