// Small dense kernels around the products with A:
//   - deterministic split-K reduction of partial blocks,
//   - column means of A (implicit centring for PCA, Sec. 4.2),
//   - the test matrix Omega (Alg. rqb step 2),
//   - Cholesky of a Gram matrix and the inverse of its factor (the economic
//     QR of Alg. rqb step 9 and Alg. subspace_iter steps 2-3, done as
//     CholeskyQR2, with a shifted first pass when the Gram matrix is too
//     ill-conditioned, Fukaya et al., SIAM J. Sci. Comput. 42, 2020),
//   - one-sided (Hestenes) Jacobi SVD of the small triangular factor of B^T
//     (the deterministic svd(B) of Alg. RSVDalgorithm step 2),
//   - the sign convention and the lift matrices for U = Q U~ (Eq. UQU),
//   - the final copies (singular values, PCA eigenvalues, info record).
#pragma once

#include "common.hpp"
#include "philox.hpp"

namespace rsvd {

// Status words are cleared by a kernel rather than a memset node, so the whole
// launch sequence stays safe to capture in a HIP graph.
__global__ void clear_u32_kernel(uint32_t* p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// ---------------------------------------------------------------- reduction
// out[r][c] = sum_s part[s][r][c] for r < rows, c < ncols (split order fixed).
template <typename T>
__global__ __launch_bounds__(256) void reduce_partials_kernel(
        const T* __restrict__ part, int S, int64_t part_stride, int64_t ldp, int64_t rows,
        int ncols, T* __restrict__ out, int64_t ldo, const uint32_t* skip_flag, uint32_t skip_mask) {
    if (skip_flag && ((*skip_flag & skip_mask) == 0u)) return;
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t r = idx / ncols;
    const int c = static_cast<int>(idx - r * ncols);
    if (r >= rows) return;
    T s = part[r * ldp + c];
    for (int k = 1; k < S; ++k) s += part[k * part_stride + r * ldp + c];
    out[r * ldo + c] = s;
}

// ------------------------------------------------------------- column means
// Partial column sums over a chunk of rows: part[s][j] = sum_{i in chunk s} A[i][j].
template <typename TA>
__global__ __launch_bounds__(256) void colsum_partial_kernel(
        const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n, int64_t rows_per_split,
        double* __restrict__ part) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (j >= n) return;
    const int64_t i0 = s * rows_per_split, i1 = min(m, i0 + rows_per_split);
    double acc = 0.0;
    for (int64_t i = i0; i < i1; ++i) acc += Conv<double>::to(A[i * lda + j]);
    part[s * n + j] = acc;
}

__global__ __launch_bounds__(256) void colmean_finish_kernel(
        const double* __restrict__ part, int S, int64_t m, int64_t n, double* __restrict__ mu) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double acc = 0.0;
    for (int s = 0; s < S; ++s) acc += part[s * n + j];
    mu[j] = acc / static_cast<double>(m);
}

// ------------------------------------------------------------------ Omega
// Omega[j][c] for j < n, c < ncols_out (entries c >= l written as zero).
template <typename T>
__global__ __launch_bounds__(256) void omega_kernel(int64_t n, int l, int ncols_out,
                                                    uint64_t seed, uint32_t stream_id, int sdist,
                                                    T* __restrict__ out, int64_t ldo) {
    const int groups = (ncols_out + 3) / 4;
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t j = idx / groups;
    const int c = static_cast<int>(idx - j * groups);
    if (j >= n) return;
    T v[4];
    omega_group<T>(static_cast<uint32_t>(j), static_cast<uint32_t>(c), seed, stream_id, sdist, v);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int col = 4 * c + t;
        if (col < ncols_out) out[j * ldo + col] = (col < l) ? v[t] : T(0);
    }
}

__global__ __launch_bounds__(256) void philox_words_kernel(int64_t n, int groups, uint64_t seed,
                                                           uint32_t stream_id, uint32_t* out) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t j = idx / groups;
    const int c = static_cast<int>(idx - j * groups);
    if (j >= n) return;
    const Philox4 w = philox4x32_10(static_cast<uint32_t>(j), static_cast<uint32_t>(c), stream_id, 0u,
                                    static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
#pragma unroll
    for (int t = 0; t < 4; ++t) out[idx * 4 + t] = w.x[t];
}

// ------------------------------------------------------- Cholesky + inverse
// One workgroup.  G = sum of the S partial Gram blocks (ldp x ldp, f64), of
// which the leading l x l block is used.  Computes G = R^T R (R upper
// triangular), writes R^{-1} (ld ldr, zero outside l x l) in precision TC and
// optionally R (f64, ld l) and Racc <- R Racc.
//
// Pass policy (CholeskyQR2 with shifted CholeskyQR3 fallback):
//   pass 1: if a pivot fails (d_j <= 100 u G_jj, d_j not finite), restart on
//           G + s I with s = 11 (m l + l (l + 1)) u tr(G) and request a 3rd pass;
//   pass 2: request a 3rd pass when the Gram is still far from the identity
//           (some d_j < G_jj / 2);
//   pass 3: runs only when requested.
// A pivot that still fails (a numerically zero column) gets a zero row in R
// and a zero column in R^{-1}; DEGENERATE is raised.
struct CholArgs {
    const double* part; int S; int64_t part_stride; int ldp;
    int l;
    int64_t mrows;
    void* rinv; int ldr;
    double* rout;             // optional R (ld l)
    double* racc;             // optional accumulated product (ld l)
    uint32_t* status;
    int pass;                 // 1, 2 or 3
    int skip_unless_pending;  // pass 3: return unless ST_SHIFT_PENDING
};

constexpr int CHOL_MAX_L = RSVD_MAX_L;
constexpr int CHOL_THREADS = 1024;

template <typename TC>
__global__ __launch_bounds__(CHOL_THREADS) void chol_kernel(CholArgs a) {
    __shared__ uint32_t s_flags;
    if (a.skip_unless_pending && ((*a.status & ST_SHIFT_PENDING) == 0u)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int l = a.l, ld = l + 1;
    double* G = reinterpret_cast<double*>(smem_raw);         // l x ld
    double* diag0 = G + l * ld;                               // l
    double* dinv = diag0 + l;                                 // l
    __shared__ double s_scalar[4];
    __shared__ int s_fail;
    const int tid = threadIdx.x, nt = blockDim.x;

    if (tid == 0) {
        uint32_t st = *a.status;
        if (a.pass == 1) st &= ~ST_SHIFT_PENDING;
        s_flags = st;
    }

    auto load_gram = [&]() {
        for (int idx = tid; idx < l * l; idx += nt) {
            const int i = idx / l, j = idx - i * l;
            double v = 0.0;
            for (int s = 0; s < a.S; ++s) v += a.part[s * a.part_stride + static_cast<int64_t>(i) * a.ldp + j];
            G[i * ld + j] = v;
        }
        __syncthreads();
        if (tid < l) diag0[tid] = G[tid * ld + tid];
        __syncthreads();
    };

    load_gram();
    if (tid == 0) {
        double tr = 0.0;
        for (int j = 0; j < l; ++j) tr += diag0[j];
        s_scalar[0] = tr;
    }
    __syncthreads();
    const double trace = s_scalar[0];
    const bool nonfinite = !isfinite(trace);
    const bool zero = (trace == 0.0);
    constexpr double u = 1.1102230246251565e-16;   // unit roundoff of the f64 Gram

    double min_ratio = 1.0;
    bool shifted = false;
    if (!nonfinite && !zero) {
        for (int attempt = 0; attempt < 2; ++attempt) {
            if (attempt == 1) {       // shifted restart
                load_gram();
                const double sh = 11.0 * (static_cast<double>(a.mrows) * l + static_cast<double>(l) * (l + 1)) * u * trace;
                if (tid < l) G[tid * ld + tid] += sh;
                __syncthreads();
                shifted = true;
            }
            if (tid == 0) s_fail = 0;
            min_ratio = 1.0;
            for (int j = 0; j < l; ++j) {
                if (tid == 0) {
                    const double d = G[j * ld + j];
                    const bool fail_pass1 = !(d > 100.0 * u * diag0[j]) || !isfinite(d);
                    const bool dead = !(d > 1e-30 * diag0[j]) || !isfinite(d) || diag0[j] == 0.0;
                    double r;
                    if (a.pass == 1 && attempt == 0 && fail_pass1) {
                        s_fail = 1; r = 0.0;
                    } else if (dead) {
                        r = 0.0;                         // numerically zero column
                        s_flags |= RSVD_FLAG_DEGENERATE;
                    } else {
                        r = sqrt(d);
                        min_ratio = fmin(min_ratio, d / diag0[j]);
                    }
                    G[j * ld + j] = r;
                    dinv[j] = (r > 0.0) ? 1.0 / r : 0.0;
                    s_scalar[1] = min_ratio;
                }
                __syncthreads();
                if (s_fail) break;
                const double rinv = dinv[j];
                for (int t = j + 1 + tid; t < l; t += nt) G[j * ld + t] *= rinv;
                __syncthreads();
                const int w = l - j - 1;
                for (int idx = tid; idx < w * w; idx += nt) {
                    const int aa = j + 1 + idx / w, bb = j + 1 + idx % w;
                    if (aa <= bb) G[aa * ld + bb] -= G[j * ld + aa] * G[j * ld + bb];
                }
                __syncthreads();
            }
            __syncthreads();
            if (!s_fail) break;
        }
        min_ratio = s_scalar[1];
    } else {
        // zero or non-finite Gram: R = 0, R^{-1} = 0
        for (int idx = tid; idx < l * ld; idx += nt) G[idx] = 0.0;
        if (tid < l) dinv[tid] = 0.0;
        if (tid == 0) s_flags |= nonfinite ? RSVD_FLAG_NONFINITE : RSVD_FLAG_DEGENERATE;
        __syncthreads();
    }
    if (tid == 0) {
        if (shifted) s_flags |= RSVD_FLAG_CHOL_SHIFT | ST_SHIFT_PENDING;
        if (a.pass == 2 && min_ratio < 0.5) s_flags |= ST_SHIFT_PENDING;
    }
    // Upper triangle of G (incl. diagonal) now holds R.  Inverse X = R^{-1}:
    // X[i][j] = -dinv[i] * sum_{t=i+1..j} R[i][t] X[t][j], X[j][j] = dinv[j];
    // X[t][j] for t < j is kept in the lower triangle at G[j][t].
    __syncthreads();
    {
        constexpr int PARTS = 8;
        const int j = tid / PARTS, part = tid % PARTS;
        for (int i = l - 2; i >= 0; --i) {
            double acc = 0.0;
            if (j > i && j < l) {
                for (int t = i + 1 + part; t <= j; t += PARTS) {
                    const double x = (t == j) ? dinv[j] : G[j * ld + t];
                    acc += G[i * ld + t] * x;
                }
            }
#pragma unroll
            for (int off = PARTS / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, PARTS);
            if (j > i && j < l && part == 0) G[j * ld + i] = -dinv[i] * acc;
            __syncthreads();
        }
    }
    // Write R^{-1} (TC) and optional R / accumulated product.
    TC* rinv = static_cast<TC*>(a.rinv);
    for (int idx = tid; idx < a.ldr * a.ldr; idx += nt) {
        const int i = idx / a.ldr, j = idx - i * a.ldr;
        double v = 0.0;
        if (i < l && j < l) v = (i == j) ? dinv[i] : (i < j ? G[j * ld + i] : 0.0);
        rinv[idx] = static_cast<TC>(v);
    }
    if (a.rout) {
        for (int idx = tid; idx < l * l; idx += nt) {
            const int i = idx / l, j = idx - i * l;
            a.rout[idx] = (i <= j) ? G[i * ld + j] : 0.0;
        }
    }
    if (a.racc) {
        // Racc <- R * Racc (both upper triangular).  Read everything first.
        constexpr int PER = (CHOL_MAX_L * CHOL_MAX_L + CHOL_THREADS - 1) / CHOL_THREADS;
        double nv[PER];
        int cnt = 0;
        for (int idx = tid; idx < l * l; idx += nt, ++cnt) {
            const int i = idx / l, j = idx - i * l;
            double v = 0.0;
            if (a.pass == 1) {
                v = (i <= j) ? G[i * ld + j] : 0.0;
            } else if (i <= j) {
                for (int t = i; t <= j; ++t) v += G[i * ld + t] * a.racc[t * l + j];
            }
            nv[cnt] = v;
        }
        __syncthreads();
        cnt = 0;
        for (int idx = tid; idx < l * l; idx += nt, ++cnt) a.racc[idx] = nv[cnt];
    }
    __syncthreads();
    if (tid == 0) *a.status = s_flags;
}

// ------------------------------------------------------ one-sided Jacobi SVD
// R (l x l, f64, ld ldr) = W diag(sigma) J^T.  Columns of W and J live
// column-major (column c at offset c * l) in LDS when they fit, otherwise in
// the global scratch provided.  Pairs are visited in round-robin order so that
// every round rotates l/2 disjoint column pairs in parallel, one 32-lane group
// per pair.  A pair is rotated when |w_a . w_b| > tol sqrt(|w_a|^2 |w_b|^2).
// Outputs (sorted by descending sigma, ties by index):
//   sigma[0..l), xv (ldx x kp, TC): xv[t][i] = W[t][perm[i]] for i < k,
//   jk (f64, l x k, ld k): jk[t][i] = J[t][perm[i]].
struct JacobiArgs {
    const double* R; int ldr; int l; int k;
    double* gw;          // global scratch for W (l*l) when LDS is too small
    double* gj;          // global scratch for J (l*l)
    double* sigma;       // l
    void* xv; int ldx; int xcols;
    double* jk;          // l x k
    uint32_t* status;
    int max_sweeps;
    double tol;
};

constexpr int JAC_THREADS = 1024;
constexpr int JAC_GROUP = 32;
constexpr size_t JAC_LDS_LIMIT = 150 * 1024;

__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int off = JAC_GROUP / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, JAC_GROUP);
    return v;
}

template <typename TC>
__global__ __launch_bounds__(JAC_THREADS) void jacobi_kernel(JacobiArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_rotated;
    __shared__ int s_perm[CHOL_MAX_L];
    __shared__ double s_sig[CHOL_MAX_L];
    const int l = a.l, tid = threadIdx.x, nt = blockDim.x;
    const size_t mat = static_cast<size_t>(l) * l * sizeof(double);
    double* W;
    double* J;
    if (2 * mat <= JAC_LDS_LIMIT) {
        W = reinterpret_cast<double*>(smem_raw);
        J = W + l * l;
    } else if (mat <= JAC_LDS_LIMIT) {
        W = reinterpret_cast<double*>(smem_raw);
        J = a.gj;
    } else {
        W = a.gw;
        J = a.gj;
    }
    for (int idx = tid; idx < l * l; idx += nt) {
        const int c = idx / l, r = idx - c * l;
        W[idx] = a.R[r * a.ldr + c];
        J[idx] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();

    const int lp = l + (l & 1);
    const int npairs = lp / 2;
    const int group = tid / JAC_GROUP, gl = tid % JAC_GROUP;
    const int ngroups = nt / JAC_GROUP;
    int sweep = 0;
    for (; sweep < a.max_sweeps; ++sweep) {
        if (tid == 0) s_rotated = 0;
        __syncthreads();
        for (int round = 0; round < lp - 1; ++round) {
            for (int p = group; p < npairs; p += ngroups) {
                int ca, cb;
                if (p == 0) { ca = round; cb = lp - 1; }
                else { ca = (round + p) % (lp - 1); cb = (round - p + lp - 1) % (lp - 1); }
                if (ca >= l || cb >= l) continue;
                double* wa = W + ca * l;
                double* wb = W + cb * l;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int r = gl; r < l; r += JAC_GROUP) {
                    const double x = wa[r], y = wb[r];
                    al += x * x; be += y * y; ga += x * y;
                }
                al = group_sum(al); be = group_sum(be); ga = group_sum(ga);
                if (ga != 0.0 && fabs(ga) > a.tol * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                    for (int r = gl; r < l; r += JAC_GROUP) {
                        const double x = wa[r], y = wb[r];
                        wa[r] = c * x - s * y;
                        wb[r] = s * x + c * y;
                    }
                    double* ja = J + ca * l;
                    double* jb = J + cb * l;
                    for (int r = gl; r < l; r += JAC_GROUP) {
                        const double x = ja[r], y = jb[r];
                        ja[r] = c * x - s * y;
                        jb[r] = s * x + c * y;
                    }
                    if (gl == 0) s_rotated = 1;
                }
            }
            __syncthreads();
        }
        if (!s_rotated) break;
        __syncthreads();
    }
    if (tid == 0 && sweep >= a.max_sweeps) atomicOr(a.status, RSVD_FLAG_JACOBI_SLOW);

    // sigma_c = |W[:, c]|; normalise the columns of W.
    for (int c = group; c < l; c += ngroups) {
        double* wc = W + c * l;
        double ss = 0.0;
        for (int r = gl; r < l; r += JAC_GROUP) ss += wc[r] * wc[r];
        ss = group_sum(ss);
        const double sg = sqrt(ss);
        const double inv = (sg > 0.0) ? 1.0 / sg : 0.0;
        for (int r = gl; r < l; r += JAC_GROUP) wc[r] *= inv;
        if (gl == 0) s_sig[c] = sg;     // unsorted for now
    }
    __syncthreads();
    // rank of each value: strictly larger ones, then equal ones with lower index
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
        if (t < l && i < a.k) v = W[s_perm[i] * l + t];
        xv[t * a.xcols + i] = static_cast<TC>(v);
    }
    for (int idx = tid; idx < l * a.k; idx += nt) {
        const int t = idx / a.k, i = idx - t * a.k;
        a.jk[idx] = J[s_perm[i] * l + t];
    }
}

// ------------------------------------------------------------- sign rule
// One workgroup per column i < k of V (n x k, ld ldv): find the entry of
// largest magnitude (lowest row on ties); if negative flip the column; then
// write the lift matrix xu[t][i] = jk[t][i] * sign * (scale ? sigma_i : 1).
template <typename TC>
__global__ __launch_bounds__(256) void sign_lift_kernel(TC* V, int64_t ldv, int64_t n, int l, int k,
                                                        const double* jk, const double* sigma,
                                                        int scale, TC* xu, int ldxu, int xcols) {
    const int i = blockIdx.x;
    const int tid = threadIdx.x;
    __shared__ double s_val[256];
    __shared__ int64_t s_idx[256];
    double best = -1.0;
    int64_t bidx = 0;
    for (int64_t r = tid; r < n; r += blockDim.x) {
        const double v = fabs(static_cast<double>(V[r * ldv + i]));
        if (v > best) { best = v; bidx = r; }
    }
    s_val[tid] = best; s_idx[tid] = bidx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
            const double ov = s_val[tid + off];
            const int64_t oi = s_idx[tid + off];
            if (ov > s_val[tid] || (ov == s_val[tid] && oi < s_idx[tid])) { s_val[tid] = ov; s_idx[tid] = oi; }
        }
        __syncthreads();
    }
    __shared__ double s_sgn;
    if (tid == 0) s_sgn = (static_cast<double>(V[s_idx[0] * ldv + i]) < 0.0) ? -1.0 : 1.0;
    __syncthreads();
    const double sgn = s_sgn;
    if (sgn < 0.0)
        for (int64_t r = tid; r < n; r += blockDim.x) V[r * ldv + i] = -V[r * ldv + i];
    const double f = sgn * (scale ? sigma[i] : 1.0);
    for (int t = tid; t < ldxu; t += blockDim.x)
        xu[t * xcols + i] = static_cast<TC>(t < l ? jk[t * k + i] * f : 0.0);
    if (i == 0)     // zero the padding columns of the lift matrix
        for (int idx = tid; idx < ldxu * (xcols - k); idx += blockDim.x) {
            const int t = idx / (xcols - k), c = k + idx % (xcols - k);
            xu[t * xcols + c] = TC(0);
        }
}

// ------------------------------------------------------------- finalize
template <typename TC>
__global__ __launch_bounds__(256) void finalize_kernel(const double* sigma, int k, double* S,
                                                       double* eigvals, double* sdev, double denom,
                                                       const double* mu, int64_t n, TC* center_out,
                                                       const uint32_t* status, rsvd_info* info,
                                                       int l, int q, int p) {
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid < k) {
        const double s = sigma[tid];
        if (S) S[tid] = s;
        if (eigvals) eigvals[tid] = s * s / denom;
        if (sdev) sdev[tid] = sqrt(s * s / denom);
    }
    if (center_out && tid < n) center_out[tid] = static_cast<TC>(mu ? mu[tid] : 0.0);
    if (info && tid == 0) {
        info->l = l; info->q = q; info->p = p;
        info->flags = *status & 0xFFFFu;
        info->est_err = 0.0;
    }
}

}  // namespace rsvd
