// Pivoted LU normalisation of a tall basis (Alg. normalized_iter, after
// Rokhlin, Szlam & Tygert 2009): Y (rows x l) <- L with Y = L U, L row-permuted
// unit lower trapezoidal, U upper triangular.  Only the span of L matters to
// the power scheme, so any stable choice of pivot rows serves; the GPU picks
// them by tournament pivoting (the "TSLU" of Grigori, Demmel & Xiang, SIAM
// J. Matrix Anal. Appl. 2011) instead of one global partial-pivoting pass,
// which would need a device-wide argmax per column:
//   1. leaves: each workgroup takes LU_ROWS consecutive rows, runs Gaussian
//      elimination with partial pivoting on them in LDS and keeps its (at
//      most l) pivot rows as candidates;
//   2. merges: each workgroup stacks G = LU_ROWS / l candidate lists (the
//      rows as they are in Y), eliminates again and keeps l pivots; repeated
//      until one list is left;
//   3. final: one workgroup factors the l chosen rows with partial pivoting
//      in f64, giving the pivot order and U, and inverts U in place;
//   4. L = Y U^-1 on the matrix cores (the same product as CholeskyQR's
//      Y R^-1), in place.
// When Y has at most LU_ROWS rows the leaf is the whole matrix and the
// pivots are those of partial pivoting on Y.  The selection phases run in
// f32 (they only decide which rows pivot); step 3 runs in f64 and the product
// in the basis precision.  A pivot at or below l eps max |Y| (eps of the
// basis precision: Y's columns dependent to working accuracy) is set to zero,
// gives a zero column of U^-1 and of L and sets RSVD_FLAG_DEGENERATE; a NaN
// pivot sets RSVD_FLAG_NONFINITE.
#pragma once

#include "common.hpp"

namespace rsvd {

constexpr int LU_ROWS = 256;     // rows per selection block
constexpr int LU_MAX_L = 128;    // widest basis
constexpr int LU_THREADS = 256;

// Argmax of v over the workgroup's threads (ties and NaN: lowest key).
// Returns the winning key in every thread.  red: 2 * (THREADS / 64) words.
__device__ __forceinline__ int lu_block_argmax(float v, int key, float* redv, int* redk) {
    for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(v, off, 64);
        const int ok = __shfl_xor(key, off, 64);
        if (ov > v || (ov == v && ok < key)) { v = ov; key = ok; }
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { redv[wave] = v; redk[wave] = key; }
    __syncthreads();
    float bv = redv[0];
    int bk = redk[0];
    for (int w = 1; w < LU_THREADS / 64; ++w)
        if (redv[w] > bv || (redv[w] == bv && redk[w] < bk)) { bv = redv[w]; bk = redk[w]; }
    __syncthreads();
    return bk;
}

// Steps 1 and 2.  Group g eliminates the rows of leaf g (cand_in null) or of
// lists g G .. g G + G - 1 of the previous level, and writes its pivot rows
// (global indices, in pivot order) to cand_out[g l ...], their number to
// cnt_out[g].
template <typename TC>
struct LuSelectBody {
    struct Args {
        const TC* Y; int64_t ldy; int64_t rows; int l;
        const int32_t* cand_in; const int32_t* cnt_in; int nlists; int G;
        int32_t* cand_out; int32_t* cnt_out;
    };
    static constexpr int THREADS = LU_THREADS;
    static int blocks(const Args& a) {
        return static_cast<int>(a.cand_in ? cdiv(a.nlists, a.G) : cdiv(a.rows, LU_ROWS));
    }
    static int ls(int l) { return l + 1; }     // odd row stride: column reads hit distinct banks
    static size_t lds(const Args& a) {
        return static_cast<size_t>(LU_ROWS) * ls(a.l) * sizeof(float) + 2 * LU_ROWS * sizeof(int32_t) +
               2 * (THREADS / 64) * sizeof(float) + 16;
    }
    static __device__ void run(const Args& a, int g) {
        extern __shared__ __align__(16) unsigned char smem_raw[];
        const int l = a.l, LS = l + 1;
        float* T = reinterpret_cast<float*>(smem_raw);
        int32_t* gid = reinterpret_cast<int32_t*>(T + static_cast<size_t>(LU_ROWS) * LS);
        int32_t* order = gid + LU_ROWS;
        float* redv = reinterpret_cast<float*>(order + LU_ROWS);
        int* redk = reinterpret_cast<int*>(redv + THREADS / 64);
        const int tid = threadIdx.x;

        int nr = 0;
        if (!a.cand_in) {
            const int64_t r0 = static_cast<int64_t>(g) * LU_ROWS;
            nr = static_cast<int>(min<int64_t>(LU_ROWS, a.rows - r0));
            for (int r = tid; r < nr; r += THREADS) gid[r] = static_cast<int32_t>(r0 + r);
        } else {
            const int t0 = g * a.G, t1 = min(a.nlists, t0 + a.G);
            for (int t = t0; t < t1; ++t) {       // every thread walks the list sizes (G is small)
                const int c = a.cnt_in[t];
                for (int i = tid; i < c; i += THREADS) gid[nr + i] = a.cand_in[static_cast<int64_t>(t) * l + i];
                nr += c;
            }
        }
        __syncthreads();
        for (int idx = tid; idx < nr * l; idx += THREADS) {
            const int r = idx / l, c = idx - r * l;
            T[r * LS + c] = static_cast<float>(a.Y[static_cast<int64_t>(gid[r]) * a.ldy + c]);
        }
        for (int r = tid; r < nr; r += THREADS) order[r] = r;
        __syncthreads();

        const int steps = min(nr, l);
        for (int j = 0; j < steps; ++j) {
            // pivot: the largest |T[., j]| over positions j..nr-1 (lowest position on ties)
            float v = -1.0f;
            int key = j;
            for (int i = j + tid; i < nr; i += THREADS) {
                const float x = fabsf(T[order[i] * LS + j]);
                if (x > v) { v = x; key = i; }
            }
            const int p = lu_block_argmax(v, key, redv, redk);
            const int pr = order[p];
            __syncthreads();
            if (tid == 0) { order[p] = order[j]; order[j] = pr; }
            __syncthreads();
            // eliminate below the pivot: each thread owns one remaining row
            const float piv = T[pr * LS + j];
            for (int i = j + 1 + tid; i < nr; i += THREADS) {
                const int r = order[i];
                const float f = (piv != 0.0f) ? T[r * LS + j] / piv : 0.0f;
                for (int c = j + 1; c < l; ++c) T[r * LS + c] = fmaf(-f, T[pr * LS + c], T[r * LS + c]);
            }
            __syncthreads();
        }
        for (int i = tid; i < steps; i += THREADS) a.cand_out[static_cast<int64_t>(g) * l + i] = gid[order[i]];
        if (tid == 0) a.cnt_out[g] = steps;
    }
};

// Step 3: the l chosen rows (cand[0 .. l)) in f64, partial pivoting among
// them, U stored to uout (l x l, ld l, f64; may be null) and U^-1 to uinv
// (TC, ld ldu); piv[i] = the row of Y that pivots at step i (may be null).
template <typename TC>
struct LuFinalBody {
    struct Args {
        const TC* Y; int64_t ldy; int l; const int32_t* cand;
        double* uout; TC* uinv; int ldu; int32_t* piv; uint32_t* status;
    };
    static constexpr int THREADS = LU_THREADS;
    static int blocks(const Args&) { return 1; }
    static size_t lds(const Args& a) {
        return static_cast<size_t>(a.l) * (a.l + 1) * sizeof(double) + a.l * sizeof(double) +
               2 * LU_MAX_L * sizeof(int32_t) + 2 * (THREADS / 64) * sizeof(float) + 16;
    }
    static __device__ void run(const Args& a, int) {
        extern __shared__ __align__(16) unsigned char smem_raw[];
        const int l = a.l, LS = l + 1;
        double* T = reinterpret_cast<double*>(smem_raw);
        double* tmp = T + static_cast<size_t>(l) * LS;
        int32_t* gid = reinterpret_cast<int32_t*>(tmp + l);
        int32_t* order = gid + LU_MAX_L;
        float* redv = reinterpret_cast<float*>(order + LU_MAX_L);
        int* redk = reinterpret_cast<int*>(redv + THREADS / 64);
        __shared__ uint32_t flags;
        const int tid = threadIdx.x;
        if (tid == 0) flags = 0;
        for (int r = tid; r < l; r += THREADS) { gid[r] = a.cand[r]; order[r] = r; }
        __syncthreads();
        float amax = 0.0f;
        for (int idx = tid; idx < l * l; idx += THREADS) {
            const int r = idx / l, c = idx - r * l;
            const double y = static_cast<double>(a.Y[static_cast<int64_t>(gid[r]) * a.ldy + c]);
            T[r * LS + c] = y;
            amax = fmaxf(amax, static_cast<float>(fabs(y)));
        }
        // pivots below l eps |Y|_max (eps of the basis precision) count as
        // zero: the rows are linearly dependent to working accuracy
        const int who = lu_block_argmax(amax, tid, redv, redk);
        __shared__ float s_amax;
        if (tid == who) s_amax = amax;
        __syncthreads();
        const double tiny = static_cast<double>(s_amax) * l *
                            (sizeof(TC) == 8 ? 2.220446049250313e-16 : 1.1920928955078125e-07);
        for (int j = 0; j < l; ++j) {
            float v = -1.0f;
            int key = j;
            for (int i = j + tid; i < l; i += THREADS) {
                const float x = static_cast<float>(fabs(T[order[i] * LS + j]));
                if (x > v) { v = x; key = i; }
            }
            // f32 magnitudes can tie where the f64 values differ: refine the
            // winner among exact f64 values in one thread (l is small)
            int p = lu_block_argmax(v, key, redv, redk);
            if (tid == 0) {
                double best = fabs(T[order[p] * LS + j]);
                for (int i = j; i < l; ++i) {
                    const double x = fabs(T[order[i] * LS + j]);
                    if (x > best) { best = x; p = i; }
                }
                const int pr = order[p];
                order[p] = order[j]; order[j] = pr;
                const double pv = T[pr * LS + j];
                if (fabs(pv) <= tiny) {
                    flags |= RSVD_FLAG_DEGENERATE;
                    T[pr * LS + j] = 0.0;
                }
                if (!(pv == pv)) flags |= RSVD_FLAG_NONFINITE;
            }
            __syncthreads();
            const int pr = order[j];
            const double piv = T[pr * LS + j];
            for (int i = j + 1 + tid; i < l; i += THREADS) {
                const int r = order[i];
                const double f = (piv != 0.0) ? T[r * LS + j] / piv : 0.0;
                for (int c = j + 1; c < l; ++c) T[r * LS + c] = fma(-f, T[pr * LS + c], T[r * LS + c]);
                T[r * LS + j] = f;
            }
            __syncthreads();
        }
        // U in pivot order: row i of U is row order[i] of T from column i on
        if (a.uout)
            for (int idx = tid; idx < l * l; idx += THREADS) {
                const int i = idx / l, c = idx - i * l;
                a.uout[idx] = (c >= i) ? T[order[i] * LS + c] : 0.0;
            }
        if (a.piv)
            for (int i = tid; i < l; i += THREADS) a.piv[i] = gid[order[i]];
        __syncthreads();
        // U^-1 in place, column by column (upper triangular): for column j,
        // x_i = -(sum_{i<t<=j} Uinv_prev[i][t] U[t][j]) ... formed as
        // x = Uinv[0:j, 0:j] U[0:j, j] scaled by -1 / U[j][j]; a zero pivot
        // gives a zero column.  Uinv[i][t] is stored in row order[i].
        for (int j = 0; j < l; ++j) {
            const double ujj = T[order[j] * LS + j];
            const double djj = (ujj != 0.0 && ujj == ujj) ? 1.0 / ujj : 0.0;
            for (int i = tid; i < j; i += THREADS) tmp[i] = T[order[i] * LS + j];
            __syncthreads();
            for (int i = tid; i < j; i += THREADS) {
                double s = 0.0;
                for (int t = i; t < j; ++t) s = fma(T[order[i] * LS + t], tmp[t], s);
                T[order[i] * LS + j] = -s * djj;
            }
            if (tid == 0) T[order[j] * LS + j] = djj;
            __syncthreads();
        }
        for (int idx = tid; idx < l * a.ldu; idx += THREADS) {
            const int i = idx / a.ldu, c = idx - i * a.ldu;
            a.uinv[idx] = static_cast<TC>((c < l && c >= i) ? T[order[i] * LS + c] : 0.0);
        }
        if (tid == 0 && flags) atomicOr(a.status, flags);
    }
};

}  // namespace rsvd
