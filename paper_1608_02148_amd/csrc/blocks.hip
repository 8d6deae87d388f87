// Kernel-level building blocks of the C ABI: Philox words, the test matrix,
// the products with A, the orthonormalisation and the small SVD.
#include "solve.hpp"

using namespace rsvd;

namespace {

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

}  // namespace

extern "C" {

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


int rsvd_block_workspace_size(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, int32_t c,
                              size_t* bytes) {
    if (!handle || !bytes || m < 1 || n < 1 || c < 1 || c > RSVD_MAX_L_SINGLE) return RSVD_ERR_INVALID;
    *bytes = block_plan(dtype, m, n, c, handle->dev.num_cu).bytes;
    return RSVD_OK;
}

}  // extern "C"

inline XPack xpack_of(const Plan& P, void* work) {
    return XPack{work ? at<uint16_t>(work, P.xpack) : nullptr, P.ldxp, P.xplane};
}

template <typename TA, typename TC>
static hipError_t gemm_nn_typed(hipStream_t st, int arith, const Plan& P, int S, int64_t m, int64_t K, int c,
                                const void* A, int64_t lda, const void* X, int64_t ldx, void* Y, int64_t ldy,
                                void* work) {
    SingleExec ex{st};
    const XPack xp = xpack_of(P, arith != 0 ? work : nullptr);
    // k-contiguous copy of X for the storage-precision streamed products
    TC* xk = work ? at<TC>(work, P.xk) : nullptr;
    const StreamTail tail = (work && P.tailslot) ? StreamTail{at<float>(work, P.tailslot),
                                                              tail_slot_bytes(P.ncu, P.Lp), P.ncu} : StreamTail{};
    if (S == 1)
        return gemm_step<TA, TC, MODE_NN>(ex, arith, 0, static_cast<const TA*>(A), lda, m, K,
                                          static_cast<const TC*>(X), ldx, c, static_cast<TC*>(Y), ldy, 1, 0,
                                          nullptr, nullptr, 0, Gate{}, xp, xk, P.ldxk, tail);
    // split n-reduction: S partial blocks (m x Lp each) summed in split order
    TC* part = at<TC>(work, P.part);
    const int64_t stride = m * P.Lp;
    RSVD_TRY((gemm_step<TA, TC, MODE_NN>(ex, arith, 0, static_cast<const TA*>(A), lda, m, K,
                                        static_cast<const TC*>(X), ldx, c, part, P.Lp, S, stride, nullptr, nullptr,
                                        0, Gate{}, xp, xk, P.ldxk, tail)));
    return reduce_step<TC>(ex, part, S, stride, P.Lp, m, c, static_cast<TC*>(Y), ldy);
}

extern "C" {

int rsvd_gemm_nn(rsvd_handle_t handle, int32_t dtype, int32_t arith, int64_t m, int64_t K, int32_t c,
                 const void* A, int64_t lda, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t splits,
                 void* work, size_t work_bytes) {
    if (!handle || m < 1 || K < 1 || c < 1 || c > RSVD_MAX_L_SINGLE || !A || !X || !Y) return RSVD_ERR_INVALID;
    if (lda < K || ldx < c || ldy < c || arith < 0 || arith > 2) return RSVD_ERR_INVALID;
    if (splits < 0 || splits > kMaxNNSplit) return RSVD_ERR_INVALID;
    if (arith != 0 && dtype == RSVD_F64) return RSVD_ERR_UNSUPPORTED;
    const Plan P = block_plan(dtype, m, K, c, handle->dev.num_cu);
    const int S = splits == 0 ? P.sp.nn : splits;
    // packed-X scratch (bf16 arithmetics) and split partial blocks live in work
    if ((arith != 0 || S > 1) && (!work || work_bytes < P.bytes)) return RSVD_ERR_INVALID;
    if (work_bytes < P.bytes) work = nullptr;     // optional: the streamed products' copy of X lives there
    hipError_t e;
    switch (dtype) {
        case RSVD_F64: e = gemm_nn_typed<double, double>(handle->stream, arith, P, S, m, K, c, A, lda, X, ldx, Y, ldy, work); break;
        case RSVD_F32: e = gemm_nn_typed<float, float>(handle->stream, arith, P, S, m, K, c, A, lda, X, ldx, Y, ldy, work); break;
        case RSVD_BF16: e = gemm_nn_typed<bf16_t, float>(handle->stream, arith, P, S, m, K, c, A, lda, X, ldx, Y, ldy, work); break;
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
    const XPack xp = xpack_of(P, work);
    TC* xk = at<TC>(work, P.xk);
    const StreamTail tail = P.tailslot ? StreamTail{at<float>(work, P.tailslot), tail_slot_bytes(P.ncu, P.Lp), P.ncu}
                                       : StreamTail{};
    if (S == 1)
        return gemm_step<TA, TC, MODE_TN>(ex, arith, 0, static_cast<const TA*>(A), lda, n, m,
                                          static_cast<const TC*>(Q), ldq, c, static_cast<TC*>(Z), ldz, 1, 0, nullptr,
                                          nullptr, 0, Gate{}, xp, xk, P.ldxk, tail);
    RSVD_TRY((gemm_step<TA, TC, MODE_TN>(ex, arith, 0, static_cast<const TA*>(A), lda, n, m,
                                        static_cast<const TC*>(Q), ldq, c, part, P.Lp, S,
                                        static_cast<int64_t>(n) * P.Lp, nullptr, nullptr, 0, Gate{}, xp, xk,
                                        P.ldxk, tail)));
    return reduce_step<TC>(ex, part, S, static_cast<int64_t>(n) * P.Lp, P.Lp, n, c, static_cast<TC*>(Z), ldz);
}

extern "C" {

int rsvd_gemm_tn(rsvd_handle_t handle, int32_t dtype, int32_t arith, int64_t m, int64_t n, int32_t c,
                 const void* A, int64_t lda, const void* Q, int64_t ldq, void* Z, int64_t ldz, void* work,
                 size_t work_bytes) {
    if (!handle || m < 1 || n < 1 || c < 1 || c > RSVD_MAX_L_SINGLE || !A || !Q || !Z || !work) return RSVD_ERR_INVALID;
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

int rsvd_lu_normalize(rsvd_handle_t handle, int32_t dtype, int64_t m, int32_t c, void* Y, int64_t ldy,
                      int32_t* piv, double* U, uint32_t* flags, void* work, size_t work_bytes) {
    if (!handle || m < 1 || c < 1 || c > RSVD_MAX_L || c > m || !Y || ldy < c || !work) return RSVD_ERR_INVALID;
    if (dtype != RSVD_F64 && dtype != RSVD_F32) return RSVD_ERR_UNSUPPORTED;
    const Plan P = block_plan(dtype, m, m, c, handle->dev.num_cu);
    if (work_bytes < P.bytes) return RSVD_ERR_INVALID;
    SingleExec ex{handle->stream};
    uint32_t* status = at<uint32_t>(work, P.status);
    hipError_t e = ex.run<ClearBody>(ClearBody::Args{status, 1});
    int32_t* cand = at<int32_t>(work, P.lucand);
    int32_t* cnt = at<int32_t>(work, P.lucnt);
    if (e == hipSuccess) {
        if (dtype == RSVD_F64)
            e = lu_normalize<double>(ex, 0, static_cast<double*>(Y), ldy, m, c, P.Lp, cand, cnt,
                                     at<double>(work, P.rinv), status, U, piv);
        else
            e = lu_normalize<float>(ex, 0, static_cast<float*>(Y), ldy, m, c, P.Lp, cand, cnt,
                                    at<float>(work, P.rinv), status, U, piv);
    }
    if (e == hipSuccess && flags) e = hipMemcpyAsync(flags, status, sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                                     handle->stream);
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
    ja.wglob = nullptr; ja.rot = nullptr; ja.outer = 0;
    e = run_jacobi<double>(ex, ja);
    if (e == hipSuccess)
        e = gemm_plain<double, double, double, MODE_TN>(ex, 0, true, R, c, c, c, wks, c, c, J, c, 1, 0, nullptr, nullptr, 0);
    if (e == hipSuccess && flags) e = hipMemcpyAsync(flags, status, sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    return hip_status(handle, e);
}

}  // extern "C"
