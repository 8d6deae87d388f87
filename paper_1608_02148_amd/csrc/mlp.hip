// Selector network for the learned choice of (q, p): 131 -> 64 -> 64 -> 15,
// ReLU, softmax, mean cross-entropy, Adam (Kingma & Ba 2015, Algorithm 1).
//
// Flat f32 parameter vector (row-major, inputs along the rows):
//   W1 131 x 64 | b1 64 | W2 64 x 64 | b2 64 | W3 64 x 15 | b3 15.
//
// Kernels (all sums in a fixed order, so results are deterministic):
//   - mlp_fwd_bwd: one 64-thread workgroup per sample; thread j owns hidden
//     unit j of both layers.  Forward values stay in LDS; with labels the same
//     workgroup forms the per-sample deltas of the three layers (softmax minus
//     one-hot, then back through W3 and W2 with the ReLU masks).
//   - mlp_grad: one thread per parameter sums input x delta over the batch in
//     sample order (the batch gradient is a sum of per-sample outer products).
//   - mlp_loss: one workgroup, strided partial sums then a fixed tree.
//   - mlp_adam: one thread per parameter.
// The products are tiny (13583 parameters, a few MFLOP per batch), so plain
// FMA code is used; there is nothing here for the matrix cores to amortise.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "philox.hpp"

namespace {

constexpr int NI = RSVD_MLP_INPUTS, NH = RSVD_MLP_HIDDEN, NO = RSVD_MLP_CLASSES;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NI * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NO, NP = OFF_B3 + NO;
static_assert(NP == RSVD_MLP_PARAMS, "parameter count");

// Per-sample buffers in the workspace (floats): h1, h2, d1, d2 (B x 64 each),
// z, d3 (B x 15 each), per-sample loss (B), then the gradient (NP).
struct MlpWork {
    float *h1, *h2, *d1, *d2, *z, *d3, *lossb, *grad;
};

inline size_t mlp_floats(int B) { return static_cast<size_t>(B) * (4 * NH + 2 * NO + 1) + NP; }

inline MlpWork carve(void* work, int B) {
    float* p = static_cast<float*>(work);
    MlpWork w;
    w.h1 = p; p += static_cast<size_t>(B) * NH;
    w.h2 = p; p += static_cast<size_t>(B) * NH;
    w.d1 = p; p += static_cast<size_t>(B) * NH;
    w.d2 = p; p += static_cast<size_t>(B) * NH;
    w.z = p; p += static_cast<size_t>(B) * NO;
    w.d3 = p; p += static_cast<size_t>(B) * NO;
    w.lossb = p; p += B;
    w.grad = p;
    return w;
}

__global__ __launch_bounds__(256) void mlp_init_kernel(float* theta, uint64_t seed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NP) return;
    int fan_in = 0;
    if (i < OFF_B1) fan_in = NI;
    else if (i >= OFF_W2 && i < OFF_B2) fan_in = NH;
    else if (i >= OFF_W3 && i < OFF_B3) fan_in = NH;
    if (fan_in == 0) { theta[i] = 0.0f; return; }       // biases start at zero
    // He-uniform: U(-a, a), a = sqrt(6 / fan_in); u from Philox word 0 of
    // counter (i, 0, 0, 0x4D4C50) under the seed.
    const rsvd::Philox4 w = rsvd::philox4x32_10(static_cast<uint32_t>(i), 0u, 0u, 0x4D4C50u,
                                                static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    const float u = (static_cast<float>(w.x[0] >> 8) + 0.5f) * (1.0f / 16777216.0f);   // (0, 1)
    theta[i] = (2.0f * u - 1.0f) * sqrtf(6.0f / static_cast<float>(fan_in));
}

__global__ __launch_bounds__(NH) void mlp_fwd_bwd_kernel(const float* __restrict__ theta, int B,
                                                         const float* __restrict__ X, const int32_t* labels,
                                                         MlpWork w, float* prob, int32_t* cls) {
    const int b = blockIdx.x, j = threadIdx.x;
    __shared__ float xs[NI], h1s[NH], h2s[NH], zs[NO], d3s[NO], d2s[NH];
    for (int i = j; i < NI; i += NH) xs[i] = X[static_cast<size_t>(b) * NI + i];
    __syncthreads();
    const float* W1 = theta + OFF_W1;
    const float* W2 = theta + OFF_W2;
    const float* W3 = theta + OFF_W3;
    float a = theta[OFF_B1 + j];
    for (int i = 0; i < NI; ++i) a = fmaf(xs[i], W1[i * NH + j], a);
    const float h1 = fmaxf(a, 0.0f);
    h1s[j] = h1;
    __syncthreads();
    a = theta[OFF_B2 + j];
    for (int i = 0; i < NH; ++i) a = fmaf(h1s[i], W2[i * NH + j], a);
    const float h2 = fmaxf(a, 0.0f);
    h2s[j] = h2;
    __syncthreads();
    if (j < NO) {
        float z = theta[OFF_B3 + j];
        for (int i = 0; i < NH; ++i) z = fmaf(h2s[i], W3[i * NO + j], z);
        zs[j] = z;
    }
    __syncthreads();
    float zmax = zs[0];
    for (int o = 1; o < NO; ++o) zmax = fmaxf(zmax, zs[o]);
    float se = 0.0f;
    for (int o = 0; o < NO; ++o) se += expf(zs[o] - zmax);
    const float lse = zmax + logf(se);
    if (j < NO) {
        const float pr = expf(zs[j] - lse);
        if (prob) prob[static_cast<size_t>(b) * NO + j] = pr;
        if (w.z) w.z[static_cast<size_t>(b) * NO + j] = zs[j];
        if (labels) {
            const float d = (pr - (j == labels[b] ? 1.0f : 0.0f)) / static_cast<float>(B);
            d3s[j] = d;
            w.d3[static_cast<size_t>(b) * NO + j] = d;
        }
    }
    if (cls && j == 0) {          // largest score, lowest index on ties
        int best = 0;
        for (int o = 1; o < NO; ++o) if (zs[o] > zs[best]) best = o;
        cls[b] = best;
    }
    if (!labels) return;
    if (j == 0) w.lossb[b] = lse - zs[labels[b]];
    w.h1[static_cast<size_t>(b) * NH + j] = h1;
    w.h2[static_cast<size_t>(b) * NH + j] = h2;
    __syncthreads();
    float d2 = 0.0f;
    for (int o = 0; o < NO; ++o) d2 = fmaf(W3[j * NO + o], d3s[o], d2);
    d2 = (h2 > 0.0f) ? d2 : 0.0f;
    d2s[j] = d2;
    w.d2[static_cast<size_t>(b) * NH + j] = d2;
    __syncthreads();
    float d1 = 0.0f;
    for (int i = 0; i < NH; ++i) d1 = fmaf(W2[j * NH + i], d2s[i], d1);
    w.d1[static_cast<size_t>(b) * NH + j] = (h1 > 0.0f) ? d1 : 0.0f;
}

// q per matrix from the network's distribution, for solves that all run with
// oversampling p_solve: pair (q', p') is covered by (q, p_solve) when q' <= q
// and p' <= p_solve, so q_b is the fewest iterations whose covered pairs hold
// probability mass >= tau; when no q reaches tau (possible for p_solve below
// the largest class value), the most iterations, q = 4.  tau <= 0: the q of
// the most probable pair.  No network: fallback_q for all.
__global__ __launch_bounds__(256) void mlp_choose_q_kernel(const float* __restrict__ prob, int B, float tau,
                                                           int p_solve, int fallback_q, int32_t* q) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    if (!prob) { q[b] = fallback_q; return; }
    const float* pb = prob + static_cast<size_t>(b) * NO;
    constexpr int kP[3] = {5, 10, 20};
    int pick = NO / 3 - 1;
    if (tau <= 0.0f) {
        int best = 0;
        for (int c = 1; c < NO; ++c) if (pb[c] > pb[best]) best = c;
        pick = best / 3;
    } else {
        double cum = 0.0;
        for (int qq = 0; qq < NO / 3; ++qq) {
            for (int j = 0; j < 3; ++j)
                if (kP[j] <= p_solve) cum += pb[3 * qq + j];
            if (cum >= tau) { pick = qq; break; }
        }
    }
    q[b] = pick;
}

// Gradient of parameter t: sum over samples of (layer input) x (layer delta).
__global__ __launch_bounds__(256) void mlp_grad_kernel(int B, const float* __restrict__ X, MlpWork w,
                                                       float* grad) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NP) return;
    const float* in = nullptr;
    const float* d = nullptr;
    int nin = 0, nout = 0, i = -1, o = 0;
    if (t < OFF_B1)      { in = X; nin = NI; d = w.d1; nout = NH; i = (t - OFF_W1) / NH; o = (t - OFF_W1) % NH; }
    else if (t < OFF_W2) { d = w.d1; nout = NH; o = t - OFF_B1; }
    else if (t < OFF_B2) { in = w.h1; nin = NH; d = w.d2; nout = NH; i = (t - OFF_W2) / NH; o = (t - OFF_W2) % NH; }
    else if (t < OFF_W3) { d = w.d2; nout = NH; o = t - OFF_B2; }
    else if (t < OFF_B3) { in = w.h2; nin = NH; d = w.d3; nout = NO; i = (t - OFF_W3) / NO; o = (t - OFF_W3) % NO; }
    else                 { d = w.d3; nout = NO; o = t - OFF_B3; }
    float s = 0.0f;
    if (in) {
        for (int b = 0; b < B; ++b)
            s = fmaf(in[static_cast<size_t>(b) * nin + i], d[static_cast<size_t>(b) * nout + o], s);
    } else {
        for (int b = 0; b < B; ++b) s += d[static_cast<size_t>(b) * nout + o];
    }
    grad[t] = s;
}

__global__ __launch_bounds__(256) void mlp_loss_kernel(int B, const float* lossb, float* loss) {
    __shared__ float part[256];
    const int tid = threadIdx.x;
    float s = 0.0f;
    for (int b = tid; b < B; b += 256) s += lossb[b];
    part[tid] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) part[tid] += part[tid + off];
        __syncthreads();
    }
    if (tid == 0) *loss = part[0] / static_cast<float>(B);
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* theta, float* m, float* v, const float* grad,
                                                       float lr, float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NP) return;
    const float g = grad[t];
    const float mt = 0.9f * m[t] + 0.1f * g;
    const float vt = 0.999f * v[t] + 0.001f * g * g;
    m[t] = mt;
    v[t] = vt;
    // c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t) (bias corrections)
    theta[t] -= lr * (mt * c1) / (sqrtf(vt * c2) + 1e-8f);
}

int status_of(rsvd_handle_t h, hipError_t e) {
    if (e == hipSuccess) return RSVD_OK;
    h->last_hip_error = static_cast<int>(e);
    return RSVD_ERR_HIP;
}

}  // namespace

namespace rsvd {

hipError_t learned_choose_q(hipStream_t st, const float* theta, int count, const float* feat, float* prob,
                            float tau, int p_solve, int fallback_q, int32_t* q) {
    if (theta) {
        MlpWork w{};
        hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3(count), dim3(NH), 0, st, theta, count, feat, nullptr, w, prob,
                           nullptr);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(mlp_choose_q_kernel, dim3((count + 255) / 256), dim3(256), 0, st, theta ? prob : nullptr,
                       count, tau, p_solve, fallback_q, q);
    return hipGetLastError();
}

}  // namespace rsvd

extern "C" {

int rsvd_mlp_workspace_size(int32_t batch, size_t* bytes) {
    if (batch < 1 || !bytes) return RSVD_ERR_INVALID;
    *bytes = mlp_floats(batch) * sizeof(float);
    return RSVD_OK;
}

int rsvd_mlp_init(rsvd_handle_t handle, float* theta, uint64_t seed) {
    if (!handle || !theta) return RSVD_ERR_INVALID;
    hipLaunchKernelGGL(mlp_init_kernel, dim3((NP + 255) / 256), dim3(256), 0, handle->stream, theta, seed);
    return status_of(handle, hipGetLastError());
}

int rsvd_mlp_forward(rsvd_handle_t handle, const float* theta, int32_t batch, const float* x, float* prob,
                     int32_t* cls) {
    if (!handle || !theta || batch < 1 || !x || (!prob && !cls)) return RSVD_ERR_INVALID;
    MlpWork w{};
    hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3(batch), dim3(NH), 0, handle->stream, theta, batch, x, nullptr, w,
                       prob, cls);
    return status_of(handle, hipGetLastError());
}

int rsvd_mlp_train_step(rsvd_handle_t handle, float* theta, float* adam_m, float* adam_v, int32_t step, float lr,
                        int32_t batch, const float* x, const int32_t* labels, float* grad, float* loss,
                        void* work, size_t work_bytes) {
    if (!handle || !theta || batch < 1 || !x || !labels || !work || step < 0) return RSVD_ERR_INVALID;
    if (step > 0 && (!adam_m || !adam_v || !(lr > 0.0f))) return RSVD_ERR_INVALID;
    if (work_bytes < mlp_floats(batch) * sizeof(float) || reinterpret_cast<uintptr_t>(work) % 16 != 0)
        return RSVD_ERR_INVALID;
    MlpWork w = carve(work, batch);
    float* g = grad ? grad : w.grad;
    hipStream_t st = handle->stream;
    hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3(batch), dim3(NH), 0, st, theta, batch, x, labels, w, nullptr,
                       nullptr);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((NP + 255) / 256), dim3(256), 0, st, batch, x, w, g);
    if (loss) hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, st, batch, w.lossb, loss);
    if (step > 0) {
        const double c1 = 1.0 / (1.0 - std::pow(0.9, step)), c2 = 1.0 / (1.0 - std::pow(0.999, step));
        hipLaunchKernelGGL(mlp_adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, st, theta, adam_m, adam_v, g,
                           lr, static_cast<float>(c1), static_cast<float>(c2));
    }
    return status_of(handle, hipGetLastError());
}

// Checkpoint file: 64-byte header (magic, u32 version, u32 parameter count,
// u32 Adam step, u64 seed, u64 training-set size, 8-byte digest, f32 tau,
// zero padding), then theta, adam_m, adam_v as little-endian f32.
int rsvd_mlp_load(rsvd_handle_t handle, const char* path, float* theta, float* adam_m, float* adam_v,
                  rsvd_mlp_header* header) {
    if (!handle || !path || (!theta && (adam_m || adam_v))) return RSVD_ERR_INVALID;
    FILE* f = std::fopen(path, "rb");
    if (!f) return RSVD_ERR_INVALID;
    const size_t want = 64 + 3 * sizeof(float) * static_cast<size_t>(NP);
    std::vector<unsigned char> raw(want + 1);
    const size_t got = std::fread(raw.data(), 1, raw.size(), f);
    std::fclose(f);
    static const char kMagic[8] = {'R', 'S', 'V', 'D', 'M', 'L', 'P', '1'};
    if (got < 36) return RSVD_ERR_INVALID;
    if (std::memcmp(raw.data(), kMagic, 8) != 0) return RSVD_ERR_UNSUPPORTED;
    uint32_t version, nparams, step;
    uint64_t seed, ntrain;
    std::memcpy(&version, raw.data() + 8, 4);
    std::memcpy(&nparams, raw.data() + 12, 4);
    std::memcpy(&step, raw.data() + 16, 4);
    std::memcpy(&seed, raw.data() + 20, 8);
    std::memcpy(&ntrain, raw.data() + 28, 8);
    if (version != 1 || nparams != static_cast<uint32_t>(NP)) return RSVD_ERR_UNSUPPORTED;
    if (got != want) return RSVD_ERR_INVALID;             // truncated or trailing bytes
    const float* vals = reinterpret_cast<const float*>(raw.data() + 64);
    for (size_t i = 0; i < 3 * static_cast<size_t>(NP); ++i)
        if (!std::isfinite(vals[i])) return RSVD_ERR_INVALID;
    if (header) {
        header->version = version; header->params = nparams; header->step = step; header->reserved = 0;
        header->seed = seed; header->n_train = ntrain;
        std::memcpy(header->digest, raw.data() + 36, 8);
        std::memcpy(&header->tau, raw.data() + 44, 4);
        header->reserved2 = 0;
    }
    if (!theta) return RSVD_OK;                           // checked only
    float* dst[3] = {theta, adam_m, adam_v};
    for (int t = 0; t < 3; ++t) {
        if (!dst[t]) continue;
        const hipError_t e = hipMemcpyAsync(dst[t], vals + static_cast<size_t>(t) * NP, sizeof(float) * NP,
                                            hipMemcpyHostToDevice, handle->stream);
        if (e != hipSuccess) return status_of(handle, e);
    }
    return status_of(handle, hipStreamSynchronize(handle->stream));
}

}  // extern "C"
