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
#include <cstdint>
#include <cstring>

#include "plan.hpp"

namespace rsvd {

int dispatch(rsvd_handle_t h, int32_t dtype, const Plan& P, const void* A, int64_t lda,
             const rsvd_params* prm, const SolveOut& o, void* work) {
    hipError_t e = hipErrorInvalidValue;
    switch (dtype) {
        case RSVD_F64: e = solve_single_f64(h, P, A, lda, prm, o, work); break;
        case RSVD_F32: e = solve_single_f32(h, P, A, lda, prm, o, work); break;
        case RSVD_BF16: e = solve_single_bf16(h, P, A, lda, prm, o, work); break;
        default: return RSVD_ERR_UNSUPPORTED;
    }
    return hip_status(h, e);
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
    if (handle) {
        for (hipEvent_t e : handle->event_pool) (void)hipEventDestroy(e);
        for (hipStream_t s : handle->side) (void)hipStreamDestroy(s);
        for (hipEvent_t e : handle->side_done) (void)hipEventDestroy(e);
        if (handle->fork) (void)hipEventDestroy(handle->fork);
        if (handle->staging) (void)hipHostFree(handle->staging);
    }
    delete handle;
    return RSVD_OK;
}

int rsvd_set_stream(rsvd_handle_t handle, void* hip_stream) {
    if (!handle) return RSVD_ERR_INVALID;
    handle->stream = static_cast<hipStream_t>(hip_stream);
    return RSVD_OK;
}

int rsvd_last_hip_error(rsvd_handle_t handle) { return handle ? handle->last_hip_error : 0; }

int rsvd_set_tile_variants(rsvd_handle_t handle, const int32_t* variants) {
    if (!handle || !variants) return RSVD_ERR_INVALID;
    for (int i = 0; i < 12; ++i)
        if (variants[i] < 0 || variants[i] > 2) return RSVD_ERR_INVALID;
    for (int i = 0; i < 12; ++i) handle->variants[i] = variants[i];
    return RSVD_OK;
}

int rsvd_get_tile_variants(rsvd_handle_t handle, int32_t* variants) {
    if (!handle || !variants) return RSVD_ERR_INVALID;
    for (int i = 0; i < 12; ++i) variants[i] = handle->variants[i];
    return RSVD_OK;
}

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
    *plan = make_plan(dtype, m, n, k, params, handle->dev.num_cu, false, handle->variants);
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

int rpca_run_ex(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                int32_t k, const rpca_options* opt, const rsvd_params* params, const rpca_outputs* out,
                void* work, size_t work_bytes, rsvd_info* info) {
    if (!opt || !out) return RSVD_ERR_INVALID;
    Plan P;
    const int c = check_common(handle, dtype, m, n, A, lda, k, params, work, work_bytes, &P);
    if (c != RSVD_OK) return c;
    if (!out->rotation || out->ldr < k || !out->eigvals || (out->x && out->ldx < k) ||
        (out->x_white && out->ldxw < k) || (out->loadings && out->ldl < k))
        return RSVD_ERR_INVALID;
    SolveOut o{};
    o.U = out->x; o.ldu = out->ldx; o.V = out->rotation; o.ldv = out->ldr; o.S = nullptr;
    o.eigvals = out->eigvals; o.sdev = out->sdev; o.center_out = out->center;
    o.scale_u = 1; o.center = opt->center ? 1 : 0; o.info = info;
    o.scale = opt->scale ? 1 : 0; o.scale_out = out->scale; o.total_var = out->total_var;
    o.loadings = out->loadings; o.ldl = out->ldl; o.xwhite = out->x_white; o.ldxw = out->ldxw;
    return dispatch(handle, dtype, P, A, lda, params, o, work);
}

int rpca_predict_workspace_size(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, int32_t k,
                                size_t* bytes) {
    if (!handle || !bytes || m < 1 || n < 1 || k < 1 || k > RSVD_MAX_L_SINGLE) return RSVD_ERR_INVALID;
    if (dtype != RSVD_F64 && dtype != RSVD_F32 && dtype != RSVD_BF16) return RSVD_ERR_UNSUPPORTED;
    *bytes = predict_plan(dtype, m, n, k, handle->dev.num_cu).bytes;
    return RSVD_OK;
}

int rpca_predict(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                 int32_t k, const void* rotation, int64_t ldr, const void* center, const void* scale, void* x,
                 int64_t ldx, void* work, size_t work_bytes) {
    if (!handle || m < 1 || n < 1 || k < 1 || k > RSVD_MAX_L_SINGLE) return RSVD_ERR_INVALID;
    if (dtype != RSVD_F64 && dtype != RSVD_F32 && dtype != RSVD_BF16) return RSVD_ERR_UNSUPPORTED;
    if (!A || lda < n || !rotation || ldr < k || !x || ldx < k || !work) return RSVD_ERR_INVALID;
    if (reinterpret_cast<uintptr_t>(work) % kAlign != 0) return RSVD_ERR_INVALID;
    const PredictPlan P = predict_plan(dtype, m, n, k, handle->dev.num_cu);
    if (work_bytes < P.bytes) return RSVD_ERR_INVALID;
    hipError_t e = hipErrorInvalidValue;
    switch (dtype) {
        case RSVD_F64: e = predict_f64(handle, P, A, lda, rotation, ldr, center, scale, x, ldx, work); break;
        case RSVD_F32: e = predict_f32(handle, P, A, lda, rotation, ldr, center, scale, x, ldx, work); break;
        case RSVD_BF16: e = predict_bf16(handle, P, A, lda, rotation, ldr, center, scale, x, ldx, work); break;
        default: return RSVD_ERR_UNSUPPORTED;
    }
    return hip_status(handle, e);
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

}  // extern "C"

// ---------------------------------------------------------------- batches
// A ragged batch runs every step of the solve as one grouped launch over all
// of its matrices.  Matrices are grouped by the column class of their product
// tiles (tile_class of l: 32, 48, 64, 80, 96, 128); each group runs its solves
// as one sequence of grouped launches with as many power iterations as its
// largest q (a member's iterations beyond its own q are switched off on the
// device), the groups spread over up to six streams (the caller's and side
// streams forked from it and joined back), and inside a group the matrices
// are ordered by descending work so that the largest tiles start first.

namespace rsvd {

struct BatchGroup {
    int tile = 0;
    int lane = 0;       // stream lane: one per size class; a lane runs its groups in order
    int q = 0;          // largest q of the members (iterations issued)
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
    // learned batches: a first phase of q = 0 sketches and selector features
    // (plans0 / groups0, workspaces at offs0), the network and the choice of
    // q on the device, then the solves (plans / groups), which start from the
    // first phase's sketches
    bool learned = false;
    std::vector<rsvd::Plan> plans0;
    std::vector<size_t> offs0;
    std::vector<rsvd::BatchGroup> groups0;
    const float* theta = nullptr;
    float tau = 0.8f;
    size_t feat_off = 0, prob_off = 0, q_off = 0;
    size_t stamps_off = 0, bytes = 0;
    void* work = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t tables_bytes = 0;            // launch tables at the start of the workspace
};

namespace rsvd {

// Records the group's steps.  host = null: the first `limit` members into the
// recorder's own arrays (planning); otherwise every member directly into the
// packed host layout at host (binding), using the step list already recorded.
// phase 0: the features phase of a learned batch; phase 1: the solves.
hipError_t record_group(rsvd_batch_s* B, BatchGroup& g, int phase, void* base, size_t limit = SIZE_MAX,
                        unsigned char* host = nullptr) {
    if (host) g.rec.begin_direct(host, static_cast<int>(g.members.size()));
    else g.rec.clear();
    const bool stamps = (B->flags & RSVD_BATCH_STAMPS) != 0;
    const std::vector<Plan>& plans = phase == 0 ? B->plans0 : B->plans;
    const std::vector<size_t>& offs = phase == 0 ? B->offs0 : B->offs;
    for (size_t mi = 0; mi < g.members.size() && mi < limit; ++mi) {
        const int i = g.members[mi];
        const rsvd_batch_desc& d = B->desc[i];
        SolveOut o{};
        o.U = d.U; o.ldu = d.ldu; o.V = d.V; o.ldv = d.ldv; o.S = d.S; o.info = d.info;
        o.stamps = stamps ? at<uint64_t>(base, B->stamps_off) + 2 * static_cast<size_t>(i) : nullptr;
        if (B->flags & RSVD_BATCH_FEATURES) { o.features = d.features; o.feat_k = d.k; o.S = nullptr; o.U = nullptr; }
        if (B->learned && phase == 0) {
            o.features = at<float>(base, B->feat_off) + static_cast<size_t>(i) * RSVD_MLP_INPUTS;
            o.feat_k = d.k; o.S = nullptr; o.U = nullptr; o.V = nullptr; o.info = nullptr;
            o.stamp_sel = 1;
        } else if (B->learned) {
            o.qsrc = at<int32_t>(base, B->q_off) + i;
            o.y0 = at<unsigned char>(base, B->offs0[i] + B->plans0[i].Y);
            o.stamp_sel = 2;
        }
        g.rec.begin_problem();
        void* w = at<unsigned char>(base, offs[i]);
        hipError_t e = hipErrorInvalidValue;
        switch (B->dtype) {
            case RSVD_F64: e = solve_record_f64(g.rec, plans[i], d.A, d.lda, &B->prm, d.stream_id, o, w); break;
            case RSVD_F32: e = solve_record_f32(g.rec, plans[i], d.A, d.lda, &B->prm, d.stream_id, o, w); break;
            case RSVD_BF16: e = solve_record_bf16(g.rec, plans[i], d.A, d.lda, &B->prm, d.stream_id, o, w); break;
        }
        RSVD_TRY(e);
        if (!g.rec.complete()) return hipErrorInvalidValue;
    }
    return hipSuccess;
}

inline hipError_t record_all(rsvd_batch_s* B, void* base, unsigned char* host) {
    for (BatchGroup& g : B->groups0) RSVD_TRY(record_group(B, g, 0, base, SIZE_MAX, host + g.table_off));
    for (BatchGroup& g : B->groups) RSVD_TRY(record_group(B, g, 1, base, SIZE_MAX, host + g.table_off));
    return hipSuccess;
}

constexpr int kLearnedFallbackQ = RSVD_LEARNED_FALLBACK_Q;
constexpr int kBatchChunks = 4;     // RSVD_BATCH_CHUNKED: chunks per size class

// Group g runs on lane g % lanes: lane 0 is the caller's stream, the others
// are side streams forked from it and joined back with events.
constexpr size_t kMaxLanes = 6;

inline size_t lanes_in(const std::vector<BatchGroup>& groups) {
    size_t n = 0;
    for (const BatchGroup& g : groups) n = std::max(n, static_cast<size_t>(g.lane) + 1);
    return std::min(n, kMaxLanes);
}

inline size_t lanes_of(const rsvd_batch_s* B) {
    return std::max(lanes_in(B->groups), lanes_in(B->groups0));
}

// One phase: fork the lanes from st, each group on its lane in order, join back.
inline hipError_t launch_groups(const rsvd_batch_s* B, const std::vector<BatchGroup>& groups, hipStream_t st) {
    const unsigned char* base = static_cast<const unsigned char*>(B->work);
    const size_t lanes = lanes_in(groups);
    rsvd_handle_t h = B->h;
    if (lanes > 1) RSVD_TRY(hipEventRecord(h->fork, st));
    for (size_t s = 1; s < lanes; ++s) RSVD_TRY(hipStreamWaitEvent(h->side[s - 1], h->fork, 0));
    for (size_t g = 0; g < groups.size(); ++g) {
        const size_t ln = static_cast<size_t>(groups[g].lane) % lanes;
        hipStream_t ls = (ln == 0) ? st : h->side[ln - 1];
        RSVD_TRY(groups[g].rec.launch(base + groups[g].table_off, ls));
    }
    for (size_t s = 1; s < lanes; ++s) {
        RSVD_TRY(hipEventRecord(h->side_done[s - 1], h->side[s - 1]));
        RSVD_TRY(hipStreamWaitEvent(st, h->side_done[s - 1], 0));
    }
    return hipSuccess;
}

// The side streams belong to the handle, so planning a batch creates none.
// A learned batch runs its features phase, then the network and the choice
// of q for every matrix, then the solves, all stream-ordered on st.
inline hipError_t launch_all(const rsvd_batch_s* B, hipStream_t st) {
    if (B->learned) {
        unsigned char* base = static_cast<unsigned char*>(B->work);
        RSVD_TRY(launch_groups(B, B->groups0, st));
        RSVD_TRY(learned_choose_q(st, B->theta, static_cast<int>(B->desc.size()), at<float>(base, B->feat_off),
                                  at<float>(base, B->prob_off), B->tau, B->prm.p, kLearnedFallbackQ,
                                  at<int32_t>(base, B->q_off)));
    }
    return launch_groups(B, B->groups, st);
}

inline hipError_t make_side_streams(rsvd_batch_s* B) {
    const size_t need = lanes_of(B) > 0 ? lanes_of(B) - 1 : 0;
    rsvd_handle_t h = B->h;
    if (need && !h->fork) RSVD_TRY(hipEventCreateWithFlags(&h->fork, hipEventDisableTiming));
    while (h->side.size() < need) {
        hipStream_t s = nullptr;
        RSVD_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        h->side.push_back(s);
        hipEvent_t e = nullptr;
        RSVD_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        h->side_done.push_back(e);
    }
    return hipSuccess;
}

// Groups of one phase by tile class, each class on its own stream lane and,
// with chunks > 1, split into up to `chunks` groups of about equal work that
// its lane runs one after another (a member's solve then spans its chunk's
// launches only, not the whole batch's).  Members are ordered by descending
// work (passes over A times the sketch width), so the largest tiles start
// first; each group issues its largest q.
inline void build_groups(std::vector<Plan>& plans, std::vector<BatchGroup>& out, int chunks = 1) {
    const int count = static_cast<int>(plans.size());
    auto work = [&](int i) {
        const Plan& p = plans[i];
        return static_cast<double>(p.m) * p.n * p.l * (p.q + 1);
    };
    int lane = 0;
    for (int tile : {128, 96, 80, 64, 48, 32}) {
        std::vector<int> members;
        for (int32_t i = 0; i < count; ++i)
            if (plans[i].tile == tile) members.push_back(i);
        if (members.empty()) continue;
        std::stable_sort(members.begin(), members.end(), [&](int a, int b) { return work(a) > work(b); });
        double total = 0.0;
        for (int i : members) total += work(i);
        double acc = 0.0;
        int c = 0;
        BatchGroup g;
        g.tile = tile;
        g.lane = lane;
        for (size_t mi = 0; mi < members.size(); ++mi) {
            const int i = members[mi];
            g.members.push_back(i);
            g.q = std::max(g.q, plans[i].q);
            acc += work(i);
            const bool cut = (c + 1 < chunks) && acc >= total * (c + 1) / chunks && mi + 1 < members.size();
            if (cut || mi + 1 == members.size()) {
                for (int j : g.members) plans[j].qmax = g.q;
                out.push_back(std::move(g));
                g = BatchGroup();
                g.tile = tile;
                g.lane = lane;
                ++c;
            }
        }
        ++lane;
    }
}

// Sizes the step tables of one phase by recording one member per group
// (every member issues the same steps, and their sizes do not depend on the
// addresses), placing them in L.
inline bool size_tables(rsvd_batch_s* B, std::vector<BatchGroup>& groups, int phase, Layout& L) {
    void* fake = reinterpret_cast<void*>(static_cast<uintptr_t>(1) << 44);
    for (BatchGroup& g : groups) {
        if (record_group(B, g, phase, fake, 1) != hipSuccess) return false;
        g.table_off = L.take(g.rec.packed_bytes_for(static_cast<int>(g.members.size())));
    }
    return true;
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
    if (flags & ~(RSVD_BATCH_GRAPH | RSVD_BATCH_STAMPS | RSVD_BATCH_FEATURES | RSVD_BATCH_OWN_QP |
                  RSVD_BATCH_CHUNKED))
        return RSVD_ERR_INVALID;
    if (params->scheme != RSVD_SCHEME_QR) return RSVD_ERR_UNSUPPORTED;   // LU: single solves only
    const bool feat = (flags & RSVD_BATCH_FEATURES) != 0;
    const bool with_u = !feat && descs[0].U != nullptr;
    std::vector<rsvd_params> prm(count, *params);
    for (int32_t i = 0; i < count; ++i) {
        const rsvd_batch_desc& d = descs[i];
        if (feat) {             // q = 0 sketch of width l0 = min(max(2k, k + 20), m, n, RSVD_MAX_L)
            prm[i].q = 0;
            const int64_t l0 = std::min<int64_t>(std::min<int64_t>(std::max(2 * d.k, d.k + 20), RSVD_MAX_L),
                                                 std::min(d.m, d.n));
            prm[i].p = static_cast<int32_t>(std::max<int64_t>(0, l0 - d.k));
        } else if (flags & RSVD_BATCH_OWN_QP) {
            prm[i].q = d.q;
            prm[i].p = d.p;
        }
        const int v = validate(dtype, d.m, d.n, d.k, &prm[i], RSVD_MAX_L);
        if (v != RSVD_OK) return v;
        if (!d.A || d.lda < d.n) return RSVD_ERR_INVALID;
        if (feat) {
            if (!d.features) return RSVD_ERR_INVALID;
            continue;
        }
        if (!d.S) return RSVD_ERR_INVALID;
        if ((d.U != nullptr) != with_u || (d.U && d.ldu < d.k) || (d.V && d.ldv < d.k)) return RSVD_ERR_INVALID;
    }
    rsvd_batch_s* B = new rsvd_batch_s();
    B->h = handle; B->dtype = dtype; B->flags = flags; B->prm = *params;
    B->desc.assign(descs, descs + count);
    B->plans.resize(count);
    for (int32_t i = 0; i < count; ++i)
        B->plans[i] = make_plan(dtype, descs[i].m, descs[i].n, descs[i].k, &prm[i], handle->dev.num_cu, true,
                                handle->variants);
    build_groups(B->plans, B->groups, (flags & RSVD_BATCH_CHUNKED) ? kBatchChunks : 1);
    B->offs.assign(count, 0);
    Layout L;
    if (!size_tables(B, B->groups, 1, L)) { delete B; return RSVD_ERR_UNSUPPORTED; }
    B->tables_bytes = L.off;
    B->stamps_off = L.take(2 * sizeof(uint64_t) * static_cast<size_t>(count));
    for (int32_t i = 0; i < count; ++i) B->offs[i] = L.take(B->plans[i].bytes);
    B->bytes = L.off;
    *batch = B;
    *work_bytes = B->bytes;
    return RSVD_OK;
}

int rsvd_batch_create_learned(rsvd_handle_t handle, int32_t dtype, int32_t count, const rsvd_batch_desc* descs,
                              const rsvd_params* params, const float* theta, float tau, int32_t flags,
                              rsvd_batch_t* batch, size_t* work_bytes) {
    if (!handle || count < 1 || !descs || !params || !batch || !work_bytes) return RSVD_ERR_INVALID;
    if (flags & ~(RSVD_BATCH_GRAPH | RSVD_BATCH_STAMPS)) return RSVD_ERR_INVALID;
    if (params->p < 0 || params->p > RSVD_LEARNED_PMAX || !(tau <= 1.0f)) return RSVD_ERR_INVALID;
    if (params->scheme != RSVD_SCHEME_QR) return RSVD_ERR_UNSUPPORTED;
    const bool with_u = descs[0].U != nullptr;
    std::vector<rsvd_params> prm0(count, *params), prm1(count, *params);
    for (int32_t i = 0; i < count; ++i) {
        const rsvd_batch_desc& d = descs[i];
        // features phase: q = 0 sketch of width l0 = min(max(2k, k + 20), m, n, RSVD_MAX_L);
        // solves: q chosen on the device (at most RSVD_LEARNED_QMAX), p = params->p
        prm0[i].q = 0;
        prm0[i].probes = 0;
        const int64_t l0 = std::min<int64_t>(std::min<int64_t>(std::max(2 * d.k, d.k + 20), RSVD_MAX_L),
                                             std::min(d.m, d.n));
        prm0[i].p = static_cast<int32_t>(std::max<int64_t>(0, l0 - d.k));
        prm1[i].q = RSVD_LEARNED_QMAX;
        int v = validate(dtype, d.m, d.n, d.k, &prm0[i], RSVD_MAX_L);
        if (v == RSVD_OK) v = validate(dtype, d.m, d.n, d.k, &prm1[i], RSVD_MAX_L);
        if (v != RSVD_OK) return v;
        if (!d.A || d.lda < d.n || !d.S) return RSVD_ERR_INVALID;
        if ((d.U != nullptr) != with_u || (d.U && d.ldu < d.k) || (d.V && d.ldv < d.k)) return RSVD_ERR_INVALID;
    }
    rsvd_batch_s* B = new rsvd_batch_s();
    B->h = handle; B->dtype = dtype; B->flags = flags; B->prm = *params;
    B->learned = true; B->theta = theta; B->tau = tau;
    B->desc.assign(descs, descs + count);
    B->plans0.resize(count);
    B->plans.resize(count);
    for (int32_t i = 0; i < count; ++i) {
        const rsvd_batch_desc& d = descs[i];
        B->plans0[i] = make_plan(dtype, d.m, d.n, d.k, &prm0[i], handle->dev.num_cu, true, handle->variants);
        // the solve's bases share the sketch's leading dimension, so its
        // first l columns are the solve's Y as they stand
        B->plans[i] = make_plan(dtype, d.m, d.n, d.k, &prm1[i], handle->dev.num_cu, true, handle->variants,
                                B->plans0[i].Lp);
        if (B->plans[i].l > B->plans0[i].l || B->plans[i].Lp != B->plans0[i].Lp) { delete B; return RSVD_ERR_UNSUPPORTED; }
    }
    build_groups(B->plans0, B->groups0);
    build_groups(B->plans, B->groups);
    B->offs0.assign(count, 0);
    B->offs.assign(count, 0);
    Layout L;
    if (!size_tables(B, B->groups0, 0, L) || !size_tables(B, B->groups, 1, L)) {
        delete B;
        return RSVD_ERR_UNSUPPORTED;
    }
    B->tables_bytes = L.off;
    B->stamps_off = L.take(2 * sizeof(uint64_t) * static_cast<size_t>(count));
    B->feat_off = L.take(static_cast<size_t>(count) * RSVD_MLP_INPUTS * sizeof(float));
    B->prob_off = L.take(static_cast<size_t>(count) * RSVD_MLP_CLASSES * sizeof(float));
    B->q_off = L.take(static_cast<size_t>(count) * sizeof(int32_t));
    for (int32_t i = 0; i < count; ++i) {
        B->offs0[i] = L.take(B->plans0[i].bytes);
        B->offs[i] = L.take(B->plans[i].bytes);
    }
    B->bytes = L.off;
    *batch = B;
    *work_bytes = B->bytes;
    return RSVD_OK;
}

int rsvd_batch_choices(rsvd_batch_t batch, int32_t* q_host) {
    if (!batch || !batch->work || !batch->learned || !q_host) return RSVD_ERR_INVALID;
    rsvd_handle_t h = batch->h;
    hipError_t e = hipMemcpyAsync(q_host, static_cast<unsigned char*>(batch->work) + batch->q_off,
                                  sizeof(int32_t) * batch->desc.size(), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return hip_status(h, e);
}

int rsvd_batch_bind(rsvd_batch_t batch, void* work, size_t work_bytes) {
    if (!batch || !work || work_bytes < batch->bytes) return RSVD_ERR_INVALID;
    if (reinterpret_cast<uintptr_t>(work) % kAlign != 0) return RSVD_ERR_INVALID;
    rsvd_handle_t h = batch->h;
    drop_graph(batch);
    batch->work = nullptr;
    hipError_t e = hipSuccess;
    if (h->staging_bytes < batch->tables_bytes) {
        if (h->staging) (void)hipHostFree(h->staging);
        h->staging = nullptr;
        h->staging_bytes = 0;
        e = hipHostMalloc(reinterpret_cast<void**>(&h->staging), batch->tables_bytes, hipHostMallocDefault);
        if (e != hipSuccess) { h->staging = nullptr; return hip_status(h, e); }
        h->staging_bytes = batch->tables_bytes;
    }
    if (record_all(batch, work, h->staging) != hipSuccess) return RSVD_ERR_UNSUPPORTED;
    for (BatchGroup& g : batch->groups) {
        e = g.rec.prepare();
        if (e != hipSuccess) return hip_status(h, e);
    }
    if (batch->tables_bytes) {
        e = hipMemcpyAsync(work, h->staging, batch->tables_bytes, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_status(h, e);
    }
    e = make_side_streams(batch);
    if (e != hipSuccess) return hip_status(h, e);
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

// ------------------------------------------------------- learned (q, p)

namespace {

const int kPChoices[3] = {5, 10, 20};

int pair_cost(int k, int c) { return (2 * (c / 3) + 2) * (k + kPChoices[c % 3]); }

// Pair a dominates pair b when it has at least as many power iterations and
// at least as much oversampling.
bool dominated(int a, int b) { return a / 3 <= b / 3 && a % 3 <= b % 3; }

// Class for one matrix from the network's distribution over the cheapest
// sufficient pair: the cheapest class c (ties: lower index) whose estimated
// chance of sufficing, the probability mass of the pairs it dominates,
// reaches tau; tau <= 0 takes the most probable class.
int decide(const float* prob, int k, float tau) {
    if (tau <= 0.0f) {
        int best = 0;
        for (int c = 1; c < RSVD_MLP_CLASSES; ++c) if (prob[c] > prob[best]) best = c;
        return best;
    }
    int pick = -1, pick_cost = 0;
    for (int c = 0; c < RSVD_MLP_CLASSES; ++c) {
        double cum = 0.0;
        for (int a = 0; a < RSVD_MLP_CLASSES; ++a) if (dominated(a, c)) cum += prob[a];
        if (cum < tau) continue;
        const int cost = pair_cost(k, c);
        if (pick < 0 || cost < pick_cost) { pick = c; pick_cost = cost; }   // c ascends: ties keep the lower
    }
    return pick < 0 ? RSVD_MLP_CLASSES - 1 : pick;
}

// Workspace: features (count x 131 f32), probabilities (count x 15 f32),
// then the sketch batch's own workspace.
struct SelectLayout {
    size_t feat_off = 0, prob_off = 0, batch_off = 0, batch_bytes = 0, bytes = 0;
};

int select_plan(rsvd_handle_t handle, int32_t dtype, int32_t count, const rsvd_batch_desc* descs,
                const rsvd_params* params, float* feat, rsvd_batch_t* b, SelectLayout* lay) {
    Layout L;
    lay->feat_off = L.take(static_cast<size_t>(count) * RSVD_MLP_INPUTS * sizeof(float));
    lay->prob_off = L.take(static_cast<size_t>(count) * RSVD_MLP_CLASSES * sizeof(float));
    lay->batch_off = L.off;
    std::vector<rsvd_batch_desc> fd(descs, descs + count);
    for (int32_t i = 0; i < count; ++i) {
        fd[i].features = feat ? feat + static_cast<size_t>(i) * RSVD_MLP_INPUTS
                              : reinterpret_cast<float*>(static_cast<uintptr_t>(256));
        fd[i].U = nullptr; fd[i].V = nullptr; fd[i].S = nullptr; fd[i].info = nullptr;
    }
    rsvd_params pp{};
    if (params) { pp = *params; pp.probes = 0; }    // features need no error estimate
    size_t bb = 0;
    const int st = rsvd_batch_create(handle, dtype, count, fd.data(), params ? &pp : nullptr, RSVD_BATCH_FEATURES,
                                     b, &bb);
    if (st != RSVD_OK) return st;
    lay->batch_bytes = bb;
    lay->bytes = lay->batch_off + bb;
    return RSVD_OK;
}

}  // namespace

extern "C" {

int rsvd_select_workspace_size(rsvd_handle_t handle, int32_t dtype, int32_t count, const rsvd_batch_desc* descs,
                               const rsvd_params* params, size_t* bytes) {
    if (!bytes || !descs || count < 1) return RSVD_ERR_INVALID;
    rsvd_batch_t b = nullptr;
    SelectLayout lay;
    const int st = select_plan(handle, dtype, count, descs, params, nullptr, &b, &lay);
    if (st != RSVD_OK) return st;
    rsvd_batch_destroy(b);
    *bytes = lay.bytes;
    return RSVD_OK;
}

int rsvd_select(rsvd_handle_t handle, int32_t dtype, int32_t count, const rsvd_batch_desc* descs,
                const rsvd_params* params, const float* theta, float tau, int32_t* q_out, int32_t* p_out,
                float* features_out, void* work, size_t work_bytes) {
    if (!handle || !theta || !q_out || !p_out || !work || count < 1 || !descs) return RSVD_ERR_INVALID;
    if (reinterpret_cast<uintptr_t>(work) % kAlign != 0) return RSVD_ERR_INVALID;
    SelectLayout lay;
    float* feat_ws = at<float>(work, 0);                 // feat_off is 0
    float* feat = features_out ? features_out : feat_ws;
    rsvd_batch_t b = nullptr;
    int st = select_plan(handle, dtype, count, descs, params, feat, &b, &lay);
    if (st != RSVD_OK) return st;
    if (work_bytes < lay.bytes) { rsvd_batch_destroy(b); return RSVD_ERR_INVALID; }
    float* prob = at<float>(work, lay.prob_off);
    st = rsvd_batch_bind(b, static_cast<unsigned char*>(work) + lay.batch_off, lay.batch_bytes);
    if (st == RSVD_OK) st = rsvd_batch_run(b);
    if (st == RSVD_OK) st = rsvd_mlp_forward(handle, theta, count, feat, prob, nullptr);
    std::vector<float> host(static_cast<size_t>(count) * RSVD_MLP_CLASSES);
    if (st == RSVD_OK) {
        hipError_t e = hipMemcpyAsync(host.data(), prob, sizeof(float) * host.size(), hipMemcpyDeviceToHost,
                                      handle->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(handle->stream);
        st = hip_status(handle, e);
    }
    rsvd_batch_destroy(b);
    if (st != RSVD_OK) return st;
    for (int32_t i = 0; i < count; ++i) {
        const int c = decide(host.data() + static_cast<size_t>(i) * RSVD_MLP_CLASSES, descs[i].k, tau);
        q_out[i] = c / 3;
        p_out[i] = kPChoices[c % 3];
    }
    return RSVD_OK;
}

}  // extern "C"
