// Execution of the solve's steps: one launch per step, either for one
// problem (arguments by value) or grouped over a batch of problems.
//
// A step is a "Body": a struct with
//   static constexpr int THREADS;                    // workgroup size
//   static int blocks(const Args&);                  // workgroups for one problem
//   static size_t lds(const Args&);                  // dynamic LDS bytes
//   static __device__ void run(const Args&, int b);  // workgroup b of the problem
// Grouped launches enumerate the workgroups of all problems of the batch in
// order; workgroup t finds its problem by binary search in the prefix sums of
// the per-problem block counts (problems with no blocks are skipped).
#pragma once

#include <cstring>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace rsvd {

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2): hardware block b runs on XCD b % 8.  For one product the logical index
// gives each XCD one contiguous range of tiles, so the row tiles of one split
// (which read the same chunk of the skinny operand) share an L2.  Grouped
// launches keep the round-robin order: their blocks are sorted by problem
// size, and contiguous ranges would give one XCD all the largest problems.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_block(int b, int total) {
    const int xcd = b % kXcds, slot = b / kXcds;
    const int per = total / kXcds, rem = total % kXcds;
    return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

template <class Body>
__global__ __launch_bounds__(Body::THREADS) void single_kernel(typename Body::Args a) {
    Body::run(a, xcd_block(blockIdx.x, gridDim.x));
}

// Bodies that run two workgroups per CU at two waves per SIMD declare
// WAVES_PER_SIMD = 2; their kernel is compiled for that register budget.
template <class Body, class = void> struct waves_per_simd { static constexpr int value = 1; };
template <class Body>
struct waves_per_simd<Body, std::void_t<decltype(Body::WAVES_PER_SIMD)>> {
    static constexpr int value = Body::WAVES_PER_SIMD;
};

template <class Body>
__global__ __launch_bounds__(Body::THREADS, 2) void single_kernel_w2(typename Body::Args a) {
    Body::run(a, xcd_block(blockIdx.x, gridDim.x));
}

template <class Body>
__global__ __launch_bounds__(Body::THREADS) void grouped_kernel(const typename Body::Args* args, const int* prefix,
                                                               int nprob) {
    const int t = blockIdx.x;
    int lo = 0, hi = nprob;               // largest lo with prefix[lo] <= t
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= t) lo = mid; else hi = mid;
    }
    Body::run(args[lo], t - prefix[lo]);
}

template <typename K>
inline hipError_t raise_lds_limit(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

// Launches each step immediately for one problem.
struct SingleExec {
    static constexpr bool kSingle = true;
    hipStream_t stream;
    template <class Body>
    hipError_t run(const typename Body::Args& a) {
        const int nb = Body::blocks(a);
        if (nb <= 0) return hipSuccess;
        const size_t lds = Body::lds(a);
        static size_t raised = 0;
        if constexpr (waves_per_simd<Body>::value == 2) {
            if (lds > raised) {
                hipError_t e = raise_lds_limit(single_kernel_w2<Body>, lds);
                if (e != hipSuccess) return e;
                raised = lds;
            }
            hipLaunchKernelGGL(single_kernel_w2<Body>, dim3(nb), dim3(Body::THREADS), lds, stream, a);
        } else {
            if (lds > raised) {
                hipError_t e = raise_lds_limit(single_kernel<Body>, lds);
                if (e != hipSuccess) return e;
                raised = lds;
            }
            hipLaunchKernelGGL(single_kernel<Body>, dim3(nb), dim3(Body::THREADS), lds, stream, a);
        }
        return hipGetLastError();
    }
};

// Records the steps of several problems; problem p must issue the same
// sequence of step kinds as problem 0 (a problem with nothing to do in a step
// records zero blocks).  upload() packs every step's argument array and block
// prefix sums into device memory; launch() then issues one grouped launch per
// step with no host synchronisation.
struct BatchRecorder {
    static constexpr bool kSingle = false;
    typedef hipError_t (*LaunchFn)(hipStream_t, const void* args, const int* prefix, int nprob, int total,
                                   size_t lds);
    typedef hipError_t (*PrepFn)(size_t lds);
    struct Step {
        LaunchFn fn = nullptr;
        PrepFn prep = nullptr;
        size_t elem = 0;
        std::vector<unsigned char> args;
        std::vector<int> prefix{0};
        size_t lds = 0;
        size_t args_off = 0, prefix_off = 0;   // offsets in the packed layout
        int total = 0;                          // workgroups over all problems
    };
    static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

    std::vector<Step> steps;
    size_t cursor = 0;
    int nprob = 0;
    bool mismatch = false;
    // Direct mode: the step list is known (recorded for one problem); every
    // problem's arguments and block counts are written straight into the
    // packed host layout at `direct`, sized for `direct_n` problems.
    unsigned char* direct = nullptr;
    int direct_n = 0;

    void begin_problem() { cursor = 0; ++nprob; }

    void begin_direct(unsigned char* host, int n) {
        size_t off = 0;
        for (Step& s : steps) {
            s.args_off = off;
            off += align256(s.elem * n);
            s.prefix_off = off;
            off += align256((n + 1) * sizeof(int));
            reinterpret_cast<int*>(host + s.prefix_off)[0] = 0;
            s.total = 0;
        }
        direct = host;
        direct_n = n;
        nprob = 0;
        cursor = 0;
        mismatch = false;
    }

    // Raises the kernel's dynamic LDS limit (a host-side attribute, done
    // before any stream capture).
    template <class Body>
    static hipError_t prepare_grouped(size_t lds) {
        static size_t raised = 0;
        if (lds > raised) {
            hipError_t e = raise_lds_limit(grouped_kernel<Body>, lds);
            if (e != hipSuccess) return e;
            raised = lds;
        }
        return hipSuccess;
    }

    template <class Body>
    static hipError_t launch_grouped(hipStream_t st, const void* args, const int* prefix, int nprob, int total,
                                     size_t lds) {
        if (total <= 0) return hipSuccess;
        hipError_t e = prepare_grouped<Body>(lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(grouped_kernel<Body>, dim3(total), dim3(Body::THREADS), lds, st,
                           static_cast<const typename Body::Args*>(args), prefix, nprob);
        return hipGetLastError();
    }

    template <class Body>
    hipError_t run(const typename Body::Args& a) {
        typedef typename Body::Args Args;
        if (direct) {
            if (cursor == steps.size() || nprob > direct_n) { mismatch = true; return hipErrorInvalidValue; }
            Step& s = steps[cursor++];
            if (s.fn != &launch_grouped<Body>) { mismatch = true; return hipErrorInvalidValue; }
            std::memcpy(direct + s.args_off + static_cast<size_t>(nprob - 1) * s.elem, &a, sizeof(Args));
            int* pre = reinterpret_cast<int*>(direct + s.prefix_off);
            pre[nprob] = pre[nprob - 1] + Body::blocks(a);
            s.total = pre[nprob];
            const size_t lds = Body::lds(a);
            if (lds > s.lds) s.lds = lds;
            return hipSuccess;
        }
        if (cursor == steps.size()) {
            if (nprob != 1) { mismatch = true; return hipErrorInvalidValue; }
            Step s;
            s.fn = &launch_grouped<Body>;
            s.prep = &prepare_grouped<Body>;
            s.elem = sizeof(Args);
            steps.push_back(std::move(s));
        }
        Step& s = steps[cursor++];
        if (s.fn != &launch_grouped<Body>) { mismatch = true; return hipErrorInvalidValue; }
        const size_t off = s.args.size();
        s.args.resize(off + sizeof(Args));
        std::memcpy(s.args.data() + off, &a, sizeof(Args));
        s.prefix.push_back(s.prefix.back() + Body::blocks(a));
        s.total = s.prefix.back();
        const size_t lds = Body::lds(a);
        if (lds > s.lds) s.lds = lds;
        return hipSuccess;
    }

    // Bytes of device memory the packed arrays need.
    size_t packed_bytes() const {
        size_t b = 0;
        for (const Step& s : steps) b += align256(s.args.size()) + align256(s.prefix.size() * sizeof(int));
        return b;
    }

    // Bytes the packed arrays need for n problems that issue the steps
    // recorded so far (the sizes do not depend on the recorded values).
    size_t packed_bytes_for(int n) const {
        size_t b = 0;
        for (const Step& s : steps) b += align256(s.elem * n) + align256((n + 1) * sizeof(int));
        return b;
    }

    // Lay the arrays out in host memory at `host` (packed_bytes() bytes); the
    // device copy of those bytes is what launch() reads.
    void pack(unsigned char* host) {
        size_t off = 0;
        for (Step& s : steps) {
            s.args_off = off;
            std::memcpy(host + off, s.args.data(), s.args.size());
            off += align256(s.args.size());
            s.prefix_off = off;
            std::memcpy(host + off, s.prefix.data(), s.prefix.size() * sizeof(int));
            off += align256(s.prefix.size() * sizeof(int));
        }
    }

    hipError_t prepare() const {
        for (const Step& s : steps) {
            hipError_t e = s.prep(s.lds);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }

    void clear() { steps.clear(); cursor = 0; nprob = 0; mismatch = false; direct = nullptr; direct_n = 0; }

    // The problem just recorded issued every step that problem 0 issued.
    bool complete() const { return !mismatch && cursor == steps.size(); }

    hipError_t launch(const void* dev, hipStream_t st) const {
        const unsigned char* base = static_cast<const unsigned char*>(dev);
        for (const Step& s : steps) {
            hipError_t e = s.fn(st, base + s.args_off, reinterpret_cast<const int*>(base + s.prefix_off), nprob,
                                s.total, s.lds);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
};

}  // namespace rsvd
