// Launch and grid-synchronisation costs on the current device, for the
// launch structure of the fused primal-dual loop (benchmark harness; not
// part of the library).  A solve runs ceil(iters / K) dependent launches;
// the alternatives to a relaunch between two groups of K iterations are a
// HIP graph of the launches, or one persistent launch that synchronises its
// whole grid (a cooperative launch with its grid barrier, or a plain launch
// of a co-resident grid with a barrier on an atomic counter).  This program
// times each on empty kernels of a given grid and prints one JSON object:
//
//   plain_us         back-to-back dependent launches, per launch
//   graph_us         the same launches replayed as a HIP graph of 6, per launch
//   coop_launch_us   cooperative launch of the grid, per launch
//   coop_sync_us     one cooperative-groups grid barrier
//   atomic_sync_us   one barrier on an atomic counter (agent scope, bounded spin)
//   atomic_xchg_us   one such barrier with a store and a reload of 16 bytes per
//                    thread around it (the halo exchange of a persistent solve)
//   cross_stream_us  what a round trip through a second stream adds to a chain
//                    of dependent launches: per group of 6 launches, an event
//                    recorded after the 2nd, waited for by a second stream that
//                    records an event of its own, which the next group's first
//                    launch waits for (work moved off the chain would pay this)
//
// usage: sync_probe BLOCKS THREADS
// Every spin is bounded: a grid that is not co-resident makes the barrier
// report a timeout (printed) instead of hanging.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>

namespace cg = cooperative_groups;

namespace {

constexpr int kSpinLimit = 200000;  // polls of about a microsecond each

#define CHECK(x)                                                                  \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            exit(1);                                                              \
        }                                                                         \
    } while (0)

__global__ void k_empty(int* sink) {
    if (sink && threadIdx.x == 0 && blockIdx.x == 0x7fffffff) sink[0] = 1;
}

__global__ void k_coop(int nsync) {
    cg::grid_group g = cg::this_grid();
    for (int k = 0; k < nsync; ++k) g.sync();
}

// Barrier number k of a launch on a counter zeroed before the launch.
__device__ bool counter_barrier(unsigned* ctr, unsigned target, int* timeout) {
    __syncthreads();
    __shared__ int ok;
    if (threadIdx.x == 0) {
        ok = 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int n = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++n > kSpinLimit) {
                ok = 0;
                atomicExch(timeout, 1);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return ok != 0;
}

// nsync barriers; with xchg each thread stores 16 bytes before a barrier and
// reads those of the same thread of the next block after it.
__global__ void k_atomic(unsigned* ctr, float4* buf, int nsync, int xchg, int* timeout) {
    const size_t n = (size_t)gridDim.x * blockDim.x;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t j = (size_t)((blockIdx.x + 1) % gridDim.x) * blockDim.x + threadIdx.x;
    float4 v = make_float4(1.0f, 2.0f, 3.0f, 4.0f);
    for (int k = 0; k < nsync; ++k) {
        float4* half = buf + (size_t)(k & 1) * n;
        if (xchg) half[i] = v;
        if (!counter_barrier(ctr, (unsigned)(k + 1) * gridDim.x, timeout)) return;
        if (xchg) {
            const float4 w = half[j];
            v = make_float4(w.x + 1.0f, w.y, w.z, w.w);
        }
    }
    if (v.x == -1.0f) buf[i] = v;  // keeps the loads
}

struct Timer {
    hipEvent_t a, b;
    Timer() {
        CHECK(hipEventCreate(&a));
        CHECK(hipEventCreate(&b));
    }
    template <class F>
    float us(hipStream_t s, int reps, F&& body) {
        body();  // warm-up
        CHECK(hipStreamSynchronize(s));
        CHECK(hipEventRecord(a, s));
        for (int r = 0; r < reps; ++r) body();
        CHECK(hipEventRecord(b, s));
        CHECK(hipEventSynchronize(b));
        float ms = 0.0f;
        CHECK(hipEventElapsedTime(&ms, a, b));
        return ms * 1e3f / reps;
    }
};

}  // namespace

int main(int argc, char** argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s BLOCKS THREADS\n", argv[0]);
        return 2;
    }
    const int nb = atoi(argv[1]), nt = atoi(argv[2]);
    if (nb < 1 || nt < 64 || nt > 1024 || nt % 64) {
        fprintf(stderr, "BLOCKS >= 1, THREADS a multiple of 64 in [64, 1024]\n");
        return 2;
    }
    CHECK(hipSetDevice(0));
    hipDeviceProp_t pr;
    CHECK(hipGetDeviceProperties(&pr, 0));
    int occ_coop = 0, occ_atomic = 0;
    CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_coop, k_coop, nt, 0));
    CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_atomic, k_atomic, nt, 0));
    const int cus = pr.multiProcessorCount;
    hipStream_t s;
    CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    Timer tm;
    const int reps = 1000;

    const float plain = tm.us(s, reps, [&] { hipLaunchKernelGGL(k_empty, dim3(nb), dim3(nt), 0, s, nullptr); });

    hipGraph_t g;
    hipGraphExec_t ge;
    CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    for (int k = 0; k < 6; ++k) hipLaunchKernelGGL(k_empty, dim3(nb), dim3(nt), 0, s, nullptr);
    CHECK(hipStreamEndCapture(s, &g));
    CHECK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    const float graph = tm.us(s, reps / 6, [&] { CHECK(hipGraphLaunch(ge, s)); }) / 6.0f;
    CHECK(hipGraphExecDestroy(ge));
    CHECK(hipGraphDestroy(g));

    float coop0 = -1.0f, coop5 = -1.0f;
    if (pr.cooperativeLaunch && occ_coop * cus >= nb) {
        int ns = 0;
        void* a0[] = {&ns};
        coop0 = tm.us(s, reps / 10, [&] {
            CHECK(hipLaunchCooperativeKernel((const void*)k_coop, dim3(nb), dim3(nt), a0, 0, s));
        });
        int n5 = 5;
        void* a5[] = {&n5};
        coop5 = tm.us(s, reps / 10, [&] {
            CHECK(hipLaunchCooperativeKernel((const void*)k_coop, dim3(nb), dim3(nt), a5, 0, s));
        });
    }

    float at0 = -1.0f, at5 = -1.0f, ax5 = -1.0f;
    int timed_out = 0;
    if (occ_atomic * cus >= nb) {
        unsigned* ctr;
        int* to;
        float4* buf;
        CHECK(hipMalloc(&ctr, 256));
        CHECK(hipMalloc(&to, 256));
        CHECK(hipMalloc(&buf, 2 * (size_t)nb * nt * sizeof(float4)));
        CHECK(hipMemset(to, 0, 256));
        CHECK(hipMemset(buf, 0, 2 * (size_t)nb * nt * sizeof(float4)));
        auto run = [&](int nsync, int xchg) {
            return tm.us(s, reps / 10, [&] {
                CHECK(hipMemsetAsync(ctr, 0, sizeof(unsigned), s));
                hipLaunchKernelGGL(k_atomic, dim3(nb), dim3(nt), 0, s, ctr, buf, nsync, xchg, to);
            });
        };
        at0 = run(0, 0);
        at5 = run(5, 0);
        ax5 = run(5, 1);
        CHECK(hipMemcpy(&timed_out, to, sizeof(int), hipMemcpyDeviceToHost));
        CHECK(hipFree(ctr));
        CHECK(hipFree(to));
        CHECK(hipFree(buf));
    }
    // cross-stream round trip inside a chain of dependent launches
    float cross = -1.0f;
    {
        hipStream_t b2;
        hipEvent_t ea, eb;
        CHECK(hipStreamCreateWithFlags(&b2, hipStreamNonBlocking));
        CHECK(hipEventCreateWithFlags(&ea, hipEventDisableTiming));
        CHECK(hipEventCreateWithFlags(&eb, hipEventDisableTiming));
        const int groups = 200;
        auto chain = [&](bool via) {
            return tm.us(s, groups, [&] {
                if (via) CHECK(hipStreamWaitEvent(s, eb, 0));
                for (int k = 0; k < 6; ++k) {
                    hipLaunchKernelGGL(k_empty, dim3(nb), dim3(nt), 0, s, nullptr);
                    if (via && k == 1) {
                        CHECK(hipEventRecord(ea, s));
                        CHECK(hipStreamWaitEvent(b2, ea, 0));
                        CHECK(hipEventRecord(eb, b2));
                    }
                }
            });
        };
        CHECK(hipEventRecord(eb, b2));
        const float plain6 = chain(false), via6 = chain(true);
        cross = via6 - plain6;
        CHECK(hipStreamSynchronize(b2));
        CHECK(hipEventDestroy(ea));
        CHECK(hipEventDestroy(eb));
        CHECK(hipStreamDestroy(b2));
    }
    auto per = [](float with, float without, int n) {
        return with < 0.0f || without < 0.0f ? -1.0f : (with - without) / n;
    };
    printf("{\"device\": \"%s\", \"cus\": %d, \"blocks\": %d, \"threads\": %d, "
           "\"coresident_blocks_per_cu\": %d, \"plain_us\": %.3f, \"graph_us\": %.3f, "
           "\"coop_launch_us\": %.3f, \"coop_sync_us\": %.3f, \"atomic_launch_us\": %.3f, "
           "\"atomic_sync_us\": %.3f, \"atomic_xchg_us\": %.3f, \"cross_stream_us\": %.3f, "
           "\"barrier_timeout\": %d}\n",
           pr.gcnArchName, cus, nb, nt, occ_atomic, plain, graph, coop0, per(coop5, coop0, 5), at0,
           per(at5, at0, 5), per(ax5, at0, 5), cross, timed_out);
    CHECK(hipStreamDestroy(s));
    return timed_out ? 3 : 0;
}
