// Device kernels for event-manifold intensity reconstruction on gfx950.
//
//   k_init          workspace initialisation
//   k_push_small    validate + scatter one push in a single workgroup
//   k_validate / k_scatter / k_push_finalize   the same for large pushes
//   k_build         data image f, time differences tx/ty, reset counts
//   k_finish        commit folded-event state / reset counts after a one-launch solve
//   k_primal, k_dual    one primal-dual iteration as two plain kernels
//   k_rotate        p into / out of each pixel's tangent frame (plain loop)
//   k_pd_fused      several iterations per HBM round trip on a register tile;
//                   its first launch of a solve (an instantiation of its own)
//                   can also bin the block's events and build f, tx, ty
//   k_pd_fused_batch    the same over the tiles of many streams
//   k_tvl1_*        timestamp denoising (FP64)
//   k_gap, k_gap_final  primal-dual gap and energy (FP64 accumulation)
//   k_time_plane, k_metric_plane   readback helpers
#include <hip/hip_ext.h>
#include <stdlib.h>

#include <atomic>

#include "kernels.h"
#include "pd_math.h"
#include "tile.h"

namespace rec {

namespace {

__device__ __forceinline__ int32_t event_error(int64_t t, int64_t prev, uint16_t x, uint16_t y,
                                               int8_t pol, int32_t W, int32_t H) {
    if (pol != 1 && pol != -1) return kErrInval;
    if (x >= W || y >= H) return kErrRange;
    if (t < prev) return kErrOrder;
    return 0;
}

__device__ __forceinline__ int64_t resolved_last(int64_t tl, int64_t t_first) {
    return tl == kNever ? t_first : tl;
}

// Fault injection for tests of the error paths: with REC_FAULT_AFTER=n in
// the environment (read at the first launch), every launch after the
// process's first n fails with hipErrorLaunchFailure and is not issued.
std::atomic<long long> g_launches{0};

long long fault_after() {
    static const long long n = [] {
        const char* e = getenv("REC_FAULT_AFTER");
        return e && *e ? atoll(e) : -1LL;
    }();
    return n;
}

// Launch with optional timing events carried by the dispatch itself.
template <typename Kern, typename... Args>
hipError_t launch(Kern kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, hipEvent_t a,
                  hipEvent_t z, Args... args) {
    const long long fa = fault_after();
    if (fa >= 0 && g_launches.fetch_add(1, std::memory_order_relaxed) >= fa)
        return hipErrorLaunchFailure;
    if (a || z)
        hipExtLaunchKernelGGL(kernel, grid, block, lds, s, a, z, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    return hipGetLastError();
}

inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

// Storage of the dual field p and of the time differences tx, ty.  The
// arithmetic is FP32 in every case; 16-bit forms round on store (RNE) and
// widen exactly on load.  tx, ty are rounded before use, so every launch
// of a solve sees the same metric.
struct StoreF32 {
    using T = float;
    static __device__ __forceinline__ float ld(const T* a, size_t k) { return a[k]; }
    static __device__ __forceinline__ void st(T* a, size_t k, float v) { a[k] = v; }
    static __device__ __forceinline__ float round(float v) { return v; }
};
// FP16 saturates at its largest finite value instead of rounding to
// infinity: a time difference above 65504 (a pixel idle for more than
// 65.5 s at T_s = 1 ms next to one that fires now) would otherwise turn the
// frame of that pixel into inf * 0 = NaN.  Such a pixel has G > 4.29e9 and
// beta = tau lambda sqrt(G) > 1.7e6, so its u is clamp(f) to within FP32
// either way; p, whose ball radius is sqrt(G), saturates likewise.  NaN
// stays NaN.
struct StoreF16 {
    using T = _Float16;
    static __device__ __forceinline__ float sat(float v) {
        constexpr float kMax = 65504.0f;
        return __builtin_fabsf(v) > kMax ? __builtin_copysignf(kMax, v) : v;
    }
    static __device__ __forceinline__ float ld(const T* a, size_t k) { return (float)a[k]; }
    static __device__ __forceinline__ void st(T* a, size_t k, float v) { a[k] = (_Float16)sat(v); }
    static __device__ __forceinline__ float round(float v) { return (float)(_Float16)sat(v); }
};
struct StoreBF16 {
    using T = uint16_t;
    static __device__ __forceinline__ uint16_t enc(float v) {  // round to nearest even
        uint32_t u = __float_as_uint(v);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    }
    static __device__ __forceinline__ float dec(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
    static __device__ __forceinline__ float ld(const T* a, size_t k) { return dec(a[k]); }
    static __device__ __forceinline__ void st(T* a, size_t k, float v) { a[k] = enc(v); }
    static __device__ __forceinline__ float round(float v) { return dec(enc(v)); }
};

// ---------------------------------------------------------------- init

__global__ void k_init(Planes P, size_t np, float u_init, int keep_u) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) {
        DevState* st = P.st;
        st->t_ref = 0;
        st->t_first = 0;
        st->first_bad = kNoBad;
        st->batch_events = 0;
        st->last_events = 0;
        st->started = 0;
        st->err = 0;
        st->pend_t_ref = 0;
        st->pend_t_first = 0;
        st->pend_events = 0;
        st->pend_accepted = 0;
        st->pend_err = 0;
    }
    if (k >= np) return;
    float u = keep_u ? P.u[0][k] : u_init;
    P.u[0][k] = u;
    P.f[k] = u;
    P.p[0][k] = 0.0f;
    P.p[0][np + k] = 0.0f;
    P.p[0][2 * np + k] = 0.0f;
    P.tx[k] = 0.0f;
    P.ty[k] = 0.0f;
    P.t_last[k] = kNever;
    P.npos[k] = 0;
    P.nneg[k] = 0;
}

// ---------------------------------------------------------------- push

__device__ __forceinline__ void scatter_one(const Planes& P, int32_t W, int64_t t, uint16_t x,
                                            uint16_t y, int8_t pol) {
    const size_t k = (size_t)y * W + x;
    if (pol > 0)
        atomicAdd(P.npos + k, 1);
    else
        atomicAdd(P.nneg + k, 1);
    atomicMax((long long*)(P.t_last + k), (long long)t);
}

__device__ __forceinline__ void accept_push(DevState* st, int64_t t0, int64_t tn, int64_t n) {
    if (!st->started) {
        st->started = 1;
        st->t_first = t0;
    }
    st->t_ref = tn;
    st->batch_events += n;
}

__device__ __forceinline__ void reject_push(DevState* st, int32_t code) {
    if (st->err == 0) st->err = code;
}

__global__ __launch_bounds__(1024) void k_push_small(Planes P, Frame fr, const int64_t* t,
                                                     const uint16_t* x, const uint16_t* y,
                                                     const int8_t* pol, int64_t n) {
    __shared__ unsigned long long first_bad;
    DevState* st = P.st;
    if (threadIdx.x == 0) first_bad = (unsigned long long)kNoBad;
    __syncthreads();
    const int64_t prev0 = st->started ? st->t_ref : INT64_MIN;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t prev = i ? t[i - 1] : prev0;
        if (event_error(t[i], prev, x[i], y[i], pol[i], fr.W, fr.H))
            atomicMin(&first_bad, (unsigned long long)i);
    }
    __syncthreads();
    const int64_t fb = (int64_t)first_bad;
    if (fb != kNoBad) {
        if (threadIdx.x == 0) {
            const int64_t prev = fb ? t[fb - 1] : prev0;
            reject_push(st, event_error(t[fb], prev, x[fb], y[fb], pol[fb], fr.W, fr.H));
        }
        return;
    }
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) scatter_one(P, fr.W, t[i], x[i], y[i], pol[i]);
    if (threadIdx.x == 0) accept_push(st, t[0], t[n - 1], n);
}

__global__ void k_validate(Planes P, Frame fr, const int64_t* t, const uint16_t* x,
                           const uint16_t* y, const int8_t* pol, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    DevState* st = P.st;
    const int64_t prev = i ? t[i - 1] : (st->started ? st->t_ref : INT64_MIN);
    if (event_error(t[i], prev, x[i], y[i], pol[i], fr.W, fr.H))
        atomicMin((unsigned long long*)&st->first_bad, (unsigned long long)i);
}

__global__ void k_scatter(Planes P, Frame fr, const int64_t* t, const uint16_t* x,
                          const uint16_t* y, const int8_t* pol, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (P.st->first_bad != kNoBad) return;
    scatter_one(P, fr.W, t[i], x[i], y[i], pol[i]);
}

__global__ void k_push_finalize(Planes P, Frame fr, const int64_t* t, const uint16_t* x,
                                const uint16_t* y, const int8_t* pol, int64_t n) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    DevState* st = P.st;
    const int64_t fb = st->first_bad;
    if (fb != kNoBad) {
        const int64_t prev = fb ? t[fb - 1] : (st->started ? st->t_ref : INT64_MIN);
        reject_push(st, event_error(t[fb], prev, x[fb], y[fb], pol[fb], fr.W, fr.H));
        st->first_bad = kNoBad;
        return;
    }
    accept_push(st, t[0], t[n - 1], n);
}

// ---------------------------------------------------------------- build

// Forward differences of the time surface from the latest timestamps of a
// pixel (tl), its right (tr) and lower (td) neighbours:
// tau(x+1) - tau(x) = (t_last(x) - t_last(x+1)) / T_s from the exact int64
// difference, divided in FP64 and rounded once; 0 on the last column / row
// and everywhere when T_s = 0 (flat manifold).
__device__ __forceinline__ void time_diffs(int64_t tl, int64_t tr, int64_t td, bool has_r,
                                           bool has_d, int64_t t0, const BuildConsts& b,
                                           float& dx, float& dy) {
    dx = 0.0f;
    dy = 0.0f;
    if (b.ts > 0.0) {
        const int64_t l = resolved_last(tl, t0);
        if (has_r) dx = (float)div_ts((double)(l - resolved_last(tr, t0)), b);
        if (has_d) dy = (float)div_ts((double)(l - resolved_last(td, t0)), b);
    }
}

__global__ void k_build(Planes P, Frame fr, int cur, BuildConsts bc, int time_mem) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    DevState* st = P.st;
    if (k == 0) {
        st->last_events = st->batch_events;
        st->batch_events = 0;
    }
    if (k >= np) return;
    const int32_t j = (int32_t)(k % fr.W), i = (int32_t)(k / fr.W);
    P.f[k] = data_image(P.u[cur][k], P.npos[k], P.nneg[k], bc.dpos, bc.dneg);
    P.npos[k] = 0;
    P.nneg[k] = 0;
    if (time_mem) return;  // tx, ty come from the timestamp denoising
    const bool hr = j < fr.W - 1, hd = i < fr.H - 1;
    float dx, dy;
    time_diffs(P.t_last[k], hr ? P.t_last[k + 1] : kNever, hd ? P.t_last[k + fr.W] : kNever, hr,
               hd, st->t_first, bc, dx, dy);
    P.tx[k] = dx;
    P.ty[k] = dy;
}

// Commits the stream state left pending by a solve's first fused launch.
__device__ __forceinline__ void commit_pending(DevState* st) {
    if (st->pend_accepted) {
        if (!st->started) {
            st->started = 1;
            st->t_first = st->pend_t_first;
        }
        st->t_ref = st->pend_t_ref;
    }
    if (st->pend_err && st->err == 0) st->err = st->pend_err;
    st->last_events = st->pend_events;
    st->batch_events = 0;
    st->pend_accepted = 0;
    st->pend_err = 0;
}

// After a solve that had a single fused launch: commit and reset counts.
__global__ void k_finish(Planes P, size_t np, int zero_counts) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) commit_pending(P.st);
    if (zero_counts && k < np) {
        P.npos[k] = 0;
        P.nneg[k] = 0;
    }
}

__global__ void k_time_plane(Planes P, Frame fr, double ts, float* out) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const DevState* st = P.st;
    const int64_t tl = resolved_last(P.t_last[k], st->t_first);
    out[k] = ts > 0.0 ? (float)((double)(st->t_ref - tl) / ts) : 0.0f;
}

// Latest timestamps with pixels that never fired resolved to the stream's
// first timestamp (0 before any event was accepted).
__global__ void k_tlast_plane(Planes P, Frame fr, int64_t* out) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    out[k] = resolved_last(P.t_last[k], P.st->t_first);
}

// State import: u, p (standard basis) and the latest timestamps into the
// current planes; counts cleared.  The stream state was written by the host
// before the launch, with t_first = INT64_MAX when started: the stream's
// first timestamp becomes the earliest imported one.
template <class S>
__global__ void k_import(Planes P, size_t np, int cur, const float* u, const float* p,
                         const int64_t* t_last, int started) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    // each thread reads its own pixel of the staging before any write, and
    // only its own pixel is written: staging and state may overlap no other
    // thread's data
    const float uu = u[k];
    const float a = p ? p[k] : 0.0f, b = p ? p[np + k] : 0.0f, c = p ? p[2 * np + k] : 0.0f;
    const int64_t tl = started ? t_last[k] : kNever;
    typename S::T* pc = (typename S::T*)P.p[cur];
    P.u[cur][k] = uu;
    S::st(pc, k, a);
    S::st(pc, np + k, b);
    S::st(pc, 2 * np + k, c);
    P.t_last[k] = tl;
    P.npos[k] = 0;
    P.nneg[k] = 0;
    if (started) atomicMin((long long*)&P.st->t_first, (long long)tl);
}

template <class S>
__global__ void k_metric_plane(Planes P, Frame fr, float* out) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const float tx = S::ld((const typename S::T*)P.tx, k), ty = S::ld((const typename S::T*)P.ty, k);
    out[k] = __builtin_fmaf(tx, tx, __builtin_fmaf(ty, ty, 1.0f));
}

// Widens n stored values to FP32 (readback of 16-bit planes).
template <class S>
__global__ void k_widen(const void* src, float* out, size_t n) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = S::ld((const typename S::T*)src, k);
}

// ---------------------------------------------------------------- event binning

// Folded events of the first launch, binned for one tile region (LDS).
struct ScanState {
    unsigned long long seg_bad[kMaxSegs];  // first event failing its own checks, per push
    int seg_ok[kMaxSegs];                  // push accepted
    int all_ok;                            // every push accepted
    long long t_first;                     // stream's first timestamp after the pushes
    long long t_ref;                       // latest accepted timestamp after the pushes
};

struct TileBins {
    ScanState* ss;
    int64_t t_ref;    // latest accepted timestamp after the pushes
    int32_t* pos;     // RH x CW counts
    int32_t* neg;
    long long* tmax;  // (RH + 1) x (CW + 1) latest timestamps (one extra column and row)
    int64_t t_first;  // stream's first timestamp after this block's events
};

// Binning of the folded pushes of a solve's first launch, for the tile
// region [rx0, rx0 + CW] x [ry0, ry0 + RH], in two calls:
//  bin_clear  lays out and zeroes the LDS bins;
//  bin_scan   validates the pushes in order (each all-or-nothing, with the
//             same error codes as a scattered push) and bins the accepted
//             events.
// The scan reads every event once: it bins each event while checking it and
// only when a push turns out to be rejected (rare) clears the bins and bins
// the accepted pushes again.  The caller issues its per-pixel loads between
// the two calls, so their latency overlaps the event loads.  Every
// workgroup takes the same decisions; the lead workgroup records the
// outcome as pending state.
__device__ void bin_clear(int RH, int CW, unsigned char* lds, TileBins& tb) {
    __shared__ ScanState ss;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid < kMaxSegs) ss.seg_bad[tid] = (unsigned long long)kNoBad;
    tb.ss = &ss;
    tb.pos = (int32_t*)lds;
    tb.neg = tb.pos + RH * CW;
    tb.tmax = (long long*)(tb.neg + RH * CW);
    for (int q = tid; q < RH * CW; q += nt) {
        tb.pos[q] = 0;
        tb.neg[q] = 0;
    }
    for (int q = tid; q < (RH + 1) * (CW + 1); q += nt) tb.tmax[q] = kNever;
    __syncthreads();
}

// Bins one event (its fields already loaded).
__device__ __forceinline__ void bin_event(int64_t t, int x, int y, int8_t pol, int RH, int CW,
                                          int rx0, int ry0, TileBins& tb) {
    const int lc = x - rx0, lr = y - ry0;
    if (lc < 0 || lc > CW || lr < 0 || lr > RH) return;
    atomicMax(&tb.tmax[lr * (CW + 1) + lc], (long long)t);
    if (lc < CW && lr < RH) atomicAdd(pol > 0 ? &tb.pos[lr * CW + lc] : &tb.neg[lr * CW + lc], 1);
}
__device__ __forceinline__ void bin_one(const EventSegs& segs, int s, int64_t i, int RH, int CW,
                                        int rx0, int ry0, TileBins& tb) {
    bin_event(segs.t[s][i], segs.x[s][i], segs.y[s][i], segs.p[s][i], RH, CW, rx0, ry0, tb);
}

__device__ void bin_scan(const Planes& P, Frame fr, const EventSegs& segs, int RH, int CW,
                         int rx0, int ry0, bool lead, TileBins& tb) {
    ScanState& ss = *tb.ss;
    const int tid = threadIdx.x, nt = blockDim.x;
    DevState* st = P.st;
    // what the in-order decisions below need for the first push (nearly
    // always the only one), loaded by thread 0 ahead of the event pass so
    // that the loads overlap it
    int32_t started = 0;
    int64_t st_ref = 0, st_first = 0, st_events = 0, t0 = 0, tn = 0;
    uint16_t x0 = 0, y0 = 0;
    int8_t p0 = 0;
    if (tid == 0) {
        started = st->started;
        st_ref = st->t_ref;
        st_first = st->t_first;
        st_events = st->batch_events;
        if (segs.count > 0) {
            t0 = segs.t[0][0];
            tn = segs.t[0][segs.n[0] - 1];
            x0 = segs.x[0][0];
            y0 = segs.y[0][0];
            p0 = segs.p[0][0];
        }
    }
    // per-event checks (each push's first event is checked against the
    // running reference time in sequence below), binning as we go
    // (all fields of an event, and the previous timestamp, are loaded before
    // any check, so that their loads are in flight together instead of
    // waiting on each other through the checks' branches)
    for (int s = 0; s < segs.count; ++s) {
        const int64_t* t = segs.t[s];
        const uint16_t* xs = segs.x[s];
        const uint16_t* ys = segs.y[s];
        const int8_t* ps = segs.p[s];
        for (int64_t i = tid; i < segs.n[s]; i += nt) {
            int64_t ti = t[i], tp = t[i > 0 ? i - 1 : 0];
            int xi = xs[i], yi = ys[i], pi = ps[i];
            asm volatile("" : "+v"(ti), "+v"(tp), "+v"(xi), "+v"(yi), "+v"(pi));
            const int64_t prev = i > 0 ? tp : INT64_MIN;
            if (event_error(ti, prev, (uint16_t)xi, (uint16_t)yi, (int8_t)pi, fr.W, fr.H))
                atomicMin(&ss.seg_bad[s], (unsigned long long)i);
            else
                bin_event(ti, xi, yi, (int8_t)pi, RH, CW, rx0, ry0, tb);
        }
    }
    __syncthreads();
    if (tid == 0) {
        int64_t ref = started ? st_ref : INT64_MIN;
        int64_t first = kNever, last = 0, accepted = 0;
        int32_t err = 0;
        int ok_all = 1;
        for (int s = 0; s < segs.count; ++s) {
            const int64_t* t = segs.t[s];
            const int64_t ts0 = s == 0 ? t0 : t[0];
            const int64_t fb = (int64_t)ss.seg_bad[s];
            int32_t code = 0;
            if (fb == 0)
                code = s == 0 ? event_error(t0, INT64_MIN, x0, y0, p0, fr.W, fr.H)
                              : event_error(t[0], INT64_MIN, segs.x[s][0], segs.y[s][0],
                                            segs.p[s][0], fr.W, fr.H);
            else if (ts0 < ref)
                code = kErrOrder;
            else if (fb != kNoBad)
                code = event_error(segs.t[s][fb], segs.t[s][fb - 1], segs.x[s][fb],
                                   segs.y[s][fb], segs.p[s][fb], fr.W, fr.H);
            ss.seg_ok[s] = code == 0;
            if (code == 0) {
                if (first == kNever) first = ts0;
                ref = s == 0 ? tn : t[segs.n[s] - 1];
                last = ref;
                accepted += segs.n[s];
            } else {
                ok_all = 0;
                if (err == 0) err = code;
            }
        }
        ss.all_ok = ok_all;
        ss.t_first = started ? st_first : (first == kNever ? 0 : first);
        ss.t_ref = accepted > 0 ? last : st_ref;
        if (lead) {
            st->pend_t_ref = last;
            st->pend_t_first = first;
            st->pend_accepted = accepted > 0;
            st->pend_events = st_events + accepted;
            st->pend_err = err;
        }
    }
    __syncthreads();
    if (!ss.all_ok) {
        // a rejected push: bin the accepted pushes again from clear bins
        for (int q = tid; q < RH * CW; q += nt) {
            tb.pos[q] = 0;
            tb.neg[q] = 0;
        }
        for (int q = tid; q < (RH + 1) * (CW + 1); q += nt) tb.tmax[q] = kNever;
        __syncthreads();
        for (int s = 0; s < segs.count; ++s) {
            if (!ss.seg_ok[s]) continue;
            for (int64_t i = tid; i < segs.n[s]; i += nt) bin_one(segs, s, i, RH, CW, rx0, ry0, tb);
        }
        __syncthreads();
    }
    tb.t_first = ss.t_first;
    tb.t_ref = ss.t_ref;
}

// ---------------------------------------------------------------- timestamp denoising

// Section 4 denoises the timestamps with a few TV-L1 iterations before the
// manifold is built: Chambolle-Pock for  min_v TV(v) + lambda |v - tau|_1
// (isotropic forward-difference TV, steps 1/sqrt(8), v_0 = tau, dual 0),
// in FP64.  tau = (t_ref - t_last) / T_s.
__global__ void k_tvl1_init(Planes P, Frame fr, double ts) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const DevState* st = P.st;
    const double t0 = (double)(st->t_ref - resolved_last(P.t_last[k], st->t_first)) / ts;
    P.tv0[k] = t0;
    P.tv[0][k] = t0;
    P.tq[k] = 0.0;
    P.tq[np + k] = 0.0;
}

// v+ = tau + shrink(v + s div q - tau, s lambda) into tv[cur ^ 1].
__global__ void k_tvl1_primal(Planes P, Frame fr, int cur, double lambda) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const int j = (int)(k % fr.W), i = (int)(k / fr.W);
    const double s = 0.35355339059327373;  // 1 / sqrt(8)
    const double* qx = P.tq;
    const double* qy = P.tq + np;
    double d = 0.0;
    if (j < fr.W - 1) d += qx[k];
    if (j > 0) d -= qx[k - 1];
    if (i < fr.H - 1) d += qy[k];
    if (i > 0) d -= qy[k - fr.W];
    const double w = P.tv[cur][k] + s * d - P.tv0[k];
    const double t = s * lambda;
    const double r = w > t ? w - t : (w < -t ? w + t : 0.0);
    P.tv[cur ^ 1][k] = P.tv0[k] + r;
}

// q+ = q / max(1, |q|) with q = q + s grad(2 v+ - v).
__global__ void k_tvl1_dual(Planes P, Frame fr, int cur) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const int j = (int)(k % fr.W), i = (int)(k / fr.W);
    const double s = 0.35355339059327373;
    const double* vo = P.tv[cur];
    const double* vn = P.tv[cur ^ 1];
    const double b = 2.0 * vn[k] - vo[k];
    const double gx = j < fr.W - 1 ? (2.0 * vn[k + 1] - vo[k + 1]) - b : 0.0;
    const double gy = i < fr.H - 1 ? (2.0 * vn[k + fr.W] - vo[k + fr.W]) - b : 0.0;
    const double a = P.tq[k] + s * gx, c = P.tq[np + k] + s * gy;
    double m = sqrt(a * a + c * c);
    if (m < 1.0) m = 1.0;
    P.tq[k] = a / m;
    P.tq[np + k] = c / m;
}

// tx, ty = forward differences of the denoised surface, rounded once.
template <class S>
__global__ void k_tvl1_finish(Planes P, Frame fr, int cur) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const int j = (int)(k % fr.W), i = (int)(k / fr.W);
    const double* v = P.tv[cur];
    const float dx = j < fr.W - 1 ? (float)(v[k + 1] - v[k]) : 0.0f;
    const float dy = i < fr.H - 1 ? (float)(v[k + fr.W] - v[k]) : 0.0f;
    S::st((typename S::T*)P.tx, k, dx);
    S::st((typename S::T*)P.ty, k, dy);
}

// The same denoising in one launch for up to kTvl1FusedMax iterations: a
// 64 x 16R register tile (R rows per lane, 16 wavefronts) with a halo of
// iters + 1 pixels runs every iteration in registers (neighbours through DPP
// and LDS, as in the primal-dual tile) and writes tx, ty of its interior.
// R = 1 spreads a small frame over more compute units (the FP64 iteration
// is bound by each unit's arithmetic), R = 2 wastes less on halos.
// Each pixel's arithmetic and its order are those of the kernels above.
// With folded pushes (segs.count > 0) the tile first validates and bins the
// block's events like the primal-dual build launch does (without recording
// any state: that launch bins them again and commits), so the surface it
// denoises already holds the block's latest timestamps.

__device__ __forceinline__ double lane_from_left_d(double v) {
    return __hiloint2double(__float_as_int(lane_from_left(__int_as_float(__double2hiint(v)))),
                            __float_as_int(lane_from_left(__int_as_float(__double2loint(v)))));
}
__device__ __forceinline__ double lane_from_right_d(double v) {
    return __hiloint2double(__float_as_int(lane_from_right(__int_as_float(__double2hiint(v)))),
                            __float_as_int(lane_from_right(__int_as_float(__double2loint(v)))));
}

template <class S, int R>
__global__ __launch_bounds__(1024) void k_tvl1_fused(Planes P, Frame fr, double ts, int iters,
                                                     double lambda, EventSegs segs, int tiles_x,
                                                     int ntiles) {
    extern __shared__ unsigned char dyn_lds[];
    constexpr int NW = 16, RH = R * NW;
    const int KH = iters + 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tile = xcd_tile(blockIdx.x, ntiles);
    const int tyi = tile / tiles_x, txi = tile - tyi * tiles_x;
    const int rx0 = txi * (64 - 2 * KH) - KH, ry0 = tyi * (RH - 2 * KH) - KH;
    const int gx = rx0 + lane;
    const int gy0 = ry0 + wave * R;
    const bool col_in = gx >= 0 && gx < fr.W;
    const bool hx = gx < fr.W - 1, lx = gx > 0;
    const DevState* st = P.st;
    int64_t t_ref = st->t_ref, t_first = st->t_first;
    const bool events = segs.count > 0;
    TileBins tb;
    tb.tmax = nullptr;
    if (events) {
        bin_clear(RH, 64, dyn_lds, tb);
        bin_scan(P, fr, segs, RH, 64, rx0, ry0, false, tb);
        t_ref = tb.t_ref;
        t_first = tb.t_first;
    }
    const double s = 0.35355339059327373;  // 1 / sqrt(8)
    const double tl = s * lambda;
    double v0[R], v[R], q1[R], q2[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int gy = gy0 + r;
        v0[r] = 0.0;
        if (col_in && gy >= 0 && gy < fr.H) {
            int64_t tl = P.t_last[(size_t)gy * fr.W + gx];
            if (events) tl = max(tl, (int64_t)tb.tmax[(wave * R + r) * 65 + lane]);
            v0[r] = (double)(t_ref - resolved_last(tl, t_first)) / ts;
        }
        v[r] = v0[r];
        q1[r] = 0.0;
        q2[r] = 0.0;
    }
    // xq[w + 1]: wavefront w's last q2 row; xb[w]: its first row of 2 vn - v
    // (then of v); xq[0] and xb[NW] stay zero
    __shared__ double xq[NW + 1][64];
    __shared__ double xb[NW + 1][64];
    if (wave == 0) xq[0][lane] = 0.0;
    if (wave == NW - 1) xb[NW][lane] = 0.0;
    for (int it = 0; it < iters; ++it) {
        double qxl[R], vn[R], b[R];
#pragma unroll
        for (int r = 0; r < R; ++r) qxl[r] = lane_from_left_d(q1[r]);
        xq[wave + 1][lane] = q2[R - 1];
        __syncthreads();
        const double qy_top = xq[wave][lane];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int gy = gy0 + r;
            double d = 0.0;
            if (hx) d += q1[r];
            if (lx) d -= qxl[r];
            if (gy < fr.H - 1) d += q2[r];
            if (gy > 0) d -= r > 0 ? q2[r - 1] : qy_top;
            const double w = v[r] + s * d - v0[r];
            const double rr = w > tl ? w - tl : (w < -tl ? w + tl : 0.0);
            vn[r] = v0[r] + rr;
            b[r] = 2.0 * vn[r] - v[r];
        }
        xb[wave][lane] = b[0];
        __syncthreads();
        const double b_bot = xb[wave + 1][lane];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int gy = gy0 + r;
            const double br = lane_from_right_d(b[r]);
            const double bd = r < R - 1 ? b[r + 1] : b_bot;
            const double gxx = hx ? br - b[r] : 0.0;
            const double gyy = gy < fr.H - 1 ? bd - b[r] : 0.0;
            const double a = q1[r] + s * gxx, c = q2[r] + s * gyy;
            double m = sqrt(a * a + c * c);
            if (m < 1.0) m = 1.0;
            q1[r] = a / m;
            q2[r] = c / m;
            v[r] = vn[r];
        }
        // the next iteration writes xq and xb only after its first barrier,
        // which every wavefront reaches after reading them here
    }
    __syncthreads();  // every wavefront has read xb before it is reused
    xb[wave][lane] = v[0];
    __syncthreads();
    const double v_bot = xb[wave + 1][lane];
    const bool col_out = col_in && lane >= KH && lane < 64 - KH;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = wave * R + r, gy = gy0 + r;
        const double vr = lane_from_right_d(v[r]);
        const double vd = r < R - 1 ? v[r + 1] : v_bot;
        if (!(col_out && row >= KH && row < RH - KH && gy >= 0 && gy < fr.H)) continue;
        const size_t k = (size_t)gy * fr.W + gx;
        const float dx = hx ? (float)(vr - v[r]) : 0.0f;
        const float dy = gy < fr.H - 1 ? (float)(vd - v[r]) : 0.0f;
        S::st((typename S::T*)P.tx, k, dx);
        S::st((typename S::T*)P.ty, k, dy);
    }
}

// ---------------------------------------------------------------- plain loop

// Coefficients of pixel k for the iteration on frame coordinates.
__device__ __forceinline__ CoefT pixel_coef(const Planes& P, Frame fr, const IterConsts& kc,
                                            size_t k, int i, int j) {
    const Basis b = make_basis(P.tx[k], P.ty[k]);
    return make_coef_t(b, P.f[k], kc.taulam, kc.sigma, j < fr.W - 1, i < fr.H - 1);
}

// Primal half-step for every pixel: needs q here, at the left and at the
// upper neighbour (0 where the neighbour is outside the image); p holds
// frame coordinates.
__global__ __launch_bounds__(256) void k_primal(Planes P, Frame fr, IterConsts kc, int cur) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (j >= fr.W || i >= fr.H) return;
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)i * fr.W + j;
    const float* p = P.p[cur];
    const CoefT c = pixel_coef(P, fr, kc, k, i, j);
    const float qx = q_x(c, p[k], p[np + k], p[2 * np + k]);
    const float qy = q_y(c, p[k], p[np + k], p[2 * np + k]);
    float qxl = 0.0f, qyu = 0.0f;
    if (j > 0) {
        const size_t kl = k - 1;
        qxl = q_x(pixel_coef(P, fr, kc, kl, i, j - 1), p[kl], p[np + kl], p[2 * np + kl]);
    }
    if (i > 0) {
        const size_t ku = k - fr.W;
        qyu = q_y(pixel_coef(P, fr, kc, ku, i - 1, j), p[ku], p[np + ku], p[2 * np + ku]);
    }
    P.u[cur ^ 1][k] = primal(P.u[cur][k], qx, qy, qxl, qyu, c, kc.ts, kc.umin, kc.umax);
}

// Dual half-step: needs the extrapolated primal here, right and below.
__global__ __launch_bounds__(256) void k_dual(Planes P, Frame fr, IterConsts kc, int cur) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (j >= fr.W || i >= fr.H) return;
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)i * fr.W + j;
    const float* uo = P.u[cur];
    const float* un = P.u[cur ^ 1];
    const float ut = extrapolate(un[k], uo[k]);
    float gx = 0.0f, gy = 0.0f;
    if (j < fr.W - 1) gx = extrapolate(un[k + 1], uo[k + 1]) - ut;
    if (i < fr.H - 1) gy = extrapolate(un[k + fr.W], uo[k + fr.W]) - ut;
    const CoefT c = pixel_coef(P, fr, kc, k, i, j);
    const float* p = P.p[cur];
    float p1 = p[k], p2 = p[np + k], p3 = p[2 * np + k];
    dual(p1, p2, p3, gx, gy, c);
    float* po = P.p[cur ^ 1];
    po[k] = p1;
    po[np + k] = p2;
    po[2 * np + k] = p3;
}

// p of every pixel into its frame (to = 1) or back to the standard basis
// (to = 0), in place (two-kernel loop; FP32 storage).
__global__ __launch_bounds__(256) void k_rotate(Planes P, Frame fr, int cur, int to) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    float* p = P.p[cur];
    const Basis b = make_basis(P.tx[k], P.ty[k]);
    float p1 = p[k], p2 = p[np + k], p3 = p[2 * np + k];
    if (to)
        to_frame(b, p1, p2, p3);
    else
        from_frame(b, p1, p2, p3);
    p[k] = p1;
    p[np + k] = p2;
    p[2 * np + k] = p3;
}

// ---------------------------------------------------------------- fused loop

// K primal-dual iterations per launch on a register tile.  A workgroup of
// NW wavefronts forms NV = NW * 64 / CW lane rows of CW lanes (CW = 64 or
// 32) and covers a CW-column x (NV*R)-row region: lane = column within its
// lane row, each lane holds R consecutive rows in registers, lane row v
// holds rows [v*R, v*R + R).  Horizontal neighbours come from adjacent
// lanes (DPP), vertical ones from the lane's own registers or, across lane
// rows, through LDS.  Each iteration widens the dependency cone by one
// pixel, so after K iterations the region minus a K-pixel border is exact;
// only that interior is written.  Reads (u, p) from buffer `cur`, writes
// `cur ^ 1`.  (32-column tiles halve the pixels per workgroup of a tile
// of the same height: small frames, whose time goes into the latency of
// each iteration on one compute unit, run faster on them.)
//
// mode & kBuild (the solve's first launch): instead of loading f, tx, ty, the
//   tile forms them from u (still u_prev), the event counts and the latest
//   timestamps with the arithmetic of k_build, and writes f, tx, ty and the
//   new latest timestamps for its interior.  With kEvents the block's
//   not-yet-scattered pushes are validated and binned in LDS first
//   (dynamic LDS); with kCounts the scattered counts are added.
// mode & kZero: resets the scattered counts of the interior at the end.
// mode & kCommit: block 0 commits the pending stream state.
// mode & kRotIn: p is loaded in the standard basis and rotated into each
//   pixel's tangent frame (the solve's first launch); otherwise p holds
//   frame coordinates already.
// mode & kRotOut: p is rotated back to the standard basis before it is
//   stored (the solve's last launch).
//
// The tile geometry uses a halo of KG >= K pixels (the batched launch keeps
// one geometry for all launches of a solve); tile (txi, tyi) covers the
// region whose interior starts at (txi, tyi) * (CW - 2 KG, NV R - 2 KG).
// `lead`: this tile does the per-stream duties (commit, pending state).
// B = (mode & kBuild): the first launch of a solve is a kernel of its own,
// so that the others carry no branch of the build path.
template <int R, int NW, int CW, class S, bool B>
__device__ __forceinline__ void pd_tile(const Planes& P, Frame fr, const IterConsts& kc,
                                        const BuildConsts& bc, const EventSegs& segs, int cur,
                                        int K, int KG, int mode, int txi, int tyi, bool lead,
                                        unsigned char* dyn_lds) {
    static_assert(CW == 64 || CW == 32, "lane rows of 64 or 32 lanes");
    constexpr int NV = NW * (64 / CW);  // lane rows
    constexpr int RH = NV * R;
    const int col = threadIdx.x & (CW - 1);
    const int v = threadIdx.x / CW;
    const int wave = threadIdx.x >> 6;
    const int OW = CW - 2 * KG, OH = RH - 2 * KG;
    const int rx0 = txi * OW - KG, ry0 = tyi * OH - KG;
    const int gx = rx0 + col;
    const int gy0 = ry0 + v * R;
    const size_t np = (size_t)fr.W * fr.H;
    const float* __restrict__ uin = P.u[cur];
    const typename S::T* __restrict__ pin = (const typename S::T*)P.p[cur];
    typename S::T* __restrict__ txs = (typename S::T*)P.tx;
    typename S::T* __restrict__ tys = (typename S::T*)P.ty;

    if ((mode & kCommit) && lead && threadIdx.x == 0) commit_pending(P.st);

    constexpr bool build = B;  // mode & kBuild (separate instantiations)
    const bool events = build && (mode & kEvents) != 0;
    TileBins tb;
    tb.ss = nullptr;
    tb.pos = tb.neg = nullptr;
    tb.tmax = nullptr;
    tb.t_first = 0;
    const bool col_in = gx >= 0 && gx < fr.W;
    const bool col_out = col_in && col >= KG && col < CW - KG;
    // Tile-relative 32-bit element offsets.  The tile's rows lie within RH
    // image rows of its first row clamped into the image (yb), so an offset
    // from the per-tile plane bases fits 32 bits for every frame size, and
    // the loads and stores take the scalar-base + vector-offset form.
    // Coordinates are clamped into the image: outside the image a lane reads
    // an edge pixel's (finite) values, which never reach a pixel inside it,
    // because the outside pixel's coefficients are zero.
    const int yb = min(max(ry0, 0), fr.H - 1);
    const size_t tb0 = (size_t)yb * fr.W;
    const uint32_t gxc = (uint32_t)min(max(gx, 0), fr.W - 1);
    auto eoff = [&](int r) -> uint32_t {  // (row offset < RH, W < 2^16: 24-bit product)
        const int gyc = min(max(gy0 + r, 0), fr.H - 1);
        return __umul24((uint32_t)(gyc - yb), (uint32_t)fr.W) + gxc;
    };
    const typename S::T* __restrict__ txb = txs + tb0;
    const typename S::T* __restrict__ tyb = tys + tb0;
    // The building launch also reads the latest timestamps of the right and
    // lower neighbours (the pixel's own where the neighbour would lie
    // outside the image: a value the time differences then do not use).
    const int64_t* __restrict__ tlb = P.t_last + tb0;
    auto eoff_r = [&](int r) -> uint32_t { return eoff(r) + (gxc + 1 < (uint32_t)fr.W ? 1u : 0u); };
    auto eoff_d = [&](int r) -> uint32_t {
        const int gyc = min(max(gy0 + r, 0), fr.H - 1);
        return eoff(r) + (gyc + 1 < fr.H ? (uint32_t)fr.W : 0u);
    };

    // First launch with few rows per lane: the pixel loads are issued
    // between clearing the bins and scanning the events, so that their
    // latency overlaps the event loads (with more rows the registers they
    // hold would cost occupancy).
    constexpr bool kEarly = B && R <= 2;
    float eu[R], ea[R], eb[R], ed[R];
    int64_t etl[R], etr[R], etd[R];
    int32_t enp[R], enn[R];
    if (events) bin_clear(RH, CW, dyn_lds, tb);
    if constexpr (kEarly) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t e = eoff(r);
            eu[r] = *at(uin + tb0, e);
            ea[r] = S::ld(at(pin + tb0, e), 0);
            eb[r] = S::ld(at(pin + np + tb0, e), 0);
            ed[r] = S::ld(at(pin + 2 * np + tb0, e), 0);
            etl[r] = *at(tlb, e);
            etr[r] = *at(tlb, eoff_r(r));
            etd[r] = *at(tlb, eoff_d(r));
            enp[r] = enn[r] = 0;
            if (mode & kCounts) {
                enp[r] = *at(P.npos + tb0, e);
                enn[r] = *at(P.nneg + tb0, e);
            }
        }
    }
    if (events) {
        bin_scan(P, fr, segs, RH, CW, rx0, ry0, lead, tb);
    } else if (build) {
        tb.t_first = P.st->t_first;
        if (lead && threadIdx.x == 0) {
            DevState* st = P.st;
            st->pend_accepted = 0;
            st->pend_err = 0;
            st->pend_events = st->batch_events;
        }
    }

    float u[R], p1[R], p2[R], p3[R], txr[R], tyr[R];
    CoefT c[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int gy = gy0 + r;
        const bool in = col_in && gy >= 0 && gy < fr.H;
        const uint32_t e = eoff(r);
        float uu, a, b, d, f, tx, ty;
        if constexpr (!build) {
            uu = *at(uin + tb0, e);
            a = S::ld(at(pin + tb0, e), 0);
            b = S::ld(at(pin + np + tb0, e), 0);
            d = S::ld(at(pin + 2 * np + tb0, e), 0);
            f = *at(P.f + tb0, e);
            tx = S::ld(at(txb, e), 0);
            ty = S::ld(at(tyb, e), 0);
        } else {
            int32_t npos = 0, nneg = 0;
            int64_t tl, tr, td;
            if constexpr (kEarly) {
                uu = eu[r];
                a = ea[r];
                b = eb[r];
                d = ed[r];
                tl = etl[r];
                tr = etr[r];
                td = etd[r];
                npos = enp[r];
                nneg = enn[r];
            } else {
                uu = *at(uin + tb0, e);
                a = S::ld(at(pin + tb0, e), 0);
                b = S::ld(at(pin + np + tb0, e), 0);
                d = S::ld(at(pin + 2 * np + tb0, e), 0);
                tl = *at(tlb, e);
                tr = *at(tlb, eoff_r(r));
                td = *at(tlb, eoff_d(r));
                if (mode & kCounts) {
                    npos = *at(P.npos + tb0, e);
                    nneg = *at(P.nneg + tb0, e);
                }
            }
            const int lr = v * R + r;
            const bool hr = in && gx < fr.W - 1, hd = in && gy < fr.H - 1;
            if (events) {
                npos += tb.pos[lr * CW + col];
                nneg += tb.neg[lr * CW + col];
                tl = max(tl, (int64_t)tb.tmax[lr * (CW + 1) + col]);
                tr = max(tr, (int64_t)tb.tmax[lr * (CW + 1) + col + 1]);
                td = max(td, (int64_t)tb.tmax[(lr + 1) * (CW + 1) + col]);
            }
            // (without events the factor is exp(0) = 1: f = u_prev exactly,
            // and a row of lanes without events skips the FP64 exp)
            f = (npos | nneg) != 0 ? data_image(uu, npos, nneg, bc.dpos, bc.dneg) : uu;
            if (mode & kTimeMem) {
                tx = S::ld(at(txb, e), 0);
                ty = S::ld(at(tyb, e), 0);
            } else {
                time_diffs(tl, tr, td, hr, hd, tb.t_first, bc, tx, ty);
                tx = S::round(tx);
                ty = S::round(ty);
            }
            if (in && col_out && lr >= KG && lr < RH - KG) {
                *at(P.f + tb0, e) = f;
                if (!(mode & kTimeMem)) {
                    S::st(at(txs + tb0, e), 0, tx);
                    S::st(at(tys + tb0, e), 0, ty);
                }
                if (events) *at(P.t_last + tb0, e) = tl;
            }
        }
        // pixels outside the image get all-zero coefficients, so their q is 0
        c[r] = make_coef_t(make_basis(tx, ty), f, kc.taulam, kc.sigma, in && gx < fr.W - 1,
                           in && gy < fr.H - 1);
        txr[r] = tx;
        tyr[r] = ty;
        u[r] = uu;
        p1[r] = a;
        p2[r] = b;
        p3[r] = d;
    }
    // (a separate pass: a branch inside the loop above would keep the
    // compiler from issuing all rows' loads ahead of the arithmetic)
    if (mode & kRotIn) {
#pragma unroll
        for (int r = 0; r < R; ++r) to_frame(make_basis(txr[r], tyr[r]), p1[r], p2[r], p3[r]);
    }

    // The output planes' bases are read before the loop and held in scalar
    // registers (read after it, their loads would sit on the launch's
    // critical path before the stores).
    float* __restrict__ uout = P.u[cur ^ 1];
    typename S::T* __restrict__ pout = (typename S::T*)P.p[cur ^ 1];
    asm volatile("" : "+s"(uout), "+s"(pout));

    // Rows that cross lane rows go through LDS.  xq[v + 1] holds lane row
    // v's last q_y row and xu[v] its first extrapolated row; xq[0] and
    // xu[NV] stay zero (nothing above the first / below the last lane row),
    // so every lane row reads its neighbour row unconditionally.
    __shared__ float xq[NV + 1][CW];
    __shared__ float xu[NV + 1][CW];
    if constexpr (NV > 1) {
        if (v == 0) xq[0][col] = 0.0f;
        if (v == NV - 1) xu[NV][col] = 0.0f;
    }

    // With up to 8 rows per lane the loop runs two iterations per trip, with
    // u alternating between two register sets, so that passing u from one
    // iteration to the next needs no register copies (8 rows: 31 instead of
    // 32 VALU instructions per pixel-iteration in the same 120 VGPRs; with
    // 16 rows the register pressure undoes the gain).  A wavefront skips the
    // iterations that cannot reach the exact interior: with 2 rows per lane
    // about a third of them at K = 13, with 4 rows a seventh (640x480 at
    // K = 13: +3.5 %), with 8 rows none up to K = 8.
    constexpr bool kSkip = NW > 1;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // med3 takes one scalar operand (umin): umax is held in a vector
    // register once, instead of being copied into one every iteration.
    float umax = kc.umax;
    asm volatile("" : "+v"(umax));
    // A skipped wavefront leaves uo as it was: it stays skipped for the rest
    // of the launch (the exact region only shrinks), its rows lie outside
    // the stored interior, and its registers feed no other row, so the stale
    // (finite) values are never used.
    auto step = [&](int it1, float (&ui)[R], float (&uo)[R]) {
        if (!kSkip || tile_rows_active<R * (64 / CW), NW>(wv, it1))
            tile_iteration<R, NV, CW>(ui, uo, p1, p2, p3, c, kc.ts, kc.umin, umax, col, v, xq,
                                      xu);
        else
            tile_skip<NW>();
    };
    int it = 0;
    if constexpr (R <= 8) {
        float ub[R];
#pragma unroll
        for (int r = 0; r < R; ++r) ub[r] = u[r];
        for (; it + 1 < K; it += 2) {
            step(it + 1, u, ub);
            step(it + 2, ub, u);
        }
    }
    for (; it < K; ++it) step(it + 1, u, u);

    // The offsets are formed again after the loop (a few instructions per
    // row) instead of being held in registers through it; a stored pixel
    // lies inside the image, so its offset needs no clamping.
    int gy0e = gy0, gxe = gx;
    asm volatile("" : "+v"(gy0e), "+v"(gxe));
    auto eoff2 = [&](int r) -> uint32_t {
        const int gyc = min(max(gy0e + r, 0), fr.H - 1);
        return __umul24((uint32_t)(gyc - yb), (uint32_t)fr.W) +
               (uint32_t)min(max(gxe, 0), fr.W - 1);
    };
    auto eoff_in = [&](int r) -> uint32_t {
        return __umul24((uint32_t)(gy0e + r - yb), (uint32_t)fr.W) + (uint32_t)gxe;
    };
    if (mode & kRotOut) {
        // tx, ty as stored (this launch wrote them if it built them)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t e = eoff2(r);
            txr[r] = S::ld(at(txb, e), 0);
            tyr[r] = S::ld(at(tyb, e), 0);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) from_frame(make_basis(txr[r], tyr[r]), p1[r], p2[r], p3[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = v * R + r;
        const int gy = gy0 + r;
        if (col_out && row >= KG && row < RH - KG && gy >= 0 && gy < fr.H) {
            const uint32_t e = eoff_in(r);
            *at(uout + tb0, e) = u[r];
            S::st(at(pout + tb0, e), 0, p1[r]);
            S::st(at(pout + np + tb0, e), 0, p2[r]);
            S::st(at(pout + 2 * np + tb0, e), 0, p3[r]);
            if (mode & kZero) {
                *at(P.npos + tb0, e) = 0;
                *at(P.nneg + tb0, e) = 0;
            }
        }
    }
}

template <int R, int NW, int CW, class S, bool B>
__global__ __launch_bounds__(64 * NW) void k_pd_fused(Planes P, Frame fr, IterConsts kc,
                                                      BuildConsts bc, EventSegs segs, int cur,
                                                      int K, int mode, int tiles_x,
                                                      Divider tiles_x_div, int ntiles) {
    extern __shared__ unsigned char dyn_lds[];
    const int tile = xcd_tile(blockIdx.x, ntiles);
    const int tyi = divide(tile, tiles_x_div), txi = tile - tyi * tiles_x;
    pd_tile<R, NW, CW, S, B>(P, fr, kc, bc, segs, cur, K, K, mode, txi, tyi, tile == 0, dyn_lds);
}

// One launch over the tiles of many streams (a work list of (stream, tile)
// pairs); every stream runs the same iterations with its own planes,
// constants and folded events.  launch = index of this launch in the solve
// (selects the stream's first-launch and second-launch modes and the
// ping-pong parity); last: the solve's last launch.
template <int R, int NW, int CW, class S, bool B>
__global__ __launch_bounds__(64 * NW) void k_pd_fused_batch(const StreamDesc* __restrict__ descs,
                                                            const int2* __restrict__ work,
                                                            int nwork, int K, int KG,
                                                            int launch, int last) {
    extern __shared__ unsigned char dyn_lds[];
    const int2 w = work[xcd_tile(blockIdx.x, nwork)];
    const StreamDesc& d = descs[w.x];
    const int tyi = divide(w.y, d.tiles_x_div), txi = w.y - tyi * d.tiles_x;
    const int mode = (launch == 0 ? d.mode0 : (launch == 1 ? d.mode1 : 0)) | (last ? kRotOut : 0);
    pd_tile<R, NW, CW, S, B>(d.P, d.fr, d.kc, d.bc, d.segs, d.cur ^ (launch & 1), K, KG, mode,
                             txi, tyi, w.y == 0, dyn_lds);
}

// After a one-launch batched solve: commit and reset counts of every stream.
__global__ void k_finish_batch(const StreamDesc* __restrict__ descs, int nstreams) {
    const int s = blockIdx.y;
    if (s >= nstreams) return;
    const StreamDesc& d = descs[s];
    const size_t np = (size_t)d.fr.W * d.fr.H;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) commit_pending(d.P.st);
    if ((d.mode1 & kZero) && k < np) {
        d.P.npos[k] = 0;
        d.P.nneg[k] = 0;
    }
}

// ---------------------------------------------------------------- gap

__device__ __forceinline__ double warp_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Per-pixel gap terms and energy in FP64 from the FP32 state:
//   term1 = s |A| - <A, p>,   A = L_g u
//   term2 = (u - v)(b + d) - b f log(u / v),  d = L_g^* p, b = lambda s,
//           v = clamp(b f / (b + d)) if b + d > 0 else u_max
//   energy = s |A| + b (u - f log u)
template <class S>
__global__ __launch_bounds__(kGapBlock) void k_gap(Planes P, Frame fr, double lambda,
                                                   double umin, double umax, int cur,
                                                   int rotated) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double g = 0.0, e = 0.0;
    if (k < np) {
        const int j = (int)(k % fr.W), i = (int)(k / fr.W);
        const float* u = P.u[cur];
        const typename S::T* p = (const typename S::T*)P.p[cur];
        const typename S::T* txs = (const typename S::T*)P.tx;
        const typename S::T* tys = (const typename S::T*)P.ty;
        // p of pixel kk in the standard basis (mid-solve the planes hold
        // frame coordinates: rotated back with the FP32 arithmetic of the
        // solve's last launch)
        auto ld_p = [&](size_t kk, double& a, double& b, double& d) {
            float p1 = S::ld(p, kk), p2 = S::ld(p, np + kk), p3 = S::ld(p, 2 * np + kk);
            if (rotated) from_frame(make_basis(S::ld(txs, kk), S::ld(tys, kk)), p1, p2, p3);
            a = p1;
            b = p2;
            d = p3;
        };
        auto qxy = [&](size_t kk, double& qx, double& qy) {
            const double tx = S::ld(txs, kk), ty = S::ld(tys, kk);
            const double G = 1.0 + tx * tx + ty * ty;
            double a, b, d;
            ld_p(kk, a, b, d);
            qx = ((1.0 + ty * ty) * a - tx * ty * b + tx * d) / G;
            qy = (-tx * ty * a + (1.0 + tx * tx) * b + ty * d) / G;
        };
        const double tx = S::ld(txs, k), ty = S::ld(tys, k);
        const double G = 1.0 + tx * tx + ty * ty;
        const double s = sqrt(G);
        const double uk = u[k];
        const double ux = j < fr.W - 1 ? (double)u[k + 1] - uk : 0.0;
        const double uy = i < fr.H - 1 ? (double)u[k + fr.W] - uk : 0.0;
        const double A1 = ((1.0 + ty * ty) * ux - tx * ty * uy) / G;
        const double A2 = ((1.0 + tx * tx) * uy - tx * ty * ux) / G;
        const double A3 = (tx * ux + ty * uy) / G;
        const double nA = sqrt(A1 * A1 + A2 * A2 + A3 * A3);
        double pk1, pk2, pk3;
        ld_p(k, pk1, pk2, pk3);
        const double t1 = s * nA - (A1 * pk1 + A2 * pk2 + A3 * pk3);
        double qx, qy, qxl = 0.0, qyu = 0.0, dummy;
        qxy(k, qx, qy);
        if (j > 0) qxy(k - 1, qxl, dummy);
        if (i > 0) qxy(k - fr.W, dummy, qyu);
        const double div = (j < fr.W - 1 ? qx : 0.0) - (j > 0 ? qxl : 0.0) +
                           (i < fr.H - 1 ? qy : 0.0) - (i > 0 ? qyu : 0.0);
        const double d = -div;
        const double b = lambda * s;
        const double f = P.f[k];
        double v = umax;
        if (b + d > 0.0) v = fmin(fmax(b * f / (b + d), umin), umax);
        const double t2 = (uk - v) * (b + d) - b * f * log(uk / v);
        g = t1 + t2;
        e = s * nA + b * (uk - f * log(uk));
    }
    __shared__ double sg[kGapBlock / 64], se[kGapBlock / 64];
    g = warp_sum(g);
    e = warp_sum(e);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sg[w] = g;
        se[w] = e;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < kGapBlock / 64; ++q) {
            a += sg[q];
            b += se[q];
        }
        P.gap_part[2 * blockIdx.x] = a;
        P.gap_part[2 * blockIdx.x + 1] = b;
    }
}

// Fixed-order sum of the per-block partials into history slot `slot`.
__global__ __launch_bounds__(256) void k_gap_final(Planes P, size_t nblocks, int slot) {
    __shared__ double sg[256], se[256];
    double a = 0.0, b = 0.0;
    for (size_t q = threadIdx.x; q < nblocks; q += 256) {
        a += P.gap_part[2 * q];
        b += P.gap_part[2 * q + 1];
    }
    sg[threadIdx.x] = a;
    se[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sg[threadIdx.x] += sg[threadIdx.x + w];
            se[threadIdx.x] += se[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        P.gap_hist[2 * slot] = sg[0];
        P.gap_hist[2 * slot + 1] = se[0];
    }
}

template <int R, int NW, int CW, class S>
hipError_t fused_launch(const Planes& P, Frame fr, IterConsts kc, BuildConsts bc,
                        const EventSegs& segs, int cur, int K, int mode, hipStream_t s,
                        LaunchEv ev) {
    const int OW = CW - 2 * K, OH = NW * (64 / CW) * R - 2 * K;
    if (K < 1 || OW <= 0 || OH <= 0) return hipErrorInvalidValue;
    const int tiles_x = (fr.W + OW - 1) / OW;
    const int tiles_y = (fr.H + OH - 1) / OH;
    const int ntiles = tiles_x * tiles_y;
    const size_t lds = fused_lds_bytes(R, NW, CW, mode);
    const Divider txd = make_divider((uint32_t)tiles_x);
    if (mode & kBuild)
        return launch(k_pd_fused<R, NW, CW, S, true>, dim3(ntiles), dim3(64 * NW), lds, s,
                      ev.start, ev.stop, P, fr, kc, bc, segs, cur, K, mode, tiles_x, txd, ntiles);
    return launch(k_pd_fused<R, NW, CW, S, false>, dim3(ntiles), dim3(64 * NW), lds, s, ev.start,
                  ev.stop, P, fr, kc, bc, segs, cur, K, mode, tiles_x, txd, ntiles);
}

template <int R, int NW, int CW, class S>
hipError_t batch_launch(const StreamDesc* descs, const int2* work, int nwork, int K, int KG,
                        int launch_idx, bool last, bool bins, hipStream_t s, LaunchEv ev) {
    constexpr int RH = NW * (64 / CW) * R;
    if (K < 1 || K > KG || CW - 2 * KG <= 0 || RH - 2 * KG <= 0) return hipErrorInvalidValue;
    // every stream's first-launch mode builds (launch 0 only)
    const size_t lds = fused_lds_bytes(R, NW, CW, bins ? kEvents : 0);
    if (launch_idx == 0)
        return launch(k_pd_fused_batch<R, NW, CW, S, true>, dim3(nwork), dim3(64 * NW), lds, s,
                      ev.start, ev.stop, descs, work, nwork, K, KG, launch_idx, last ? 1 : 0);
    return launch(k_pd_fused_batch<R, NW, CW, S, false>, dim3(nwork), dim3(64 * NW), lds, s,
                  ev.start, ev.stop, descs, work, nwork, K, KG, launch_idx, last ? 1 : 0);
}

}  // namespace

size_t gap_blocks(size_t np) { return (np + kGapBlock - 1) / kGapBlock; }

size_t fused_lds_bytes(int rows, int waves, int cols, int mode) {
    if (!(mode & kEvents)) return 0;
    const size_t RH = (size_t)rows * waves * (64 / cols), CW = cols;
    return 2 * RH * CW * sizeof(int32_t) + (RH + 1) * (CW + 1) * sizeof(long long);
}

int fused_tiles(Frame fr, int rows, int waves, int cols, int iters) {
    const int OW = cols - 2 * iters, OH = rows * waves * (64 / cols) - 2 * iters;
    if (OW <= 0 || OH <= 0) return -1;
    return ((fr.W + OW - 1) / OW) * ((fr.H + OH - 1) / OH);
}

hipError_t launch_init(const Planes& P, Frame fr, float u_init, bool keep_u, hipStream_t s) {
    const size_t np = (size_t)fr.W * fr.H;
    return launch(k_init, dim3(blocks_for(np, 256)), dim3(256), 0, s, nullptr, nullptr, P, np,
                  u_init, keep_u ? 1 : 0);
}

hipError_t launch_push(const Planes& P, Frame fr, const int64_t* t, const uint16_t* x,
                       const uint16_t* y, const int8_t* pol, int64_t n, hipStream_t s,
                       LaunchEv ev) {
    if (n <= 0) return hipSuccess;
    if (n <= kSmallPush)
        return launch(k_push_small, dim3(1), dim3(1024), 0, s, ev.start, ev.stop, P, fr, t, x, y,
                      pol, n);
    const unsigned g = blocks_for((size_t)n, 256);
    hipError_t e = launch(k_validate, dim3(g), dim3(256), 0, s, ev.start, nullptr, P, fr, t, x, y,
                          pol, n);
    if (e == hipSuccess)
        e = launch(k_scatter, dim3(g), dim3(256), 0, s, nullptr, nullptr, P, fr, t, x, y, pol, n);
    if (e == hipSuccess)
        e = launch(k_push_finalize, dim3(1), dim3(64), 0, s, nullptr, ev.stop, P, fr, t, x, y, pol,
                   n);
    return e;
}

hipError_t launch_build(const Planes& P, Frame fr, int cur, BuildConsts bc, bool time_mem,
                        hipStream_t s, LaunchEv ev) {
    const size_t np = (size_t)fr.W * fr.H;
    return launch(k_build, dim3(blocks_for(np, 256)), dim3(256), 0, s, ev.start, ev.stop, P, fr,
                  cur, bc, time_mem ? 1 : 0);
}

namespace {
// Tiles of the one-launch denoiser with R rows per lane (64 x 16R pixels,
// halo iters + 1), or -1 if the halo leaves no interior.
int tvl1_tiles_r(Frame fr, int iters, int R) {
    const int kh = iters + 1, ow = 64 - 2 * kh, oh = 16 * R - 2 * kh;
    if (ow <= 0 || oh <= 0) return -1;
    return ((fr.W + ow - 1) / ow) * ((fr.H + oh - 1) / oh);
}

// One row per lane when those tiles fit on the compute units at once (one
// 1024-lane workgroup each; MI355X has 256), else two.
constexpr int kTvl1OneRowTiles = 256;
int tvl1_rows(Frame fr, int iters) {
    const int n1 = tvl1_tiles_r(fr, iters, 1);
    return n1 > 0 && n1 <= kTvl1OneRowTiles ? 1 : 2;
}
}  // namespace

int tvl1_tiles(Frame fr, int iters) {
    if (iters > kTvl1FusedMax) return -1;
    return tvl1_tiles_r(fr, iters, tvl1_rows(fr, iters));
}

hipError_t launch_tvl1(const Planes& P, Frame fr, double ts, int iters, double lambda,
                       int storage, const EventSegs& segs, hipStream_t s, LaunchEv ev) {
    const size_t np = (size_t)fr.W * fr.H;
    if (iters <= kTvl1FusedMax) {
        const int kh = iters + 1, R = tvl1_rows(fr, iters);
        const int tiles_x = (fr.W + 64 - 2 * kh - 1) / (64 - 2 * kh);
        const int nt = tvl1_tiles(fr, iters);
        if (nt <= 0) return hipErrorInvalidValue;
        const dim3 gt(nt), bt(1024);
        const size_t lds = segs.count > 0 ? fused_lds_bytes(R, 16, 64, kEvents) : 0;
        if (R == 1) {
            if (storage == kStoreF16)
                return launch(k_tvl1_fused<StoreF16, 1>, gt, bt, lds, s, ev.start, ev.stop, P,
                              fr, ts, iters, lambda, segs, tiles_x, nt);
            if (storage == kStoreBF16)
                return launch(k_tvl1_fused<StoreBF16, 1>, gt, bt, lds, s, ev.start, ev.stop, P,
                              fr, ts, iters, lambda, segs, tiles_x, nt);
            return launch(k_tvl1_fused<StoreF32, 1>, gt, bt, lds, s, ev.start, ev.stop, P, fr,
                          ts, iters, lambda, segs, tiles_x, nt);
        }
        if (storage == kStoreF16)
            return launch(k_tvl1_fused<StoreF16, 2>, gt, bt, lds, s, ev.start, ev.stop, P, fr,
                          ts, iters, lambda, segs, tiles_x, nt);
        if (storage == kStoreBF16)
            return launch(k_tvl1_fused<StoreBF16, 2>, gt, bt, lds, s, ev.start, ev.stop, P, fr,
                          ts, iters, lambda, segs, tiles_x, nt);
        return launch(k_tvl1_fused<StoreF32, 2>, gt, bt, lds, s, ev.start, ev.stop, P, fr, ts,
                      iters, lambda, segs, tiles_x, nt);
    }
    if (segs.count > 0) return hipErrorInvalidValue;  // pushes must be scattered first
    const dim3 g(blocks_for(np, 256)), b(256);
    hipError_t e = launch(k_tvl1_init, g, b, 0, s, ev.start, nullptr, P, fr, ts);
    int cur = 0;
    for (int it = 0; it < iters && e == hipSuccess; ++it) {
        e = launch(k_tvl1_primal, g, b, 0, s, nullptr, nullptr, P, fr, cur, lambda);
        if (e == hipSuccess) e = launch(k_tvl1_dual, g, b, 0, s, nullptr, nullptr, P, fr, cur);
        cur ^= 1;
    }
    if (e != hipSuccess) return e;
    if (storage == kStoreF16)
        return launch(k_tvl1_finish<StoreF16>, g, b, 0, s, nullptr, ev.stop, P, fr, cur);
    if (storage == kStoreBF16)
        return launch(k_tvl1_finish<StoreBF16>, g, b, 0, s, nullptr, ev.stop, P, fr, cur);
    return launch(k_tvl1_finish<StoreF32>, g, b, 0, s, nullptr, ev.stop, P, fr, cur);
}

hipError_t launch_finish(const Planes& P, Frame fr, bool zero_counts, hipStream_t s,
                         LaunchEv ev) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t n = zero_counts ? np : 1;
    return launch(k_finish, dim3(blocks_for(n, 256)), dim3(256), 0, s, ev.start, ev.stop, P, np,
                  zero_counts ? 1 : 0);
}

hipError_t launch_rotate(const Planes& P, Frame fr, int cur, bool to_frame, hipStream_t s,
                         LaunchEv ev) {
    const size_t np = (size_t)fr.W * fr.H;
    return launch(k_rotate, dim3(blocks_for(np, 256)), dim3(256), 0, s, ev.start, ev.stop, P, fr,
                  cur, to_frame ? 1 : 0);
}

hipError_t launch_pd_plain(const Planes& P, Frame fr, IterConsts kc, int cur, hipStream_t s,
                           LaunchEv ev) {
    const dim3 grid((fr.W + 63) / 64, (fr.H + 3) / 4);
    hipError_t e = launch(k_primal, grid, dim3(256), 0, s, ev.start, nullptr, P, fr, kc, cur);
    if (e == hipSuccess) e = launch(k_dual, grid, dim3(256), 0, s, nullptr, ev.stop, P, fr, kc, cur);
    return e;
}

bool fused_shape_supported(int rows, int waves, int cols, int storage) {
    const int key = rows * 100 + waves;
    if (cols == 32) {
        if (storage != kStoreF32) return key == 208;
        switch (key) {
            case 108: case 116: case 204: case 208: case 216: case 308: case 404: case 408:
                return true;
            default:
                return false;
        }
    }
    if (cols != 64) return false;
    if (storage != kStoreF32)
        return key == 216 || key == 416 || key == 804 || key == 808 || key == 408;
    switch (key) {
        case 202: case 204: case 208: case 216: case 316:
        case 401: case 402: case 404: case 408: case 416: case 508: case 608:
        case 801: case 802: case 804: case 808:
        case 1601: case 1602: case 1604:
            return true;
        default:
            return false;
    }
}

#define REC_FUSED_CASE(R, NW, CW)                                                               \
    case (CW == 32 ? 10000 : 0) + R * 100 + NW:                                                \
        return fused_launch<R, NW, CW, StoreF32>(P, fr, kc, bc, segs, cur, iters, mode, s, ev);
#define REC_FUSED_CASE16(R, NW, CW)                                                             \
    case (CW == 32 ? 10000 : 0) + R * 100 + NW:                                                \
        return storage == kStoreF16                                                             \
                   ? fused_launch<R, NW, CW, StoreF16>(P, fr, kc, bc, segs, cur, iters, mode, s, \
                                                       ev)                                      \
                   : fused_launch<R, NW, CW, StoreBF16>(P, fr, kc, bc, segs, cur, iters, mode,  \
                                                        s, ev);

hipError_t launch_pd_fused(const Planes& P, Frame fr, IterConsts kc, BuildConsts bc,
                           const EventSegs& segs, int cur, int iters, int mode, int rows,
                           int waves, int cols, int storage, hipStream_t s, LaunchEv ev) {
    if (!fused_shape_supported(rows, waves, cols, storage)) return hipErrorInvalidValue;
    const int key = (cols == 32 ? 10000 : 0) + rows * 100 + waves;
    if (storage != kStoreF32) {
        switch (key) {
            REC_FUSED_CASE16(2, 16, 64)
            REC_FUSED_CASE16(4, 16, 64)
            REC_FUSED_CASE16(4, 8, 64)
            REC_FUSED_CASE16(8, 4, 64)
            REC_FUSED_CASE16(8, 8, 64)
            REC_FUSED_CASE16(2, 8, 32)
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
        REC_FUSED_CASE(2, 2, 64)
        REC_FUSED_CASE(2, 4, 64)
        REC_FUSED_CASE(2, 8, 64)
        REC_FUSED_CASE(2, 16, 64)
        REC_FUSED_CASE(3, 16, 64)
        REC_FUSED_CASE(4, 1, 64)
        REC_FUSED_CASE(4, 2, 64)
        REC_FUSED_CASE(4, 4, 64)
        REC_FUSED_CASE(4, 8, 64)
        REC_FUSED_CASE(4, 16, 64)
        REC_FUSED_CASE(5, 8, 64)
        REC_FUSED_CASE(6, 8, 64)
        REC_FUSED_CASE(8, 1, 64)
        REC_FUSED_CASE(8, 2, 64)
        REC_FUSED_CASE(8, 4, 64)
        REC_FUSED_CASE(8, 8, 64)
        REC_FUSED_CASE(16, 1, 64)
        REC_FUSED_CASE(16, 2, 64)
        REC_FUSED_CASE(16, 4, 64)
        REC_FUSED_CASE(1, 8, 32)
        REC_FUSED_CASE(1, 16, 32)
        REC_FUSED_CASE(2, 4, 32)
        REC_FUSED_CASE(2, 8, 32)
        REC_FUSED_CASE(2, 16, 32)
        REC_FUSED_CASE(3, 8, 32)
        REC_FUSED_CASE(4, 4, 32)
        REC_FUSED_CASE(4, 8, 32)
        default: return hipErrorInvalidValue;
    }
}
#undef REC_FUSED_CASE
#undef REC_FUSED_CASE16

#define REC_BATCH_CASE(R, NW, CW)                                                               \
    case (CW == 32 ? 10000 : 0) + R * 100 + NW:                                                \
        return batch_launch<R, NW, CW, StoreF32>(descs, work, nwork, K, KG, li, last, bins, s,  \
                                                 ev);
#define REC_BATCH_CASE16(R, NW, CW)                                                             \
    case (CW == 32 ? 10000 : 0) + R * 100 + NW:                                                \
        return storage == kStoreF16                                                             \
                   ? batch_launch<R, NW, CW, StoreF16>(descs, work, nwork, K, KG, li, last,     \
                                                       bins, s, ev)                             \
                   : batch_launch<R, NW, CW, StoreBF16>(descs, work, nwork, K, KG, li, last,    \
                                                        bins, s, ev);

hipError_t launch_pd_batch(const StreamDesc* descs, const int2* work, int nwork, int K, int KG,
                           int li, bool last, bool bins, int rows, int waves, int cols,
                           int storage, hipStream_t s, LaunchEv ev) {
    if (!batch_shape_supported(rows, waves, cols, storage) || nwork <= 0)
        return hipErrorInvalidValue;
    const int key = (cols == 32 ? 10000 : 0) + rows * 100 + waves;
    if (storage != kStoreF32) {
        switch (key) {
            REC_BATCH_CASE16(2, 16, 64)
            REC_BATCH_CASE16(4, 16, 64)
            REC_BATCH_CASE16(4, 8, 64)
            REC_BATCH_CASE16(8, 4, 64)
            REC_BATCH_CASE16(8, 8, 64)
            REC_BATCH_CASE16(2, 8, 32)
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
        REC_BATCH_CASE(2, 16, 64)
        REC_BATCH_CASE(4, 8, 64)
        REC_BATCH_CASE(4, 16, 64)
        REC_BATCH_CASE(6, 8, 64)
        REC_BATCH_CASE(8, 4, 64)
        REC_BATCH_CASE(8, 8, 64)
        REC_BATCH_CASE(1, 16, 32)
        REC_BATCH_CASE(2, 8, 32)
        default: return hipErrorInvalidValue;
    }
}
#undef REC_BATCH_CASE
#undef REC_BATCH_CASE16

bool batch_shape_supported(int rows, int waves, int cols, int storage) {
    const int key = rows * 100 + waves;
    if (cols == 32) return key == 208 || (storage == kStoreF32 && key == 116);
    if (cols != 64) return false;
    if (storage == kStoreF32 && key == 608) return true;
    return key == 216 || key == 408 || key == 416 || key == 804 || key == 808;
}

hipError_t launch_finish_batch(const StreamDesc* descs, int nstreams, size_t max_np,
                               hipStream_t s) {
    return launch(k_finish_batch, dim3(blocks_for(max_np, 256), nstreams), dim3(256), 0, s,
                  nullptr, nullptr, descs, nstreams);
}

hipError_t launch_gap(const Planes& P, Frame fr, double lambda, double umin, double umax,
                      int cur, bool rotated, int slot, int storage, hipStream_t s, LaunchEv ev) {
    const size_t np = (size_t)fr.W * fr.H;
    const size_t nb = gap_blocks(np);
    const dim3 g((unsigned)nb), b(kGapBlock);
    const int rot = rotated ? 1 : 0;
    hipError_t e =
        storage == kStoreF16
            ? launch(k_gap<StoreF16>, g, b, 0, s, ev.start, nullptr, P, fr, lambda, umin, umax,
                     cur, rot)
        : storage == kStoreBF16
            ? launch(k_gap<StoreBF16>, g, b, 0, s, ev.start, nullptr, P, fr, lambda, umin, umax,
                     cur, rot)
            : launch(k_gap<StoreF32>, g, b, 0, s, ev.start, nullptr, P, fr, lambda, umin, umax,
                     cur, rot);
    if (e == hipSuccess)
        e = launch(k_gap_final, dim3(1), dim3(256), 0, s, nullptr, ev.stop, P, nb, slot);
    return e;
}

hipError_t launch_time_plane(const Planes& P, Frame fr, double time_unit_us, float* out,
                             hipStream_t s) {
    const size_t np = (size_t)fr.W * fr.H;
    return launch(k_time_plane, dim3(blocks_for(np, 256)), dim3(256), 0, s, nullptr, nullptr, P,
                  fr, time_unit_us, out);
}

hipError_t launch_tlast_plane(const Planes& P, Frame fr, int64_t* out, hipStream_t s) {
    const size_t np = (size_t)fr.W * fr.H;
    return launch(k_tlast_plane, dim3(blocks_for(np, 256)), dim3(256), 0, s, nullptr, nullptr, P,
                  fr, out);
}

hipError_t launch_metric_plane(const Planes& P, Frame fr, int storage, float* out, hipStream_t s) {
    const size_t np = (size_t)fr.W * fr.H;
    const dim3 g(blocks_for(np, 256)), b(256);
    if (storage == kStoreF16)
        return launch(k_metric_plane<StoreF16>, g, b, 0, s, nullptr, nullptr, P, fr, out);
    if (storage == kStoreBF16)
        return launch(k_metric_plane<StoreBF16>, g, b, 0, s, nullptr, nullptr, P, fr, out);
    return launch(k_metric_plane<StoreF32>, g, b, 0, s, nullptr, nullptr, P, fr, out);
}

hipError_t launch_import(const Planes& P, Frame fr, int cur, int storage, const float* u,
                         const float* p, const int64_t* t_last, bool started, hipStream_t s) {
    const size_t np = (size_t)fr.W * fr.H;
    const dim3 g(blocks_for(np, 256)), b(256);
    const int st = started ? 1 : 0;
    if (storage == kStoreF16)
        return launch(k_import<StoreF16>, g, b, 0, s, nullptr, nullptr, P, np, cur, u, p, t_last,
                      st);
    if (storage == kStoreBF16)
        return launch(k_import<StoreBF16>, g, b, 0, s, nullptr, nullptr, P, np, cur, u, p, t_last,
                      st);
    return launch(k_import<StoreF32>, g, b, 0, s, nullptr, nullptr, P, np, cur, u, p, t_last, st);
}

hipError_t launch_widen(const void* src, int storage, float* out, size_t n, hipStream_t s) {
    const dim3 g(blocks_for(n, 256)), b(256);
    if (storage == kStoreF16)
        return launch(k_widen<StoreF16>, g, b, 0, s, nullptr, nullptr, src, out, n);
    if (storage == kStoreBF16)
        return launch(k_widen<StoreBF16>, g, b, 0, s, nullptr, nullptr, src, out, n);
    return launch(k_widen<StoreF32>, g, b, 0, s, nullptr, nullptr, src, out, n);
}

}  // namespace rec
