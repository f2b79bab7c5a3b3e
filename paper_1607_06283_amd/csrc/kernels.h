// Internal interface between the C ABI (rec_api.hip) and the device kernels
// (kernels.hip).  Not part of the public header.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rec {

constexpr int64_t kNever = INT64_MIN;   // t_last of a pixel that never fired
constexpr int64_t kNoBad = INT64_MAX;   // no rejected event in the current push

// Error codes stored by device-side validation (same values as REC_E*).
constexpr int32_t kErrInval = -1;
constexpr int32_t kErrRange = -2;
constexpr int32_t kErrOrder = -3;

// Device-resident stream state (first 256 bytes of the workspace).
struct alignas(256) DevState {
    int64_t t_ref;          // timestamp of the last accepted event
    int64_t t_first;        // first accepted timestamp of the stream
    int64_t first_bad;      // index of the first invalid event of the running push
    int64_t batch_events;   // events accepted since the last solve (scattered pushes)
    int64_t last_events;    // events consumed by the last solve
    int32_t started;        // 1 once an event was accepted
    int32_t err;            // first deferred push error not yet reported (0 = none)
    // Outcome of the events folded into a solve's first launch; written by
    // that launch's block 0 and committed to the fields above by the next
    // launch (no block of the first launch may see the update).
    int64_t pend_t_ref;
    int64_t pend_t_first;
    int64_t pend_events;
    int32_t pend_accepted;  // 1 if at least one folded event was accepted
    int32_t pend_err;
};

// Device pointers carved from the caller's workspace.
struct Planes {
    DevState* st;
    float* u[2];            // primal image, ping-pong
    float* p[2];            // dual field, 3 consecutive planes, ping-pong
    float* f;               // data image of the current block
    float* tx;              // forward differences of the time surface
    float* ty;
    int64_t* t_last;        // latest timestamp per pixel (kNever if none)
    int32_t* npos;          // event counts of scattered pushes
    int32_t* nneg;
    int64_t* ev_t;          // staging for host-pointer pushes
    uint16_t* ev_x;
    uint16_t* ev_y;
    int8_t* ev_p;
    double* gap_part;       // per-block (gap, energy) partial sums
    double* gap_hist;       // (gap, energy) per sample of the running solve
    double* tv0;            // timestamp denoising (when enabled): raw surface,
    double* tv[2];          //   iterate (ping-pong),
    double* tq;             //   dual field (2 planes)
};

struct Frame {
    int32_t W, H;
};

// FP32 constants of the iteration: ts = tau / sigma (the primal step on the
// sigma-scaled coefficients), sigma, tau * lambda, the clamp range.
struct IterConsts {
    float ts, sigma, taulam, umin, umax;
};

// Constants of the data image and time-surface build (FP64).
struct BuildConsts {
    double dpos, dneg;  // contrast thresholds Delta+, Delta-
    double ts;          // microseconds per unit of tau (0: flat manifold)
    double its;         // 1 / ts rounded to nearest, or 0 where a division is used instead
};
// Build constants of a stream; its is set for 2^-100 <= ts <= 2^100, where
// x / ts for any |x| < 2^63 stays clear of overflow and underflow.
inline BuildConsts make_build_consts(double dpos, double dneg, double ts) {
    const bool ok = ts >= 0x1p-100 && ts <= 0x1p100;
    return BuildConsts{dpos, dneg, ts, ok ? 1.0 / ts : 0.0};
}

// x / ts in FP64, rounded to nearest.  With its = RN(1 / ts), q = RN(x its)
// is within an ulp of the quotient, the remainder x - q ts is exact in one
// fused multiply-add, and RN(q + r its) is the correctly rounded quotient
// (Markstein, "Computation of elementary functions on the IBM RISC
// System/6000 processor", 1990), so this equals the IEEE division, at three
// FP64 operations instead of the division's sequence.
__host__ __device__ __forceinline__ double div_ts(double x, const BuildConsts& b) {
    if (b.its == 0.0) return x / b.ts;
    const double q = x * b.its;
    const double r = __builtin_fma(-q, b.ts, x);
    return __builtin_fma(r, b.its, q);
}

// Division by a launch constant d (1 <= d < 2^31) of any 0 <= n < 2^31 with
// a multiply-high, an add and a shift (Granlund and Montgomery, "Division by
// invariant integers using multiplication", 1994: with l = ceil(log2 d) and
// m' = ceil(2^(32+l) / d), floor(n / d) = floor(n m' / 2^(32+l)); m' - 2^32
// fits 32 bits and n + mulhi(n, m' - 2^32) does not overflow for n < 2^31).
// A tile index turns into its tile row and column this way at the start of
// every fused launch, where a general integer division would delay the
// first loads.
struct Divider {
    uint32_t m;  // m' - 2^32
    uint32_t l;
};
inline Divider make_divider(uint32_t d) {
    if (d <= 1) return Divider{0, 0};  // n / 1 (0 is no divisor: it maps to 1)
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    const unsigned __int128 num = (unsigned __int128)1 << (32 + l);
    const uint64_t mp = (uint64_t)((num + d - 1) / d);
    return Divider{(uint32_t)(mp - (1ull << 32)), l};
}
__host__ __device__ __forceinline__ int divide(int n, Divider dv) {
    const uint32_t un = (uint32_t)n;
    const uint32_t hi = (uint32_t)(((uint64_t)un * dv.m) >> 32);  // mulhi
    return (int)((un + hi) >> dv.l);
}

// Device-pointer pushes not scattered yet: consumed by the first fused
// launch of the next solve, in order, each all-or-nothing.
constexpr int kMaxSegs = 4;
struct EventSegs {
    const int64_t* t[kMaxSegs];
    const uint16_t* x[kMaxSegs];
    const uint16_t* y[kMaxSegs];
    const int8_t* p[kMaxSegs];
    int64_t n[kMaxSegs];
    int32_t count;
};

// Modes of the fused primal-dual launch (bit set).
constexpr int kBuild = 1;   // form f, tx, ty (and the new t_last) first
constexpr int kZero = 2;    // reset the scattered event counts of the interior at the end
constexpr int kEvents = 4;  // with kBuild: validate and bin the folded events in LDS
constexpr int kCommit = 8;  // commit the pending stream state of the previous launch
constexpr int kCounts = 16; // with kBuild: add the scattered event counts
constexpr int kTimeMem = 32; // with kBuild: tx, ty were written by the timestamp denoising
constexpr int kRotIn = 64;   // p is loaded in the standard basis: rotate it into the frame
constexpr int kRotOut = 128; // rotate p back to the standard basis before storing it

constexpr int kGapBlock = 256;
constexpr int kGapHistCap = 4096;
constexpr int kSmallPush = 4096;   // pushes up to this size use one workgroup

// Storage of p and tx, ty (arithmetic is FP32 in every case).
constexpr int kStoreF32 = 0;
constexpr int kStoreBF16 = 1;
constexpr int kStoreF16 = 2;

// One stream of a batched solve (device copy, written before the solve).
struct StreamDesc {
    Planes P;
    Frame fr;
    IterConsts kc;
    BuildConsts bc;
    EventSegs segs;
    int32_t cur;     // ping-pong parity at the start of the solve
    int32_t mode0;   // mode of the solve's first launch
    int32_t mode1;   // mode of its second launch
    int32_t tiles_x; // tiles per row for the batch's tile geometry
    Divider tiles_x_div;  // the same as a divider
};

// Optional timing events around a launch (recorded by the launch packet).
struct LaunchEv {
    hipEvent_t start = nullptr, stop = nullptr;
};

size_t gap_blocks(size_t np);
size_t fused_lds_bytes(int rows, int waves, int cols, int mode);
int fused_tiles(Frame fr, int rows, int waves, int cols, int iters);

// Launchers: return the first HIP error (launch errors only; no sync).
hipError_t launch_init(const Planes& P, Frame fr, float u_init, bool keep_u, hipStream_t s);
hipError_t launch_push(const Planes& P, Frame fr, const int64_t* t, const uint16_t* x,
                       const uint16_t* y, const int8_t* pol, int64_t n, hipStream_t s,
                       LaunchEv ev = {});
hipError_t launch_build(const Planes& P, Frame fr, int cur, BuildConsts bc, bool time_mem,
                        hipStream_t s, LaunchEv ev = {});
// Timestamp denoising: `iters` TV-L1 iterations on the surface, then tx, ty
// (in the given storage) from the denoised surface.
// Timestamp denoising; with folded pushes (segs.count > 0, only up to
// kTvl1FusedMax iterations) the launch bins the block's events itself.
constexpr int kTvl1FusedMax = 14;
int tvl1_tiles(Frame fr, int iters);  // tiles of the one-launch form, -1 beyond it
hipError_t launch_tvl1(const Planes& P, Frame fr, double ts, int iters, double lambda,
                       int storage, const EventSegs& segs, hipStream_t s, LaunchEv ev = {});
hipError_t launch_finish(const Planes& P, Frame fr, bool zero_counts, hipStream_t s,
                         LaunchEv ev = {});
// The two-kernel loop iterates on frame coordinates of p: launch_rotate
// brings p into the frame (to_frame) before the first iteration of a solve
// and back after the last.
hipError_t launch_rotate(const Planes& P, Frame fr, int cur, bool to_frame, hipStream_t s,
                         LaunchEv ev = {});
hipError_t launch_pd_plain(const Planes& P, Frame fr, IterConsts k, int cur, hipStream_t s,
                           LaunchEv ev = {});
hipError_t launch_pd_fused(const Planes& P, Frame fr, IterConsts k, BuildConsts bc,
                           const EventSegs& segs, int cur, int iters, int mode, int rows,
                           int waves, int cols, int storage, hipStream_t s, LaunchEv ev = {});
bool fused_shape_supported(int rows, int waves, int cols, int storage);
// rotated: p holds frame coordinates (between the launches of a solve).
hipError_t launch_gap(const Planes& P, Frame fr, double lambda, double umin, double umax,
                      int cur, bool rotated, int slot, int storage, hipStream_t s,
                      LaunchEv ev = {});
hipError_t launch_time_plane(const Planes& P, Frame fr, double time_unit_us, float* out,
                             hipStream_t s);
hipError_t launch_metric_plane(const Planes& P, Frame fr, int storage, float* out, hipStream_t s);
hipError_t launch_tlast_plane(const Planes& P, Frame fr, int64_t* out, hipStream_t s);
hipError_t launch_widen(const void* src, int storage, float* out, size_t n, hipStream_t s);
// State import into the current planes (u, p in the standard basis or NULL
// for zero, latest timestamps; kNever everywhere when !started); the
// stream state must have been written first, with t_first = INT64_MAX when
// started (the launch lowers it to the earliest imported timestamp).
hipError_t launch_import(const Planes& P, Frame fr, int cur, int storage, const float* u,
                         const float* p, const int64_t* t_last, bool started, hipStream_t s);
// Batched solve: one launch over the work list of (stream, tile) pairs.
// K iterations in this launch, KG the halo of the tile geometry (K <= KG),
// li the launch's index within the solve, bins: some stream folds events.
hipError_t launch_pd_batch(const StreamDesc* descs, const int2* work, int nwork, int K, int KG,
                           int li, bool last, bool bins, int rows, int waves, int cols,
                           int storage, hipStream_t s, LaunchEv ev = {});
bool batch_shape_supported(int rows, int waves, int cols, int storage);
hipError_t launch_finish_batch(const StreamDesc* descs, int nstreams, size_t max_np,
                               hipStream_t s);

}  // namespace rec
