// C ABI of the reconstruction library: parameter and event validation,
// workspace layout, context state and launch sequencing.  All arithmetic of
// the method runs in the kernels of kernels.hip.
//
// Per block of events the device work is:
//   - device-pointer pushes are recorded, not launched; the first fused
//     primal-dual launch of the next solve validates and bins them itself
//     (up to kMaxSegs pushes and kFoldMaxEvents events; beyond that, and for
//     host-pointer pushes, the events are scattered by their own kernels);
//     with timestamp denoising the one-launch denoiser bins them too;
//   - the solve's first fused launch builds f, tx, ty and iterates; the
//     next launches iterate; the second one commits the stream state (or a
//     small finishing kernel does, when the solve has one launch).
// So a block of a small sensor costs ceil(iters / K) launches and no events.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "kernels.h"
#include "shape.h"
#include "staging.h"
#include "rec.h"

using rec::Planes;

namespace {

constexpr size_t kAlign = 256;
constexpr int kProfClasses = 4;  // push, build, primal-dual, gap
constexpr size_t kProfFlush = 1u << 15;
constexpr int64_t kFoldMaxEvents = 16384;   // events binned in the first launch at most
constexpr int64_t kFoldMaxWork = 1 << 24;   // events x tiles scanned in it at most

inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Bytes of each half of the staging ring: one packed record of ne events.
inline size_t stage_half(size_t ne) { return align_up(ne * 13); }

// Lays the workspace out (base == nullptr: only sizes it).  Returns bytes.
size_t carve(const rec_params* prm, char* base, Planes* P) {
    const size_t np = (size_t)prm->width * (size_t)prm->height;
    const size_t ne = (size_t)prm->max_events;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = align_up(off);
        char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    Planes q;
    q.st = (rec::DevState*)take(sizeof(rec::DevState));
    q.u[0] = (float*)take(np * 4);
    q.u[1] = (float*)take(np * 4);
    q.p[0] = (float*)take(3 * np * 4);
    q.p[1] = (float*)take(3 * np * 4);
    q.f = (float*)take(np * 4);
    q.tx = (float*)take(np * 4);
    q.ty = (float*)take(np * 4);
    q.t_last = (int64_t*)take(np * 8);
    q.npos = (int32_t*)take(np * 4);
    q.nneg = (int32_t*)take(np * 4);
    // staging ring of host-pointer pushes: two halves of 13 bytes per event
    // (a push of max_events events fills one); ev_x .. ev_p: the planes of
    // such a push at the start of the first half
    char* ring = take(2 * stage_half(ne));
    q.ev_t = (int64_t*)ring;
    q.ev_x = ring ? (uint16_t*)(ring + 8 * ne) : nullptr;
    q.ev_y = ring ? (uint16_t*)(ring + 10 * ne) : nullptr;
    q.ev_p = ring ? (int8_t*)(ring + 12 * ne) : nullptr;
    q.gap_part = (double*)take(rec::gap_blocks(np) * 2 * sizeof(double));
    q.gap_hist = (double*)take((size_t)rec::kGapHistCap * 2 * sizeof(double));
    const size_t nt = prm->tvl1_iters > 0 ? np : 0;  // denoising planes only when enabled
    q.tv0 = (double*)take(nt * 8);
    q.tv[0] = (double*)take(nt * 8);
    q.tv[1] = (double*)take(nt * 8);
    q.tq = (double*)take(2 * nt * 8);
    if (P) *P = q;
    return align_up(off);
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

// A roctx range around an entry point, so that a marker trace
// (rocprofv3 --marker-trace) shows each call beside the kernels it enqueues.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

struct Seg {
    const int64_t* t;
    const uint16_t* x;
    const uint16_t* y;
    const int8_t* p;
    int64_t n;
};

}  // namespace

struct rec_ctx {
    rec_params prm;
    Planes P;
    rec::Frame fr;
    rec::IterConsts kc;
    hipStream_t stream;
    int device;
    int cur;                 // which ping-pong buffers hold the current (u, p)
    int rows, waves, cols;   // fused tile shape
    int kmax;                // iterations per fused launch (at most)
    // Host-pointer pushes are staged as packed records (t, x, y, polarity of
    // one push, back to back) in a ring of two halves: the pinned host buffer
    // and the workspace's staging ring hold a record at the same offset, and
    // a copy kernel moves it.  Records fill the current half (stage_cur) up
    // to stage_used; stage_done[h]: the last copy out of half h.  The copies
    // are recorded (pulls; pull_halves: the halves they read) and launched
    // together before anything reads the records: by the solve (a batched
    // solve launches the copies of all its contexts at once), or by a call
    // that scatters the records.
    char* pinned;
    const char* pinned_dev;  // its device address
    size_t stage_used;
    int stage_cur;
    hipEvent_t stage_done[2];
    bool stage_busy[2];
    std::vector<rec::PullDesc> pulls;
    unsigned pull_halves;
    // device-pointer pushes recorded but not scattered yet (in order)
    std::vector<Seg> deferred;
    int64_t deferred_events;
    bool counts_dirty;       // scattered pushes left counts for the next solve
    // host mirror of the device stream state (valid while only host pushes ran)
    bool mirror_known;
    bool mirror_started;
    int64_t mirror_tref;
    int gap_samples;
    int batch_refs;          // live batches holding this context (rec_destroy refuses while > 0)
    // profiling
    bool prof_on;
    std::vector<hipEvent_t> prof_pool;
    std::vector<int> prof_cls;   // class of each (start, stop) pair
    std::vector<int64_t> prof_work;
    size_t prof_used;
    double prof_ms[kProfClasses];
    int64_t prof_launches[kProfClasses];
    int64_t prof_pd_px_iters;
};

namespace {

int dev_err(hipError_t e) { return e == hipSuccess ? REC_OK : REC_EDEVICE; }

hipEvent_t prof_event(rec_ctx* c) {
    if (c->prof_used == c->prof_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->prof_pool.push_back(e);
    }
    return c->prof_pool[c->prof_used++];
}

int prof_flush(rec_ctx* c) {
    if (!c->prof_used) return REC_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return REC_EDEVICE;
    for (size_t q = 0; q < c->prof_cls.size(); ++q) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->prof_pool[2 * q], c->prof_pool[2 * q + 1]) != hipSuccess)
            return REC_EDEVICE;
        const int k = c->prof_cls[q];
        c->prof_ms[k] += ms;
        c->prof_launches[k] += 1;
        if (k == 2) c->prof_pd_px_iters += c->prof_work[q];
    }
    c->prof_cls.clear();
    c->prof_work.clear();
    c->prof_used = 0;
    return REC_OK;
}

// Runs one launch; when profiling, the launch packet itself records a
// (start, stop) timing event pair, so the pair measures the kernel(s) only.
template <class F>
int timed(rec_ctx* c, int cls, int64_t work, F&& launch) {
    if (!c->prof_on) return dev_err(launch(rec::LaunchEv{}));
    if (c->prof_used + 2 > kProfFlush) {
        const int rc = prof_flush(c);
        if (rc) return rc;
    }
    rec::LaunchEv ev;
    ev.start = prof_event(c);
    ev.stop = prof_event(c);
    if (!ev.start || !ev.stop) return REC_EDEVICE;
    if (launch(ev) != hipSuccess) return REC_EDEVICE;
    c->prof_cls.push_back(cls);
    c->prof_work.push_back(work);
    return REC_OK;
}

// Reads the device state after synchronising; reports and clears a deferred
// push error.
int read_state(rec_ctx* c, rec::DevState* out) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return REC_EDEVICE;
    rec::DevState st;
    if (hipMemcpy(&st, c->P.st, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return REC_EDEVICE;
    if (out) *out = st;
    if (st.err != 0) {
        const int32_t zero = 0;
        if (hipMemcpy(&c->P.st->err, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
            return REC_EDEVICE;
        return st.err;
    }
    return REC_OK;
}

// Marks the copies recorded for c as launched: the host may rewrite the
// pinned bytes of a half they read once stage_done of that half has passed.
int pulls_launched(rec_ctx* c) {
    for (int h = 0; h < 2; ++h) {
        if (!((c->pull_halves >> h) & 1u)) continue;
        if (hipEventRecord(c->stage_done[h], c->stream) != hipSuccess) return REC_EDEVICE;
        c->stage_busy[h] = true;
    }
    c->pulls.clear();
    c->pull_halves = 0;
    return REC_OK;
}

// Launches the recorded copies of host-pointer pushes (one launch per
// kMaxPulls copies) on the context's stream.
int flush_pulls(rec_ctx* c) {
    for (size_t a = 0; a < c->pulls.size(); a += rec::kMaxPulls) {
        const int m = (int)std::min(c->pulls.size() - a, (size_t)rec::kMaxPulls);
        const int rc = timed(c, 0, 0, [&](rec::LaunchEv ev) {
            return rec::launch_pulls(c->pulls.data() + a, m, c->stream, ev.start, ev.stop);
        });
        if (rc) return rc;
    }
    return pulls_launched(c);
}

// Scatters the recorded pushes with their own kernels (the copies of host
// pushes first).
int flush_deferred(rec_ctx* c) {
    const int rc0 = flush_pulls(c);
    if (rc0) return rc0;
    for (const Seg& s : c->deferred) {
        const int rc = timed(c, 0, s.n, [&](rec::LaunchEv ev) {
            return rec::launch_push(c->P, c->fr, s.t, s.x, s.y, s.p, s.n, c->stream, ev);
        });
        if (rc) return rc;
        c->counts_dirty = true;
    }
    c->deferred.clear();
    c->deferred_events = 0;
    return REC_OK;
}

// Copies the n events of a host-pointer push (at most max_events) into the
// staging ring as one packed record: written to the pinned buffer, with its
// copy to the device recorded (launched later, with the others, by
// flush_pulls or a batched solve); *out gets the record's four device
// arrays.  When the current half is full, the record starts the other one:
// the pushes still recorded in that half are scattered first (the copy,
// enqueued after them, then overwrites nothing still to be read), and the
// host waits for the half's last copy before rewriting its pinned bytes, so
// it runs at most about a half ahead of the device.
int stage_events(rec_ctx* c, const int64_t* t, const uint16_t* x, const uint16_t* y,
                 const int8_t* p, int64_t n, Seg* out) {
    const size_t m = (size_t)n, need = 13 * m, half = stage_half((size_t)c->prm.max_events);
    if (c->stage_used + need > half) {
        const int o = c->stage_cur ^ 1;
        const char* lo = (const char*)c->P.ev_t + (size_t)o * half;
        for (const Seg& s : c->deferred) {
            if ((const char*)s.t >= lo && (const char*)s.t < lo + half) {
                const int rc = flush_deferred(c);
                if (rc) return rc;
                break;
            }
        }
        if ((c->pull_halves >> o) & 1u) {  // its last copy is still to be launched
            const int rc = flush_pulls(c);
            if (rc) return rc;
        }
        if (c->stage_busy[o] && hipEventSynchronize(c->stage_done[o]) != hipSuccess)
            return REC_EDEVICE;
        c->stage_busy[o] = false;
        c->stage_cur = o;
        c->stage_used = 0;
    }
    const int hh = c->stage_cur;
    const size_t off = (size_t)hh * half + c->stage_used;
    char* h = c->pinned + off;
    memcpy(h, t, m * 8);
    memcpy(h + 8 * m, x, m * 2);
    memcpy(h + 10 * m, y, m * 2);
    memcpy(h + 12 * m, p, m);
    char* d = (char*)c->P.ev_t + off;
    // whole 16-byte words: the slot extends to the next 256-byte boundary
    c->pulls.push_back(rec::PullDesc{c->pinned_dev + off, d, (need + 15) & ~(size_t)15});
    c->pull_halves |= 1u << hh;
    c->stage_used = align_up(c->stage_used + need);
    *out = Seg{(const int64_t*)d, (const uint16_t*)(d + 8 * m), (const uint16_t*)(d + 10 * m),
               (const int8_t*)(d + 12 * m), n};
    return REC_OK;
}

}  // namespace

extern "C" {

void rec_default_params(rec_params* prm, int32_t width, int32_t height) {
    if (!prm) return;
    memset(prm, 0, sizeof(*prm));
    prm->width = width;
    prm->height = height;
    prm->lambda = 90.0;
    prm->delta_pos = 0.2;
    prm->delta_neg = 0.2;
    prm->u_min = 1.0;
    prm->u_max = exp(1.0);
    prm->tau = 1.0 / sqrt(8.0 + 4.0 * sqrt(2.0));
    prm->sigma = prm->tau;
    prm->time_unit_us = 1000.0;
    prm->u_init = sqrt(prm->u_min * prm->u_max);
    prm->iters = 50;
    prm->gap_every = 0;
    prm->fuse_iters = -1;
    prm->max_events = 65536;
    prm->tile_rows = 0;
    prm->tile_waves = 0;
    prm->storage = REC_STORE_F32;
    prm->tvl1_iters = 0;
    prm->tvl1_lambda = 1.0;
}

int rec_check_params(const rec_params* prm) {
    if (!prm) return REC_EINVAL;
    if (prm->width < 1 || prm->height < 1 || prm->width > 65535 || prm->height > 65535)
        return REC_EINVAL;
    if (!finite_pos(prm->lambda) || !finite_pos(prm->delta_pos) || !finite_pos(prm->delta_neg))
        return REC_EINVAL;
    if (!finite_pos(prm->u_min) || !isfinite(prm->u_max) || !(prm->u_max > prm->u_min))
        return REC_EINVAL;
    if (!finite_pos(prm->tau) || !finite_pos(prm->sigma)) return REC_EINVAL;
    if (prm->tau * prm->sigma * (8.0 + 4.0 * sqrt(2.0)) > 1.0 + 1e-12) return REC_EINVAL;
    if (!isfinite(prm->time_unit_us) || prm->time_unit_us < 0.0) return REC_EINVAL;
    if (!finite_pos(prm->u_init)) return REC_EINVAL;
    if (prm->iters < 0 || prm->gap_every < 0) return REC_EINVAL;
    if (prm->fuse_iters < -1 || prm->fuse_iters > 31) return REC_EINVAL;
    if (prm->max_events < 1 || prm->max_events > (1 << 28)) return REC_EINVAL;
    if (prm->storage != REC_STORE_F32 && prm->storage != REC_STORE_BF16 &&
        prm->storage != REC_STORE_F16)
        return REC_EINVAL;
    if (prm->storage != REC_STORE_F32 && prm->fuse_iters == 0) return REC_EINVAL;
    if (prm->tvl1_iters < 0 || prm->tvl1_iters > 10000) return REC_EINVAL;
    if (prm->tvl1_iters > 0 && !finite_pos(prm->tvl1_lambda)) return REC_EINVAL;
    if ((prm->tile_rows == 0) != (prm->tile_waves == 0)) return REC_EINVAL;
    if (prm->tile_cols != 0 && (prm->tile_rows == 0 || (prm->tile_cols != 64 &&
                                                        prm->tile_cols != 32)))
        return REC_EINVAL;
    if (prm->tile_rows &&
        !rec::fused_shape_supported(prm->tile_rows, prm->tile_waves,
                                    prm->tile_cols ? prm->tile_cols : 64, prm->storage))
        return REC_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (prm->reserved[i] != 0) return REC_EINVAL;
    return REC_OK;
}

size_t rec_workspace_bytes(const rec_params* prm) {
    if (rec_check_params(prm) != REC_OK) return 0;
    return carve(prm, nullptr, nullptr);
}

int rec_check_events(const int64_t* t_us, const uint16_t* x, const uint16_t* y,
                     const int8_t* polarity, int64_t n, int32_t width, int32_t height,
                     int64_t t_prev) {
    if (n < 0 || width < 1 || height < 1) return REC_EINVAL;
    if (n == 0) return REC_OK;
    if (!t_us || !x || !y || !polarity) return REC_EINVAL;
    // Blocks of events are checked with branch-free flags (a loop the
    // compiler vectorises); a block with a failing event is checked again
    // in order, which gives the code of the first failing check of the
    // first failing event.
    constexpr int64_t kBlock = 512;
    int64_t prev = t_prev;
    for (int64_t a = 0; a < n; a += kBlock) {
        const int64_t m = n - a < kBlock ? n - a : kBlock;
        const int64_t* t = t_us + a;
        const uint16_t* xs = x + a;
        const uint16_t* ys = y + a;
        const int8_t* ps = polarity + a;
        unsigned bad = t[0] < prev;
        for (int64_t i = 1; i < m; ++i) bad |= (unsigned)(t[i] < t[i - 1]);
        for (int64_t i = 0; i < m; ++i) {
            // polarity +-1: (p + 1) is 0 or 2
            bad |= (unsigned)((((int)ps[i] + 1) & ~2) != 0);
            bad |= (unsigned)(xs[i] >= width) | (unsigned)(ys[i] >= height);
        }
        if (bad) {
            for (int64_t i = 0; i < m; ++i) {
                if (ps[i] != 1 && ps[i] != -1) return REC_EINVAL;
                if (xs[i] >= width || ys[i] >= height) return REC_ERANGE;
                if (t[i] < prev) return REC_EORDER;
                prev = t[i];
            }
        }
        prev = t[m - 1];
    }
    return REC_OK;
}

int rec_init(const rec_params* prm, void* dev_workspace, size_t ws_bytes, void* hip_stream,
             const float* u0, rec_ctx** out) {
    Range range("rec_init");
    if (!out) return REC_EINVAL;
    *out = nullptr;
    int rc = rec_check_params(prm);
    if (rc) return rc;
    if (!dev_workspace || ((uintptr_t)dev_workspace & (kAlign - 1))) return REC_EINVAL;
    const size_t need = carve(prm, nullptr, nullptr);
    if (ws_bytes < need) return REC_ENOMEM;
    const size_t np = (size_t)prm->width * prm->height;
    if (u0) {
        for (size_t k = 0; k < np; ++k)
            if (!(isfinite(u0[k]) && u0[k] > 0.0f)) return REC_EINVAL;
    }
    rec_ctx* c = new (std::nothrow) rec_ctx();
    if (!c) return REC_ENOMEM;
    c->prm = *prm;
    carve(prm, (char*)dev_workspace, &c->P);
    c->fr = {prm->width, prm->height};
    c->kc.ts = (float)(prm->tau / prm->sigma);
    c->kc.sigma = (float)prm->sigma;
    c->kc.taulam = (float)(prm->tau * prm->lambda);
    c->kc.umin = (float)prm->u_min;
    c->kc.umax = (float)prm->u_max;
    c->stream = (hipStream_t)hip_stream;
    c->cur = 0;
    rec::choose_shape(prm, (int64_t)prm->width * prm->height, true, &c->rows, &c->waves, &c->cols,
                 &c->kmax);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return REC_EDEVICE;
    }
    const size_t ne = (size_t)prm->max_events;
    // coherent: the copy kernel reads each byte once, and no GPU cache line
    // of it can outlive the host's rewrite of a half (non-coherent memory
    // measured the same)
    if (hipHostMalloc((void**)&c->pinned, 2 * stage_half(ne), hipHostMallocCoherent) !=
        hipSuccess) {
        delete c;
        return REC_ENOMEM;
    }
    if (hipHostGetDevicePointer((void**)&c->pinned_dev, c->pinned, 0) != hipSuccess) {
        rec_destroy(c);
        return REC_EDEVICE;
    }
    for (hipEvent_t* e : {&c->stage_done[0], &c->stage_done[1]}) {
        if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
            rec_destroy(c);
            return REC_EDEVICE;
        }
    }
    c->mirror_known = true;
    c->mirror_started = false;
    c->mirror_tref = 0;
    if (u0) {
        if (hipMemcpyAsync(c->P.u[0], u0, np * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
            rec_destroy(c);
            return REC_EDEVICE;
        }
    }
    rc = dev_err(rec::launch_init(c->P, c->fr, (float)prm->u_init, u0 != nullptr, c->stream));
    if (!rc && u0 && hipStreamSynchronize(c->stream) != hipSuccess) rc = REC_EDEVICE;
    if (rc) {
        rec_destroy(c);
        return rc;
    }
    *out = c;
    return REC_OK;
}

int rec_push_events(rec_ctx* c, const int64_t* t_us, const uint16_t* x, const uint16_t* y,
                    const int8_t* polarity, int64_t n, int on_device) {
    Range range("rec_push_events");
    if (!c || n < 0) return REC_EINVAL;
    if (n == 0) return REC_OK;
    if (!t_us || !x || !y || !polarity) return REC_EINVAL;
    if (on_device) {
        c->mirror_known = false;
        if (c->prm.fuse_iters == 0) {
            // the unfused loop has no first launch to fold the events into
            c->counts_dirty = true;
            return timed(c, 0, n, [&](rec::LaunchEv ev) {
                return rec::launch_push(c->P, c->fr, t_us, x, y, polarity, n, c->stream, ev);
            });
        }
        if ((int)c->deferred.size() == rec::kMaxSegs) {
            const int rc = flush_deferred(c);
            if (rc) return rc;
        }
        c->deferred.push_back(Seg{t_us, x, y, polarity, n});
        c->deferred_events += n;
        return REC_OK;
    }
    // host pointers: validated here against the host mirror of the stream
    // state (earlier device pushes go first, to learn their outcome), then
    // staged as one packed record with one copy
    int rc;
    if (!c->mirror_known) {
        rc = flush_deferred(c);
        if (rc) return rc;
        rec::DevState st;
        rc = read_state(c, &st);
        if (rc) return rc;
        c->mirror_known = true;
        c->mirror_started = st.started != 0;
        c->mirror_tref = st.t_ref;
    }
    rc = rec_check_events(t_us, x, y, polarity, n, c->prm.width, c->prm.height,
                          c->mirror_started ? c->mirror_tref : INT64_MIN);
    if (rc) return rc;
    const int64_t cap = c->prm.max_events;
    if (c->prm.fuse_iters != 0 && n <= cap) {
        // like a device push: binned by the next solve's first launch
        if ((int)c->deferred.size() == rec::kMaxSegs) {
            rc = flush_deferred(c);
            if (rc) return rc;
        }
        Seg sg;
        rc = stage_events(c, t_us, x, y, polarity, n, &sg);
        if (rc) return rc;
        c->deferred.push_back(sg);
        c->deferred_events += n;
    } else {
        // the unfused loop, or a push beyond the staging: scattered now
        rc = flush_deferred(c);
        if (rc) return rc;
        for (int64_t a = 0; a < n; a += cap) {
            const int64_t m = (n - a < cap) ? n - a : cap;
            Seg sg;
            rc = stage_events(c, t_us + a, x + a, y + a, polarity + a, m, &sg);
            if (!rc) rc = flush_pulls(c);
            if (rc) return rc;
            rc = timed(c, 0, m, [&](rec::LaunchEv ev) {
                return rec::launch_push(c->P, c->fr, sg.t, sg.x, sg.y, sg.p, m, c->stream, ev);
            });
            if (rc) return rc;
        }
        c->counts_dirty = true;
    }
    c->mirror_started = true;
    c->mirror_tref = t_us[n - 1];
    return REC_OK;
}

int rec_solve(rec_ctx* c, int32_t iters, rec_stats* stats) {
    Range range("rec_solve");
    if (!c) return REC_EINVAL;
    if (iters <= 0) iters = c->prm.iters;
    const int64_t np = (int64_t)c->fr.W * c->fr.H;
    const rec::BuildConsts bc =
        rec::make_build_consts(c->prm.delta_pos, c->prm.delta_neg, c->prm.time_unit_us);
    const bool fused = c->prm.fuse_iters != 0 && iters > 0;
    const bool denoise = c->prm.tvl1_iters > 0 && c->prm.time_unit_us > 0.0;
    int rc;
    rec::EventSegs segs;
    memset(&segs, 0, sizeof(segs));
    bool fold = false;
    // with denoising the one-launch denoiser bins the pushes as well (it
    // needs the block's timestamps before the metric is built)
    const int64_t dn_tiles =
        denoise ? rec::tvl1_tiles(c->fr, c->prm.tvl1_iters) : 0;
    if (fused && dn_tiles >= 0 && !c->deferred.empty()) {
        const int first_k = iters < c->kmax ? iters : c->kmax;
        const int64_t tiles = rec::fused_tiles(c->fr, c->rows, c->waves, c->cols, first_k);
        fold = c->deferred_events <= kFoldMaxEvents && tiles > 0 &&
               c->deferred_events * (tiles > dn_tiles ? tiles : dn_tiles) <= kFoldMaxWork;
    }
    if (fold) {
        // the copies of the host pushes' records go first
        rc = flush_pulls(c);
        if (rc) return rc;
        for (size_t s = 0; s < c->deferred.size(); ++s) {
            segs.t[s] = c->deferred[s].t;
            segs.x[s] = c->deferred[s].x;
            segs.y[s] = c->deferred[s].y;
            segs.p[s] = c->deferred[s].p;
            segs.n[s] = c->deferred[s].n;
        }
        segs.count = (int32_t)c->deferred.size();
        c->deferred.clear();
        c->deferred_events = 0;
    } else {
        rc = flush_deferred(c);
        if (rc) return rc;
    }
    if (denoise) {
        // the denoised surface needs every timestamp of the block first:
        // scattered above, or binned by the denoising launch itself
        rc = timed(c, 1, np, [&](rec::LaunchEv ev) {
            return rec::launch_tvl1(c->P, c->fr, c->prm.time_unit_us, c->prm.tvl1_iters,
                                    c->prm.tvl1_lambda, c->prm.storage, segs, c->stream, ev);
        });
        if (rc) return rc;
    }
    if (!fused) {
        rc = timed(c, 1, np, [&](rec::LaunchEv ev) {
            return rec::launch_build(c->P, c->fr, c->cur, bc, denoise, c->stream, ev);
        });
        if (rc) return rc;
        c->counts_dirty = false;
    }
    const bool counts = c->counts_dirty;
    const int ge = c->prm.gap_every;
    int samples = 0;
    int launch = 0;
    // iterations are cut into segments ending at gap samples; each segment
    // is split evenly into launches of at most kmax iterations
    for (int it = 0; it < iters;) {
        int seg = iters - it;
        if (ge > 0 && seg > ge - it % ge) seg = ge - it % ge;
        if (!fused) {
            // the iterations run on p in each pixel's tangent frame
            if (it == 0) {
                rc = timed(c, 1, np, [&](rec::LaunchEv ev) {
                    return rec::launch_rotate(c->P, c->fr, c->cur, true, c->stream, ev);
                });
                if (rc) return rc;
            }
            for (int q = 0; q < seg; ++q) {
                rc = timed(c, 2, np, [&](rec::LaunchEv ev) {
                    return rec::launch_pd_plain(c->P, c->fr, c->kc, c->cur, c->stream, ev);
                });
                if (rc) return rc;
                c->cur ^= 1;
            }
            if (it + seg == iters) {
                rc = timed(c, 1, np, [&](rec::LaunchEv ev) {
                    return rec::launch_rotate(c->P, c->fr, c->cur, false, c->stream, ev);
                });
                if (rc) return rc;
            }
        } else {
            const int nl = (seg + c->kmax - 1) / c->kmax;
            for (int q = 0; q < nl; ++q) {
                const int m = seg / nl + (q < seg % nl ? 1 : 0);
                int mode = 0;
                if (launch == 0)
                    mode = rec::kBuild | (fold ? rec::kEvents : 0) | (counts ? rec::kCounts : 0) |
                           (denoise ? rec::kTimeMem : 0) | rec::kRotIn;
                else if (launch == 1)
                    mode = rec::kCommit | (counts ? rec::kZero : 0);
                if (it + seg == iters && q == nl - 1) mode |= rec::kRotOut;
                rc = timed(c, 2, np * m, [&](rec::LaunchEv ev) {
                    return rec::launch_pd_fused(c->P, c->fr, c->kc, bc, segs, c->cur, m, mode,
                                                c->rows, c->waves, c->cols, c->prm.storage,
                                                c->stream, ev);
                });
                if (rc) return rc;
                c->cur ^= 1;
                if (launch == 0 && iters <= m) {
                    // a single launch: commit and reset counts in their own kernel
                    rc = timed(c, 1, np, [&](rec::LaunchEv ev) {
                        return rec::launch_finish(c->P, c->fr, counts, c->stream, ev);
                    });
                    if (rc) return rc;
                }
                ++launch;
            }
            c->counts_dirty = false;
        }
        it += seg;
        if (ge > 0 && it % ge == 0) {
            const int slot = samples < rec::kGapHistCap ? samples : rec::kGapHistCap - 1;
            rc = timed(c, 3, np, [&](rec::LaunchEv ev) {
                return rec::launch_gap(c->P, c->fr, c->prm.lambda, c->prm.u_min, c->prm.u_max,
                                       c->cur, it < iters, slot, c->prm.storage, c->stream, ev);
            });
            if (rc) return rc;
            ++samples;
        }
    }
    c->gap_samples = samples;
    if (!stats) return REC_OK;
    rec::DevState st;
    rc = read_state(c, &st);
    stats->iters_run = iters;
    stats->gap_samples = samples;
    stats->t_ref_us = st.t_ref;
    stats->events_in_batch = st.last_events;
    stats->gap = NAN;
    stats->energy = NAN;
    if (rc) return rc;
    if (samples > 0) {
        const int slot = samples < rec::kGapHistCap ? samples - 1 : rec::kGapHistCap - 1;
        double ge2[2];
        if (hipMemcpy(ge2, c->P.gap_hist + 2 * slot, sizeof(ge2), hipMemcpyDeviceToHost) != hipSuccess)
            return REC_EDEVICE;
        stats->gap = ge2[0];
        stats->energy = ge2[1];
        if (!isfinite(ge2[0]) || !isfinite(ge2[1])) return REC_ENUMERIC;
    }
    return REC_OK;
}

int rec_get_image(rec_ctx* c, int32_t which, void* out, int on_device) {
    Range range("rec_get_image");
    if (!c || !out || which < REC_U || which > REC_T_LAST) return REC_EINVAL;
    const size_t np = (size_t)c->fr.W * c->fr.H;
    // a synchronising call: recorded device-pointer pushes are scattered
    // first, so the caller may release their arrays once this returns (and
    // planes that pushes write see every push)
    int rc = flush_deferred(c);
    if (rc) return rc;
    const void* src = nullptr;
    size_t bytes = np * 4;
    hipError_t e = hipSuccess;
    // derived planes go through a spare ping-pong buffer unless written in place
    float* spare = c->P.u[c->cur ^ 1];
    float* spare3 = c->P.p[c->cur ^ 1];  // 3 planes, FP32-sized whatever the storage
    const bool narrow = c->prm.storage != REC_STORE_F32;
    switch (which) {
        case REC_U: src = c->P.u[c->cur]; break;
        case REC_F: src = c->P.f; break;
        case REC_TX:
        case REC_TY:
        case REC_STATE_P: {
            const void* raw = which == REC_TX ? (const void*)c->P.tx
                            : which == REC_TY ? (const void*)c->P.ty : (const void*)c->P.p[c->cur];
            const size_t n = which == REC_STATE_P ? 3 * np : np;
            bytes = n * 4;
            if (!narrow) {
                src = raw;
                break;
            }
            float* dst = on_device ? (float*)out : (which == REC_STATE_P ? spare3 : spare);
            e = rec::launch_widen(raw, c->prm.storage, dst, n, c->stream);
            src = on_device ? nullptr : dst;
            break;
        }
        case REC_COUNT_POS: src = c->P.npos; break;
        case REC_COUNT_NEG: src = c->P.nneg; break;
        case REC_T_LAST: {
            // pixels that never fired read as the stream's first timestamp
            // (8 bytes per pixel: the spare dual planes hold 12)
            int64_t* dst = on_device ? (int64_t*)out : (int64_t*)spare3;
            e = rec::launch_tlast_plane(c->P, c->fr, dst, c->stream);
            src = on_device ? nullptr : dst;
            bytes = np * 8;
            break;
        }
        case REC_TIME: {
            float* dst = on_device ? (float*)out : spare;
            e = rec::launch_time_plane(c->P, c->fr, c->prm.time_unit_us, dst, c->stream);
            src = on_device ? nullptr : spare;
            break;
        }
        case REC_METRIC_G: {
            float* dst = on_device ? (float*)out : spare;
            e = rec::launch_metric_plane(c->P, c->fr, c->prm.storage, dst, c->stream);
            src = on_device ? nullptr : spare;
            break;
        }
        default: return REC_EINVAL;
    }
    if (e != hipSuccess) return REC_EDEVICE;
    if (src) {
        e = hipMemcpyAsync(out, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           c->stream);
        if (e != hipSuccess) return REC_EDEVICE;
    }
    return read_state(c, nullptr);
}

int rec_gap_history(rec_ctx* c, double* gap, double* energy, int32_t cap) {
    if (!c || cap < 0) return REC_EINVAL;
    int rc = flush_deferred(c);
    if (rc) return rc;
    rc = read_state(c, nullptr);
    if (rc) return rc;
    int n = c->gap_samples < rec::kGapHistCap ? c->gap_samples : rec::kGapHistCap;
    if (n > cap) n = cap;
    if (n > 0) {
        std::vector<double> buf(2 * (size_t)n);
        if (hipMemcpy(buf.data(), c->P.gap_hist, buf.size() * sizeof(double), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return REC_EDEVICE;
        for (int i = 0; i < n; ++i) {
            if (gap) gap[i] = buf[2 * i];
            if (energy) energy[i] = buf[2 * i + 1];
        }
    }
    return n;
}

int rec_sync(rec_ctx* c) {
    if (!c) return REC_EINVAL;
    const int rc = flush_deferred(c);
    if (rc) return rc;
    return read_state(c, nullptr);
}

int rec_profile(rec_ctx* c, int enable) {
    if (!c) return REC_EINVAL;
    if (enable) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return REC_EDEVICE;
        c->prof_cls.clear();
        c->prof_work.clear();
        c->prof_used = 0;
        for (int k = 0; k < kProfClasses; ++k) {
            c->prof_ms[k] = 0.0;
            c->prof_launches[k] = 0;
        }
        c->prof_pd_px_iters = 0;
    }
    c->prof_on = enable != 0;
    return REC_OK;
}

int rec_profile_read(rec_ctx* c, rec_profile_t* out) {
    if (!c || !out) return REC_EINVAL;
    int rc = flush_deferred(c);
    if (rc) return rc;
    rc = prof_flush(c);
    if (rc) return rc;
    for (int k = 0; k < kProfClasses; ++k) {
        out->ms[k] = c->prof_ms[k];
        out->launches[k] = c->prof_launches[k];
    }
    out->pd_pixel_iters = c->prof_pd_px_iters;
    return REC_OK;
}

int rec_get_times(rec_ctx* c, int64_t* t_first, int64_t* t_ref, int32_t* started) {
    Range range("rec_get_times");
    if (!c) return REC_EINVAL;
    int rc = flush_deferred(c);
    if (rc) return rc;
    rec::DevState st;
    rc = read_state(c, &st);
    if (rc) return rc;
    if (t_first) *t_first = st.started ? st.t_first : 0;
    if (t_ref) *t_ref = st.started ? st.t_ref : 0;
    if (started) *started = st.started;
    return REC_OK;
}

int rec_set_state(rec_ctx* c, const float* u, const float* p, const int64_t* t_last,
                  int64_t t_ref, int on_device) {
    Range range("rec_set_state");
    if (!c || !u) return REC_EINVAL;
    const bool started = t_ref != INT64_MIN;
    if (started && !t_last) return REC_EINVAL;
    // only between blocks: no pushed events may be pending
    if (!c->deferred.empty() || c->counts_dirty) return REC_ESTATE;
    const size_t np = (size_t)c->fr.W * c->fr.H;
    if (!on_device) {
        for (size_t k = 0; k < np; ++k)
            if (!(isfinite(u[k]) && u[k] > 0.0f)) return REC_EINVAL;
        for (size_t k = 0; p && k < 3 * np; ++k)
            if (!isfinite(p[k])) return REC_EINVAL;
        for (size_t k = 0; started && k < np; ++k)
            if (t_last[k] > t_ref) return REC_EORDER;
    }
    // host arrays go straight into the current planes (the import kernel
    // then rewrites each pixel from its own value) or, for p in 16-bit
    // storage, through the spare FP32-sized dual planes
    const float* du = u;
    const float* dp = p;
    const int64_t* dt = t_last;
    hipError_t e = hipSuccess;
    if (!on_device) {
        const bool f32 = c->prm.storage == rec::kStoreF32;
        float* pst = f32 ? c->P.p[c->cur] : c->P.p[c->cur ^ 1];
        e = hipMemcpyAsync(c->P.u[c->cur], u, np * 4, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && p)
            e = hipMemcpyAsync(pst, p, 3 * np * 4, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && started)
            e = hipMemcpyAsync(c->P.t_last, t_last, np * 8, hipMemcpyHostToDevice, c->stream);
        du = c->P.u[c->cur];
        dp = p ? pst : nullptr;
        dt = started ? c->P.t_last : nullptr;
    }
    // the stream state, written once the copies above are done
    rec::DevState st;
    memset(&st, 0, sizeof(st));
    st.t_ref = started ? t_ref : 0;
    st.t_first = started ? INT64_MAX : 0;
    st.first_bad = rec::kNoBad;
    st.started = started ? 1 : 0;
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(c->P.st, &st, sizeof(st), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = rec::launch_import(c->P, c->fr, c->cur, c->prm.storage, du, dp, dt, started,
                               c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return REC_EDEVICE;
    c->mirror_known = true;
    c->mirror_started = started;
    c->mirror_tref = started ? t_ref : 0;
    c->gap_samples = 0;
    return REC_OK;
}

int rec_destroy(rec_ctx* c) {
    if (!c) return REC_OK;
    if (c->batch_refs > 0) return REC_ESTATE;  // a live batch still uses it
    int rc = REC_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) rc = REC_EDEVICE;
    for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->stage_done)
        if (e) (void)hipEventDestroy(e);
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
    return rc;
}

const char* rec_strerror(int code) {
    switch (code) {
        case REC_OK: return "success";
        case REC_EINVAL: return "invalid argument, parameter or event polarity";
        case REC_ERANGE: return "event coordinate outside the image";
        case REC_EORDER: return "event timestamp lower than the previous one";
        case REC_EDEVICE: return "HIP runtime error";
        case REC_ENUMERIC: return "non-finite gap or energy";
        case REC_ESTATE: return "call not valid in the current state";
        case REC_ENOMEM: return "workspace too small, allocation failed, or input beyond a static scratch limit";
        default: return "unknown status code";
    }
}

}  // extern "C"

// ------------------------------------------------------------------------
// Batched solves: many streams, one launch chain per tile-geometry class.
//
// Streams are grouped into classes (one per sensor size, at most
// kMaxClasses); every class has its own tile geometry and iterations per
// launch and a work list of its (stream, tile) pairs, so a solve runs one
// chain of ceil(iters / K_c) launches per class.  The chains run one after
// another on the batch's stream (REC_BATCH_SERIAL), concurrently on one
// stream per class forked from and joined back into the batch's stream
// (REC_BATCH_STREAMS), or as a HIP graph of that fork/join captured once
// per (iterations, descriptor buffer, folded-event classes) and replayed
// (REC_BATCH_GRAPH).  The descriptors are uploaded before the chains, into
// one of two fixed device buffers, so a captured graph stays valid.
// ------------------------------------------------------------------------

namespace {

struct Shape {
    int rows, waves, cols, k;
    bool operator==(const Shape& o) const {
        return rows == o.rows && waves == o.waves && cols == o.cols && k == o.k;
    }
};

constexpr int kMaxClasses = 8;
constexpr int kMaxGraphs = 8;

// Candidate tile geometries of the batched launch (rows per lane x
// wavefronts x columns) and iterations per launch.
std::vector<Shape> batch_candidates(int storage) {
    std::vector<Shape> v;
    const int shapes[][3] = {{2, 16, 64}, {4, 8, 64}, {4, 16, 64}, {6, 8, 64},
                             {8, 4, 64},  {8, 8, 64}, {1, 16, 32}, {2, 8, 32}};
    const int ks[] = {4, 6, 8, 9, 10, 13, 15};
    for (auto& sh : shapes) {
        if (!rec::batch_shape_supported(sh[0], sh[1], sh[2], storage)) continue;
        const int rh = sh[0] * sh[1] * (64 / sh[2]);
        for (int k : ks)
            if (k <= (rh - 1) / 2 && k <= (sh[2] - 1) / 2)
                v.push_back(Shape{sh[0], sh[1], sh[2], k});
    }
    return v;
}

int shape_tiles(rec::Frame fr, Shape sh) {
    return rec::fused_tiles(fr, sh.rows, sh.waves, sh.cols, sh.k);
}

}  // namespace

// Streams of one sensor size (or one run of sizes) and their geometry.
struct BatchGroup {
    std::vector<rec_ctx*> ctx;
    Shape shape;
    size_t max_np;          // largest frame of the group (pixels)
    int64_t px;             // pixels of all its streams
};

// Streams sharing one tile geometry: the groups of equal geometry, whose
// tiles one launch chain covers.
struct BatchClass {
    Shape shape;
    int s0, ns;             // its streams: descriptors s0 .. s0 + ns - 1
    int64_t work0;          // its (stream, tile) pairs: work list entries work0 ..
    int nwork;              //   work0 + nwork - 1
    size_t max_np;          // largest frame of the class (pixels)
};

struct GraphEntry {
    int iters, q;
    unsigned fold;          // classes whose first launch bins folded events
    hipGraphExec_t exec;
};

struct rec_batch {
    rec_ctx* lead;               // the caller's first context: holds the profiling state
    std::vector<BatchGroup> grp;
    std::vector<rec_ctx*> ctx;   // in descriptor order: grouped by class
    std::vector<BatchClass> cls;
    hipStream_t side[kMaxClasses];  // class ci > 0 runs on side[ci] (concurrent chains)
    hipEvent_t done[kMaxClasses];   //   and records done[ci] after its chain
    hipStream_t stream;
    int storage;
    int mode;                    // REC_BATCH_SERIAL, _STREAMS or _GRAPH
    double tuned_us;             // measured time of the tuned schedule (0: not tuned)
    // device workspace
    rec::StreamDesc* d_desc[2];  // alternating per solve
    int2* d_work;
    int64_t work_cap;
    // pinned staging of the descriptors (h_desc_dev: their device addresses)
    rec::StreamDesc* h_desc[2];
    const void* h_desc_dev[2];
    hipEvent_t copied[2];
    bool copy_used[2];
    int parity;
    hipEvent_t fork;
    // graphs are captured on and replayed in a stream of the batch's own
    // (the contexts' stream may be the null stream, which cannot capture),
    // ordered after and before the contexts' stream by two events
    hipStream_t cap;
    hipEvent_t pre, post;
    std::vector<GraphEntry> graphs;
    bool holds_refs;             // the contexts count this batch as a user
};

namespace {

size_t batch_desc_bytes(int n) { return align_up((size_t)n * sizeof(rec::StreamDesc)); }

// Groups the contexts into classes: one per distinct sensor size, or, with
// more sizes than kMaxClasses, runs of sizes ordered by pixel count.
// Returns the class index of every context.
std::vector<int> group_sizes(rec_ctx* const* ctxs, int n, int* nclasses) {
    std::vector<int64_t> keys;
    for (int i = 0; i < n; ++i) {
        const int64_t key = ((int64_t)ctxs[i]->fr.W << 32) | (uint32_t)ctxs[i]->fr.H;
        bool seen = false;
        for (int64_t k : keys) seen = seen || k == key;
        if (!seen) keys.push_back(key);
    }
    // sizes ordered by pixel count (then width)
    auto px = [](int64_t key) { return (key >> 32) * (key & 0xffffffff); };
    for (size_t i = 1; i < keys.size(); ++i)
        for (size_t j = i; j > 0 && (px(keys[j]) < px(keys[j - 1]) ||
                                     (px(keys[j]) == px(keys[j - 1]) && keys[j] < keys[j - 1]));
             --j) {
            const int64_t t = keys[j];
            keys[j] = keys[j - 1];
            keys[j - 1] = t;
        }
    const int nk = (int)keys.size();
    const int nc = nk < kMaxClasses ? nk : kMaxClasses;
    std::vector<int> out(n);
    for (int i = 0; i < n; ++i) {
        const int64_t key = ((int64_t)ctxs[i]->fr.W << 32) | (uint32_t)ctxs[i]->fr.H;
        int r = 0;
        while (keys[r] != key) ++r;
        out[i] = (int)((int64_t)r * nc / nk);  // consecutive sizes share a class
    }
    *nclasses = nc;
    return out;
}

// Classes from the groups' geometries: groups of equal geometry form one
// class (one launch chain); the descriptor order follows the classes.
void build_classes(rec_batch* b) {
    std::vector<int> order(b->grp.size());
    for (size_t g = 0; g < order.size(); ++g) order[g] = (int)g;
    auto key = [&](int g) {
        const Shape& sh = b->grp[g].shape;
        return ((int64_t)sh.rows << 24) | ((int64_t)sh.waves << 16) | ((int64_t)sh.cols << 8) |
               sh.k;
    };
    for (size_t i = 1; i < order.size(); ++i)  // stable: equal geometries keep group order
        for (size_t j = i; j > 0 && key(order[j]) < key(order[j - 1]); --j) {
            const int t = order[j];
            order[j] = order[j - 1];
            order[j - 1] = t;
        }
    b->ctx.clear();
    b->cls.clear();
    for (int g : order) {
        const BatchGroup& gr = b->grp[g];
        if (b->cls.empty() || !(b->cls.back().shape == gr.shape)) {
            BatchClass c{};
            c.shape = gr.shape;
            c.s0 = (int)b->ctx.size();
            b->cls.push_back(c);
        }
        BatchClass& c = b->cls.back();
        for (rec_ctx* x : gr.ctx) b->ctx.push_back(x);
        c.ns += (int)gr.ctx.size();
        if (gr.max_np > c.max_np) c.max_np = gr.max_np;
    }
}

int upload_work(rec_batch* b) {
    std::vector<int2> w;
    for (BatchClass& c : b->cls) {
        c.work0 = (int64_t)w.size();
        for (int s = c.s0; s < c.s0 + c.ns; ++s) {
            const int t = shape_tiles(b->ctx[s]->fr, c.shape);
            if (t <= 0) return REC_EINVAL;
            for (int q = 0; q < t; ++q) w.push_back(make_int2(s, q));
        }
        c.nwork = (int)((int64_t)w.size() - c.work0);
    }
    if ((int64_t)w.size() > b->work_cap) return REC_ENOMEM;
    if (hipMemcpy(b->d_work, w.data(), w.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess)
        return REC_EDEVICE;
    return REC_OK;
}

// Descriptors of every stream; *fold receives the classes (bit mask) in
// which some stream folds pushed events into its first launch.
void fill_desc(rec_batch* b, rec::StreamDesc* d, unsigned* fold) {
    *fold = 0;
    for (size_t ci = 0; ci < b->cls.size(); ++ci) {
        const BatchClass& cl = b->cls[ci];
        for (int s = cl.s0; s < cl.s0 + cl.ns; ++s) {
            rec_ctx* c = b->ctx[s];
            rec::StreamDesc& e = d[s];
            memset(&e, 0, sizeof(e));
            e.P = c->P;
            e.fr = c->fr;
            e.kc = c->kc;
            e.bc = rec::make_build_consts(c->prm.delta_pos, c->prm.delta_neg, c->prm.time_unit_us);
            e.cur = c->cur;
            const int ow = cl.shape.cols - 2 * cl.shape.k;
            e.tiles_x = (c->fr.W + ow - 1) / ow;
            e.tiles_x_div = rec::make_divider((uint32_t)e.tiles_x);
            const bool f = !c->deferred.empty();
            if (f) {
                for (size_t q = 0; q < c->deferred.size(); ++q) {
                    e.segs.t[q] = c->deferred[q].t;
                    e.segs.x[q] = c->deferred[q].x;
                    e.segs.y[q] = c->deferred[q].y;
                    e.segs.p[q] = c->deferred[q].p;
                    e.segs.n[q] = c->deferred[q].n;
                }
                e.segs.count = (int32_t)c->deferred.size();
                *fold |= 1u << ci;
            }
            e.mode0 = rec::kBuild | (f ? rec::kEvents : 0) |
                      (c->counts_dirty ? rec::kCounts : 0) | rec::kRotIn;
            e.mode1 = rec::kCommit | (c->counts_dirty ? rec::kZero : 0);
        }
    }
}

// Enqueues the launch chains of every class for `iters` iterations on the
// descriptors in buffer q, on stream `main`.  concurrent: each class but the
// first runs on its own stream, forked from and joined back into `main`.
// timing: side-effect-free launches for the autotuner (every launch reads
// the current buffers and writes the others, modes 0, no folded events).
int enqueue_chains(rec_batch* b, hipStream_t main, int q, int iters, unsigned fold,
                   bool concurrent, bool timing) {
    const bool fork = concurrent && b->cls.size() > 1;
    if (fork) {
        if (hipEventRecord(b->fork, main) != hipSuccess) return REC_EDEVICE;
        for (size_t ci = 1; ci < b->cls.size(); ++ci)
            if (hipStreamWaitEvent(b->side[ci], b->fork, 0) != hipSuccess) return REC_EDEVICE;
    }
    rec_ctx* c0 = b->lead;
    for (size_t ci = 0; ci < b->cls.size(); ++ci) {
        const BatchClass& cl = b->cls[ci];
        hipStream_t s = (fork && ci > 0) ? b->side[ci] : main;
        const int K = cl.shape.k;
        const int nl = (iters + K - 1) / K;
        for (int li = 0; li < nl; ++li) {
            const int m = iters / nl + (li < iters % nl ? 1 : 0);
            int64_t work = 0;
            if (c0->prof_on && !timing)
                for (int si = cl.s0; si < cl.s0 + cl.ns; ++si)
                    work += (int64_t)b->ctx[si]->fr.W * b->ctx[si]->fr.H * m;
            auto go = [&](rec::LaunchEv ev) {
                return rec::launch_pd_batch(b->d_desc[q], b->d_work + cl.work0, cl.nwork, m, K,
                                            timing ? 2 : li, !timing && li == nl - 1,
                                            !timing && li == 0 && ((fold >> ci) & 1u),
                                            cl.shape.rows, cl.shape.waves, cl.shape.cols,
                                            b->storage, s, ev);
            };
            const int rc = timing ? dev_err(go(rec::LaunchEv{})) : timed(c0, 2, work, go);
            if (rc) return rc;
        }
        if (nl == 1 && !timing &&
            hipSuccess != rec::launch_finish_batch(b->d_desc[q] + cl.s0, cl.ns, cl.max_np, s))
            return REC_EDEVICE;
        if (fork && ci > 0 && hipEventRecord(b->done[ci], s) != hipSuccess) return REC_EDEVICE;
    }
    if (fork)
        for (size_t ci = 1; ci < b->cls.size(); ++ci)
            if (hipStreamWaitEvent(main, b->done[ci], 0) != hipSuccess) return REC_EDEVICE;
    return REC_OK;
}

// Time `reps` side-effect-free runs of the whole schedule of the current
// geometries (concurrent chains, `iters` iterations): the least time of
// a run, in microseconds.
int time_schedule(rec_batch* b, int iters, int reps, double* us) {
    build_classes(b);
    int rc = upload_work(b);
    if (rc) return rc;
    rec::StreamDesc* h = b->h_desc[0];
    unsigned fold = 0;
    fill_desc(b, h, &fold);
    for (size_t s = 0; s < b->ctx.size(); ++s) h[s].mode0 = h[s].mode1 = 0;
    if (hipMemcpy(b->d_desc[0], h, b->ctx.size() * sizeof(rec::StreamDesc), hipMemcpyHostToDevice) !=
        hipSuccess)
        return REC_EDEVICE;
    // one event between runs: the time of a run is the least of `reps`
    // (each run's chains are joined back into the stream before the next
    // forks, so consecutive events bracket one run)
    constexpr int kMaxReps = 8;
    if (reps < 1 || reps > kMaxReps) return REC_EINVAL;
    hipEvent_t ev[kMaxReps + 1];
    int nev = 0;
    for (; nev <= reps; ++nev)
        if (hipEventCreate(&ev[nev]) != hipSuccess) break;
    if (nev <= reps) rc = REC_EDEVICE;
    if (!rc) rc = enqueue_chains(b, b->stream, 0, iters, 0, true, true);  // warm-up run
    if (!rc && hipEventRecord(ev[0], b->stream) != hipSuccess) rc = REC_EDEVICE;
    for (int r = 0; r < reps && !rc; ++r) {
        rc = enqueue_chains(b, b->stream, 0, iters, 0, true, true);
        if (!rc && hipEventRecord(ev[r + 1], b->stream) != hipSuccess) rc = REC_EDEVICE;
    }
    if (!rc && hipStreamSynchronize(b->stream) != hipSuccess) rc = REC_EDEVICE;
    float best = 0.0f;
    for (int r = 0; r < reps && !rc; ++r) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev[r], ev[r + 1]) != hipSuccess)
            rc = REC_EDEVICE;
        else if (r == 0 || ms < best)
            best = ms;
    }
    for (int i = 0; i < nev; ++i) (void)hipEventDestroy(ev[i]);
    if (!rc) *us = (double)best * 1e3;
    return rc;
}

void drop_graphs(rec_batch* b) {
    for (GraphEntry& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
}

// The captured fork/join of a solve (built on first use).
int graph_for(rec_batch* b, int q, int iters, unsigned fold, hipGraphExec_t* out) {
    for (const GraphEntry& g : b->graphs)
        if (g.iters == iters && g.q == q && g.fold == fold) {
            *out = g.exec;
            return REC_OK;
        }
    if ((int)b->graphs.size() == kMaxGraphs) drop_graphs(b);
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed) != hipSuccess)
        return REC_EDEVICE;
    const int rc = enqueue_chains(b, b->cap, q, iters, fold, true, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : REC_EDEVICE;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return REC_EDEVICE;
    b->graphs.push_back(GraphEntry{iters, q, fold, exec});
    *out = exec;
    return REC_OK;
}

}  // namespace

extern "C" {

size_t rec_batch_workspace_bytes(rec_ctx* const* ctxs, int32_t n) {
    if (!ctxs || n < 1) return 0;
    for (int i = 0; i < n; ++i)
        if (!ctxs[i]) return 0;
    // every stream may get any candidate geometry
    const std::vector<Shape> cand = batch_candidates(ctxs[0]->prm.storage);
    int64_t tiles = 0;
    for (int i = 0; i < n; ++i) {
        int64_t t = 0;
        for (const Shape& sh : cand) {
            const int64_t ti = shape_tiles(ctxs[i]->fr, sh);
            if (ti > t) t = ti;
        }
        tiles += t;
    }
    return 2 * batch_desc_bytes(n) + align_up((size_t)tiles * sizeof(int2));
}

int rec_batch_init(rec_ctx* const* ctxs, int32_t n, void* dev_workspace, size_t ws_bytes,
                   int32_t tune_iters, rec_batch** out) {
    Range range("rec_batch_init");
    if (!out) return REC_EINVAL;
    *out = nullptr;
    if (!ctxs || n < 1 || tune_iters < 0) return REC_EINVAL;
    for (int i = 0; i < n; ++i) {
        rec_ctx* c = ctxs[i];
        if (!c || c->stream != ctxs[0]->stream || c->device != ctxs[0]->device) return REC_EINVAL;
        if (c->prm.storage != ctxs[0]->prm.storage || c->prm.fuse_iters == 0 ||
            c->prm.tvl1_iters > 0 || c->prm.gap_every > 0)
            return REC_EINVAL;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return REC_EINVAL;
    }
    if (!dev_workspace || ((uintptr_t)dev_workspace & (kAlign - 1))) return REC_EINVAL;
    const size_t need = rec_batch_workspace_bytes(ctxs, n);
    if (ws_bytes < need) return REC_ENOMEM;
    rec_batch* b = new (std::nothrow) rec_batch();
    if (!b) return REC_ENOMEM;
    b->stream = ctxs[0]->stream;
    b->storage = ctxs[0]->prm.storage;
    b->mode = REC_BATCH_STREAMS;
    b->lead = ctxs[0];
    int ng = 0;
    const std::vector<int> grp_of = group_sizes(ctxs, n, &ng);
    b->grp.resize(ng);
    for (int i = 0; i < n; ++i) {
        BatchGroup& g = b->grp[grp_of[i]];
        g.ctx.push_back(ctxs[i]);
        const size_t np = (size_t)ctxs[i]->fr.W * ctxs[i]->fr.H;
        if (np > g.max_np) g.max_np = np;
        g.px += (int64_t)np;
    }
    // default geometry, one for every group: the automatic choice for a frame
    // of the batch's total pixel count (64-column tiles)
    {
        int64_t total = 0;
        for (const BatchGroup& g : b->grp) total += g.px;
        int r, w, cw, k;
        rec::choose_shape(&ctxs[0]->prm, total, false, &r, &w, &cw, &k);
        if (!rec::batch_shape_supported(r, w, cw, b->storage)) {
            r = 4;
            w = 8;
            cw = 64;
            if (k > 15) k = 15;
        }
        for (BatchGroup& g : b->grp) g.shape = Shape{r, w, cw, k};
    }
    build_classes(b);
    char* base = (char*)dev_workspace;
    b->d_desc[0] = (rec::StreamDesc*)base;
    b->d_desc[1] = (rec::StreamDesc*)(base + batch_desc_bytes(n));
    b->d_work = (int2*)(base + 2 * batch_desc_bytes(n));
    b->work_cap = (int64_t)((ws_bytes - 2 * batch_desc_bytes(n)) / sizeof(int2));
    int rc = REC_OK;
    for (int q = 0; q < 2 && !rc; ++q) {
        // as long as the device buffer (the copy kernel reads whole 16-byte
        // words); coherent, like the push staging
        if (hipHostMalloc((void**)&b->h_desc[q], batch_desc_bytes(n), hipHostMallocCoherent) !=
            hipSuccess)
            rc = REC_ENOMEM;
        else if (hipHostGetDevicePointer((void**)&b->h_desc_dev[q], b->h_desc[q], 0) !=
                     hipSuccess ||
                 hipEventCreateWithFlags(&b->copied[q], hipEventDisableTiming) != hipSuccess)
            rc = REC_EDEVICE;
    }
    if (!rc && (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&b->pre, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&b->post, hipEventDisableTiming) != hipSuccess ||
                hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess))
        rc = REC_EDEVICE;
    for (int ci = 1; ci < ng && !rc; ++ci) {
        // default priority (work on streams of different priorities is not mixed)
        if (hipStreamCreateWithFlags(&b->side[ci], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->done[ci], hipEventDisableTiming) != hipSuccess)
            rc = REC_EDEVICE;
    }
    // all streams' pending work must be on the stream before timing reads it
    if (!rc && hipStreamSynchronize(b->stream) != hipSuccess) rc = REC_EDEVICE;
    if (!rc && tune_iters > 0) {
        // autotuner on the measured time of the whole schedule (all class
        // chains, concurrent) for tune_iters iterations:
        //  1. one geometry for every group (one launch chain): best candidate;
        //  2. coordinate descent over the groups, largest first, each trying
        //     every candidate with the others fixed (groups that end up
        //     with equal geometries share one launch chain).
        const std::vector<Shape> cand = batch_candidates(b->storage);
        auto measure = [&](double* us) {
            const int r = time_schedule(b, tune_iters, 5, us);
            return r == REC_ENOMEM || r == REC_EINVAL ? 1 : r;  // 1: does not fit
        };
        double best = 1e300;
        std::vector<Shape> keep(ng);
        for (int g = 0; g < ng; ++g) keep[g] = b->grp[g].shape;
        for (size_t ci = 0; ci < cand.size() && (rc == REC_OK || rc == 1); ++ci) {
            for (BatchGroup& g : b->grp) g.shape = cand[ci];
            double us = 0.0;
            rc = measure(&us);
            if (rc == REC_OK && us < best) {
                best = us;
                for (int g = 0; g < ng; ++g) keep[g] = cand[ci];
            }
        }
        if (rc == 1) rc = REC_OK;
        std::vector<int> order(ng);
        for (int g = 0; g < ng; ++g) order[g] = g;
        for (int i = 1; i < ng; ++i)
            for (int j = i; j > 0 && b->grp[order[j]].px > b->grp[order[j - 1]].px; --j) {
                const int t = order[j];
                order[j] = order[j - 1];
                order[j - 1] = t;
            }
        for (int oi = 0; oi < ng && ng > 1 && !rc; ++oi) {
            const int g = order[oi];
            for (const Shape& sh : cand) {
                if (sh == keep[g]) continue;
                for (int h = 0; h < ng; ++h) b->grp[h].shape = h == g ? sh : keep[h];
                double us = 0.0;
                rc = measure(&us);
                if (rc == 1) {
                    rc = REC_OK;
                    continue;
                }
                if (rc) break;
                if (us < best) {
                    best = us;
                    keep[g] = sh;
                }
            }
        }
        for (int g = 0; g < ng; ++g) b->grp[g].shape = keep[g];
        b->tuned_us = best < 1e300 ? best : 0.0;
        build_classes(b);
    }
    if (!rc) rc = upload_work(b);
    if (rc) {
        rec_batch_destroy(b);
        return rc;
    }
    for (rec_ctx* c : b->ctx) ++c->batch_refs;
    b->holds_refs = true;
    *out = b;
    return REC_OK;
}

int rec_batch_solve(rec_batch* b, int32_t iters) {
    Range range("rec_batch_solve");
    if (!b || iters < 1) return REC_EINVAL;
    int rc;
    // pushes the first launch cannot fold are scattered first
    for (const BatchClass& cl : b->cls)
        for (int s = cl.s0; s < cl.s0 + cl.ns; ++s) {
            rec_ctx* c = b->ctx[s];
            const int64_t tiles = shape_tiles(c->fr, cl.shape);
            if (c->deferred_events > kFoldMaxEvents || c->deferred_events * tiles > kFoldMaxWork) {
                rc = flush_deferred(c);
                if (rc) return rc;
            }
        }
    const int q = b->parity;
    if (b->copy_used[q] && hipEventSynchronize(b->copied[q]) != hipSuccess) return REC_EDEVICE;
    unsigned fold = 0;
    fill_desc(b, b->h_desc[q], &fold);
    const size_t n = b->ctx.size();
    // one copy kernel (per kMaxPulls copies) moves the descriptors and the
    // records of every context's host pushes
    std::vector<rec::PullDesc> pl;
    pl.push_back(rec::PullDesc{b->h_desc_dev[q], b->d_desc[q],
                               (n * sizeof(rec::StreamDesc) + 15) & ~(size_t)15});
    for (rec_ctx* c : b->ctx) pl.insert(pl.end(), c->pulls.begin(), c->pulls.end());
    for (size_t a = 0; a < pl.size(); a += rec::kMaxPulls) {
        const int m = (int)std::min(pl.size() - a, (size_t)rec::kMaxPulls);
        rc = timed(b->lead, 0, 0, [&](rec::LaunchEv ev) {
            return rec::launch_pulls(pl.data() + a, m, b->stream, ev.start, ev.stop);
        });
        if (rc) return rc;
    }
    for (rec_ctx* c : b->ctx) {
        rc = pulls_launched(c);
        if (rc) return rc;
    }
    if (hipEventRecord(b->copied[q], b->stream) != hipSuccess) return REC_EDEVICE;
    b->copy_used[q] = true;
    b->parity ^= 1;
    if (b->mode == REC_BATCH_GRAPH && !b->lead->prof_on) {
        hipGraphExec_t exec = nullptr;
        rc = graph_for(b, q, iters, fold, &exec);
        if (rc) return rc;
        if (hipEventRecord(b->pre, b->stream) != hipSuccess ||
            hipStreamWaitEvent(b->cap, b->pre, 0) != hipSuccess ||
            hipGraphLaunch(exec, b->cap) != hipSuccess ||
            hipEventRecord(b->post, b->cap) != hipSuccess ||
            hipStreamWaitEvent(b->stream, b->post, 0) != hipSuccess)
            return REC_EDEVICE;
    } else {
        rc = enqueue_chains(b, b->stream, q, iters, fold, b->mode != REC_BATCH_SERIAL, false);
        if (rc) return rc;
    }
    for (const BatchClass& cl : b->cls) {
        const int nl = (iters + cl.shape.k - 1) / cl.shape.k;
        for (int s = cl.s0; s < cl.s0 + cl.ns; ++s) {
            rec_ctx* c = b->ctx[s];
            c->cur ^= (nl & 1);
            c->deferred.clear();
            c->deferred_events = 0;
            c->counts_dirty = false;
            c->gap_samples = 0;
        }
    }
    return REC_OK;
}

int rec_batch_classes(const rec_batch* b) {
    if (!b) return REC_EINVAL;
    return (int)b->cls.size();
}

int rec_batch_config(const rec_batch* b, int32_t cls, rec_batch_class* out) {
    if (!b || !out || cls < 0 || cls >= (int)b->cls.size()) return REC_EINVAL;
    const BatchClass& cl = b->cls[cls];
    out->width = b->ctx[cl.s0]->fr.W;
    out->height = b->ctx[cl.s0]->fr.H;
    out->streams = cl.ns;
    out->rows = cl.shape.rows;
    out->waves = cl.shape.waves;
    out->cols = cl.shape.cols;
    out->kiters = cl.shape.k;
    out->tiles = cl.nwork;
    out->tuned_us = b->tuned_us;
    return REC_OK;
}

int rec_batch_set_geometry(rec_batch* b, int32_t width, int32_t height, int32_t rows,
                           int32_t waves, int32_t cols, int32_t kiters) {
    Range range("rec_batch_set_geometry");
    if (!b || !rec::batch_shape_supported(rows, waves, cols, b->storage) || kiters < 1 ||
        kiters > (cols - 1) / 2 || kiters > (rows * waves * (64 / cols) - 1) / 2)
        return REC_EINVAL;
    BatchGroup* grp = nullptr;
    for (BatchGroup& g : b->grp)
        for (rec_ctx* c : g.ctx)
            if (c->fr.W == width && c->fr.H == height) grp = &g;
    if (!grp) return REC_EINVAL;
    // the work list may still be read by the previous solve's launches
    if (hipStreamSynchronize(b->stream) != hipSuccess) return REC_EDEVICE;
    const Shape old = grp->shape;
    grp->shape = Shape{rows, waves, cols, kiters};
    drop_graphs(b);
    build_classes(b);
    int rc = upload_work(b);
    if (rc) {
        grp->shape = old;
        build_classes(b);
        const int r2 = upload_work(b);
        return rc ? rc : r2;
    }
    return REC_OK;
}

int rec_batch_set_mode(rec_batch* b, int32_t mode) {
    if (!b || (mode != REC_BATCH_SERIAL && mode != REC_BATCH_STREAMS && mode != REC_BATCH_GRAPH))
        return REC_EINVAL;
    b->mode = mode;
    return REC_OK;
}

int rec_batch_destroy(rec_batch* b) {
    if (!b) return REC_OK;
    int rc = REC_OK;
    if (hipStreamSynchronize(b->stream) != hipSuccess) rc = REC_EDEVICE;
    if (b->holds_refs)
        for (rec_ctx* c : b->ctx) --c->batch_refs;
    drop_graphs(b);
    for (int ci = 0; ci < kMaxClasses; ++ci) {
        if (b->side[ci]) {
            if (hipStreamSynchronize(b->side[ci]) != hipSuccess) rc = REC_EDEVICE;
            (void)hipStreamDestroy(b->side[ci]);
        }
        if (b->done[ci]) (void)hipEventDestroy(b->done[ci]);
    }
    if (b->cap) {
        if (hipStreamSynchronize(b->cap) != hipSuccess) rc = REC_EDEVICE;
        (void)hipStreamDestroy(b->cap);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->pre) (void)hipEventDestroy(b->pre);
    if (b->post) (void)hipEventDestroy(b->post);
    for (int q = 0; q < 2; ++q) {
        if (b->copied[q]) (void)hipEventDestroy(b->copied[q]);
        if (b->h_desc[q]) (void)hipHostFree(b->h_desc[q]);
    }
    delete b;
    return rc;
}

}  // extern "C"
