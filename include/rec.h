/*
 * rec.h - C ABI of the MI355X (gfx950) intensity-image reconstruction for
 * event cameras on the event manifold (Reinbacher, Graber, Pock, BMVC 2016).
 *
 * For each block of events the library
 *   1. scatters the events into per-pixel polarity counts and the latest
 *      timestamp of every pixel (Section 3: e^n = (x^n, y^n, theta^n, t^n)),
 *   2. forms the data image f = u_prev * exp(Delta+ n+ - Delta- n-)
 *      (eqn. intensity_update applied for every event of the block),
 *   3. forms the time surface tau = (t_ref - t_last) / T_s and its forward
 *      differences, which define the metric g = I + grad tau grad tau^T
 *      (Section 3.1, eqns. 1-2; discrete operator L_g of eqn. 3),
 *   4. runs Chambolle-Pock primal-dual iterations for eqn. (5), the
 *      manifold TV with the generalised Kullback-Leibler data term on
 *      [u_min, u_max], with the closed-form proximal maps of Section 3.2,
 *      warm-started from the previous block's (u, p).
 *
 * Conventions
 *   - Images are H x W, row-major, x = column index (fast), y = row index.
 *   - Timestamps are int64 microseconds and must not decrease (ties allowed),
 *     also across pushes.  Relative times are formed from exact int64
 *     differences, divided in FP64, and only then rounded to FP32.
 *   - The primal image u and the data image f are FP32 in device memory.
 *     The dual field p (3 planes) and the time differences tx, ty are FP32,
 *     or BF16 / FP16 with rec_params.storage; the arithmetic is FP32 in
 *     every case, and the primal-dual gap is accumulated in FP64.
 *   - Every function returns an int status: REC_OK (0) or a negative REC_E*
 *     code.  No C++ exception crosses this interface.
 *
 * Ownership
 *   - The caller allocates the device workspace (rec_workspace_bytes) and
 *     keeps it alive until rec_destroy; the library never allocates device
 *     memory.  It allocates the host-side context and a pinned host staging
 *     buffer for host-pointer pushes, both released by rec_destroy.
 *   - Event arrays and output buffers belong to the caller.  Host arrays
 *     only need to stay valid for the duration of the call.  A device-
 *     pointer push records the pointers: the arrays must stay valid, and
 *     unchanged, until the next rec_solve (or rec_batch_solve) has completed
 *     on the context's stream, or until one of the synchronising calls
 *     below has returned (each scatters the recorded pushes first).
 *
 * Streams and synchronisation
 *   - All device work of a context -- pushes, builds, iterations, gap
 *     evaluations and readbacks -- is enqueued in order on the one
 *     hipStream_t given to rec_init (NULL = the default stream); only a
 *     batch (rec_batch_init) creates streams of its own, which it forks from
 *     and joins back into that stream within each solve.  Work the caller
 *     enqueues on that stream after a call returns is ordered after that
 *     call's work.
 *   - Device-pointer pushes are not launched when made: the first fused
 *     launch of the next rec_solve validates and bins them itself (or, for
 *     more pushes or events than it takes, they are scattered by kernels of
 *     their own at that point).  Host-pointer pushes are validated on the
 *     host and written to the pinned staging buffer; one copy kernel on the
 *     context's stream moves all such records pending into the workspace's
 *     staging ring when they are first needed (by the next solve -- for a
 *     batch, one launch for all its contexts -- or a call that scatters
 *     them); from there they take the same way (the unfused loop, and a
 *     push of more than max_events events, scatter them at once).  The
 *     ring has room for two pushes of max_events events: a push that starts
 *     a half waits on the host for the last copy out of that half.
 *   - rec_push_events and rec_solve without stats do not synchronise.
 *     rec_solve with stats, rec_get_image, rec_gap_history, rec_get_times,
 *     rec_set_state, rec_profile_read, rec_sync and rec_destroy synchronise
 *     the stream.
 *   - Errors found on the device (device-pointer pushes) are reported by the
 *     next synchronising call; the rejected push changes no state.
 *   - After REC_EDEVICE the context's state is undefined: destroy it, or
 *     restore a checkpoint with rec_set_state.  (Tests force this path with
 *     REC_FAULT_AFTER=n in the environment: every launch after the process's
 *     first n fails without being issued.)
 *
 * Threading: a context must not be used from two threads at once; distinct
 * contexts are independent.  The only global state of the library is the
 * static device array of rec_diff_forward_noalloc and the per-device
 * address of it that the library looks up once (see there).
 */
#ifndef REC_H
#define REC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    REC_OK = 0,
    REC_EINVAL = -1,   /* bad argument or parameter, polarity not in {-1, +1} */
    REC_ERANGE = -2,   /* event coordinate outside the image */
    REC_EORDER = -3,   /* timestamp lower than the previous one */
    REC_EDEVICE = -4,  /* a HIP runtime call failed */
    REC_ENUMERIC = -5, /* non-finite gap or energy */
    REC_ESTATE = -6,   /* call not valid in the object's state: rec_destroy of a
                          context that a live batch still holds, rec_set_state
                          with pushes pending */
    REC_ENOMEM = -7    /* workspace too small, host allocation failed, or input larger
                          than the static array of rec_diff_forward_noalloc */
};

/* Planes readable with rec_get_image. */
enum {
    REC_U = 0,         /* float[H*W]  reconstructed image u */
    REC_F = 1,         /* float[H*W]  data image f of the last solved block */
    REC_TIME = 2,      /* float[H*W]  tau = (t_ref - t_last) / T_s, now */
    REC_METRIC_G = 3,  /* float[H*W]  G = 1 + tx^2 + ty^2 of the last block */
    REC_STATE_P = 4,   /* float[3*H*W] dual field p, planes p1, p2, p3 */
    REC_TX = 5,        /* float[H*W]  tau(x+1, y) - tau(x, y), 0 on the last column */
    REC_TY = 6,        /* float[H*W]  tau(x, y+1) - tau(x, y), 0 on the last row */
    REC_COUNT_POS = 7, /* int32[H*W]  positive events of the pending block */
    REC_COUNT_NEG = 8, /* int32[H*W]  negative events of the pending block */
    REC_T_LAST = 9     /* int64[H*W]  latest timestamp; a pixel that never fired reads
                          as the stream's first timestamp (0 before any event) */
};

/* Storage of the dual field and the time differences (rec_params.storage). */
enum { REC_STORE_F32 = 0, REC_STORE_BF16 = 1, REC_STORE_F16 = 2 };

typedef struct rec_ctx rec_ctx;

/* Method and launch parameters.  rec_default_params fills every field. */
typedef struct {
    int32_t width, height;   /* image size, 1 .. 65535 each */
    double lambda;           /* data-term weight lambda (eqn. 5); default 90 */
    double delta_pos;        /* contrast thresholds Delta+, Delta- (Section 3); */
    double delta_neg;        /*   default 0.2 each */
    double u_min, u_max;     /* intensity range (eqn. data_term); default 1, e */
    double tau, sigma;       /* primal / dual steps; tau*sigma*(8 + 4 sqrt 2) <= 1
                                (Section 3.2); default (8 + 4 sqrt 2)^(-1/2) each */
    double time_unit_us;     /* T_s: microseconds per unit of tau; default 1000;
                                0 switches the manifold off (t = const, Section 4.2) */
    double u_init;           /* constant initial image if rec_init gets no u0;
                                default sqrt(u_min * u_max) */
    int32_t iters;           /* iterations per rec_solve when called with 0; default 50 */
    int32_t gap_every;       /* gap / energy every this many iterations; 0 = never */
    int32_t fuse_iters;      /* iterations per fused launch: -1 = chosen from the frame
                                size (default), 0 = unfused two-kernel loop, k >= 1 = at
                                most k (also capped by the tile height) */
    int32_t max_events;      /* largest host-pointer push handled in one piece (larger
                                pushes are split); sizes the staging ring, 26 bytes per
                                event of workspace and of pinned memory; default 65536 */
    int32_t tile_rows;       /* fused tile: rows per lane x wavefronts per workgroup, one of */
    int32_t tile_waves;      /*   2x2 2x4 2x8 2x16 3x16 4x1 4x2 4x4 4x8 4x16 5x8 6x8 8x1
                                  8x2 8x4 8x8 16x1 16x2 16x4 (16-bit storage: 2x16 4x8 4x16
                                  8x4 8x8) with 64 columns; set both or neither.  0, 0 =
                                  automatic by frame size (tile_cols 0 too): up to 60k
                                  pixels 1x16 of 32 columns, up to 120k 2x8 of 32 columns,
                                  up to 400k 4x16, up to 600k 2x8 of 32 columns, larger 8x8
                                  (16-bit storage: 2x8 of 32 columns for the 32-column
                                  cases) */
    int32_t storage;         /* storage of the dual field p and of tx, ty: REC_STORE_F32
                                (default), REC_STORE_BF16 or REC_STORE_F16; the arithmetic
                                is FP32 in every case (16-bit forms need the fused loop) */
    int32_t tvl1_iters;      /* timestamp denoising before the metric is built (Section 4
                                applies a small number of TV-L1 iterations and gives neither
                                count nor weight): FP64 Chambolle-Pock iterations for
                                min TV(v) + tvl1_lambda |v - tau|_1; 0 = off (default) */
    double tvl1_lambda;      /* L1 weight of the denoising, > 0; default 1 */
    int32_t tile_cols;       /* fused tile width: 64 (one row of 64 lanes per wavefront) or
                                32 (two rows of 32 lanes per wavefront; shapes 1x8 1x16 2x4
                                2x8 2x16 3x8 4x4 4x8, 16-bit storage 2x8; the tile covers
                                32 columns x 2 * rows * waves rows); 0 = 64 when tile_rows
                                is set, automatic otherwise; set only with tile_rows */
    int32_t reserved[3];     /* must be 0 */
} rec_params;

/* Statistics of one rec_solve (filled when stats are requested). */
typedef struct {
    double gap;              /* last sampled primal-dual gap (NaN if none sampled) */
    double energy;           /* energy of eqn. (5) at the same iterate */
    int32_t iters_run;
    int32_t gap_samples;
    int64_t t_ref_us;        /* timestamp of the last event pushed so far */
    int64_t events_in_batch; /* events consumed by this solve */
} rec_stats;

/* Per-kernel-class device time, collected when profiling is on. */
typedef struct {
    double ms[4];            /* 0 push, 1 build, 2 primal-dual, 3 gap */
    int64_t launches[4];
    int64_t pd_pixel_iters;  /* pixel-iterations done by the primal-dual launches */
} rec_profile_t;

/* Fill *prm with the defaults for a width x height sensor. */
void rec_default_params(rec_params* prm, int32_t width, int32_t height);

/* Validate parameters on the host; REC_OK or REC_EINVAL.  No device call. */
int rec_check_params(const rec_params* prm);

/* Device workspace bytes needed for prm (0 if prm is invalid). */
size_t rec_workspace_bytes(const rec_params* prm);

/* Host validation of an event array (no device call): polarity in {-1, +1}
 * (REC_EINVAL), x < width and y < height (REC_ERANGE), t non-decreasing and
 * t[0] >= t_prev (REC_EORDER; pass INT64_MIN for no previous timestamp).
 * The first failing event decides the code. */
int rec_check_events(const int64_t* t_us, const uint16_t* x, const uint16_t* y,
                     const int8_t* polarity, int64_t n, int32_t width, int32_t height,
                     int64_t t_prev);

/* Create a context on the current HIP device: the reconstruction state of
 * one event camera of width x height pixels (the image domain Omega of
 * Section 3), with u initialised to prm->u_init or to the caller's first
 * image u0 (Section 3 notes that the first image cannot be recovered from
 * events; a known u0 is the case the paper integrates from), p = 0, no
 * event seen.
 *   dev_workspace  device memory of at least rec_workspace_bytes(prm)
 *                  bytes, 256-byte aligned; owned by the caller.
 *   ws_bytes       its size in bytes.
 *   hip_stream     a hipStream_t or NULL (default stream).
 *   u0             optional host image, H*W floats row-major, each finite
 *                  and > 0; copied before the call returns.
 *   out            receives the context.
 * Errors: REC_EINVAL (bad parameters, NULL or misaligned workspace, a u0
 * value <= 0 or non-finite), REC_ENOMEM (short workspace, host allocation),
 * REC_EDEVICE (HIP call failed).  On error *out is NULL and nothing is
 * left allocated.  The workspace is initialised asynchronously on the
 * stream (with u0 the call synchronises once). */
int rec_init(const rec_params* prm, void* dev_workspace, size_t ws_bytes, void* hip_stream,
             const float* u0, rec_ctx** out);

/* Add n events e^k = (x^k, y^k, theta^k, t^k) (Section 3: pixel, polarity
 * +-1, timestamp) to the pending block.  SoA arrays of n elements each:
 * t_us int64 microseconds, non-decreasing within the push and across
 * pushes; x < width and y < height; polarity in {-1, +1}.  Host memory if
 * on_device == 0, device memory otherwise (see Ownership).
 * All-or-nothing: a rejected push changes no state.  Host pointers are
 * validated on the host before anything is enqueued (REC_EINVAL bad
 * polarity or NULL array, REC_ERANGE coordinate outside the image,
 * REC_EORDER timestamp below the previous one; the first failing event
 * decides); device pointers are validated on the device and the same codes
 * are reported by the next synchronising call.  n == 0 is a no-op. */
int rec_push_events(rec_ctx* c, const int64_t* t_us, const uint16_t* x, const uint16_t* y,
                    const int8_t* polarity, int64_t n, int on_device);

/* Solve the pending block.
 *   1. f = u_prev * exp(Delta+ n+ - Delta- n-) per pixel, n+- the block's
 *      event counts (eqn. intensity_update applied for every event);
 *   2. tau = (t_ref - t_last) / T_s and its forward differences tx, ty,
 *      which define the metric g = I + grad tau grad tau^T, G = det g and
 *      the operator L_g (Section 3.1, eqns. 1-3);
 *   3. `iters` Chambolle-Pock iterations for eqn. (5) with the closed-form
 *      proximal maps of Section 3.2 (eqns. cont_iterates, update_rules),
 *      warm-started from the previous block's (u, p); prm->iters if
 *      iters <= 0.
 * Without stats the call only enqueues work.  With stats != NULL it
 * synchronises and fills *stats; REC_ENUMERIC if the last sampled gap or
 * energy is not finite (gap sampling needs prm->gap_every > 0), and any
 * deferred push error is returned.  REC_EDEVICE if a launch fails. */
int rec_solve(rec_ctx* c, int32_t iters, rec_stats* stats);

/* Copy a plane of the state into out (the REC_U.. list gives type and
 * size): the reconstructed image u : Omega -> [u_min, u_max] (Section 3,
 * eqn. 5) and the inputs and intermediates of the last solve.  out is host
 * memory if on_device == 0, device memory otherwise; the call synchronises
 * in both cases and reports deferred push errors.  Recorded device-pointer
 * pushes are scattered first, so count, time and latest-timestamp planes
 * include them.  REC_EINVAL for an unknown plane or NULL out. */
int rec_get_image(rec_ctx* c, int32_t which, void* out, int on_device);

/* The stream's first and latest accepted timestamps (0, 0 and *started = 0
 * before any event).  Synchronises; scatters recorded device pushes first and
 * reports deferred push errors.  Any output may be NULL. */
int rec_get_times(rec_ctx* c, int64_t* t_first, int64_t* t_ref, int32_t* started);

/* Checkpoint / resume (not in the paper, whose state between blocks is the
 * warm start (u, p) of Section 3.2 and the time surface of Section 3.1):
 * replace the context's state with u (float[H*W], each finite and > 0), p
 * (float[3*H*W] in the standard basis, planes p1, p2, p3, as rec_get_image
 * REC_STATE_P returns it; NULL for zero) and the latest timestamps t_last
 * (int64[H*W], as REC_T_LAST returns it) with t_ref the stream's latest
 * timestamp (rec_get_times); t_ref == INT64_MIN imports a stream that has
 * seen no event (t_last ignored, may be NULL).  With the planes exported
 * from another context of the same parameters after a solve, the next
 * pushes and solves give the same bits as that context would.  Planes of
 * the last solve (f, tx, ty, G) are not imported: the next solve rebuilds
 * them; the stream's first timestamp becomes the earliest imported one.
 * Host arrays (on_device == 0) are validated: REC_EINVAL for a bad u
 * or p value, REC_EORDER for a t_last above t_ref; device arrays are not
 * and must not overlap the workspace.  REC_ESTATE while pushes are pending
 * (solve them first).  Synchronises. */
int rec_set_state(rec_ctx* c, const float* u, const float* p, const int64_t* t_last,
                  int64_t t_ref, int on_device);

/* Gap and energy samples of the last rec_solve, in order; returns the number
 * of samples (>= 0) or an error.  At most cap values are written. */
int rec_gap_history(rec_ctx* c, double* gap, double* energy, int32_t cap);

/* Wait for the context's stream and report deferred device errors. */
int rec_sync(rec_ctx* c);

/* Turn per-launch device timing on (1) or off (0); turning it on clears the
 * totals.  Timing adds an event pair around every launch. */
int rec_profile(rec_ctx* c, int enable);

/* Read the timing totals collected since profiling was turned on (synchronises). */
int rec_profile_read(rec_ctx* c, rec_profile_t* out);

/* Release the context (after synchronising its stream).  NULL is a no-op.
 * REC_ESTATE, and nothing is released, while a live batch (rec_batch_init
 * without rec_batch_destroy yet) holds the context. */
int rec_destroy(rec_ctx* c);

/* Static description of a status code. */
const char* rec_strerror(int code);

/* ---------------------------------------------------------------------
 * Batched solves.  Many independent streams (cameras of different sizes
 * and event rates) are solved together.  Every sensor size (or run of
 * sizes by pixel count, when there are more than 8 sizes) gets a tile
 * geometry and iterations per launch K; the sizes sharing a geometry form
 * a class, and a solve runs one chain of ceil(iters / K_c) launches per
 * class, every launch covering the tiles of all streams of the class.
 * Results are the same bits as solving each stream alone (the per-pixel
 * arithmetic does not depend on the tiling or on K).  (Not in the paper,
 * which reconstructs one camera.)
 * ------------------------------------------------------------------- */
typedef struct rec_batch rec_batch;

/* How a batched solve issues the class chains. */
enum {
    REC_BATCH_SERIAL = 0,   /* one after another on the contexts' stream */
    REC_BATCH_STREAMS = 1,  /* concurrently: every class but the first on a stream of
                               the batch's own, forked from the contexts' stream after
                               the solve's descriptor upload and joined back into it
                               (default) */
    REC_BATCH_GRAPH = 2     /* the fork/join of REC_BATCH_STREAMS captured once into a
                               HIP graph per (iterations, descriptor buffer, classes
                               with folded events) and replayed on a stream of the
                               batch's own, ordered after the contexts' stream and
                               before its later work; the descriptor upload stays
                               outside the graph */
};

/* One class of a batch (rec_batch_config). */
typedef struct {
    int32_t width, height;  /* sensor size of the class's first stream */
    int32_t streams;        /* streams in the class */
    int32_t rows, waves;    /* tile geometry: rows per lane, wavefronts per workgroup, */
    int32_t cols;           /*   columns (64 or 32) */
    int32_t kiters;         /* iterations per launch K_c */
    int32_t tiles;          /* workgroups per launch of the class */
    double tuned_us;        /* autotuner's time of the whole tuned schedule for its
                               tune_iters iterations, least of five runs (0 when not
                               tuned) */
} rec_batch_class;

/* Device workspace bytes for a batch of these contexts (0 if invalid). */
size_t rec_batch_workspace_bytes(rec_ctx* const* ctxs, int32_t n);

/* Group n contexts.  They must share device, stream and storage, use the
 * fused loop, and have no timestamp denoising and no gap sampling.  The
 * contexts stay owned by the caller and must outlive the batch.  Without
 * tuning (tune_iters == 0) all sizes share the automatic geometry of a
 * frame of the batch's total pixel count (one class).  With tune_iters > 0
 * an autotuner times the whole schedule of tune_iters iterations (the
 * least of five runs after a warm-up run) for every
 * candidate geometry shared by all sizes, keeps the fastest, then runs a
 * coordinate descent over the sizes (largest first), each trying every
 * candidate (rows, waves, columns, K) with the others fixed; sizes that end
 * with equal geometries share one class.  The timed launches read the
 * streams' current state and write only their spare buffers, so no state
 * changes (synchronises).
 * The batch creates one stream (default priority, non-blocking) per class
 * beyond the first and one for graph replays, released by
 * rec_batch_destroy.  REC_EINVAL for mixed or
 * repeated contexts, REC_ENOMEM for a short workspace or host allocation,
 * REC_EDEVICE for a failed HIP call. */
int rec_batch_init(rec_ctx* const* ctxs, int32_t n, void* dev_workspace, size_t ws_bytes,
                   int32_t tune_iters, rec_batch** out);

/* Solve the pending block of every stream of the batch with `iters`
 * iterations (each stream's pushes since its last solve; a stream without
 * new events smooths its previous image).  Does not synchronise: work the
 * caller enqueues on the contexts' stream afterwards is ordered after every
 * class chain. */
int rec_batch_solve(rec_batch* b, int32_t iters);

/* Number of classes of the batch (>= 1), or REC_EINVAL. */
int rec_batch_classes(const rec_batch* b);

/* The geometry of class cls (0 .. rec_batch_classes - 1). */
int rec_batch_config(const rec_batch* b, int32_t cls, rec_batch_class* out);

/* Set the geometry of the streams of one sensor size (of every size that
 * shares its group when the batch has more than 8 sizes), instead of the
 * automatic or tuned one: rows per lane, wavefronts, columns (64 or 32) as
 * listed for rec_params.tile_rows / tile_cols in the batched launch's set
 * (64 columns: 2x16 4x8 4x16 6x8 8x4 8x8, 32 columns: 1x16 2x8; 16-bit
 * storage without 6x8 and 1x16), and iterations per launch
 * 1 <= kiters <= (min(columns, tile rows) - 1) / 2.  For instance to reuse
 * an earlier tuning without timing again.  The classes are formed again;
 * synchronises.  REC_EINVAL for an unsupported geometry or a size not in
 * the batch, REC_ENOMEM if the tiles exceed the workspace. */
int rec_batch_set_geometry(rec_batch* b, int32_t width, int32_t height, int32_t rows,
                           int32_t waves, int32_t cols, int32_t kiters);

/* Select how solves issue the class chains (REC_BATCH_*); the same bits in
 * every mode.  While profiling is on (rec_profile on the first context of
 * the batch) REC_BATCH_GRAPH solves issue the chains directly. */
int rec_batch_set_mode(rec_batch* b, int32_t mode);

/* Release the batch (after synchronising its streams).  NULL is a no-op. */
int rec_batch_destroy(rec_batch* b);

/* -------------------------------------------------------------------
 * Differentiable unrolled solve (training through the reconstruction).
 *
 * Not in the paper: the K primal-dual iterations of Section 3.2 on one
 * block of data, unrolled as a function of its inputs, with a hand-written
 * reverse sweep.  For a batch of B images of W x H:
 *
 *   f     = u0 * exp(dpos n+ - dneg n-)            (eqn. intensity_update)
 *   ubar  = u_k - tau L_g^* p_k
 *   u_k+1 = clamp(prox_{tau D}(ubar), u_min, u_max)  with the data term
 *           lambda * w * (u - f log u) * sqrt(G) per pixel
 *   p_k+1 = proj_{|.| <= sqrt(G)}(p_k + sigma L_g (2 u_k+1 - u_k))
 *
 * from (u0, p0), with L_g, G from the time differences (tx, ty) (eqn. 3).
 * w = 1 is the paper's model; with w = 1 and p0 = 0 the result has the same
 * bits as rec_solve on the same block (both carry p in each pixel's tangent
 * frame between the first and the last iteration).  rec_diff_forward returns (u_K, p_K) and keeps
 * checkpoints of (u, p) every ckpt_every iterations in the workspace;
 * rec_diff_backward, given dJ/du_K (and optionally dJ/dp_K), recomputes each
 * segment from its checkpoint and runs the adjoint iterations backwards,
 * returning dJ/du0 (through u0 and through f), dJ/dp0, dJ/dw and
 * dJ/d(lambda, dpos, dneg).  The derivative of the clamped prox is zero on
 * clamped pixels; the projection contributes (s/|q|)(I - q q^T/|q|^2)
 * where it is active (q the point projected).  Arithmetic is FP32 as in the
 * forward solve; the scalar gradients are reduced in FP64.
 *
 * Layouts (device memory, row-major, x fastest):
 *   image planes  float / int32 [B][H][W]
 *   dual fields   float [B][3][H][W]   (the 3 components of p per image)
 *   theta         double [3] = (lambda, delta_pos, delta_neg), device memory
 *                 so that it can itself be a trained parameter; lambda > 0
 *                 and finite deltas are the caller's to ensure.
 * ------------------------------------------------------------------- */
typedef struct rec_diff_desc {
    int32_t width, height;  /* 1..65535 */
    int32_t batch;          /* images, 1..65535 */
    int32_t iters;          /* unrolled iterations K >= 0 */
    int32_t ckpt_every;     /* checkpoint interval, 1..max(K, 1); 1 keeps every
                               state (16 bytes per pixel per iteration) and
                               the backward recomputes nothing */
    int32_t unfused;        /* 0: fused register-tile kernels (several
                               iterations per launch); 1: one launch per
                               half-step (reference form, same bits) */
    double tau, sigma;      /* steps: tau sigma (8 + 4 sqrt 2) <= 1 */
    double u_min, u_max;    /* 0 < u_min < u_max */
} rec_diff_desc;

typedef struct rec_diff_inputs {
    const float* u0;        /* initial image and u_prev of f; > 0; required */
    const float* p0;        /* initial dual field, or NULL for zero */
    const int32_t* npos;    /* event counts of the block; required */
    const int32_t* nneg;
    const float* tx;        /* forward differences of the time surface; required */
    const float* ty;
    const float* w;         /* data weights, or NULL for all 1 */
    const double* theta;    /* (lambda, delta_pos, delta_neg); required */
} rec_diff_inputs;

typedef struct rec_diff_grads {
    float* u0;              /* dJ/du0 [B][H][W], or NULL */
    float* p0;              /* dJ/dp0 [B][3][H][W], or NULL */
    float* w;               /* dJ/dw [B][H][W], or NULL */
    double* theta;          /* dJ/d(lambda, delta_pos, delta_neg) [3], or NULL */
} rec_diff_grads;

/* Device workspace bytes (0 if the descriptor is invalid): the data image,
 * ceil(K / ckpt_every) + 1 checkpoints and ckpt_every - 1 recomputed states
 * of 16 bytes per pixel each, and the adjoint planes. */
size_t rec_diff_workspace_bytes(const rec_diff_desc* d);

/* Forward: (u_K, p_K) into u_out [B][H][W] (required) and p_out
 * [B][3][H][W] (or NULL), and checkpoints into the workspace (256-byte
 * aligned, rec_diff_workspace_bytes long, owned by the caller).  Enqueued on
 * `stream` (a hipStream_t, NULL = default); no synchronisation, no
 * allocation.  REC_EINVAL for a bad descriptor or a missing required
 * pointer, REC_ENOMEM for a short workspace, REC_EDEVICE if a launch fails.
 * The outputs must not alias the inputs or the workspace. */
int rec_diff_forward(const rec_diff_desc* d, const rec_diff_inputs* in, float* u_out,
                     float* p_out, void* dev_workspace, size_t ws_bytes, void* stream);

/* Forward without any device allocation or workspace, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  Same descriptor, inputs and outputs as
 * rec_diff_forward and the same bits of (u_K, p_K), but no checkpoints are
 * kept (ckpt_every is validated and otherwise ignored), so no
 * rec_diff_backward can follow it.  The data image and two ping-pong
 * states live in a static device array of 36 MiB that every device the
 * library runs on holds until the process ends; it takes at most
 * width * height * batch <= 1048576 pixels per call (REC_ENOMEM beyond
 * that; split the batch).  The array is shared by all calls on a device
 * and keeps the last call's contents: calls that overlap in time on one
 * device (different streams or threads) race and must be ordered by the
 * caller.  Enqueued on `stream`, no synchronisation.  REC_EINVAL for a bad
 * descriptor or a missing required pointer, REC_EDEVICE if the array's
 * address cannot be found or a launch fails. */
int rec_diff_forward_noalloc(const rec_diff_desc* d, const rec_diff_inputs* in, float* u_out,
                             float* p_out, void* stream);

/* Backward: g_u = dJ/du_K [B][H][W] and g_p = dJ/dp_K [B][3][H][W] (either
 * may be NULL for zero); the gradients requested in `out` are overwritten.
 * Must follow rec_diff_forward with the same descriptor, the same inputs
 * (unchanged in between) and the same workspace, on the same stream or
 * ordered after it.  Same errors as rec_diff_forward. */
int rec_diff_backward(const rec_diff_desc* d, const rec_diff_inputs* in, const float* g_u,
                      const float* g_p, const rec_diff_grads* out, void* dev_workspace,
                      size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* REC_H */
