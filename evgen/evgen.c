/*
 * Seeded synthetic event-camera streams (input generator only).
 *
 * This file models the *sensor*, not the reconstruction: a smooth periodic
 * log-intensity texture L(x, y, t) in [0, 1] is moved rigidly across the
 * W x H pixel grid, and every pixel emits an event each time its log
 * intensity crosses the next contrast level (threshold Delta above or below
 * its last reference level), the behaviour the paper assumes of a DVS
 * (Section 3: an event marks a log-intensity change of one threshold).
 * It holds none of the reconstruction method's arithmetic; both the FP64
 * oracle and the GPU path consume its output as plain arrays.
 *
 * Texture: 32 Gaussian blobs with seeded centres, widths and signed
 * amplitudes, summed over the 3x3 periodic images of the W x H cell so the
 * pattern tiles the plane; min-max normalised on the t = 0 pixel grid, then
 * clipped to [0, 1].  Each Gaussian is truncated at 9 sigma (relative weight
 * below 3e-18), which is part of the definition of L.
 *
 * Motion: L(p, t) = T(R(-w t)(p - c) + c - v t) with c the frame centre,
 * i.e. the texture translates with velocity v and rotates at w rad/s.  Because
 * rotations preserve distances, each blob stays a blob whose centre moves, so
 * every frame is a sum of separable Gaussians (row factor x column factor).
 *
 * Emission: pixels are sampled on a uniform time grid of dt microseconds.  A
 * pixel keeps an integer level k; its reference is R0 + Delta k, where the
 * initial reference R0 = L(t = 0) - Delta (2 phi - 1) carries a seeded
 * per-pixel phase phi in [0, 1), so pixels do not all fire in lock-step at
 * the start of the stream (|L(0) - R0| < Delta, as after any event).  Between two samples, every crossing of
 * R0 + Delta (k+1) (resp. k-1) emits a +1 (resp. -1) event at the linearly
 * interpolated time, floored to an integer microsecond and offset by t0.
 * Hence, for noise-free streams, |L - (R0 + Delta (n+ - n-))| < Delta holds
 * at every sample time, and exp(R0) is the exactly known starting image from
 * which integrating the events reproduces the scene up to the threshold.
 *
 * Noise: optionally, a fraction of extra events with uniform pixel, uniform
 * integer time in the stream window and uniform polarity; they do not touch
 * the reference levels.
 *
 * Order: events are sorted by (timestamp, pixel index y*W + x, generation
 * sequence number); the key is unique, so the order is fully determined.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) with the
 * standard increment and mixing constants; doubles are (z >> 11) * 2^-53.
 * Results do not depend on the OpenMP thread count: every pixel is computed
 * independently with a fixed summation order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t width, height;
    uint64_t seed;
    int32_t n_blobs;        /* 32 */
    double sigma_lo;        /* blob width range, fraction of min(W, H) */
    double sigma_hi;
    double threshold;       /* contrast threshold Delta in log intensity */
    double speed_px_s;      /* translation speed; direction drawn from seed */
    double omega_rad_s;     /* rotation rate about the frame centre */
    int64_t t0_us;          /* absolute timestamp of t = 0 */
    int64_t dt_us;          /* sampling step */
    int64_t duration_us;    /* stream length */
    double noise_frac;      /* extra uniform noise events, fraction of signal */
} evg_params;

typedef struct {
    int64_t t;
    int32_t pix;
    int8_t pol;
    uint8_t noise;
    uint16_t pad;
    int64_t seq;
} evg_event;

typedef struct {
    evg_event* ev;
    int64_t n, cap;
    double max_step_dl;     /* largest per-pixel |L(t_k) - L(t_{k-1})| seen */
    int64_t n_signal, n_noise;
} evg_stream;

typedef struct {
    int32_t n;              /* number of blobs */
    double* cx;
    double* cy;
    double* sig;
    double* amp;
    double vx, vy;          /* translation velocity px/s */
    double lo, hi;          /* normalisation (raw min / max at t = 0) */
} texture;

static uint64_t sm64_next(uint64_t* s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double sm64_unit(uint64_t* s) { return (double)(sm64_next(s) >> 11) * 0x1.0p-53; }

/* Raw (un-normalised) texture at relative time t_s seconds into `out` (H*W). */
static void raw_frame(const evg_params* P, const texture* T, double t_s, double* out) {
    const int W = P->width, H = P->height;
    const double ccx = 0.5 * (W - 1), ccy = 0.5 * (H - 1);
    const double th = P->omega_rad_s * t_s;
    const double cs = cos(th), sn = sin(th);
    const int nterm = T->n * 9;
    double* ex = (double*)malloc(sizeof(double) * nterm);
    double* ey = (double*)malloc(sizeof(double) * nterm);
    double* inv2s2 = (double*)malloc(sizeof(double) * nterm);
    double* a = (double*)malloc(sizeof(double) * nterm);
    int* x0 = (int*)malloc(sizeof(int) * nterm);
    int* x1 = (int*)malloc(sizeof(int) * nterm);
    int* y0 = (int*)malloc(sizeof(int) * nterm);
    int* y1 = (int*)malloc(sizeof(int) * nterm);
    for (int k = 0; k < T->n; ++k) {
        double bx = fmod(T->cx[k] + T->vx * t_s, (double)W);
        double by = fmod(T->cy[k] + T->vy * t_s, (double)H);
        if (bx < 0) bx += W;
        if (by < 0) by += H;
        for (int m = -1; m <= 1; ++m)
            for (int n = -1; n <= 1; ++n) {
                int j = k * 9 + (m + 1) * 3 + (n + 1);
                double dx = bx + m * (double)W - ccx, dy = by + n * (double)H - ccy;
                ex[j] = ccx + cs * dx - sn * dy;
                ey[j] = ccy + sn * dx + cs * dy;
                inv2s2[j] = 1.0 / (2.0 * T->sig[k] * T->sig[k]);
                a[j] = T->amp[k];
                double r = 9.0 * T->sig[k];
                double lo = ceil(ex[j] - r), hi = floor(ex[j] + r) + 1;
                x0[j] = lo < 0 ? 0 : (lo > W ? W : (int)lo);
                x1[j] = hi < 0 ? 0 : (hi > W ? W : (int)hi);
                lo = ceil(ey[j] - r); hi = floor(ey[j] + r) + 1;
                y0[j] = lo < 0 ? 0 : (lo > H ? H : (int)lo);
                y1[j] = hi < 0 ? 0 : (hi > H ? H : (int)hi);
            }
    }
    /* column factors per term, computed once per frame */
    double* colf = (double*)malloc(sizeof(double) * (size_t)nterm * W);
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < nterm; ++j)
        for (int x = 0; x < W; ++x) {
            double d = x - ex[j];
            colf[(size_t)j * W + x] = (x >= x0[j] && x < x1[j]) ? exp(-d * d * inv2s2[j]) : 0.0;
        }
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        double* row = out + (size_t)y * W;
        for (int x = 0; x < W; ++x) row[x] = 0.0;
        for (int j = 0; j < nterm; ++j) {
            if (y < y0[j] || y >= y1[j]) continue;
            double d = y - ey[j];
            double w = a[j] * exp(-d * d * inv2s2[j]);
            const double* cf = colf + (size_t)j * W;
            for (int x = x0[j]; x < x1[j]; ++x) row[x] += w * cf[x];
        }
    }
    free(colf); free(ex); free(ey); free(inv2s2); free(a);
    free(x0); free(x1); free(y0); free(y1);
}

static void make_texture(const evg_params* P, texture* T) {
    uint64_t s = P->seed;
    const int W = P->width, H = P->height;
    const double m = W < H ? W : H;
    T->n = P->n_blobs;
    T->cx = (double*)malloc(sizeof(double) * T->n);
    T->cy = (double*)malloc(sizeof(double) * T->n);
    T->sig = (double*)malloc(sizeof(double) * T->n);
    T->amp = (double*)malloc(sizeof(double) * T->n);
    for (int k = 0; k < T->n; ++k) {
        T->cx[k] = sm64_unit(&s) * W;
        T->cy[k] = sm64_unit(&s) * H;
        T->sig[k] = (P->sigma_lo + (P->sigma_hi - P->sigma_lo) * sm64_unit(&s)) * m;
        T->amp[k] = 2.0 * sm64_unit(&s) - 1.0;
    }
    double ang = 2.0 * M_PI * sm64_unit(&s);
    T->vx = P->speed_px_s * cos(ang);
    T->vy = P->speed_px_s * sin(ang);
    T->lo = 0.0; T->hi = 1.0;
    double* f0 = (double*)malloc(sizeof(double) * (size_t)W * H);
    raw_frame(P, T, 0.0, f0);
    double lo = f0[0], hi = f0[0];
    for (size_t i = 1; i < (size_t)W * H; ++i) {
        if (f0[i] < lo) lo = f0[i];
        if (f0[i] > hi) hi = f0[i];
    }
    T->lo = lo;
    T->hi = hi > lo ? hi : lo + 1.0;
    free(f0);
}

static void free_texture(texture* T) { free(T->cx); free(T->cy); free(T->sig); free(T->amp); }

/* Normalised, clipped log-intensity frame at relative time t_us. */
static void norm_frame(const evg_params* P, const texture* T, int64_t t_us, double* out) {
    const size_t np = (size_t)P->width * P->height;
    raw_frame(P, T, (double)t_us * 1e-6, out);
    const double sc = 1.0 / (T->hi - T->lo);
    for (size_t i = 0; i < np; ++i) {
        double v = (out[i] - T->lo) * sc;
        out[i] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
    }
}

/* Initial reference levels R0 from the t = 0 frame L (see header). */
static void ref0(const evg_params* P, const double* L, double* R0) {
    uint64_t s = P->seed ^ 0x8CB92BA72F3D8DD7ull;
    const size_t np = (size_t)P->width * P->height;
    for (size_t i = 0; i < np; ++i) R0[i] = L[i] - P->threshold * (2.0 * sm64_unit(&s) - 1.0);
}

static int push_event(evg_stream* S, int64_t t, int32_t pix, int8_t pol, uint8_t noise) {
    if (S->n == S->cap) {
        int64_t nc = S->cap ? S->cap * 2 : 1 << 16;
        evg_event* ne = (evg_event*)realloc(S->ev, sizeof(evg_event) * nc);
        if (!ne) return -1;
        S->ev = ne; S->cap = nc;
    }
    evg_event* e = &S->ev[S->n];
    e->t = t; e->pix = pix; e->pol = pol; e->noise = noise; e->pad = 0; e->seq = S->n;
    S->n++;
    return 0;
}

static int cmp_event(const void* a, const void* b) {
    const evg_event* x = (const evg_event*)a;
    const evg_event* y = (const evg_event*)b;
    if (x->t != y->t) return x->t < y->t ? -1 : 1;
    if (x->pix != y->pix) return x->pix < y->pix ? -1 : 1;
    if (x->seq != y->seq) return x->seq < y->seq ? -1 : 1;
    return 0;
}

/* Log-intensity frame at relative time t_us (H*W doubles, row-major). */
int evg_frame(const evg_params* P, int64_t t_us, double* out) {
    if (!P || !out || P->width <= 0 || P->height <= 0 || P->n_blobs <= 0) return -1;
    texture T;
    make_texture(P, &T);
    norm_frame(P, &T, t_us, out);
    free_texture(&T);
    return 0;
}

/* Initial reference levels R0 (H*W doubles): log of the known initial image. */
int evg_ref0(const evg_params* P, double* out) {
    if (!P || !out || P->width <= 0 || P->height <= 0 || P->n_blobs <= 0) return -1;
    const size_t np = (size_t)P->width * P->height;
    double* f0 = (double*)malloc(sizeof(double) * np);
    texture T;
    make_texture(P, &T);
    norm_frame(P, &T, 0, f0);
    ref0(P, f0, out);
    free(f0);
    free_texture(&T);
    return 0;
}

/* Generate a stream; returns an opaque handle (NULL on error). */
evg_stream* evg_run(const evg_params* P) {
    if (!P || P->width <= 0 || P->height <= 0 || P->width > 65535 || P->height > 65535 ||
        P->n_blobs <= 0 || P->dt_us <= 0 || P->duration_us < 0 || !(P->threshold > 0))
        return NULL;
    const int W = P->width, H = P->height;
    const size_t np = (size_t)W * H;
    texture T;
    make_texture(P, &T);
    evg_stream* S = (evg_stream*)calloc(1, sizeof(evg_stream));
    double* R0 = (double*)malloc(sizeof(double) * np);
    double* La = (double*)malloc(sizeof(double) * np);
    double* Lb = (double*)malloc(sizeof(double) * np);
    int32_t* level = (int32_t*)calloc(np, sizeof(int32_t));
    norm_frame(P, &T, 0, La);
    ref0(P, La, R0);
    const double D = P->threshold;
    for (int64_t ta = 0; ta < P->duration_us; ta += P->dt_us) {
        int64_t tb = ta + P->dt_us;
        if (tb > P->duration_us) tb = P->duration_us;
        const double span = (double)(tb - ta);
        norm_frame(P, &T, tb, Lb);
        for (size_t i = 0; i < np; ++i) {
            const double a = La[i], b = Lb[i];
            const double dl = fabs(b - a);
            if (dl > S->max_step_dl) S->max_step_dl = dl;
            int32_t k = level[i];
            while (b - (R0[i] + D * (k + 1)) >= 0.0) {
                double v = R0[i] + D * (k + 1);
                double tc = (double)ta + (v - a) / (b - a) * span;
                if (push_event(S, P->t0_us + (int64_t)floor(tc), (int32_t)i, 1, 0)) goto fail;
                ++k;
            }
            while (b - (R0[i] + D * (k - 1)) <= 0.0) {
                double v = R0[i] + D * (k - 1);
                double tc = (double)ta + (v - a) / (b - a) * span;
                if (push_event(S, P->t0_us + (int64_t)floor(tc), (int32_t)i, -1, 0)) goto fail;
                --k;
            }
            level[i] = k;
        }
        double* tmp = La; La = Lb; Lb = tmp;
    }
    S->n_signal = S->n;
    if (P->noise_frac > 0.0) {
        uint64_t s = P->seed ^ 0xD1B54A32D192ED03ull;
        int64_t nn = (int64_t)llround(P->noise_frac * (double)S->n_signal);
        for (int64_t q = 0; q < nn; ++q) {
            int32_t pix = (int32_t)(sm64_next(&s) % (uint64_t)np);
            int64_t t = (int64_t)(sm64_next(&s) % (uint64_t)(P->duration_us + 1));
            int8_t pol = (sm64_next(&s) >> 63) ? 1 : -1;
            if (push_event(S, P->t0_us + t, pix, pol, 1)) goto fail;
        }
    }
    S->n_noise = S->n - S->n_signal;
    qsort(S->ev, (size_t)S->n, sizeof(evg_event), cmp_event);
    free(R0); free(La); free(Lb); free(level);
    free_texture(&T);
    return S;
fail:
    free(R0); free(La); free(Lb); free(level);
    free_texture(&T);
    free(S->ev); free(S);
    return NULL;
}

int64_t evg_count(const evg_stream* S) { return S ? S->n : -1; }
double evg_max_step_dl(const evg_stream* S) { return S ? S->max_step_dl : -1.0; }
int64_t evg_noise_count(const evg_stream* S) { return S ? S->n_noise : -1; }

/* Copy the sorted stream out as SoA arrays (any output may be NULL). */
int evg_copy(const evg_stream* S, int32_t width, int64_t* t, uint16_t* x, uint16_t* y,
             int8_t* pol, uint8_t* is_noise) {
    if (!S || width <= 0) return -1;
    for (int64_t i = 0; i < S->n; ++i) {
        const evg_event* e = &S->ev[i];
        if (t) t[i] = e->t;
        if (x) x[i] = (uint16_t)(e->pix % width);
        if (y) y[i] = (uint16_t)(e->pix / width);
        if (pol) pol[i] = e->pol;
        if (is_noise) is_noise[i] = e->noise;
    }
    return 0;
}

void evg_free(evg_stream* S) {
    if (!S) return;
    free(S->ev);
    free(S);
}
