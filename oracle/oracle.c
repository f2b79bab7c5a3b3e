/*
 * FP64 CPU oracle for intensity reconstruction on the event manifold
 * (Reinbacher, Graber, Pock, BMVC 2016).  TEST INFRASTRUCTURE ONLY: the
 * tests, the smoke check and the CPU-baseline leg of the benchmark call it;
 * the product path never does.  It shares no code with the GPU library.
 *
 * Everything is plain loops over whole images in double precision, one
 * function per step of the method, in the paper's order and notation:
 *
 *   events  e^n = (x^n, y^n, theta^n, t^n)                     Section 3
 *   data image f^n = u^{n-1} * c1 (theta > 0) or * c2 (theta < 0),
 *        c1 = exp(Delta+), c2 = exp(-Delta-)          eqn. intensity_update
 *   time surface t(x, y): time since the last event at each pixel;
 *        metric g = I + grad t grad t^T, G = det g                eqns. 1-2
 *   L_g: R^{HxW} -> R^{HxWx3}, forward differences L_x, L_y     eqn. (3)
 *   energy  ||L_g u||_g + lambda sum (u - f log u) sqrt(G),
 *        u in [u_min, u_max]                                      eqn. (5)
 *   Chambolle-Pock iterations with the closed-form proximal maps
 *        (KL prox with beta = tau lambda sqrt(G); dual projection
 *         onto the ball of radius sqrt(G))   eqns. cont_iterates, update_rules
 *
 * Readings of points the paper leaves open (each is a parameter or a
 * documented default, shared with the GPU library by value only):
 *   - t(x, y) is the int64 microsecond timestamp of the most recent event;
 *     the surface used is tau = (t_ref - t_last) / T_s with t_ref the last
 *     pushed timestamp (the metric only sees squares and products of the
 *     differences, so a surface of last-event times and one of elapsed
 *     times give the same g).
 *     Pixels that never fired count as having fired at the stream's first
 *     timestamp.  T_s = 0 switches the manifold off (t = const).
 *   - L_x, L_y are forward differences with h = 1 and a zero difference on
 *     the last column / row (Chambolle 2004); div is minus their adjoint.
 *     The time differences are formed from the exact int64 differences of
 *     timestamps, divided by T_s.
 *   - Several events at one pixel in one block multiply their factors, in
 *     any order: f = u_prev * exp(Delta+ n+ - Delta- n-).
 *   - KL prox in the algebraically identical form that avoids cancellation:
 *     with a = ubar - beta, d = sqrt(a^2 + 4 beta f):
 *     a >= 0: (a + d) / 2;  a < 0: 2 beta f / (d - a).  Then clamp.
 *   - Warm start: u and p carry over between blocks; p starts at 0.
 *   - Timestamp denoising (Section 4 runs a small number of TV-L1
 *     iterations on the timestamps and gives neither their count nor the
 *     weight): optional, off by default.  When on, tau is replaced by the result of n
 *     Chambolle-Pock iterations for  min_v TV(v) + lambda_t |v - tau|_1
 *     started at v = tau, dual 0, steps 1/sqrt(8), before the differences
 *     are taken.
 *   - Optional slope cap (not in the paper; off by default): the time
 *     differences are clipped to [-cap, cap], the reading used for storage
 *     formats of bounded range (FP16 saturates at 65504).
 *
 * Optional per-pixel data weights w (not in the paper; they make the data
 * term lambda sum w (u - f log u) sqrt(G) and are the weights a learned
 * reconstruction would differentiate; w = 1 is the paper's model).
 *
 * Primal-dual gap (not in the paper; standard Fenchel duality for eqn. (5)),
 * per pixel, with A = L_g u, d = (L_g^* p), s = sqrt(G), b = lambda s:
 *   term1 = s |A| - <A, p>                                  (>= 0 if |p| <= s)
 *   term2 = (u - v)(b + d) - b f log(u / v),
 *           v = clamp(b f / (b + d)) if b + d > 0 else u_max    (>= 0)
 * The gap is the sum of both terms over all pixels.
 *
 * Built twice from this one file: single-threaded, and with OpenMP (the
 * pragmas below split the per-pixel loops of the operators and of the
 * iteration over threads; every pixel's value is computed by the same
 * operations either way, and the gap and energy sums stay serial, so both
 * builds give the same bits).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ERANGE (-2)
#define ORC_EORDER (-3)

#define ORC_NEVER INT64_MIN

typedef struct {
    int32_t width, height;
    double lambda;
    double delta_pos, delta_neg;
    double u_min, u_max;
    double tau, sigma;
    double time_unit_us;   /* T_s; 0 = flat manifold */
    double u_init;
    int32_t tvl1_iters;    /* timestamp denoising iterations; 0 = off */
    double tvl1_lambda;    /* its L1 data weight */
    double slope_cap;      /* > 0: time differences clipped to [-cap, cap]; 0 = none */
} orc_params;

typedef struct {
    orc_params P;
    size_t np;
    double *u, *p1, *p2, *p3;        /* primal image, dual field (3 planes) */
    double *f;                       /* data image of the current block */
    double *w;                       /* per-pixel data weights (NULL: all 1) */
    double *tau_s, *tx, *ty;         /* time surface and its forward differences */
    float *tau32, *tx32, *ty32;      /* the same, rounded once to FP32 */
    int32_t *npos, *nneg;            /* events of the pending block */
    int64_t *t_last;                 /* latest timestamp per pixel, ORC_NEVER if none */
    int64_t t_first, t_ref;
    int started;
    int64_t pending;
} orc_state;

/* ------------------------------------------------------------------ */
/* Operators                                                           */
/* ------------------------------------------------------------------ */

/* A time difference limited to [-cap, cap] (cap = 0: unlimited).  Not in
 * the paper: it models storing the differences in a format whose largest
 * finite value is cap (FP16: 65504), which saturates instead of overflowing. */
static double clip_slope(double d, double cap) {
    if (cap > 0.0) {
        if (d > cap) return cap;
        if (d < -cap) return -cap;
    }
    return d;
}

/* Forward differences with zero on the last column / row (Chambolle 2004). */
void orc_grad(int W, int H, const double* v, double* gx, double* gy) {
#pragma omp parallel for
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t k = (size_t)i * W + j;
            gx[k] = (j < W - 1) ? v[k + 1] - v[k] : 0.0;
            gy[k] = (i < H - 1) ? v[k + W] - v[k] : 0.0;
        }
}

/* div = -grad^T: backward differences with the matching boundary rows. */
void orc_div(int W, int H, const double* qx, const double* qy, double* out) {
#pragma omp parallel for
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t k = (size_t)i * W + j;
            double d = 0.0;
            if (j < W - 1) d += qx[k];
            if (j > 0) d -= qx[k - 1];
            if (i < H - 1) d += qy[k];
            if (i > 0) d -= qy[k - W];
            out[k] = d;
        }
}

/* L_g u, eqn. (3): per pixel, the 3-vector of the manifold gradient in
 * local coordinates, built from (L_x u, L_y u) and (L_x t, L_y t). */
void orc_apply_Lg(int W, int H, const double* tx, const double* ty, const double* u,
                  double* a1, double* a2, double* a3) {
    size_t np = (size_t)W * H;
    double* ux = (double*)malloc(sizeof(double) * np);
    double* uy = (double*)malloc(sizeof(double) * np);
    orc_grad(W, H, u, ux, uy);
#pragma omp parallel for
    for (size_t k = 0; k < np; ++k) {
        double G = 1.0 + tx[k] * tx[k] + ty[k] * ty[k];
        a1[k] = ((1.0 + ty[k] * ty[k]) * ux[k] - tx[k] * ty[k] * uy[k]) / G;
        a2[k] = ((1.0 + tx[k] * tx[k]) * uy[k] - tx[k] * ty[k] * ux[k]) / G;
        a3[k] = (tx[k] * ux[k] + ty[k] * uy[k]) / G;
    }
    free(ux);
    free(uy);
}

/* L_g^* p: the adjoint of L_g = M grad, where M is the per-pixel 3x2 matrix
 * of eqn. (3).  L_g^* p = grad^T (M^T p) = -div(M^T p). */
void orc_apply_LgT(int W, int H, const double* tx, const double* ty, const double* p1,
                   const double* p2, const double* p3, double* out) {
    size_t np = (size_t)W * H;
    double* qx = (double*)calloc(np, sizeof(double));
    double* qy = (double*)calloc(np, sizeof(double));
#pragma omp parallel for
    for (size_t k = 0; k < np; ++k) {
        double G = 1.0 + tx[k] * tx[k] + ty[k] * ty[k];
        /* columns of M: M[:,0] = (1+ty^2, -tx ty, tx)/G, M[:,1] = (-tx ty, 1+tx^2, ty)/G */
        qx[k] = ((1.0 + ty[k] * ty[k]) * p1[k] - tx[k] * ty[k] * p2[k] + tx[k] * p3[k]) / G;
        qy[k] = (-tx[k] * ty[k] * p1[k] + (1.0 + tx[k] * tx[k]) * p2[k] + ty[k] * p3[k]) / G;
    }
    orc_div(W, H, qx, qy, out);
#pragma omp parallel for
    for (size_t k = 0; k < np; ++k) out[k] = -out[k];
    free(qx);
    free(qy);
}

/* prox_{tau D} of the KL data term at one pixel, eqn. update_rules. */
double orc_prox_kl(double ubar, double beta, double f, double umin, double umax) {
    double a = ubar - beta;
    double d = sqrt(a * a + 4.0 * beta * f);
    double u = (a >= 0.0) ? 0.5 * (a + d) : 2.0 * beta * f / (d - a);
    if (u < umin) u = umin;
    if (u > umax) u = umax;
    return u;
}

/* prox_{sigma R^*}: projection of one dual 3-vector onto the ball of radius s. */
void orc_project(double* q1, double* q2, double* q3, double s) {
    double n = sqrt(*q1 * *q1 + *q2 * *q2 + *q3 * *q3);
    double m = n / s;
    if (m < 1.0) m = 1.0;
    *q1 /= m;
    *q2 /= m;
    *q3 /= m;
}

/* TV-L1 denoising of an image f by Chambolle-Pock (2011):
 *   v_{k+1} = prox(v_k + s div q_k),  prox(w) = f + shrink(w - f, s lambda)
 *   q_{k+1} = q / max(1, |q|) with q = q_k + s grad(2 v_{k+1} - v_k)
 * with s = 1/sqrt(8) (||grad||^2 <= 8), v_0 = f, q_0 = 0. */
void orc_tvl1(int W, int H, const double* f, int iters, double lambda, double* v) {
    const size_t n = (size_t)W * H;
    const double s = 1.0 / sqrt(8.0);
    double* qx = (double*)calloc(n, sizeof(double));
    double* qy = (double*)calloc(n, sizeof(double));
    double* d = (double*)malloc(sizeof(double) * n);
    double* vn = (double*)malloc(sizeof(double) * n);
    double* vb = (double*)malloc(sizeof(double) * n);
    double* gx = (double*)malloc(sizeof(double) * n);
    double* gy = (double*)malloc(sizeof(double) * n);
    for (size_t k = 0; k < n; ++k) v[k] = f[k];
    for (int it = 0; it < iters; ++it) {
        orc_div(W, H, qx, qy, d);
        for (size_t k = 0; k < n; ++k) {
            double w = v[k] + s * d[k] - f[k];
            double t = s * lambda;
            double r = w > t ? w - t : (w < -t ? w + t : 0.0);
            vn[k] = f[k] + r;
            vb[k] = 2.0 * vn[k] - v[k];
        }
        orc_grad(W, H, vb, gx, gy);
        for (size_t k = 0; k < n; ++k) {
            double a = qx[k] + s * gx[k], b = qy[k] + s * gy[k];
            double m = sqrt(a * a + b * b);
            if (m < 1.0) m = 1.0;
            qx[k] = a / m;
            qy[k] = b / m;
            v[k] = vn[k];
        }
    }
    free(qx); free(qy); free(d); free(vn); free(vb); free(gx); free(gy);
}

/* ------------------------------------------------------------------ */
/* State                                                               */
/* ------------------------------------------------------------------ */

int orc_check_params(const orc_params* P) {
    if (!P) return ORC_EINVAL;
    if (P->width <= 0 || P->height <= 0 || P->width > 65535 || P->height > 65535) return ORC_EINVAL;
    if (!(P->u_min > 0.0) || !(P->u_max > P->u_min) || !isfinite(P->u_max)) return ORC_EINVAL;
    if (!(P->lambda > 0.0) || !isfinite(P->lambda)) return ORC_EINVAL;
    if (!(P->delta_pos > 0.0) || !(P->delta_neg > 0.0)) return ORC_EINVAL;
    if (!(P->tau > 0.0) || !(P->sigma > 0.0)) return ORC_EINVAL;
    if (!(P->time_unit_us >= 0.0) || !isfinite(P->time_unit_us)) return ORC_EINVAL;
    if (!(P->u_init > 0.0) || !isfinite(P->u_init)) return ORC_EINVAL;
    if (P->tvl1_iters < 0) return ORC_EINVAL;
    if (P->tvl1_iters > 0 && !(P->tvl1_lambda > 0.0)) return ORC_EINVAL;
    if (!(P->slope_cap >= 0.0)) return ORC_EINVAL;
    return ORC_OK;
}

void orc_free(orc_state* S) {
    if (!S) return;
    free(S->u); free(S->p1); free(S->p2); free(S->p3); free(S->f);
    free(S->tau_s); free(S->tx); free(S->ty);
    free(S->tau32); free(S->tx32); free(S->ty32);
    free(S->npos); free(S->nneg); free(S->t_last); free(S->w);
    free(S);
}

orc_state* orc_create(const orc_params* P, const double* u0) {
    if (orc_check_params(P) != ORC_OK) return NULL;
    orc_state* S = (orc_state*)calloc(1, sizeof(orc_state));
    if (!S) return NULL;
    S->P = *P;
    S->np = (size_t)P->width * P->height;
    size_t n = S->np;
    S->u = (double*)malloc(sizeof(double) * n);
    S->p1 = (double*)calloc(n, sizeof(double));
    S->p2 = (double*)calloc(n, sizeof(double));
    S->p3 = (double*)calloc(n, sizeof(double));
    S->f = (double*)malloc(sizeof(double) * n);
    S->tau_s = (double*)calloc(n, sizeof(double));
    S->tx = (double*)calloc(n, sizeof(double));
    S->ty = (double*)calloc(n, sizeof(double));
    S->tau32 = (float*)calloc(n, sizeof(float));
    S->tx32 = (float*)calloc(n, sizeof(float));
    S->ty32 = (float*)calloc(n, sizeof(float));
    S->npos = (int32_t*)calloc(n, sizeof(int32_t));
    S->nneg = (int32_t*)calloc(n, sizeof(int32_t));
    S->t_last = (int64_t*)malloc(sizeof(int64_t) * n);
    if (!S->u || !S->p1 || !S->p2 || !S->p3 || !S->f || !S->tau_s || !S->tx || !S->ty ||
        !S->tau32 || !S->tx32 || !S->ty32 || !S->npos || !S->nneg || !S->t_last) {
        orc_free(S);
        return NULL;
    }
    for (size_t k = 0; k < n; ++k) {
        S->u[k] = u0 ? u0[k] : P->u_init;
        S->f[k] = S->u[k];
        S->t_last[k] = ORC_NEVER;
    }
    S->t_first = 0;
    S->t_ref = 0;
    S->started = 0;
    return S;
}

/* Add events to the pending block.  All-or-nothing: a push with any bad
 * event changes nothing.  Timestamps must not decrease, also across pushes. */
int orc_push(orc_state* S, const int64_t* t, const uint16_t* x, const uint16_t* y,
             const int8_t* pol, int64_t n) {
    if (!S || n < 0) return ORC_EINVAL;
    if (n == 0) return ORC_OK;
    if (!t || !x || !y || !pol) return ORC_EINVAL;
    int64_t prev = S->started ? S->t_ref : INT64_MIN;
    for (int64_t e = 0; e < n; ++e) {
        if (pol[e] != 1 && pol[e] != -1) return ORC_EINVAL;
        if (x[e] >= S->P.width || y[e] >= S->P.height) return ORC_ERANGE;
        if (t[e] < prev) return ORC_EORDER;
        prev = t[e];
    }
    if (!S->started) {
        S->t_first = t[0];
        S->started = 1;
    }
    for (int64_t e = 0; e < n; ++e) {
        size_t k = (size_t)y[e] * S->P.width + x[e];
        if (pol[e] > 0) S->npos[k] += 1; else S->nneg[k] += 1;
        if (t[e] > S->t_last[k]) S->t_last[k] = t[e];
        S->t_ref = t[e];
    }
    S->pending += n;
    return ORC_OK;
}

/* Steps before the iterations: data image f, time surface, its differences.
 * Consumes the pending block. */
void orc_build(orc_state* S) {
    const int W = S->P.width, H = S->P.height;
    const double Ts = S->P.time_unit_us;
    /* data image, eqn. intensity_update applied for every event of the block */
    for (size_t k = 0; k < S->np; ++k) {
        S->f[k] = S->u[k] * exp(S->P.delta_pos * S->npos[k] - S->P.delta_neg * S->nneg[k]);
        S->npos[k] = 0;
        S->nneg[k] = 0;
    }
    S->pending = 0;
    /* time surface (time since the last event) and forward differences */
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t k = (size_t)i * W + j;
            int64_t tl = S->t_last[k] == ORC_NEVER ? S->t_first : S->t_last[k];
            S->tau_s[k] = (Ts > 0.0) ? (double)(S->t_ref - tl) / Ts : 0.0;
            S->tau32[k] = (float)S->tau_s[k];
        }
    if (Ts > 0.0 && S->P.tvl1_iters > 0) {
        /* denoised surface (Section 4), then plain differences of it */
        double* v = (double*)malloc(sizeof(double) * S->np);
        orc_tvl1(W, H, S->tau_s, S->P.tvl1_iters, S->P.tvl1_lambda, v);
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j) {
                size_t k = (size_t)i * W + j;
                S->tx[k] = clip_slope((j < W - 1) ? v[k + 1] - v[k] : 0.0, S->P.slope_cap);
                S->ty[k] = clip_slope((i < H - 1) ? v[k + W] - v[k] : 0.0, S->P.slope_cap);
                S->tx32[k] = (float)S->tx[k];
                S->ty32[k] = (float)S->ty[k];
            }
        free(v);
        return;
    }
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            size_t k = (size_t)i * W + j;
            int64_t tl = S->t_last[k] == ORC_NEVER ? S->t_first : S->t_last[k];
            double dx = 0.0, dy = 0.0;
            if (Ts > 0.0 && j < W - 1) {
                int64_t tr = S->t_last[k + 1] == ORC_NEVER ? S->t_first : S->t_last[k + 1];
                dx = (double)(tl - tr) / Ts;   /* tau(j+1) - tau(j) */
            }
            if (Ts > 0.0 && i < H - 1) {
                int64_t td = S->t_last[k + W] == ORC_NEVER ? S->t_first : S->t_last[k + W];
                dy = (double)(tl - td) / Ts;   /* tau(i+1) - tau(i) */
            }
            S->tx[k] = dx = clip_slope(dx, S->P.slope_cap);
            S->ty[k] = dy = clip_slope(dy, S->P.slope_cap);
            S->tx32[k] = (float)dx;
            S->ty32[k] = (float)dy;
        }
}

/* Gap and energy at the current (u, p); see the header for the formula. */
void orc_gap_energy(const orc_state* S, double* gap, double* energy) {
    const int W = S->P.width, H = S->P.height;
    const size_t n = S->np;
    double* a1 = (double*)malloc(sizeof(double) * n);
    double* a2 = (double*)malloc(sizeof(double) * n);
    double* a3 = (double*)malloc(sizeof(double) * n);
    double* ls = (double*)malloc(sizeof(double) * n);
    orc_apply_Lg(W, H, S->tx, S->ty, S->u, a1, a2, a3);
    orc_apply_LgT(W, H, S->tx, S->ty, S->p1, S->p2, S->p3, ls);
    double g = 0.0, e = 0.0;
    for (size_t k = 0; k < n; ++k) {
        double s = sqrt(1.0 + S->tx[k] * S->tx[k] + S->ty[k] * S->ty[k]);
        double na = sqrt(a1[k] * a1[k] + a2[k] * a2[k] + a3[k] * a3[k]);
        double t1 = s * na - (a1[k] * S->p1[k] + a2[k] * S->p2[k] + a3[k] * S->p3[k]);
        double b = S->P.lambda * (S->w ? S->w[k] : 1.0) * s;
        double d = ls[k];
        double u = S->u[k], f = S->f[k];
        double v;
        if (b + d > 0.0) {
            v = b * f / (b + d);
            if (v < S->P.u_min) v = S->P.u_min;
            if (v > S->P.u_max) v = S->P.u_max;
        } else {
            v = S->P.u_max;
        }
        double t2 = (u - v) * (b + d) - b * f * log(u / v);
        g += t1 + t2;
        e += s * na + b * (u - f * log(u));
    }
    *gap = g;
    *energy = e;
    free(a1); free(a2); free(a3); free(ls);
}

/* `iters` Chambolle-Pock iterations on the current block, eqn. cont_iterates:
 *   u_{k+1} = prox_{tau D}(u_k - tau L_g^* p_k)
 *   p_{k+1} = prox_{sigma R^*}(p_k + sigma L_g (2 u_{k+1} - u_k))
 * If gap_every > 0, after every gap_every-th iteration the gap and energy
 * are written to gaps[m], energies[m] (m = 0, 1, ...). */
void orc_iterate(orc_state* S, int iters, int gap_every, double* gaps, double* energies) {
    const int W = S->P.width, H = S->P.height;
    const size_t n = S->np;
    const double tau = S->P.tau, sigma = S->P.sigma, lam = S->P.lambda;
    double* ls = (double*)malloc(sizeof(double) * n);
    double* unew = (double*)malloc(sizeof(double) * n);
    double* ut = (double*)malloc(sizeof(double) * n);
    double* a1 = (double*)malloc(sizeof(double) * n);
    double* a2 = (double*)malloc(sizeof(double) * n);
    double* a3 = (double*)malloc(sizeof(double) * n);
    int m = 0;
    for (int it = 0; it < iters; ++it) {
        /* primal step */
        orc_apply_LgT(W, H, S->tx, S->ty, S->p1, S->p2, S->p3, ls);
#pragma omp parallel for
        for (size_t k = 0; k < n; ++k) {
            double s = sqrt(1.0 + S->tx[k] * S->tx[k] + S->ty[k] * S->ty[k]);
            double beta = tau * lam * (S->w ? S->w[k] : 1.0) * s;
            double ubar = S->u[k] - tau * ls[k];
            unew[k] = orc_prox_kl(ubar, beta, S->f[k], S->P.u_min, S->P.u_max);
            ut[k] = 2.0 * unew[k] - S->u[k];
        }
        /* dual step on the extrapolated primal */
        orc_apply_Lg(W, H, S->tx, S->ty, ut, a1, a2, a3);
#pragma omp parallel for
        for (size_t k = 0; k < n; ++k) {
            double s = sqrt(1.0 + S->tx[k] * S->tx[k] + S->ty[k] * S->ty[k]);
            double q1 = S->p1[k] + sigma * a1[k];
            double q2 = S->p2[k] + sigma * a2[k];
            double q3 = S->p3[k] + sigma * a3[k];
            orc_project(&q1, &q2, &q3, s);
            S->p1[k] = q1;
            S->p2[k] = q2;
            S->p3[k] = q3;
            S->u[k] = unew[k];
        }
        if (gap_every > 0 && (it + 1) % gap_every == 0) {
            double g, e;
            orc_gap_energy(S, &g, &e);
            if (gaps) gaps[m] = g;
            if (energies) energies[m] = e;
            ++m;
        }
    }
    free(ls); free(unew); free(ut); free(a1); free(a2); free(a3);
}

/* One reconstruction: consume the pending block, then iterate. */
void orc_solve(orc_state* S, int iters, int gap_every, double* gaps, double* energies) {
    orc_build(S);
    orc_iterate(S, iters, gap_every, gaps, energies);
}

/* ------------------------------------------------------------------ */
/* Access for the tests                                                */
/* ------------------------------------------------------------------ */

enum { ORC_U = 0, ORC_F = 1, ORC_TAU = 2, ORC_TX = 3, ORC_TY = 4, ORC_P1 = 5, ORC_P2 = 6,
       ORC_P3 = 7, ORC_TAU32 = 8, ORC_TX32 = 9, ORC_TY32 = 10, ORC_NPOS = 11, ORC_NNEG = 12,
       ORC_TLAST = 13 };

int orc_get(const orc_state* S, int which, void* out) {
    if (!S || !out) return ORC_EINVAL;
    size_t n = S->np;
    switch (which) {
        case ORC_U: memcpy(out, S->u, n * sizeof(double)); break;
        case ORC_F: memcpy(out, S->f, n * sizeof(double)); break;
        case ORC_TAU: memcpy(out, S->tau_s, n * sizeof(double)); break;
        case ORC_TX: memcpy(out, S->tx, n * sizeof(double)); break;
        case ORC_TY: memcpy(out, S->ty, n * sizeof(double)); break;
        case ORC_P1: memcpy(out, S->p1, n * sizeof(double)); break;
        case ORC_P2: memcpy(out, S->p2, n * sizeof(double)); break;
        case ORC_P3: memcpy(out, S->p3, n * sizeof(double)); break;
        case ORC_TAU32: memcpy(out, S->tau32, n * sizeof(float)); break;
        case ORC_TX32: memcpy(out, S->tx32, n * sizeof(float)); break;
        case ORC_TY32: memcpy(out, S->ty32, n * sizeof(float)); break;
        case ORC_NPOS: memcpy(out, S->npos, n * sizeof(int32_t)); break;
        case ORC_NNEG: memcpy(out, S->nneg, n * sizeof(int32_t)); break;
        case ORC_TLAST: {
            int64_t* o = (int64_t*)out;
            for (size_t k = 0; k < n; ++k) o[k] = S->t_last[k] == ORC_NEVER ? S->t_first : S->t_last[k];
            break;
        }
        default: return ORC_EINVAL;
    }
    return ORC_OK;
}

int64_t orc_t_ref(const orc_state* S) { return S ? S->t_ref : 0; }

/* Overwrite the iterate (u, p) — for pins that start from a chosen point. */
int orc_set_state(orc_state* S, const double* u, const double* p1, const double* p2,
                  const double* p3) {
    if (!S) return ORC_EINVAL;
    size_t n = S->np;
    if (u) memcpy(S->u, u, n * sizeof(double));
    if (p1) memcpy(S->p1, p1, n * sizeof(double));
    if (p2) memcpy(S->p2, p2, n * sizeof(double));
    if (p3) memcpy(S->p3, p3, n * sizeof(double));
    return ORC_OK;
}

/* Per-pixel data weights (NULL restores w = 1). */
int orc_set_weights(orc_state* S, const double* w) {
    if (!S) return ORC_EINVAL;
    if (!w) {
        free(S->w);
        S->w = NULL;
        return ORC_OK;
    }
    if (!S->w) S->w = (double*)malloc(sizeof(double) * S->np);
    if (!S->w) return ORC_EINVAL;
    memcpy(S->w, w, S->np * sizeof(double));
    return ORC_OK;
}

/* Overwrite the block data (f and the time differences) — for pins on a
 * chosen manifold (flat, ramp) without going through events. */
int orc_set_data(orc_state* S, const double* f, const double* tx, const double* ty) {
    if (!S) return ORC_EINVAL;
    size_t n = S->np;
    if (f) memcpy(S->f, f, n * sizeof(double));
    if (tx) memcpy(S->tx, tx, n * sizeof(double));
    if (ty) memcpy(S->ty, ty, n * sizeof(double));
    return ORC_OK;
}
