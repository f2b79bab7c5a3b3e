// Differentiable unrolled primal-dual loop: forward with checkpoints and the
// hand-written reverse sweep (C ABI rec_diff_*).
//
// Forward (per iteration, Section 3.2, eqn. cont_iterates, with per-pixel
// data weights w):
//   ubar = u - tau L_g^* p,   u+ = clamp(prox(ubar; beta, f)),  beta = tau lambda w s
//   p+   = proj_s(pbar),      pbar = p + sigma L_g (2 u+ - u)
// Reverse (adjoints written with a hat; h_u, h_p those of (u+, p+)):
//   q      = J_proj(pbar)^T h_p          J = I inside the ball,
//                                        (s/|pbar|)(I - n n^T) outside
//   ut_hat = sigma L_g^* q
//   H      = h_u + 2 ut_hat              adjoint of u+ including the extrapolation
//   ub_hat = (u+/r) H,  beta_hat = ((f - u+)/r) H,  f_hat = (beta/r) H
//                                        (derivatives of the root u+ of
//                                        u^2 - a u - beta f = 0, a = ubar - beta,
//                                        r = sqrt(a^2 + 4 beta f); all 0 where
//                                        the clamp is active)
//   hat u  = ub_hat - ut_hat,   hat p = q - tau L_g ub_hat
// and after the last reverse step
//   dJ/du0 = hat u_0 + f_hat_sum * exp(dpos n+ - dneg n-)   (f = u0 exp(...))
//   dJ/dw  = tau lambda s beta_hat_sum,  dJ/dlambda = sum tau w s beta_hat_sum
//   dJ/ddpos = sum f_hat_sum f n+,  dJ/ddneg = -sum f_hat_sum f n-.
// The reverse step needs (u_k, p_k, u_k+1): every ckpt_every-th state is a
// checkpoint of the forward; the states between two checkpoints are
// recomputed, bit for bit, by the same forward kernels before the segment's
// reverse steps run.
//
// With iters > 0 every stored state (checkpoints, recorded states) holds p
// in each pixel's tangent frame (p' = U^T p, U = [e1 e2 n] of the time
// surface; see pd_math.h), as the stream solve does between its launches:
// the forward rotates p0 in and p_K out, the reverse rotates dJ/dp_K in and
// dJ/dp0 out, and the adjoint q of p lives in the same coordinates (U is
// orthogonal, so the adjoint of the rotation is its transpose).  The
// forward then produces the same bits as the stream solve of the block.
//
// Two forms, same bits:
//  - fused (default): register tiles as in the forward solve.  The forward
//    runs a segment's iterations per launch; the recomputation of a segment
//    also records every intermediate state; the reverse sweep runs several
//    reverse steps per launch on a tile with the adjoint state in registers
//    (a K-step launch reads a K-pixel halo; each step reads the recorded
//    state it needs).
//  - unfused (reference): one thread per pixel, 64 x 4 pixels per
//    workgroup, blockIdx.z = image, one launch per half-step.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <atomic>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "kernels.h"
#include "pd_math.h"
#include "rec.h"
#include "tile.h"

namespace rec {
namespace {

constexpr int kTileX = 64, kTileY = 4, kThreads = kTileX * kTileY;

struct Dims {
    int32_t W, H;
    size_t np;  // W * H
};

// One (u, p) state of the whole batch: u [B][np], p [B][3][np].
struct State {
    float* u;
    float* p;
};

struct Steps {
    double tau_d;  // tau in FP64 (for tau * lambda, as the forward solve forms it)
    float ts;      // tau / sigma (the primal step on the sigma-scaled coefficients)
    float sigma, umin, umax;
    int rot;       // iters > 0: states carry p in the tangent frame
};

// Coefficients of a pixel for the iteration on frame coordinates.
__device__ __forceinline__ CoefT coef(float tx, float ty, float f, float taulam, float sigma,
                                      bool has_x, bool has_y) {
    return make_coef_t(make_basis(tx, ty), f, taulam, sigma, has_x, has_y);
}

__device__ __forceinline__ bool pixel(const Dims& d, int& i, int& j, size_t& o, size_t& b) {
    j = blockIdx.x * kTileX + (threadIdx.x & (kTileX - 1));
    i = blockIdx.y * kTileY + (threadIdx.x >> 6);
    b = blockIdx.z;
    o = b * d.np + (size_t)i * d.W + j;
    return j < d.W && i < d.H;
}

// tau * lambda * w of one pixel (FP32, the product the forward solve uses
// when w = 1).
__device__ __forceinline__ float taulam_w(const double* theta, double tau, const float* w,
                                          size_t o) {
    const float tl = (float)(tau * theta[0]);
    return w ? tl * w[o] : tl;
}

// q_x of the left neighbour / q_y of the upper neighbour of field v
// (3 planes of stride np starting at v; coefficients sigma M), 0 outside the
// image.
__device__ __forceinline__ float qx_left(const Dims& d, int i, int j, size_t o, const float* tx,
                                         const float* ty, const float* v1, size_t np,
                                         float sigma) {
    if (j == 0) return 0.0f;
    const size_t l = o - 1;
    const CoefT c = coef(tx[l], ty[l], 0.0f, 0.0f, sigma, true, i < d.H - 1);
    return q_x(c, v1[l], v1[np + l], v1[2 * np + l]);
}
__device__ __forceinline__ float qy_up(const Dims& d, int i, int j, size_t o, const float* tx,
                                       const float* ty, const float* v1, size_t np, float sigma) {
    if (i == 0) return 0.0f;
    const size_t l = o - d.W;
    const CoefT c = coef(tx[l], ty[l], 0.0f, 0.0f, sigma, j < d.W - 1, true);
    return q_y(c, v1[l], v1[np + l], v1[2 * np + l]);
}

// Offset of pixel o of image b in a 3-plane field [B][3][np]: component m
// is at base + m * np.
__device__ __forceinline__ size_t field(const Dims& d, size_t b, size_t o) {
    return o + 2 * b * d.np;  // b * 3 np + (o - b np)
}

// ------------------------------------------------------------------ forward

// f = u0 exp(dpos n+ - dneg n-); state 0 = (u0, p0 or 0), p0 rotated into
// the frame when rot.
__global__ __launch_bounds__(kThreads) void k_diff_init(Dims d, const float* __restrict__ u0,
                                                        const float* __restrict__ p0,
                                                        const int32_t* __restrict__ npos,
                                                        const int32_t* __restrict__ nneg,
                                                        const double* __restrict__ theta,
                                                        const float* __restrict__ tx,
                                                        const float* __restrict__ ty, int rot,
                                                        float* __restrict__ f, State s0) {
    int i, j;
    size_t o, b;
    if (!pixel(d, i, j, o, b)) return;
    const float u = u0[o];
    f[o] = data_image(u, npos[o], nneg[o], theta[1], theta[2]);
    s0.u[o] = u;
    const size_t q = field(d, b, o);
    float p1 = 0.0f, p2 = 0.0f, p3 = 0.0f;
    if (p0) {
        p1 = p0[q];
        p2 = p0[q + d.np];
        p3 = p0[q + 2 * d.np];
        if (rot) to_frame(make_basis(tx[o], ty[o]), p1, p2, p3);
    }
    s0.p[q] = p1;
    s0.p[q + d.np] = p2;
    s0.p[q + 2 * d.np] = p3;
}

// Primal half-step from state a into b.u.
__global__ __launch_bounds__(kThreads) void k_diff_primal(Dims d, State a, State b_,
                                                          const float* __restrict__ f,
                                                          const float* __restrict__ tx,
                                                          const float* __restrict__ ty,
                                                          const float* __restrict__ w,
                                                          const double* __restrict__ theta,
                                                          Steps st) {
    int i, j;
    size_t o, b;
    if (!pixel(d, i, j, o, b)) return;
    const size_t q = field(d, b, o);
    const float* p = a.p + (q - o);  // image b's field, indexed by o
    const CoefT c = coef(tx[o], ty[o], f[o], taulam_w(theta, st.tau_d, w, o), st.sigma,
                         j < d.W - 1, i < d.H - 1);
    const float qx = q_x(c, p[o], p[d.np + o], p[2 * d.np + o]);
    const float qy = q_y(c, p[o], p[d.np + o], p[2 * d.np + o]);
    const float qxl = qx_left(d, i, j, o, tx, ty, p, d.np, st.sigma);
    const float qyu = qy_up(d, i, j, o, tx, ty, p, d.np, st.sigma);
    b_.u[o] = primal(a.u[o], qx, qy, qxl, qyu, c, st.ts, st.umin, st.umax);
}

// Dual half-step: p of state a, primal a.u -> b.u, into b.p.
__global__ __launch_bounds__(kThreads) void k_diff_dual(Dims d, State a, State b_,
                                                        const float* __restrict__ tx,
                                                        const float* __restrict__ ty, Steps st) {
    int i, j;
    size_t o, b;
    if (!pixel(d, i, j, o, b)) return;
    const float ut = extrapolate(b_.u[o], a.u[o]);
    float gx = 0.0f, gy = 0.0f;
    if (j < d.W - 1) gx = extrapolate(b_.u[o + 1], a.u[o + 1]) - ut;
    if (i < d.H - 1) gy = extrapolate(b_.u[o + d.W], a.u[o + d.W]) - ut;
    const CoefT c = coef(tx[o], ty[o], 0.0f, 0.0f, st.sigma, j < d.W - 1, i < d.H - 1);
    const size_t q = field(d, b, o);
    float p1 = a.p[q], p2 = a.p[q + d.np], p3 = a.p[q + 2 * d.np];
    dual(p1, p2, p3, gx, gy, c);
    b_.p[q] = p1;
    b_.p[q + d.np] = p2;
    b_.p[q + 2 * d.np] = p3;
}

// (u_K, p_K), p rotated back to the standard basis when rot.
__global__ __launch_bounds__(kThreads) void k_diff_out(Dims d, State s,
                                                       const float* __restrict__ tx,
                                                       const float* __restrict__ ty, int rot,
                                                       float* __restrict__ u,
                                                       float* __restrict__ p) {
    int i, j;
    size_t o, b;
    if (!pixel(d, i, j, o, b)) return;
    u[o] = s.u[o];
    if (p) {
        const size_t q = field(d, b, o);
        float p1 = s.p[q], p2 = s.p[q + d.np], p3 = s.p[q + 2 * d.np];
        if (rot) from_frame(make_basis(tx[o], ty[o]), p1, p2, p3);
        p[q] = p1;
        p[q + d.np] = p2;
        p[q + 2 * d.np] = p3;
    }
}

// ------------------------------------------------------------------ reverse

// Adjoint planes of the reverse sweep.
struct Adj {
    float* q;      // [B][3][np] J_proj^T h_p of the latest reverse step
    float* ub;     // [B][np] ub_hat of the latest reverse step
    float* uh;     // [B][np] hat u of the latest reverse step
    float* gbeta;  // [B][np] sum of beta_hat over the steps
    float* gf;     // [B][np] sum of f_hat over the steps
};

// hat p of the state after the latest reverse step, at one pixel, in frame
// coordinates when st.rot: q - tau L_g ub_hat = q - ts sigma M grad ub_hat,
// ts = tau / sigma (first = no step yet: g_p rotated into the frame, or 0).
__device__ __forceinline__ void adj_p(const Dims& d, int i, int j, size_t o, size_t q,
                                      const CoefT& c, const float* tx, const float* ty,
                                      const Adj& A, const float* g_p, bool first,
                                      const Steps& st, float& h1, float& h2, float& h3) {
    if (first) {
        h1 = g_p ? g_p[q] : 0.0f;
        h2 = g_p ? g_p[q + d.np] : 0.0f;
        h3 = g_p ? g_p[q + 2 * d.np] : 0.0f;
        if (g_p && st.rot) to_frame(make_basis(tx[o], ty[o]), h1, h2, h3);
        return;
    }
    const float ubc = A.ub[o];
    const float gx = j < d.W - 1 ? A.ub[o + 1] - ubc : 0.0f;
    const float gy = i < d.H - 1 ? A.ub[o + d.W] - ubc : 0.0f;
    float v1, v2;
    ascent_dir(c, gx, gy, v1, v2);
    h1 = __builtin_fmaf(-st.ts, v1, A.q[q]);
    h2 = __builtin_fmaf(-st.ts, v2, A.q[q + d.np]);
    h3 = A.q[q + 2 * d.np];
}

// Reverse of the dual half-step of the iteration a -> b: q = J_proj^T h_p.
__global__ __launch_bounds__(kThreads) void k_adj_dual(Dims d, State a, State b_,
                                                       const float* __restrict__ tx,
                                                       const float* __restrict__ ty, Adj A,
                                                       const float* __restrict__ g_p, int first,
                                                       Steps st) {
    int i, j;
    size_t o, b;
    if (!pixel(d, i, j, o, b)) return;
    const size_t q = field(d, b, o);
    const CoefT c = coef(tx[o], ty[o], 0.0f, 0.0f, st.sigma, j < d.W - 1, i < d.H - 1);
    float h1, h2, h3;
    adj_p(d, i, j, o, q, c, tx, ty, A, g_p, first != 0, st, h1, h2, h3);
    // pbar of the forward step, recomputed
    const float ut = extrapolate(b_.u[o], a.u[o]);
    const float gx = j < d.W - 1 ? extrapolate(b_.u[o + 1], a.u[o + 1]) - ut : 0.0f;
    const float gy = i < d.H - 1 ? extrapolate(b_.u[o + d.W], a.u[o + d.W]) - ut : 0.0f;
    float b1, b2, b3;
    dual_ascent(c, gx, gy, a.p[q], a.p[q + d.np], a.p[q + 2 * d.np], b1, b2, b3);
    const float n2 = norm2(b1, b2, b3);
    const float sc = c.s * rsq(n2);
    if (sc < 1.0f) {  // the forward projected this point (same test as its min)
        const float t = __builtin_fmaf(b3, h3, __builtin_fmaf(b2, h2, b1 * h1)) * rcp(n2);
        h1 = sc * __builtin_fmaf(-t, b1, h1);
        h2 = sc * __builtin_fmaf(-t, b2, h2);
        h3 = sc * __builtin_fmaf(-t, b3, h3);
    }
    A.q[q] = h1;
    A.q[q + d.np] = h2;
    A.q[q + 2 * d.np] = h3;
}

// Reverse of the primal half-step and the extrapolation of the iteration
// starting at state a.
__global__ __launch_bounds__(kThreads) void k_adj_primal(Dims d, State a,
                                                         const float* __restrict__ f,
                                                         const float* __restrict__ tx,
                                                         const float* __restrict__ ty,
                                                         const float* __restrict__ w,
                                                         const double* __restrict__ theta, Adj A,
                                                         const float* __restrict__ g_u,
                                                         int first, Steps st) {
    int i, j;
    size_t o, b;
    if (!pixel(d, i, j, o, b)) return;
    const size_t q = field(d, b, o);
    const float* qf = A.q + (q - o);
    const float* p = a.p + (q - o);
    const float fo = f[o];
    const CoefT c = coef(tx[o], ty[o], fo, taulam_w(theta, st.tau_d, w, o), st.sigma,
                         j < d.W - 1, i < d.H - 1);
    // ut_hat = sigma L_g^* q = -div(sigma M^T q)
    const float qx = q_x(c, qf[o], qf[d.np + o], qf[2 * d.np + o]);
    const float qy = q_y(c, qf[o], qf[d.np + o], qf[2 * d.np + o]);
    const float divq = (qx - qx_left(d, i, j, o, tx, ty, qf, d.np, st.sigma)) +
                       (qy - qy_up(d, i, j, o, tx, ty, qf, d.np, st.sigma));
    const float ut_hat = -divq;
    const float hu = first ? (g_u ? g_u[o] : 0.0f) : A.uh[o];
    const float H = __builtin_fmaf(2.0f, ut_hat, hu);
    // the forward's root, recomputed
    const float px = q_x(c, p[o], p[d.np + o], p[2 * d.np + o]);
    const float py = q_y(c, p[o], p[d.np + o], p[2 * d.np + o]);
    float r;
    const float un = prox_root(a.u[o], px, py, qx_left(d, i, j, o, tx, ty, p, d.np, st.sigma),
                               qy_up(d, i, j, o, tx, ty, p, d.np, st.sigma), c.hb, c.bf, st.ts,
                               r);
    const bool active = un >= st.umin && un <= st.umax;
    const float hr = active ? H * rcp(r) : 0.0f;
    const float ub_hat = un * hr;
    A.ub[o] = ub_hat;
    A.uh[o] = ub_hat - ut_hat;
    A.gbeta[o] += (fo - un) * hr;
    A.gf[o] += prox_beta(c) * hr;
}

__global__ __launch_bounds__(kThreads) void k_adj_zero(Dims d, Adj A) {
    int i, j;
    size_t o, b;
    if (!pixel(d, i, j, o, b)) return;
    A.gbeta[o] = 0.0f;
    A.gf[o] = 0.0f;
}

// Gradients of the inputs; per-workgroup FP64 partial sums of the scalar
// gradients (lambda, dpos, dneg) into part[3 * block].
__global__ __launch_bounds__(kThreads) void k_adj_final(
    Dims d, const float* __restrict__ f, const float* __restrict__ tx,
    const float* __restrict__ ty, const float* __restrict__ w, const int32_t* __restrict__ npos,
    const int32_t* __restrict__ nneg, const double* __restrict__ theta, Adj A,
    const float* __restrict__ g_u, const float* __restrict__ g_p, int first, Steps st,
    float* __restrict__ gu0, float* __restrict__ gp0, float* __restrict__ gw,
    double* __restrict__ part) {
    __shared__ double red[3][kThreads];
    int i, j;
    size_t o, b;
    double s_lam = 0.0, s_dp = 0.0, s_dn = 0.0;
    if (pixel(d, i, j, o, b)) {
        const size_t q = field(d, b, o);
        const CoefT c = coef(tx[o], ty[o], 0.0f, 0.0f, st.sigma, j < d.W - 1, i < d.H - 1);
        if (gp0) {
            float h1, h2, h3;
            adj_p(d, i, j, o, q, c, tx, ty, A, g_p, first != 0, st, h1, h2, h3);
            if (st.rot) from_frame(make_basis(tx[o], ty[o]), h1, h2, h3);
            gp0[q] = h1;
            gp0[q + d.np] = h2;
            gp0[q + 2 * d.np] = h3;
        }
        const double gb = first ? 0.0 : (double)A.gbeta[o];
        const double gfo = first ? 0.0 : (double)A.gf[o];
        const int32_t np_ = npos[o], nn_ = nneg[o];
        if (gu0) {
            const double e = exp(theta[1] * (double)np_ - theta[2] * (double)nn_);
            const double hu = first ? (g_u ? (double)g_u[o] : 0.0) : (double)A.uh[o];
            gu0[o] = (float)(hu + gfo * e);
        }
        const double tws = st.tau_d * (double)c.s;  // d beta / d(lambda w)
        const double wo = w ? (double)w[o] : 1.0;
        if (gw) gw[o] = (float)(tws * theta[0] * gb);
        s_lam = tws * wo * gb;
        const double ff = gfo * (double)f[o];
        s_dp = ff * (double)np_;
        s_dn = -ff * (double)nn_;
    }
    const int t = threadIdx.x;
    red[0][t] = s_lam;
    red[1][t] = s_dp;
    red[2][t] = s_dn;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int m = 0; m < 3; ++m) red[m][t] += red[m][t + h];
        __syncthreads();
    }
    if (t < 3) {
        const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        part[3 * blk + t] = red[t][0];
    }
}

// Sum of the partials in a fixed order (one workgroup).
__global__ __launch_bounds__(kThreads) void k_adj_reduce(const double* __restrict__ part,
                                                         size_t nblk, double* __restrict__ out) {
    __shared__ double red[3][kThreads];
    const int t = threadIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    for (size_t k = t; k < nblk; k += kThreads)
        for (int m = 0; m < 3; ++m) s[m] += part[3 * k + m];
    for (int m = 0; m < 3; ++m) red[m][t] = s[m];
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int m = 0; m < 3; ++m) red[m][t] += red[m][t + h];
        __syncthreads();
    }
    if (t < 3) out[t] = red[t][0];
}

// ------------------------------------------------------------------ fused

// Tiles of a fused launch: each image is cut into tiles_x x tiles_y regions
// of 64 x RH pixels whose interiors (the region minus a KG-pixel border)
// partition the image.
struct TileGrid {
    int tiles_x, per_image, total;
    int kg;  // halo = iterations (or reverse steps) of the launch
    Divider tiles_x_div, per_image_div;  // the same as dividers
};

// Intermediate states recorded by a forward launch: the state after
// iteration it (it < K - 1) goes to (u + it * stride, p + it * stride).
struct Trail {
    float* u;
    float* p;
    size_t stride;
};

// Where a tile sits; interior(): the pixel is written by this tile.
// Planes are addressed from per-tile bases with 32-bit offsets: the tile's
// rows lie within RH image rows of its first row clamped into the image
// (yb), so an offset from plane + tb (image planes) or plane + tbf + c np
// (component c of a field) fits 32 bits for every size.
struct TilePos {
    int lane, wave, gx, gy0, b, yb;
    size_t img, fld;  // offsets of image b in an image plane / a 3-plane field
    size_t tb, tbf;   // the tile's bases: img + yb W, fld + yb W
    uint32_t gxc;     // gx clamped into the image
    bool col_in, col_out;
};

template <int R, int NW>
__device__ __forceinline__ TilePos tile_pos(const Dims& d, const TileGrid& g) {
    constexpr int RH = NW * R;
    TilePos t;
    t.lane = threadIdx.x & 63;
    t.wave = threadIdx.x >> 6;
    const int tile = xcd_tile(blockIdx.x, g.total);
    t.b = divide(tile, g.per_image_div);
    const int tt = tile - t.b * g.per_image;
    const int tyi = divide(tt, g.tiles_x_div), txi = tt - tyi * g.tiles_x;
    const int OW = 64 - 2 * g.kg, OH = RH - 2 * g.kg;
    t.gx = txi * OW - g.kg + t.lane;
    t.gy0 = tyi * OH - g.kg + t.wave * R;
    t.img = (size_t)t.b * d.np;
    t.fld = 3 * t.img;
    t.yb = min(max(tyi * OH - g.kg, 0), d.H - 1);
    t.tb = t.img + (size_t)t.yb * d.W;
    t.tbf = t.fld + (size_t)t.yb * d.W;
    t.gxc = (uint32_t)min(max(t.gx, 0), d.W - 1);
    t.col_in = t.gx >= 0 && t.gx < d.W;
    t.col_out = t.col_in && t.lane >= g.kg && t.lane < 64 - g.kg;
    return t;
}

// Offset of row r of the lane from the tile's bases, the coordinates
// clamped into the image: outside the image a lane reads an edge pixel's
// (finite) values, which reach no pixel inside, because the coefficients of
// a pixel outside the image are zero.
__device__ __forceinline__ uint32_t eoff(const Dims& d, const TilePos& t, int r) {
    const int gyc = min(max(t.gy0 + r, 0), d.H - 1);
    return __umul24((uint32_t)(gyc - t.yb), (uint32_t)d.W) + t.gxc;
}

template <int R, int NW>
__device__ __forceinline__ bool interior(const Dims& d, const TileGrid& g, const TilePos& t,
                                         int r) {
    constexpr int RH = NW * R;
    const int row = t.wave * R + r, gy = t.gy0 + r;
    return t.col_out && row >= g.kg && row < RH - g.kg && gy >= 0 && gy < d.H;
}

template <int R, int NW>
__device__ __forceinline__ void store_state(const Dims& d, const TileGrid& g, const TilePos& t,
                                            float* U, float* P, const float (&u)[R],
                                            const float (&p1)[R], const float (&p2)[R],
                                            const float (&p3)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!interior<R, NW>(d, g, t, r)) continue;
        const uint32_t e = __umul24((uint32_t)(t.gy0 + r - t.yb), (uint32_t)d.W) + (uint32_t)t.gx;
        *at(U + t.tb, e) = u[r];
        *at(P + t.tbf, e) = p1[r];
        *at(P + t.tbf + d.np, e) = p2[r];
        *at(P + t.tbf + 2 * d.np, e) = p3[r];
    }
}

// Metric constants of a tile's rows (pixels outside the image: zero
// coefficients, as in the forward solve's tiles).
template <int R>
__device__ __forceinline__ void tile_coefs(const Dims& d, const TilePos& t, const float* f,
                                           const float* tx, const float* ty, const float* w,
                                           float tl, float sigma, CoefT (&c)[R], float (&fr)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int gy = t.gy0 + r;
        const bool in = t.col_in && gy >= 0 && gy < d.H;
        const uint32_t e = eoff(d, t, r);
        const float ff = *at(f + t.tb, e);
        const float tlw = w ? tl * *at(w + t.tb, e) : tl;
        fr[r] = ff;
        c[r] = coef(*at(tx + t.tb, e), *at(ty + t.tb, e), ff, tlw, sigma,
                    in && t.gx < d.W - 1, in && gy < d.H - 1);
    }
}

// Forward: K iterations from state `in` to state `out`; with rec.u set,
// also the K - 1 intermediate states.
template <int R, int NW>
__global__ __launch_bounds__(64 * NW) void k_dfwd_fused(Dims d, TileGrid g, State in, State out,
                                                        Trail rec, const float* __restrict__ f,
                                                        const float* __restrict__ tx,
                                                        const float* __restrict__ ty,
                                                        const float* __restrict__ w,
                                                        const double* __restrict__ theta,
                                                        Steps st) {
    const TilePos t = tile_pos<R, NW>(d, g);
    const int K = g.kg;
    float u[R], p1[R], p2[R], p3[R], fr[R];
    CoefT c[R];
    tile_coefs<R>(d, t, f, tx, ty, w, (float)(st.tau_d * theta[0]), st.sigma, c,
                 fr);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t e = eoff(d, t, r);
        u[r] = *at(in.u + t.tb, e);
        p1[r] = *at(in.p + t.tbf, e);
        p2[r] = *at(in.p + t.tbf + d.np, e);
        p3[r] = *at(in.p + t.tbf + 2 * d.np, e);
    }
    __shared__ float xq[NW + 1][64];
    __shared__ float xu[NW + 1][64];
    if (t.wave == 0) xq[0][t.lane] = 0.0f;
    if (t.wave == NW - 1) xu[NW][t.lane] = 0.0f;
    for (int it = 0; it < K; ++it) {
        tile_iteration<R, NW>(u, u, p1, p2, p3, c, st.ts, st.umin, st.umax, t.lane, t.wave, xq,
                              xu);
        if (rec.u && it < K - 1)
            store_state<R, NW>(d, g, t, rec.u + it * rec.stride, rec.p + it * rec.stride, u, p1,
                               p2, p3);
    }
    store_state<R, NW>(d, g, t, out.u, out.p, u, p1, p2, p3);
}

// States j0 .. j0 + K of a reverse launch (local index 0 .. K).
constexpr int kMaxRev = 8;
struct StateSeq {
    float* u[kMaxRev + 1];
    float* p[kMaxRev + 1];
};

// Adjoint planes read or written by a reverse launch (ping-pong between
// launches: tiles read their halo from `in` while others write `out`).
struct AdjIO {
    float* q;   // [B][3][np]
    float* ub;  // [B][np]
    float* uh;  // [B][np]
};

// Reverse steps j0 + K - 1 down to j0 on a register tile: the adjoint state
// (q, ub_hat, hat u) comes from `ain` (or from g_p, 0, g_u when `first`)
// and goes to `aout`; the sums of beta_hat and f_hat are accumulated into
// gbeta, gf (interior pixels, in place).  (Unrolling the steps completely,
// with K a template parameter, needs 176 registers per lane instead of 127
// and measured 25 % slower.)
template <int R, int NW>
__global__ __launch_bounds__(64 * NW) void k_adj_fused(
    Dims d, TileGrid g, StateSeq S, AdjIO ain, AdjIO aout, float* __restrict__ gbeta,
    float* __restrict__ gf, const float* __restrict__ g_u, const float* __restrict__ g_p,
    int first, const float* __restrict__ f, const float* __restrict__ tx,
    const float* __restrict__ ty, const float* __restrict__ w, const double* __restrict__ theta,
    Steps st) {
    const TilePos t = tile_pos<R, NW>(d, g);
    const int K = g.kg;
    const int lane = t.lane, wave = t.wave;
    float fr[R];
    CoefT c[R];
    tile_coefs<R>(d, t, f, tx, ty, w, (float)(st.tau_d * theta[0]), st.sigma, c,
                 fr);
    float u1[R], Q1[R], Q2[R], Q3[R], UB[R], UH[R], GB[R], GF[R];
    uint32_t ee[R];  // offsets of the lane's rows from the tile's bases (clamped)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int gy = t.gy0 + r;
        const bool inside = t.col_in && gy >= 0 && gy < d.H;
        const uint32_t e = ee[r] = eoff(d, t, r);
        u1[r] = *at(S.u[K] + t.tb, e);
        Q1[r] = Q2[r] = Q3[r] = UB[r] = UH[r] = 0.0f;
        if (first) {
            // the adjoints of the last state: zero outside the image
            if (inside) {
                if (g_p) {
                    Q1[r] = *at(g_p + t.tbf, e);
                    Q2[r] = *at(g_p + t.tbf + d.np, e);
                    Q3[r] = *at(g_p + t.tbf + 2 * d.np, e);
                    if (st.rot)
                        to_frame(make_basis(*at(tx + t.tb, e), *at(ty + t.tb, e)), Q1[r], Q2[r],
                                 Q3[r]);
                }
                if (g_u) UH[r] = *at(g_u + t.tb, e);
            }
        } else {
            Q1[r] = *at(ain.q + t.tbf, e);
            Q2[r] = *at(ain.q + t.tbf + d.np, e);
            Q3[r] = *at(ain.q + t.tbf + 2 * d.np, e);
            UB[r] = *at(ain.ub + t.tb, e);
            UH[r] = *at(ain.uh + t.tb, e);
        }
        const bool own = interior<R, NW>(d, g, t, r);
        GB[r] = own ? *at(gbeta + t.tb, e) : 0.0f;
        GF[r] = own ? *at(gf + t.tb, e) : 0.0f;
    }
    __shared__ float xa[NW][64], xb[NW][64], xc[NW][64], xd[NW][64];
    // the state of the next step is loaded one step ahead
    float nu[R], na[R], nb[R], nc[R];
    auto load_state = [&](int j) {
        const float* su = S.u[j] + t.tb;
        const float* sp = S.p[j] + t.tbf;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            nu[r] = *at(su, ee[r]);
            na[r] = *at(sp, ee[r]);
            nb[r] = *at(sp + d.np, ee[r]);
            nc[r] = *at(sp + 2 * d.np, ee[r]);
        }
    };
    load_state(K - 1);
    for (int s = 0; s < K; ++s) {
        float u0[R], pa[R], pb[R], pc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            u0[r] = nu[r];
            pa[r] = na[r];
            pb[r] = nb[r];
            pc[r] = nc[r];
        }
        if (s + 1 < K) load_state(K - 2 - s);
        // reverse of the dual half-step: needs ub_hat and the extrapolated
        // primal at the right and lower neighbours
        float ut[R];
#pragma unroll
        for (int r = 0; r < R; ++r) ut[r] = extrapolate(u1[r], u0[r]);
        float ub_bot = 0.0f, ut_bot = 0.0f;
        if constexpr (NW > 1) {
            xa[wave][lane] = UB[0];
            xb[wave][lane] = ut[0];
            __syncthreads();
            if (wave < NW - 1) {
                ub_bot = xa[wave + 1][lane];
                ut_bot = xb[wave + 1][lane];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const CoefT& cc = c[r];
            const float ubr = lane_from_right(UB[r]);
            const float ubd = r < R - 1 ? UB[r + 1] : ub_bot;
            const float gx = ubr - UB[r], gy = ubd - UB[r];
            float v1, v2;
            ascent_dir(cc, gx, gy, v1, v2);
            float h1 = __builtin_fmaf(-st.ts, v1, Q1[r]);
            float h2 = __builtin_fmaf(-st.ts, v2, Q2[r]);
            float h3 = Q3[r];
            const float utr = lane_from_right(ut[r]);
            const float utd = r < R - 1 ? ut[r + 1] : ut_bot;
            float b1, b2, b3;
            dual_ascent(cc, utr - ut[r], utd - ut[r], pa[r], pb[r], pc[r], b1, b2, b3);
            const float n2 = norm2(b1, b2, b3);
            const float sc = cc.s * rsq(n2);
            if (sc < 1.0f) {
                const float tt = __builtin_fmaf(b3, h3, __builtin_fmaf(b2, h2, b1 * h1)) * rcp(n2);
                h1 = sc * __builtin_fmaf(-tt, b1, h1);
                h2 = sc * __builtin_fmaf(-tt, b2, h2);
                h3 = sc * __builtin_fmaf(-tt, b3, h3);
            }
            Q1[r] = h1;
            Q2[r] = h2;
            Q3[r] = h3;
        }
        // reverse of the primal half-step: needs M^T q and M^T p at the left
        // and upper neighbours
        float qxq[R], qyq[R], qxp[R], qyp[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            qxq[r] = q_x(c[r], Q1[r], Q2[r], Q3[r]);
            qyq[r] = q_y(c[r], Q1[r], Q2[r], Q3[r]);
            qxp[r] = q_x(c[r], pa[r], pb[r], pc[r]);
            qyp[r] = q_y(c[r], pa[r], pb[r], pc[r]);
        }
        float qyq_top = 0.0f, qyp_top = 0.0f;
        if constexpr (NW > 1) {
            xc[wave][lane] = qyq[R - 1];
            xd[wave][lane] = qyp[R - 1];
            __syncthreads();
            if (wave > 0) {
                qyq_top = xc[wave - 1][lane];
                qyp_top = xd[wave - 1][lane];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float qxl = lane_from_left(qxq[r]);
            const float qyu = r > 0 ? qyq[r - 1] : qyq_top;
            const float ut_hat = -((qxq[r] - qxl) + (qyq[r] - qyu));
            const float H = __builtin_fmaf(2.0f, ut_hat, UH[r]);
            const float pxl = lane_from_left(qxp[r]);
            const float pyu = r > 0 ? qyp[r - 1] : qyp_top;
            float rr;
            const float un =
                prox_root(u0[r], qxp[r], qyp[r], pxl, pyu, c[r].hb, c[r].bf, st.ts, rr);
            const bool active = un >= st.umin && un <= st.umax;
            const float hr = active ? H * rcp(rr) : 0.0f;
            const float ub = un * hr;
            UB[r] = ub;
            UH[r] = ub - ut_hat;
            GB[r] += (fr[r] - un) * hr;
            GF[r] += prox_beta(c[r]) * hr;
            u1[r] = u0[r];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!interior<R, NW>(d, g, t, r)) continue;
        const uint32_t e = ee[r];  // (an interior pixel's offset needs no clamping)
        *at(aout.q + t.tbf, e) = Q1[r];
        *at(aout.q + t.tbf + d.np, e) = Q2[r];
        *at(aout.q + t.tbf + 2 * d.np, e) = Q3[r];
        *at(aout.ub + t.tb, e) = UB[r];
        *at(aout.uh + t.tb, e) = UH[r];
        *at(gbeta + t.tb, e) = GB[r];
        *at(gf + t.tb, e) = GF[r];
    }
}

// ------------------------------------------------------------------ host

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool desc_ok(const rec_diff_desc* d) {
    if (!d) return false;
    if (d->width < 1 || d->width > 65535 || d->height < 1 || d->height > 65535) return false;
    if (d->batch < 1 || d->batch > 65535 || d->iters < 0) return false;
    if (d->unfused != 0 && d->unfused != 1) return false;
    if (d->ckpt_every < 1 || d->ckpt_every > (d->iters > 0 ? d->iters : 1)) return false;
    if (!(d->tau > 0.0) || !(d->sigma > 0.0) || !isfinite(d->tau) || !isfinite(d->sigma))
        return false;
    if (d->tau * d->sigma * (8.0 + 4.0 * sqrt(2.0)) > 1.0 + 1e-12) return false;
    if (!(d->u_min > 0.0) || !(d->u_max > d->u_min) || !isfinite(d->u_max)) return false;
    return true;
}

int segments(const rec_diff_desc* d) {
    return d->iters == 0 ? 0 : (d->iters + d->ckpt_every - 1) / d->ckpt_every;
}

dim3 grid_of(const rec_diff_desc* d) {
    return dim3((unsigned)((d->width + kTileX - 1) / kTileX),
                (unsigned)((d->height + kTileY - 1) / kTileY), (unsigned)d->batch);
}

size_t blocks_of(const rec_diff_desc* d) {
    const dim3 g = grid_of(d);
    return (size_t)g.x * g.y * g.z;
}

// Workspace carve: f | checkpoints (C + 1 states) | segment (k - 1 states) |
// adjoint planes (q, ub, uh twice for the fused ping-pong; the two sums) |
// partial sums.
struct Carve {
    float* f;
    State ck0;        // checkpoint c at ck0 + c * state_stride
    State seg0;       // segment slot j at seg0 + j * state_stride
    size_t state_floats;
    Adj A;            // q, ub, uh of side 0 and the sums
    AdjIO B;          // q, ub, uh of side 1
    double* part;
    size_t bytes;
};

Carve carve(const rec_diff_desc* d, char* base) {
    Carve c{};
    const size_t n = (size_t)d->width * d->height * d->batch;
    const size_t plane = align_up(n * sizeof(float));
    const size_t state = 4 * plane;
    size_t off = 0;
    c.f = (float*)(base + off);
    off += plane;
    c.state_floats = state / sizeof(float);
    c.ck0.u = (float*)(base + off);
    c.ck0.p = (float*)(base + off + plane);
    off += state * (size_t)(segments(d) + 1);
    c.seg0.u = (float*)(base + off);
    c.seg0.p = (float*)(base + off + plane);
    off += state * (size_t)(d->ckpt_every - 1);
    c.A.q = (float*)(base + off);
    off += 3 * plane;
    c.A.ub = (float*)(base + off);
    off += plane;
    c.A.uh = (float*)(base + off);
    off += plane;
    c.A.gbeta = (float*)(base + off);
    off += plane;
    c.A.gf = (float*)(base + off);
    off += plane;
    c.B.q = (float*)(base + off);
    off += 3 * plane;
    c.B.ub = (float*)(base + off);
    off += plane;
    c.B.uh = (float*)(base + off);
    off += plane;
    c.part = (double*)(base + off);
    off += align_up(blocks_of(d) * 3 * sizeof(double));
    c.bytes = off;
    return c;
}

State at(State s0, size_t stride, int k) {
    return State{s0.u + (size_t)k * stride, s0.p + (size_t)k * stride};
}

// Fused tile shapes: forward (rows per lane, wavefronts) by the batch's
// pixel count; the reverse keeps its adjoint state in registers (about 3x
// the forward's per row) on 4 rows per lane x 8 wavefronts, 5 steps per
// launch.  Measured on 16 x 346x260 (forward+backward, 100 iterations):
// reverse 4x8 with 5 steps 2.73 ms; 2x16 with 3/4/5/6/8 steps 3.07/2.96/
// 2.94/2.87/3.23 ms; forward 8x4 or 2x16 instead of 4x16: 3.63, 3.27 ms.
// With the current kernels (2.41 ms): reverse 4x16 with 5 or 8 steps 2.50,
// 2.47 ms (one 1024-lane workgroup per compute unit); 4x8 with up to 7
// steps (7 + 3 per checkpoint segment) 2.39-2.40 ms, within run-to-run
// spread of the 5 + 5 split.
struct FusedShape {
    int fr, fw, fk;  // forward rows, waves, max iterations per launch
    int rr, rw, rk;  // reverse rows, waves, max steps per launch
};

FusedShape fused_shape(const rec_diff_desc* d) {
    const size_t n = (size_t)d->width * d->height * d->batch;
    FusedShape f;
    if (n > 250000) {
        f.fr = 4; f.fw = 16; f.fk = 16;
    } else {
        f.fr = 2; f.fw = 16; f.fk = 15;
    }
    f.rr = 4; f.rw = 8; f.rk = 5;
    return f;
}

struct Ctx {
    const rec_diff_desc* d;
    const rec_diff_inputs* in;
    Carve cv;
    Dims dims;
    Steps st;
    dim3 grid;
    FusedShape fs;
    hipStream_t s;
};

TileGrid tile_grid(const Ctx& x, int rh, int kg) {
    TileGrid g;
    const int ow = 64 - 2 * kg, oh = rh - 2 * kg;
    g.tiles_x = (x.d->width + ow - 1) / ow;
    const int ty = (x.d->height + oh - 1) / oh;
    g.per_image = g.tiles_x * ty;
    g.total = g.per_image * x.d->batch;
    g.kg = kg;
    g.tiles_x_div = make_divider((uint32_t)g.tiles_x);
    g.per_image_div = make_divider((uint32_t)g.per_image);
    return g;
}

// K fused forward iterations from `a` into `b`, recording the K - 1
// intermediate states into rec (if rec.u).
void fwd_fused(const Ctx& x, State a, State b, int K, Trail rec) {
    const TileGrid g = tile_grid(x, x.fs.fr * x.fs.fw, K);
    const dim3 grid((unsigned)g.total), blk(64 * x.fs.fw);
    const rec_diff_inputs* in = x.in;
    if (x.fs.fr == 4)
        hipLaunchKernelGGL((k_dfwd_fused<4, 16>), grid, blk, 0, x.s, x.dims, g, a, b, rec,
                           x.cv.f, in->tx, in->ty, in->w, in->theta, x.st);
    else
        hipLaunchKernelGGL((k_dfwd_fused<2, 16>), grid, blk, 0, x.s, x.dims, g, a, b, rec,
                           x.cv.f, in->tx, in->ty, in->w, in->theta, x.st);
}

bool inputs_ok(const rec_diff_desc* d, const rec_diff_inputs* in) {
    return desc_ok(d) && in && in->u0 && in->npos && in->nneg && in->tx && in->ty && in->theta;
}

void set_consts(const rec_diff_desc* d, Ctx& x) {
    x.dims = Dims{d->width, d->height, (size_t)d->width * d->height};
    x.st = Steps{d->tau, (float)(d->tau / d->sigma), (float)d->sigma, (float)d->u_min,
                 (float)d->u_max, d->iters > 0 ? 1 : 0};
    x.grid = grid_of(d);
    x.fs = fused_shape(d);
}

int check_call(const rec_diff_desc* d, const rec_diff_inputs* in, void* ws, size_t bytes,
               Ctx& x) {
    if (!inputs_ok(d, in)) return REC_EINVAL;
    if (!ws || ((uintptr_t)ws % kAlign) != 0) return REC_EINVAL;
    x.d = d;
    x.in = in;
    x.cv = carve(d, (char*)ws);
    if (bytes < x.cv.bytes) return REC_ENOMEM;
    set_consts(d, x);
    return REC_OK;
}

// One forward iteration from state a into b.
void step(const Ctx& x, State a, State b) {
    hipLaunchKernelGGL(k_diff_primal, x.grid, dim3(kThreads), 0, x.s, x.dims, a, b, x.cv.f,
                       x.in->tx, x.in->ty, x.in->w, x.in->theta, x.st);
    hipLaunchKernelGGL(k_diff_dual, x.grid, dim3(kThreads), 0, x.s, x.dims, a, b, x.in->tx,
                       x.in->ty, x.st);
}

// State j of segment c (0 = its checkpoint, m = the next checkpoint).
State seg_state(const Ctx& x, int c, int j, int m) {
    if (j == 0) return at(x.cv.ck0, x.cv.state_floats, c);
    if (j == m) return at(x.cv.ck0, x.cv.state_floats, c + 1);
    return at(x.cv.seg0, x.cv.state_floats, j - 1);
}

// States a -> b of segment c by fused launches of at most fk iterations;
// with `record`, every state in between is written to its segment slot.
void fwd_segment(const Ctx& x, int c, int a, int b, int m, bool record) {
    while (a < b) {
        const int K = b - a < x.fs.fk ? b - a : x.fs.fk;
        Trail rec{nullptr, nullptr, 0};
        if (record && K > 1) {
            const State r0 = seg_state(x, c, a + 1, m);  // a + 1 < b <= m: a slot
            rec = Trail{r0.u, r0.p, x.cv.state_floats};
        }
        fwd_fused(x, seg_state(x, c, a, m), seg_state(x, c, a + K, m), K, rec);
        a += K;
    }
}

// Reverse steps j = jtop - 1 down to j0 in one fused launch; state_of(j)
// gives the stored state j.
template <class StateOf>
void rev_fused(const Ctx& x, StateOf state_of, int j0, int jtop, const float* g_u,
               const float* g_p, int first, int& side) {
    const int K = jtop - j0;
    StateSeq S;
    for (int i = 0; i <= K; ++i) {
        const State st = state_of(j0 + i);
        S.u[i] = st.u;
        S.p[i] = st.p;
    }
    const AdjIO A0{x.cv.A.q, x.cv.A.ub, x.cv.A.uh};
    const AdjIO ain = side ? x.cv.B : A0, aout = side ? A0 : x.cv.B;
    const TileGrid g = tile_grid(x, x.fs.rr * x.fs.rw, K);
    const rec_diff_inputs* in = x.in;
    hipLaunchKernelGGL((k_adj_fused<4, 8>), dim3((unsigned)g.total), dim3(64 * 8), 0, x.s,
                       x.dims, g, S, ain, aout, x.cv.A.gbeta, x.cv.A.gf, g_u, g_p, first, x.cv.f,
                       in->tx, in->ty, in->w, in->theta, x.st);
    side ^= 1;
}

// The forward that allocates nothing (rec_diff_forward_noalloc) keeps the
// data image and two ping-pong states (u and the three planes of p) of at
// most kScratchPixels pixels in this file-scope array: 9 planes of 4 MiB.
// Each device holds its own copy, at its own address, until the process
// ends; host code uses the address hipGetSymbolAddress returns for the
// current device, never the array's name.
constexpr size_t kScratchPixels = size_t(1) << 20;
constexpr size_t kScratchPlanes = 9;
constexpr size_t kScratchBytes = kScratchPlanes * kScratchPixels * sizeof(float);
static_assert(kScratchPixels * sizeof(float) % kAlign == 0, "planes stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch_addr[kMaxDevices];

// Device address of `scratch` on the current device, looked up once per
// device (two threads racing on the first lookup store the same address).
int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return REC_EDEVICE;
    void* p = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (!p) {
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return REC_EDEVICE;
        g_scratch_addr[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return REC_OK;
}

}  // namespace
}  // namespace rec

using namespace rec;

namespace {
// A roctx range around an entry point (rocprofv3 --marker-trace).
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};
}  // namespace

extern "C" {

size_t rec_diff_workspace_bytes(const rec_diff_desc* d) {
    if (!desc_ok(d)) return 0;
    return carve(d, nullptr).bytes;
}

int rec_diff_forward(const rec_diff_desc* d, const rec_diff_inputs* in, float* u_out,
                     float* p_out, void* dev_workspace, size_t ws_bytes, void* stream) {
    Range range("rec_diff_forward");
    Ctx x;
    int rc = check_call(d, in, dev_workspace, ws_bytes, x);
    if (rc != REC_OK) return rc;
    if (!u_out) return REC_EINVAL;
    x.s = (hipStream_t)stream;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_diff_init, x.grid, dim3(kThreads), 0, x.s, x.dims, in->u0, in->p0,
                       in->npos, in->nneg, in->theta, in->tx, in->ty, x.st.rot, x.cv.f, x.cv.ck0);
    const int C = segments(d), k = d->ckpt_every;
    const size_t sf = x.cv.state_floats;
    if (k == 1 && !d->unfused) {
        // every state is kept: fused launches of up to fk iterations that
        // record their intermediate states straight into the checkpoints
        for (int a = 0; a < d->iters;) {
            const int K = d->iters - a < x.fs.fk ? d->iters - a : x.fs.fk;
            const State r0 = at(x.cv.ck0, sf, a + 1);
            fwd_fused(x, at(x.cv.ck0, sf, a), at(x.cv.ck0, sf, a + K), K,
                      K > 1 ? Trail{r0.u, r0.p, sf} : Trail{nullptr, nullptr, 0});
            a += K;
        }
    }
    for (int c = 0; c < C && !(k == 1 && !d->unfused); ++c) {
        const int m = (d->iters - c * k) < k ? d->iters - c * k : k;
        if (d->unfused) {
            for (int j = 0; j < m; ++j)
                step(x, seg_state(x, c, j, m), seg_state(x, c, j + 1, m));
        } else {
            fwd_segment(x, c, 0, m, m, false);
        }
    }
    hipLaunchKernelGGL(k_diff_out, x.grid, dim3(kThreads), 0, x.s, x.dims,
                       at(x.cv.ck0, x.cv.state_floats, C), in->tx, in->ty, x.st.rot, u_out, p_out);
    return hipGetLastError() == hipSuccess ? REC_OK : REC_EDEVICE;
}

int rec_diff_forward_noalloc(const rec_diff_desc* d, const rec_diff_inputs* in, float* u_out,
                             float* p_out, void* stream) {
    Range range("rec_diff_forward_noalloc");
    if (!inputs_ok(d, in) || !u_out) return REC_EINVAL;
    const size_t n = (size_t)d->width * d->height * d->batch;
    if (n > kScratchPixels) return REC_ENOMEM;
    void* base = nullptr;
    const int rc = scratch_address(&base);
    if (rc != REC_OK) return rc;
    Ctx x;
    x.d = d;
    x.in = in;
    set_consts(d, x);
    x.s = (hipStream_t)stream;
    // f | state 0 | state 1, each state u and p1..p3 (planes of n floats,
    // 256-byte aligned; every value is written before it is read, so no
    // earlier call's contents matter)
    const size_t plane = align_up(n * sizeof(float));
    char* b = (char*)base;
    x.cv = Carve{};
    x.cv.f = (float*)b;
    x.cv.state_floats = 4 * plane / sizeof(float);
    x.cv.ck0 = State{(float*)(b + plane), (float*)(b + 2 * plane)};
    const size_t sf = x.cv.state_floats;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_diff_init, x.grid, dim3(kThreads), 0, x.s, x.dims, in->u0, in->p0,
                       in->npos, in->nneg, in->theta, in->tx, in->ty, x.st.rot, x.cv.f, x.cv.ck0);
    int side = 0;
    for (int a = 0; a < d->iters;) {
        const State from = at(x.cv.ck0, sf, side), to = at(x.cv.ck0, sf, side ^ 1);
        int K = 1;
        if (d->unfused) {
            step(x, from, to);
        } else {
            K = d->iters - a < x.fs.fk ? d->iters - a : x.fs.fk;
            fwd_fused(x, from, to, K, Trail{nullptr, nullptr, 0});
        }
        a += K;
        side ^= 1;
    }
    hipLaunchKernelGGL(k_diff_out, x.grid, dim3(kThreads), 0, x.s, x.dims, at(x.cv.ck0, sf, side),
                       in->tx, in->ty, x.st.rot, u_out, p_out);
    return hipGetLastError() == hipSuccess ? REC_OK : REC_EDEVICE;
}

int rec_diff_backward(const rec_diff_desc* d, const rec_diff_inputs* in, const float* g_u,
                      const float* g_p, const rec_diff_grads* out, void* dev_workspace,
                      size_t ws_bytes, void* stream) {
    Range range("rec_diff_backward");
    Ctx x;
    int rc = check_call(d, in, dev_workspace, ws_bytes, x);
    if (rc != REC_OK) return rc;
    if (!out) return REC_EINVAL;
    x.s = (hipStream_t)stream;
    (void)hipGetLastError();
    const dim3 blk(kThreads);
    hipLaunchKernelGGL(k_adj_zero, x.grid, blk, 0, x.s, x.dims, x.cv.A);
    const int C = segments(d), k = d->ckpt_every;
    int first = 1, side = 0;
    if (k == 1 && !d->unfused) {
        // every state is stored: no recomputation, reverse chunks run across
        // checkpoint boundaries
        const size_t sf = x.cv.state_floats;
        auto ck = [&](int j) { return at(x.cv.ck0, sf, j); };
        for (int jtop = d->iters; jtop > 0;) {
            const int j0 = jtop > x.fs.rk ? jtop - x.fs.rk : 0;
            rev_fused(x, ck, j0, jtop, g_u, g_p, first, side);
            first = 0;
            jtop = j0;
        }
    }
    for (int c = C - 1; c >= 0 && !d->unfused && k > 1; --c) {
        const int m = (d->iters - c * k) < k ? d->iters - c * k : k;
        if (m >= 2) fwd_segment(x, c, 0, m - 1, m, true);  // states 1 .. m-1
        auto seg = [&](int j) { return seg_state(x, c, j, m); };
        for (int jtop = m; jtop > 0;) {
            const int j0 = jtop > x.fs.rk ? jtop - x.fs.rk : 0;
            rev_fused(x, seg, j0, jtop, g_u, g_p, first, side);
            first = 0;
            jtop = j0;
        }
    }
    for (int c = C - 1; c >= 0 && d->unfused; --c) {
        const int m = (d->iters - c * k) < k ? d->iters - c * k : k;
        for (int j = 0; j + 1 < m; ++j)  // recompute the states inside the segment
            step(x, seg_state(x, c, j, m), seg_state(x, c, j + 1, m));
        for (int j = m - 1; j >= 0; --j) {
            const State a = seg_state(x, c, j, m), b = seg_state(x, c, j + 1, m);
            hipLaunchKernelGGL(k_adj_dual, x.grid, blk, 0, x.s, x.dims, a, b, in->tx, in->ty,
                               x.cv.A, g_p, first, x.st);
            hipLaunchKernelGGL(k_adj_primal, x.grid, blk, 0, x.s, x.dims, a, x.cv.f, in->tx,
                               in->ty, in->w, in->theta, x.cv.A, g_u, first, x.st);
            first = 0;
        }
    }
    Adj cur = x.cv.A;  // the side holding the latest adjoint state
    if (side) {
        cur.q = x.cv.B.q;
        cur.ub = x.cv.B.ub;
        cur.uh = x.cv.B.uh;
    }
    hipLaunchKernelGGL(k_adj_final, x.grid, blk, 0, x.s, x.dims, x.cv.f, in->tx, in->ty, in->w,
                       in->npos, in->nneg, in->theta, cur, g_u, g_p, first, x.st, out->u0,
                       out->p0, out->w, x.cv.part);
    if (out->theta)
        hipLaunchKernelGGL(k_adj_reduce, dim3(1), blk, 0, x.s, x.cv.part, blocks_of(d),
                           out->theta);
    return hipGetLastError() == hipSuccess ? REC_OK : REC_EDEVICE;
}

}  // extern "C"
