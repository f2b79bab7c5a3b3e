// Per-pixel arithmetic of the primal-dual iteration on the event manifold.
//
// Every kernel that updates (u, p) -- the two-kernel loop, the fused
// temporally-blocked loop and the differentiable solve -- calls these inline
// functions, so a pixel's update is the same sequence of FP32 operations
// whichever kernel runs it (the library is compiled with -ffp-contract=off
// and every fused multiply-add below is explicit).
//
// Notation (Section 3.1-3.2 of the paper):
//   tx, ty      forward differences of the time surface tau
//   G           1 + tx^2 + ty^2 = det g;  s = sqrt(G)
//   M           3x2 matrix of eqn. (3), L_g u = M (L_x u, L_y u):
//               M = (1/G) [[1+ty^2, -tx ty], [-tx ty, 1+tx^2], [tx, ty]]
//   beta        tau * lambda * s            (KL prox, eqn. update_rules)
//
// The dual variable in a per-pixel orthonormal frame.  The columns of M span
// the tangent plane of the surface (x, y, tau(x, y)): with a = sqrt(1 + ty^2),
//   e1 = (1 + ty^2, -tx ty, tx) / (a s),  e2 = (0, 1, ty) / a,
//   n  = (-tx, -ty, 1) / s              (unit normal)
// form an orthonormal basis U = [e1 e2 n] and M = [e1 e2] T with the upper
// triangular T = [[e1x, e1y], [0, e2y]] (e1x = a / s, e1y = -tx ty / (a s),
// e2y = 1 / a).  Writing p = U p' (p' = U^T p):
//   M^T p = T^T (p'1, p'2),   U^T (p + sigma M g) = p' + sigma (T g, 0),
// and the projection onto the ball of radius s is the same in p' (U is
// orthogonal).  So the iteration runs on p' with the three coefficients of
// sigma T: q = sigma M^T p costs three operations, the dual ascent three.
// The adjoint is L_g^* p = -div(M^T p), so the primal step u - tau L_g^* p
// is u + (tau / sigma) div q.  A solve rotates p into the frame once at its
// start and back at its end (the frame depends on the block's time surface
// only).
//
// Boundary handling.  The forward differences vanish on the last column
// (L_x) and the last row (L_y).  Since L_g u = M (L_x u, L_y u), a vanishing
// L_x u is the same as a zero first column of M at that pixel, and the
// adjoint's matching backward difference drops q_x there too; likewise for
// the second column on the last row.  So the column of T that multiplies a
// difference leaving the image is stored as zero ("masked"), and pixels
// outside the image carry zero coefficients.  The update formulas then need
// no per-pixel boundary branches: the neighbour terms they read are exactly
// zero wherever the operator has no such term.
#pragma once

#include <hip/hip_runtime.h>

namespace rec {

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Data image of one pixel: f = u_prev * exp(Delta+ n+ - Delta- n-)
// (eqn. intensity_update for every event of the block), formed in FP64 and
// rounded once.
__device__ __forceinline__ float data_image(float u_prev, int npos, int nneg, double dpos,
                                            double dneg) {
    const double e = dpos * (double)npos - dneg * (double)nneg;
    return (float)((double)u_prev * exp(e));
}

// The frame of one pixel.
struct Basis {
    float e1x, e1y, e1z;  // e1
    float e2y, e2z;       // e2 (e2x = 0)
    float nx, ny, nz;     // n
    float s;              // sqrt(G)
};

__device__ __forceinline__ Basis make_basis(float tx, float ty) {
    Basis b;
    const float a2 = __builtin_fmaf(ty, ty, 1.0f);  // 1 + ty^2
    const float G = __builtin_fmaf(tx, tx, a2);     // 1 + tx^2 + ty^2
    const float ia = rsq(a2), is = rsq(G);
    const float ias = ia * is;
    b.e1x = a2 * ias;
    b.e1y = -(tx * ty) * ias;
    b.e1z = tx * ias;
    b.e2y = ia;
    b.e2z = ty * ia;
    b.nx = -tx * is;
    b.ny = -ty * is;
    b.nz = is;
    b.s = G * is;
    return b;
}

// Metric-dependent constants of one pixel (computed once per launch; they
// depend on the block's tau and f only).  sigma: the dual step size folded
// into the coefficients.  has_x: the pixel has a right neighbour inside the
// image (so L_x is a real difference); has_y: it has a lower neighbour.
struct CoefT {
    float k11;      // sigma T11, 0 if the first column is masked
    float k12, k22; // sigma T12, sigma T22, 0 if the second column is masked
    float s;        // ball radius sqrt(G)
    float hb, bf;   // KL prox constants beta / 2 and beta f
};

// beta itself (exact: hb is beta / 2).
__device__ __forceinline__ float prox_beta(const CoefT& c) { return 2.0f * c.hb; }

__device__ __forceinline__ CoefT make_coef_t(const Basis& b, float f, float taulam, float sigma,
                                             bool has_x, bool has_y) {
    CoefT c;
    c.k11 = has_x ? sigma * b.e1x : 0.0f;
    c.k12 = has_y ? sigma * b.e1y : 0.0f;
    c.k22 = has_y ? sigma * b.e2y : 0.0f;
    c.s = b.s;
    const float beta = taulam * b.s;
    c.hb = 0.5f * beta;
    c.bf = beta * f;
    return c;
}

// p' = U^T p and p = U p'.
__device__ __forceinline__ void to_frame(const Basis& b, float& p1, float& p2, float& p3) {
    const float r1 = __builtin_fmaf(b.e1z, p3, __builtin_fmaf(b.e1y, p2, b.e1x * p1));
    const float r2 = __builtin_fmaf(b.e2z, p3, b.e2y * p2);
    const float r3 = __builtin_fmaf(b.nz, p3, __builtin_fmaf(b.ny, p2, b.nx * p1));
    p1 = r1;
    p2 = r2;
    p3 = r3;
}
__device__ __forceinline__ void from_frame(const Basis& b, float& p1, float& p2, float& p3) {
    const float x = __builtin_fmaf(b.nx, p3, b.e1x * p1);
    const float y = __builtin_fmaf(b.ny, p3, __builtin_fmaf(b.e2y, p2, b.e1y * p1));
    const float z = __builtin_fmaf(b.nz, p3, __builtin_fmaf(b.e2z, p2, b.e1z * p1));
    p1 = x;
    p2 = y;
    p3 = z;
}

// q = sigma M^T p from the frame coordinates p' (p'3 does not enter; zero
// components where the column is masked).
__device__ __forceinline__ float q_x(const CoefT& c, float p1, float, float) {
    return c.k11 * p1;
}
__device__ __forceinline__ float q_y(const CoefT& c, float p1, float p2, float) {
    return __builtin_fmaf(c.k22, p2, c.k12 * p1);
}

// Primal step u_{k+1} = prox_{tau D}(u_k - tau L_g^* p_k) at one pixel, with
// ubar = u + ts div q, ts = tau / sigma, and
// div q = (q_x - q_x(left)) + (q_y - q_y(up)) (backward differences; the
// neighbour values are 0 outside the image).  The KL prox is the positive
// root of u^2 - a u - beta f = 0, a = ubar - beta, in the cancellation-free
// form: with r = sqrt(a^2 + 4 beta f) and d = r + |a|, the root is d / 2 for
// a >= 0 and 2 beta f / d for a < 0 (d is r + a in the first case and r - a
// in the second, so neither branch subtracts nearly equal numbers); then it
// is clamped to [umin, umax].  Everything is evaluated at half scale,
// h = a / 2 = (u + (ts div - beta)) / 2, r / 2 = sqrt(h^2 + beta f),
// d / 2 = r / 2 + |h|: the root is d / 2 itself, or beta f / (d / 2), so no
// halving is left in the loop.
// prox_root returns the unclamped root and r (the reverse sweep of the
// unrolled loop needs both); primal clamps it.
__device__ __forceinline__ float prox_root(float u, float qx, float qy, float qx_left, float qy_up,
                                           float hb, float bf, float ts, float& r) {
    // (operands ordered so that the values that arrive last -- the upper
    // neighbour's q_y from another lane row, then div -- enter last)
    const float div = ((qx - qx_left) + qy) - qy_up;
    const float h = __builtin_fmaf(0.5f * ts, div, __builtin_fmaf(0.5f, u, -hb));
    const float rh = sqrt_(__builtin_fmaf(h, h, bf));
    const float dh = rh + __builtin_fabsf(h);
    r = 2.0f * rh;
    return h >= 0.0f ? dh : bf * rcp(dh);
}

__device__ __forceinline__ float primal(float u, float qx, float qy, float qx_left, float qy_up,
                                        const CoefT& c, float ts, float umin, float umax) {
    float r;
    const float un = prox_root(u, qx, qy, qx_left, qy_up, c.hb, c.bf, ts, r);
    return __builtin_amdgcn_fmed3f(un, umin, umax);  // clamp (umin <= umax, un not NaN)
}

// Over-relaxed primal 2 u_{k+1} - u_k.
__device__ __forceinline__ float extrapolate(float un, float u) {
    return __builtin_fmaf(2.0f, un, -u);
}

// Dual ascent in the frame: pbar' = p' + (sigma T g, 0), with (gx, gy) the
// forward differences of the extrapolated primal (any finite value where
// the column of T is masked).
__device__ __forceinline__ void dual_ascent(const CoefT& c, float gx, float gy, float p1, float p2,
                                            float p3, float& b1, float& b2, float& b3) {
    b1 = __builtin_fmaf(c.k12, gy, __builtin_fmaf(c.k11, gx, p1));  // gy (lower row) last
    b2 = __builtin_fmaf(c.k22, gy, p2);
    b3 = p3;
}

// |b|^2 with the terms that do not wait for b1 formed first.
__device__ __forceinline__ float norm2(float b1, float b2, float b3) {
    return __builtin_fmaf(b1, b1, __builtin_fmaf(b2, b2, b3 * b3));
}

// sigma M (gx, gy) in frame coordinates (third component 0).
__device__ __forceinline__ void ascent_dir(const CoefT& c, float gx, float gy, float& v1,
                                           float& v2) {
    v1 = __builtin_fmaf(c.k12, gy, c.k11 * gx);
    v2 = c.k22 * gy;
}

// Dual step p_{k+1} = prox_{sigma R^*}(pbar) in the frame: the ascent, then
// the projection onto the ball of radius s, p / max(1, |p| / s), computed as
// p * min(1, s / |p|).
__device__ __forceinline__ void dual(float& p1, float& p2, float& p3, float gx, float gy,
                                     const CoefT& c) {
    float b1, b2, b3;
    dual_ascent(c, gx, gy, p1, p2, p3, b1, b2, b3);
    const float n2 = norm2(b1, b2, b3);
    const float sc = __builtin_fminf(1.0f, c.s * rsq(n2));
    p1 = b1 * sc;
    p2 = b2 * sc;
    p3 = b3 * sc;
}

}  // namespace rec
