// Per-pixel arithmetic of the primal-dual iteration on the event manifold.
//
// Every kernel that updates (u, p) -- the two-kernel loop, the fused
// temporally-blocked loop and the gap evaluation -- calls these inline
// functions, so a pixel's update is the same sequence of FP32 operations
// whichever kernel runs it (the library is compiled with -ffp-contract=off
// and every fused multiply-add below is explicit).
//
// Notation (Section 3.1-3.2 of the paper):
//   tx, ty      forward differences of the time surface tau
//   G           1 + tx^2 + ty^2 = det g;  s = sqrt(G)
//   M           3x2 matrix of eqn. (3), L_g u = M (L_x u, L_y u):
//               M = (1/G) [[1+ty^2, -tx ty], [-tx ty, 1+tx^2], [tx, ty]]
//   q           M^T p; the adjoint is L_g^* p = -div q
//   beta        tau * lambda * s            (KL prox, eqn. update_rules)
//   c4          4 beta f
#pragma once

#include <hip/hip_runtime.h>

namespace rec {

struct Coef {
    float m11, m12, m22, m31, m32;  // M entries (m12 is shared by rows 1 and 2)
    float G, s;                     // det g and sqrt(det g)
    float beta, c4;                 // KL prox constants
};

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Metric-dependent constants of one pixel (computed once per block of
// iterations; they depend on the block's tau and f only).
__device__ __forceinline__ Coef make_coef(float tx, float ty, float f, float taulam) {
    Coef c;
    const float ax = __builtin_fmaf(tx, tx, 1.0f);  // 1 + tx^2
    const float ay = __builtin_fmaf(ty, ty, 1.0f);  // 1 + ty^2
    const float G = __builtin_fmaf(tx, tx, ay);     // 1 + tx^2 + ty^2
    const float iG = rcp(G);
    c.m11 = ay * iG;
    c.m22 = ax * iG;
    c.m12 = -(tx * ty) * iG;
    c.m31 = tx * iG;
    c.m32 = ty * iG;
    c.G = G;
    c.s = sqrt_(G);
    c.beta = taulam * c.s;
    c.c4 = (4.0f * c.beta) * f;
    return c;
}

// q = M^T p at one pixel.
__device__ __forceinline__ float q_x(const Coef& c, float p1, float p2, float p3) {
    return __builtin_fmaf(c.m31, p3, __builtin_fmaf(c.m12, p2, c.m11 * p1));
}
__device__ __forceinline__ float q_y(const Coef& c, float p1, float p2, float p3) {
    return __builtin_fmaf(c.m32, p3, __builtin_fmaf(c.m22, p2, c.m12 * p1));
}

// Primal step u_{k+1} = prox_{tau D}(u_k - tau L_g^* p_k) at one pixel.
// div q uses backward differences with the boundary of the forward
// differences' adjoint: +q_x here unless on the last column, -q_x of the
// left neighbour unless on the first column; likewise along y.
// The KL prox uses the cancellation-free form of the closed-form root:
// a = ubar - beta, r = sqrt(a^2 + 4 beta f):
//   a >= 0: (a + r) / 2,   a < 0: 2 beta f / (r - a);   then clamp.
__device__ __forceinline__ float primal(float u, float qx, float qy, float qx_left,
                                        float qy_up, bool has_r, bool has_l, bool has_d,
                                        bool has_u, const Coef& c, float tau, float umin,
                                        float umax) {
    const float dx = (has_r ? qx : 0.0f) - (has_l ? qx_left : 0.0f);
    const float dy = (has_d ? qy : 0.0f) - (has_u ? qy_up : 0.0f);
    const float ubar = __builtin_fmaf(tau, dx + dy, u);
    const float a = ubar - c.beta;
    const float r = sqrt_(__builtin_fmaf(a, a, c.c4));
    const float pos = 0.5f * (a + r);
    const float neg = (0.5f * c.c4) * rcp(r - a);
    const float un = a >= 0.0f ? pos : neg;
    return __builtin_fminf(__builtin_fmaxf(un, umin), umax);
}

// Over-relaxed primal 2 u_{k+1} - u_k.
__device__ __forceinline__ float extrapolate(float un, float u) {
    return __builtin_fmaf(2.0f, un, -u);
}

// Dual step p_{k+1} = prox_{sigma R^*}(p_k + sigma L_g ubar) at one pixel, with
// (gx, gy) the forward differences of the extrapolated primal; the prox is
// the projection onto the ball of radius s: p / max(1, |p| / s).
__device__ __forceinline__ void dual(float& p1, float& p2, float& p3, float gx, float gy,
                                     const Coef& c, float sigma) {
    const float v1 = __builtin_fmaf(c.m12, gy, c.m11 * gx);
    const float v2 = __builtin_fmaf(c.m22, gy, c.m12 * gx);
    const float v3 = __builtin_fmaf(c.m32, gy, c.m31 * gx);
    float b1 = __builtin_fmaf(sigma, v1, p1);
    float b2 = __builtin_fmaf(sigma, v2, p2);
    float b3 = __builtin_fmaf(sigma, v3, p3);
    const float n2 = __builtin_fmaf(b3, b3, __builtin_fmaf(b2, b2, b1 * b1));
    const float sc = c.s * rsq(n2);
    const bool out = n2 > c.G;
    p1 = out ? b1 * sc : b1;
    p2 = out ? b2 * sc : b2;
    p3 = out ? b3 * sc : b3;
}

}  // namespace rec
