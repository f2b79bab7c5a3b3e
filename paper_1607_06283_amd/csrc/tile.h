// Register-tile building blocks shared by the fused loops: the forward
// primal-dual iteration of a tile, and the plane-addressing, lane and XCD
// helpers.
//
// Tile layout: a workgroup's lanes form NV rows of CW lanes ("lane rows";
// CW = 64: one per wavefront, CW = 32: two per wavefront) and cover CW
// columns x (NV * R) rows; lane = column within its lane row, each lane
// holds R consecutive rows in registers and lane row v holds rows
// [v R, v R + R).  Horizontal neighbours come from adjacent lanes (DPP
// whole-wavefront shifts), vertical ones from the lane's own registers or,
// across lane rows, through LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "pd_math.h"

namespace rec {

// Element e of a plane addressed from a base pointer with a 32-bit offset
// (byte offset computed in 32 bits), so that the load or store takes the
// scalar-base + 32-bit vector-offset form.  The base passes through the
// global address space: the planes are device memory, and pointers that a
// kernel reads from memory (the batched launch's descriptors) would
// otherwise be accessed with flat instructions.
using gchar = __attribute__((address_space(1))) char;
template <class T>
__device__ __forceinline__ const T* at(const T* base, uint32_t e) {
    return (const T*)((const gchar*)base + e * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ T* at(T* base, uint32_t e) {
    return (T*)((gchar*)base + e * (uint32_t)sizeof(T));
}

// blockIdx -> tile such that each of the 8 XCDs (which receive blocks
// round-robin) works on one contiguous run of tiles, so halo rows shared by
// neighbouring tiles are fetched into the same L2.
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
    const int q = ntiles >> 3, rem = ntiles & 7;
    const int xcd = b & 7, idx = b >> 3;
    return xcd * q + min(xcd, rem) + idx;
}

// Whole-wavefront lane shifts by one lane (DPP wave_shr:1 / wave_shl:1);
// the lane without a source receives 0.  With two lane rows per wavefront
// the first column of the second lane row receives the last column of the
// first (and vice versa): both are halo columns of the tile, whose values
// are not exact anyway, and every such value is finite.
__device__ __forceinline__ float lane_from_left(float v) {   // value of lane - 1
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_from_right(float v) {  // value of lane + 1
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}

// Makes the value available at this point of the program: an empty asm
// statement that reads it, so the compiler cannot sink its computation past
// a following barrier.
__device__ __forceinline__ void settle(float x) { asm volatile("" ::"v"(x)); }

// Whether wavefront `wave` must compute iteration `it` (1-based) of a
// launch.  After `it` iterations of a tile started from exact values
// everywhere, rows [it, RH - it) are exact (each iteration reads one row
// above and below), so a wavefront whose rows all lie outside
// [it - 1, RH - it + 1) cannot influence any row that will be exact later.
// It may skip the iteration's arithmetic but must still take part in its
// two barriers (tile_skip); the LDS rows it leaves stale are read only by
// rows that are themselves outside the exact region.
// (R: rows per wavefront, NW: wavefronts of the tile.)
template <int R, int NW>
__device__ __forceinline__ bool tile_rows_active(int wave, int it) {
    constexpr int RH = NW * R;
    return wave * R + R >= it && wave * R <= RH - it;
}

template <int NW>
__device__ __forceinline__ void tile_skip() {
    if constexpr (NW > 1) {
        __syncthreads();
        __syncthreads();
    }
}

// One primal-dual iteration of a tile held in registers (u, p in frame
// coordinates, metric constants c per row; ts = tau / sigma) with NV lane
// rows of CW lanes; the new u goes to uo (which may be u itself);
// `col` is the lane's column and `v` its lane row.  Rows that cross lane
// rows go through LDS: xq[v + 1] receives lane row v's last q_y row and
// xu[v] its first extrapolated row (NV + 1 rows of CW floats each); xq[0]
// and xu[NV] must hold zeros.  Pixels outside the image carry all-zero
// coefficients, so every neighbour term they contribute is 0.
// The rows whose neighbours are in the lane's own registers are updated
// before each barrier, so that only one row's update waits for the
// exchange (the result does not depend on this order).
template <int R, int NV, int CW = 64>
__device__ __forceinline__ void tile_iteration(float (&u)[R], float (&uo)[R], float (&p1)[R],
                                               float (&p2)[R], float (&p3)[R],
                                               const CoefT (&c)[R], float ts,
                                               float umin, float umax, int col, int v,
                                               float (*xq)[CW], float (*xu)[CW]) {
    float qx[R], qy[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        qx[r] = q_x(c[r], p1[r], p2[r], p3[r]);
        qy[r] = q_y(c[r], p1[r], p2[r], p3[r]);
    }
    if constexpr (NV > 1) xq[v + 1][col] = qy[R - 1];
    float un[R], ut[R];
#pragma unroll
    for (int r = 1; r < R; ++r) {
        un[r] = primal(u[r], qx[r], qy[r], lane_from_left(qx[r]), qy[r - 1], c[r], ts, umin, umax);
        ut[r] = extrapolate(un[r], u[r]);
        settle(ut[r]);
    }
    float qy_top = 0.0f;
    if constexpr (NV > 1) {
        __syncthreads();
        qy_top = xq[v][col];
    }
    un[0] = primal(u[0], qx[0], qy[0], lane_from_left(qx[0]), qy_top, c[0], ts, umin, umax);
    ut[0] = extrapolate(un[0], u[0]);
    if constexpr (NV > 1) xu[v][col] = ut[0];
#pragma unroll
    for (int r = 0; r < R - 1; ++r) {
        dual(p1[r], p2[r], p3[r], lane_from_right(ut[r]) - ut[r], ut[r + 1] - ut[r], c[r]);
        uo[r] = un[r];
        settle(p1[r]);
        settle(p2[r]);
        settle(p3[r]);
    }
    float ut_bot = 0.0f;
    if constexpr (NV > 1) {
        __syncthreads();
        ut_bot = xu[v + 1][col];
    }
    dual(p1[R - 1], p2[R - 1], p3[R - 1], lane_from_right(ut[R - 1]) - ut[R - 1],
         ut_bot - ut[R - 1], c[R - 1]);
    uo[R - 1] = un[R - 1];
}

}  // namespace rec
