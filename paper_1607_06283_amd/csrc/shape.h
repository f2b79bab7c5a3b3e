// The fused loop's automatic tile shape (a host function of the library).
// It lives apart from the C ABI's source so that the files that decide
// which kernels a solve launches on which tiles (this one, the kernels and
// their headers) are separate from the rest of the library.
#pragma once

#include <stdint.h>

#include "kernels.h"
#include "rec.h"

namespace rec {

// Fused tile shape (rows per lane, wavefronts per workgroup, columns) and
// iterations per launch.  Small and mid-size frames are limited by the
// latency of each iteration on a compute unit and by the fixed cost of each
// launch, large frames by VALU issue and HBM.  Measured on MI355X, 50
// iterations per block, pixel-iterations/s (shape = rows x waves x columns,
// K = iterations per launch):
//   64x64 and 128x128: 1x16x32 K 10: 5.4 and 21.4 G (2x16x64 K 13: 4.5, 17.9)
//   240x180:           1x16x32 K 9: 49 G (2x16x64 K 13: 45 G)
//   320x240, 346x260:  2x8x32 K 8: 69, 69 G (best of 18 shapes 74, 74 G;
//                      2x16x64 K 13: 54, 51 G)
//   0.12-1 Mpx:        4x16x64 (since a wavefront of a 4-row tile skips the
//                      iterations that cannot reach the exact interior),
//                      K by the count below: 640x480 K 13 215 G (K 11:
//                      203 G), 720x576 K 10 265 G (K 9: 247 G; 2x8x32
//                      K 8: 203 G), 800x600 K 9 280 G (K 8 / 10 / 13:
//                      266 / 195 / 208 G; 2x8x32 K 8: 211 G), 960x720
//                      K 13 291 G (K 10: 272 G), 1024x768 K 10 298 G,
//                      1280x720 K 10 360 G (BF16 380, FP16 377; 8x8x64
//                      K 10: 331 G)
//   1-16 Mpx:          4x16x64 K 8: 1600x1200 417 G (K 9 / 10: 380 /
//                      343 G; 8x8x64: 332 G), 1920x1080 392 G (K 9:
//                      407-410 G; 8x8x64: 380 G), 2560x1440 468 G (455 G),
//                      3840x2160 469 G (461 G); with many tiles a compute
//                      unit's share of them no longer decides, and no
//                      simple count picked the best K on all of these
//   5120x5760:         8x8x64 K 8: 484 G (6x8x64 K 6: 440 G, 8x8x64 K 10: 432 G;
//                      later 508 G against 503 G for 4x16x64 K 8)
//   with BF16 storage: 1280x720 8x8x64 K 10 304 G, 5120x5760 8x8x64 K 8 478 G
//                      (4x8x64 K 6: 284 G, 448 G)
// `narrow` allows 32-column tiles (the untuned batch keeps 64 columns: it
// takes 2x16 K 13 up to 250k pixels and the large-frame shape beyond).
//
// Iterations per launch K (8..13) of the 4x16x64 tile (64 x 64 pixels, one
// 1024-lane workgroup; a compute unit holds two) on a W x H frame solved
// `iters` iterations at a time: the least launches x rounds, launches =
// ceil(iters / K), rounds = ceil(tiles / 256) (the compute units that hold
// one tile more than others set the pace of every iteration); on a tie the
// fewer tiles.  Measured to pick the best K on the frames of 0.12-1 Mpx
// listed above.
inline int tile4x16_k(int W, int H, int iters) {
    if (iters <= 0) iters = 50;
    int best = 13;
    long best_cost = 0, best_tiles = 0;
    for (int K = 8; K <= 13; ++K) {
        const int ow = 64 - 2 * K;
        const long tiles = (long)((W + ow - 1) / ow) * (long)((H + ow - 1) / ow);
        const long cost = (long)((iters + K - 1) / K) * ((tiles + 255) / 256);
        if (K == 8 || cost < best_cost || (cost == best_cost && tiles < best_tiles)) {
            best = K;
            best_cost = cost;
            best_tiles = tiles;
        }
    }
    return best;
}

inline void choose_shape(const rec_params* prm, int64_t np, bool narrow, int* rows, int* waves,
                  int* cols, int* kiters) {
    int r = prm->tile_rows, w = prm->tile_waves, cw = prm->tile_cols ? prm->tile_cols : 64, k;
    const bool f32 = prm->storage == kStoreF32;
    int ar, aw, acw;  // automatic shape
    if (!narrow) {
        if (np <= 250000) {
            ar = 2, aw = 16, acw = 64, k = 13;
        } else {
            ar = f32 ? 6 : 4, aw = 8, acw = 64, k = 6;
        }
    } else if (np <= 24000) {
        ar = 1, aw = 16, acw = 32, k = 10;
    } else if (np <= 60000) {
        ar = 1, aw = 16, acw = 32, k = 9;
    } else if (np <= 120000) {
        ar = 2, aw = 8, acw = 32, k = 8;
    } else if (np <= 1000000) {
        ar = 4, aw = 16, acw = 64, k = tile4x16_k(prm->width, prm->height, prm->iters);
    } else if (np <= 16000000) {
        ar = 4, aw = 16, acw = 64, k = 8;
    } else {
        ar = 8, aw = 8, acw = 64, k = 8;
    }
    if (!fused_shape_supported(ar, aw, acw, prm->storage)) {
        // 16-bit storage has 2x8 as its only 32-column tile
        ar = 2, aw = 8, acw = 32;
    }
    if (!r) {
        r = ar;
        w = aw;
        cw = acw;
    }
    if (prm->fuse_iters > 0) k = prm->fuse_iters;
    const int rh = r * w * (64 / cw);
    const int kmax = (rh - 1) / 2 < (cw - 1) / 2 ? (rh - 1) / 2 : (cw - 1) / 2;
    if (k > kmax) k = kmax;
    *rows = r;
    *waves = w;
    *cols = cw;
    *kiters = k;
}

}  // namespace rec
