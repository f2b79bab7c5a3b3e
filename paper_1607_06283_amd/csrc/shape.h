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
//   480x360, 640x480:  4x16x64 K 13: 97, 162 G (best 103, 162 G)
//   800x600:           2x8x32 K 8: 153 G (best 154 G)
//   0.6-16 Mpx:        4x16x64 (since a wavefront of a 4-row tile skips the
//                      iterations that cannot reach the exact interior),
//                      K 10 up to 1 Mpx, K 8 beyond: 960x720 267 G,
//                      1024x768 298 G, 1280x720 360 G (BF16 380, FP16
//                      377; 8x8x64 K 10: 252, 280, 331 G); 1600x1200
//                      414 G (K 9 / 10: 380 / 343 G); 1920x1080 388 G
//                      (K 9: 407-410 G, K 10: 371 G; 8x8x64 K 8: 379 G);
//                      2560x1440 459 G (448 G); 3840x2160 464 G (455 G).
//                      Which K wins depends on how the tiles fall on the
//                      256 compute units, which no simple count predicted
//                      on all of these frames
//   5120x5760:         8x8x64 K 8: 484 G (6x8x64 K 6: 440 G, 8x8x64 K 10: 432 G;
//                      later 508 G against 503 G for 4x16x64 K 8)
//   with BF16 storage: 1280x720 8x8x64 K 10 304 G, 5120x5760 8x8x64 K 8 478 G
//                      (4x8x64 K 6: 284 G, 448 G)
// `narrow` allows 32-column tiles (the untuned batch keeps 64 columns: it
// takes 2x16 K 13 up to 250k pixels and the large-frame shape beyond).
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
    } else if (np <= 400000) {
        ar = 4, aw = 16, acw = 64, k = 13;
    } else if (np <= 600000) {
        ar = 2, aw = 8, acw = 32, k = 8;
    } else if (np <= 1000000) {
        ar = 4, aw = 16, acw = 64, k = 10;
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
