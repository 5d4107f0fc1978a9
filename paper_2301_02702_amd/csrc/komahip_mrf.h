// Internal layout of the MRF matching kernels (komahip_mrf.hip), shared
// with the host code. Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace koma {

struct MrfArgs {
    const uint16_t *xh;    // [n_pix_pad][kp] fingerprints, binary16 bits (re, im) interleaved
    const uint16_t *dh;    // [n_ent_tiles * 128][kp] entries, same layout
    const float *inv_norm2;  // [n_ent_tiles * 128] 1 / ||entry||^2 (-1: padding or zero entry)
    const int32_t *x_exp;  // [n_pix_pad] power-of-two exponent applied to each fingerprint
    int64_t kp;            // padded contraction length (halfs), multiple of 32
    int64_t n_pix, n_pix_pad;  // pixels, padded to a multiple of 128
    int64_t n_ent_tiles;   // 128-entry tiles
    int64_t n_split, tiles_per_split;  // grid.y and entry tiles per workgroup
    int64_t n_planes;      // partial planes: 2 per split (the two entry halves of a tile)
    float *part_score;     // [n_planes][n_pix_pad]
    int32_t *part_idx;     // [n_planes][n_pix_pad]
};

int launch_mrf_pack(const float2 *src, int64_t n_rows, int64_t n_rows_pad, int64_t n_t, int64_t kp,
                    uint16_t *dst, int32_t *exps, float *inv_norm2, void *stream);
int launch_mrf_match(const MrfArgs &a, void *stream);
int launch_mrf_final(const MrfArgs &a, int32_t *best, double *proj, void *stream);

}  // namespace koma
