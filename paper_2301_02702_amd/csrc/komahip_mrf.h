// Internal layout of the MRF matching kernels (komahip_mrf.hip), shared
// with the host code. Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace koma {

struct MrfArgs {
    const uint16_t *xh;    // [n_pix_pad][kp] fingerprints, binary16 bits (re, im) interleaved
    const uint16_t *dh;    // [n_ent_tiles * mrf_ent_tile()][kp] entries, same layout
    const float *inv_norm2;  // [n_ent_tiles * mrf_ent_tile()] 1 / ||entry||^2 (-1: padding or zero entry)
    const int32_t *x_exp;  // [n_pix_pad] power-of-two exponent applied to each fingerprint
    int64_t kp;            // padded contraction length (halfs), multiple of 32
    int64_t n_pix, n_pix_pad;  // pixels, padded to a multiple of mrf_pix_tile()
    int64_t n_ent_tiles;   // entry tiles of mrf_ent_tile() entries
    int64_t n_split, tiles_per_split;  // entry splits and entry tiles per workgroup
    int64_t n_planes;      // partial planes: mrf_ent_tile() / 64 per split (one per 64 entries of a tile)
    float *part_score;     // [n_planes][n_pix_pad]
    int32_t *part_idx;     // [n_planes][n_pix_pad]
};

int launch_mrf_pack(const float2 *src, int64_t n_rows, int64_t n_rows_pad, int64_t n_t, int64_t kp,
                    uint16_t *dst, int32_t *exps, float *inv_norm2, void *stream);
int launch_mrf_match(const MrfArgs &a, void *stream);
// pixels and entries of one matching workgroup tile (multiples of 64)
int mrf_pix_tile();
int mrf_ent_tile();
int launch_mrf_final(const MrfArgs &a, int32_t *best, double *proj, void *stream);

}  // namespace koma
