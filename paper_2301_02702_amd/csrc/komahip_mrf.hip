// MR-fingerprinting dictionary matching on the matrix cores (gfx950).
//
// The paper's MRF experiment assigns every pixel's fingerprint x the
// dictionary entry with the maximum dot product against the normalised
// entries: best(x) = argmax_e |<d_e, x>|^2 / ||d_e||^2 with
// <d, x> = sum_t conj(d_t) x_t. Over all pixels and entries this is one
// dense complex contraction over the TR axis, so it runs as a GEMM on the
// MFMA units with the argmax fused into the epilogue:
//
//   k_mrf_pack   every row (fingerprint or entry) is scaled by an exact
//                power of two so that its largest |Re|, |Im| is in [0.5, 1)
//                and rounded to binary16, interleaved (re, im) along the
//                contraction axis and zero-padded; entries also get
//                1 / ||rounded entry||^2.
//   k_mrf_match  a workgroup owns 128 pixels (one 32-pixel slab per
//                wavefront) and a range of entries; per 64-entry tile each
//                wavefront accumulates Re and Im of <d, x> for 32 x 64
//                (pixel, entry) pairs with v_mfma_f32_32x32x16_f16
//                (FP32 accumulation), then scores the tile and keeps the
//                running best entry of each of its pixels (ties: lower
//                index). Re <d, x> = [xr, xi] . [dr, di] and
//                Im <d, x> = [xr, xi] . [-di, dr]: the second operand is
//                formed from the first in registers.
//   k_mrf_final  the best of the workgroups' partial results per pixel, in
//                entry order, and the projection <d, x> / ||d|| in the
//                caller's units.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "komahip_mrf.h"

namespace koma {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMrfWG = 256;
constexpr int kMrfWaves = 4;
constexpr int kPixTile = 32 * kMrfWaves;  // pixels per workgroup
constexpr int kEntTile = 64;              // entries per tile (two 32-wide MFMA columns)

// ---------------------------------------------------------------- packing

// One row per workgroup: the row's largest component magnitude, its
// power-of-two exponent, the binary16 copy and (entries) 1 / ||copy||^2.
__global__ __launch_bounds__(kMrfWG) void k_mrf_pack(const float2 *src, int64_t n_rows, int64_t n_t, int64_t kp,
                                                    _Float16 *dst, int32_t *exps, float *inv_norm2) {
    __shared__ float red[kMrfWG];
    const int64_t row = blockIdx.x;
    const int tid = threadIdx.x;
    _Float16 *out = dst + row * kp;
    if (row >= n_rows) {  // padding rows: zeros, excluded from the argmax
        for (int64_t k = tid; k < kp; k += kMrfWG) out[k] = (_Float16)0.0f;
        if (tid == 0) {
            exps[row] = 0;
            if (inv_norm2) inv_norm2[row] = -1.0f;
        }
        return;
    }
    const float2 *in = src + row * n_t;
    float m = 0.0f;
    for (int64_t t = tid; t < n_t; t += kMrfWG) {
        const float2 v = in[t];
        m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    red[tid] = m;
    __syncthreads();
    for (int s = kMrfWG / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
        __syncthreads();
    }
    m = red[0];
    __syncthreads();
    int e = 0;
    if (m > 0.0f) (void)frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
    const float scale = ldexpf(1.0f, -e);  // exact power of two
    float n2 = 0.0f;
    for (int64_t t = tid; t < n_t; t += kMrfWG) {
        const float2 v = in[t];
        const _Float16 re = (_Float16)(v.x * scale), im = (_Float16)(v.y * scale);
        out[2 * t] = re;
        out[2 * t + 1] = im;
        const float fr = (float)re, fi = (float)im;
        n2 = fmaf(fr, fr, fmaf(fi, fi, n2));
    }
    for (int64_t k = 2 * n_t + tid; k < kp; k += kMrfWG) out[k] = (_Float16)0.0f;
    if (inv_norm2) {
        red[tid] = n2;
        __syncthreads();
        for (int s = kMrfWG / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
    }
    if (tid == 0) {
        exps[row] = -e;
        // an all-zero entry can never be the best match
        if (inv_norm2) inv_norm2[row] = red[0] > 0.0f ? 1.0f / red[0] : -1.0f;
    }
}

// ---------------------------------------------------------------- matching

struct Best {
    float score;
    int32_t idx;
    float re, im;
};

__device__ __forceinline__ bool better(float s, int32_t i, float bs, int32_t bi) {
    return s > bs || (s == bs && i < bi);
}

// (Re, Im) pair of binary16 values -> (-Im, Re): rotate the halves of each
// dword and flip the sign of the new low half.
__device__ __forceinline__ half8 times_i_conj(half8 v) {
    uint32_t w[4];
    __builtin_memcpy(w, &v, 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = ((w[q] << 16) | (w[q] >> 16)) ^ 0x00008000u;
    half8 r;
    __builtin_memcpy(&r, w, 16);
    return r;
}

// Grid: x = pixel tiles of 128, y = entry splits. Each workgroup scans entry
// tiles [y * tiles_per_split, ...) and writes one partial best per pixel.
__global__ __launch_bounds__(kMrfWG) void k_mrf_match(MrfArgs a) {
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t p0 = (int64_t)blockIdx.x * kPixTile + 32 * wave;  // this wave's 32 pixels
    const int64_t kp = a.kp;
    const int half = lane >> 5;   // which 8-wide k slice of a 16-wide step this lane feeds
    const int col = lane & 31;    // MFMA row (A) / column (B) index of this lane
    const half8 *xa = reinterpret_cast<const half8 *>(a.xh + (p0 + col) * kp + 8 * half);

    // running best of the 16 rows this lane holds (rows 8(r/4) + 4 half + r % 4)
    Best best[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) best[r] = Best{-1.0f, 0x7fffffff, 0.0f, 0.0f};

    const int64_t t0 = (int64_t)blockIdx.y * a.tiles_per_split;
    const int64_t t1 = min(t0 + a.tiles_per_split, a.n_ent_tiles);
    for (int64_t et = t0; et < t1; ++et) {
        const int64_t e0 = et * kEntTile;
        const half8 *db0 = reinterpret_cast<const half8 *>(a.dh + (e0 + col) * kp + 8 * half);
        const half8 *db1 = reinterpret_cast<const half8 *>(a.dh + (e0 + 32 + col) * kp + 8 * half);
        f32x16 re0 = {}, im0 = {}, re1 = {}, im1 = {};
        // k advances 16 halfs (8 complex TR values) per MFMA step; a half8 is 16 of them
        for (int64_t k = 0; k < kp; k += 16) {
            const int64_t q = k >> 3;  // half8 index
            const half8 av = xa[q];
            const half8 b0 = db0[q];
            const half8 b1 = db1[q];
            re0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, b0, re0, 0, 0, 0);
            im0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, times_i_conj(b0), im0, 0, 0, 0);
            re1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, b1, re1, 0, 0, 0);
            im1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, times_i_conj(b1), im1, 0, 0, 0);
        }
        // score the tile: lane holds column e0 + col (and + 32) for its 16 rows
        const float w0 = a.inv_norm2[e0 + col], w1 = a.inv_norm2[e0 + 32 + col];
        const int32_t i0 = (int32_t)(e0 + col), i1 = (int32_t)(e0 + 32 + col);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float s0 = (re0[r] * re0[r] + im0[r] * im0[r]) * w0;
            float s1 = (re1[r] * re1[r] + im1[r] * im1[r]) * w1;
            if (w0 < 0.0f) s0 = -1.0f;
            if (w1 < 0.0f) s1 = -1.0f;
            Best c = better(s1, i1, s0, i0) ? Best{s1, i1, re1[r], im1[r]} : Best{s0, i0, re0[r], im0[r]};
            // best over the 32 columns of this half wave (fixed butterfly; ties -> lower index)
#pragma unroll
            for (int m = 1; m < 32; m <<= 1) {
                const float os = __shfl_xor(c.score, m, 32);
                const int32_t oi = __shfl_xor(c.idx, m, 32);
                const float ore = __shfl_xor(c.re, m, 32);
                const float oim = __shfl_xor(c.im, m, 32);
                if (better(os, oi, c.score, c.idx)) c = Best{os, oi, ore, oim};
            }
            if (better(c.score, c.idx, best[r].score, best[r].idx)) best[r] = c;
        }
    }
    // one lane per half wave writes its 16 rows
    if (col == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t p = p0 + 8 * (r >> 2) + 4 * half + (r & 3);
            const int64_t o = (int64_t)blockIdx.y * a.n_pix_pad + p;
            a.part_score[o] = best[r].score;
            a.part_idx[o] = best[r].idx;
            a.part_ip[o] = make_float2(best[r].re, best[r].im);
        }
    }
}

// Best over the splits (in split order, i.e. entry order) and the output in
// the caller's units.
__global__ __launch_bounds__(kMrfWG) void k_mrf_final(MrfArgs a, int32_t *best, double *proj) {
    const int64_t p = (int64_t)blockIdx.x * kMrfWG + threadIdx.x;
    if (p >= a.n_pix) return;
    float bs = -1.0f;
    int32_t bi = 0x7fffffff;
    float2 ip = make_float2(0.0f, 0.0f);
    for (int64_t s = 0; s < a.n_split; ++s) {
        const int64_t o = s * a.n_pix_pad + p;
        const float sc = a.part_score[o];
        const int32_t id = a.part_idx[o];
        if (better(sc, id, bs, bi)) {
            bs = sc;
            bi = id;
            ip = a.part_ip[o];
        }
    }
    if (bi == 0x7fffffff || bs < 0.0f) {  // no valid entry
        best[p] = -1;
        proj[2 * p] = 0.0;
        proj[2 * p + 1] = 0.0;
        return;
    }
    best[p] = bi;
    // <d, x>/||d|| on the scaled operands is 2^kx times the caller's value
    const double f = sqrt((double)a.inv_norm2[bi]) * ldexp(1.0, -a.x_exp[p]);
    proj[2 * p] = (double)ip.x * f;
    proj[2 * p + 1] = (double)ip.y * f;
}

static int check_launch() { return hipGetLastError() == hipSuccess ? 0 : -1; }

int launch_mrf_pack(const float2 *src, int64_t n_rows, int64_t n_rows_pad, int64_t n_t, int64_t kp,
                    _Float16 *dst, int32_t *exps, float *inv_norm2, void *stream) {
    if (n_rows_pad <= 0) return 0;
    if (n_rows_pad > 0x7fffffff || kp < 2 * n_t || kp % 16) return -1;
    hipLaunchKernelGGL(k_mrf_pack, dim3((unsigned)n_rows_pad), dim3(kMrfWG), 0, (hipStream_t)stream, src, n_rows,
                       n_t, kp, dst, exps, inv_norm2);
    return check_launch();
}

int launch_mrf_match(const MrfArgs &a, void *stream) {
    if (a.n_pix_pad % kPixTile || a.n_ent_tiles <= 0 || a.kp % 16 || a.n_split <= 0 || a.n_split > 65535) return -1;
    dim3 grid((unsigned)(a.n_pix_pad / kPixTile), (unsigned)a.n_split);
    hipLaunchKernelGGL(k_mrf_match, grid, dim3(kMrfWG), 0, (hipStream_t)stream, a);
    return check_launch();
}

int launch_mrf_final(const MrfArgs &a, int32_t *best, double *proj, void *stream) {
    if (a.n_pix <= 0) return 0;
    dim3 grid((unsigned)((a.n_pix + kMrfWG - 1) / kMrfWG));
    hipLaunchKernelGGL(k_mrf_final, grid, dim3(kMrfWG), 0, (hipStream_t)stream, a, best, proj);
    return check_launch();
}

}  // namespace koma
