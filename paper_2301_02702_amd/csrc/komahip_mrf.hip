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
//   k_mrf_match  a workgroup owns 128 pixels and a range of 128-entry
//                tiles; operand slices are staged through LDS (double
//                buffered) and each wavefront accumulates Re and Im of
//                <d, x> for 64 x 64 (pixel, entry) pairs with
//                v_mfma_f32_32x32x16_f16 (FP32 accumulation), then scores
//                the tile and keeps, per lane and pixel, the best entry seen
//                (ties: lower index). Re <d, x> = [xr, xi] . [dr, di] and
//                Im <d, x> = [xr, xi] . [-di, dr]: the second operand is
//                formed from the first in registers.
//   k_mrf_final  the best of the partial results per pixel, and the
//                projection <d, x> / ||d|| recomputed in FP64 from the
//                binary16 operands, in the caller's units.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "komahip_mrf.h"

namespace koma {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
// 16-byte chunks as a native vector (HIP's uint4 is a struct whose copies
// the compiler routes through private memory here)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMrfWG = 256;  // packing and final kernels
constexpr int kMrfWaves = 4;
#ifndef KOMA_MRF_PT
#define KOMA_MRF_PT 256
#endif
#ifndef KOMA_MRF_ET
#define KOMA_MRF_ET 128
#endif
constexpr int kPixTile = KOMA_MRF_PT;  // pixels per matching workgroup
constexpr int kEntTile = KOMA_MRF_ET;  // entries per matching workgroup tile
constexpr int kPixWaves = kPixTile / 64, kEntWaves = kEntTile / 64;
constexpr int kMatchWG = 64 * kPixWaves * kEntWaves;  // one 64 x 64 block per wavefront

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

__device__ __forceinline__ bool better(float s, int32_t i, float bs, int32_t bi) {
    return s > bs || (s == bs && i < bi);
}

// (Re, Im) pair of binary16 values -> (-Im, Re): rotate the halves of each
// dword and flip the sign of the new low half (2 vector instructions per
// dword, which the binary16 matrix instructions partly overlap).
__device__ __forceinline__ half8 times_i_conj(half8 v) {
    uint32_t w[4];
    __builtin_memcpy(w, &v, 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = ((w[q] << 16) | (w[q] >> 16)) ^ 0x00008000u;
    half8 r;
    __builtin_memcpy(&r, w, 16);
    return r;
}

// Workgroup tile: kPixTile pixels x kEntTile entries, staged through LDS in
// slices of kSlice binary16 values of the contraction axis, double buffered.
// Wavefront w owns pixels 64 (w % kPixWaves) .. +63 and entries
// 64 (w / kPixWaves) .. +63 of the tile:
// 2 x 2 blocks of 32 x 32 with the entries as the MFMA rows and the pixels as
// its columns, each with a Re and an Im accumulator (8 accumulators of 16
// floats per lane). Lane l then holds one pixel (column l % 32) of each pixel
// block and 16 entries (rows 8 (r / 4) + 4 (l / 32) + r % 4) of each entry
// block, so its running best is one (score, entry) pair per pixel block: few
// registers, and two wavefronts per SIMD.
#ifndef KOMA_MRF_SLICE
#define KOMA_MRF_SLICE 64
#endif
#ifndef KOMA_MRF_MINW
#define KOMA_MRF_MINW 2
#endif
#ifndef KOMA_MRF_SWIZZLE
#define KOMA_MRF_SWIZZLE 1
#endif
constexpr int kSlice = KOMA_MRF_SLICE;  // halfs of the contraction axis per stage
constexpr int kLdsRow = kSlice + 8;     // padded row against bank conflicts

// One staged slice: kSlice / 16 steps of the 2 x 2 blocks of one wavefront,
// Re and Im. FIRST: the slice that starts the sums (C operand zero).
template <bool FIRST>
__device__ __forceinline__ void mma_slice(f32x16 (&acc)[2][2][2], const _Float16 *la, const _Float16 *lb, int wp,
                                          int we, int col, int half) {
#pragma unroll
    for (int kk = 0; kk < kSlice; kk += 16) {
        half8 dv[2], dw[2], xv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            dv[i] = *reinterpret_cast<const half8 *>(lb + (we + 32 * i + col) * kLdsRow + kk + 8 * half);
            dw[i] = times_i_conj(dv[i]);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
            xv[j] = *reinterpret_cast<const half8 *>(la + (wp + 32 * j + col) * kLdsRow + kk + 8 * half);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const bool z = FIRST && kk == 0;
                acc[i][j][0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(dv[i], xv[j], z ? f32x16{} : acc[i][j][0], 0, 0, 0);
                acc[i][j][1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(dw[i], xv[j], z ? f32x16{} : acc[i][j][1], 0, 0, 0);
            }
    }
}

__global__ __launch_bounds__(kMatchWG, KOMA_MRF_MINW) void k_mrf_match(MrfArgs a) {
    __shared__ __attribute__((aligned(16))) _Float16 ldsa[2][kPixTile * kLdsRow];  // [stage] pixels
    __shared__ __attribute__((aligned(16))) _Float16 ldsb[2][kEntTile * kLdsRow];  // [stage] entries
    // 1 / ||entry||^2 by tile parity; -inf for padding and all-zero entries, whose
    // scores 0 * -inf are NaN and never win a comparison
    __shared__ __attribute__((aligned(16))) float lw[2][kEntTile];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int half = lane >> 5;  // k offset 8 * half within a 16-wide MFMA step
    const int col = lane & 31;   // MFMA row (A) / column (B) index of this lane
    const int wp = (wave % kPixWaves) * 64, we = (wave / kPixWaves) * 64;
    // Work item w = (pixel tile, split) with the split fastest. Workgroups
    // are dispatched to the eight XCDs in turn (workgroup L to XCD L % 8), and
    // each XCD has its own L2: XCD x takes a contiguous range of the work
    // order, so the workgroups resident on one XCD at a time are a few pixel
    // tiles times every split and share the fingerprint slices (one pixel
    // tile, all splits) and the dictionary slices (one split, several pixel
    // tiles) in their L2.
    const int64_t L = blockIdx.x, n_wg = gridDim.x;
#if KOMA_MRF_SWIZZLE
    const int64_t per = n_wg / 8;
    const int64_t w = L < 8 * per ? (L % 8) * per + L / 8 : L;
#else
    const int64_t w = L;
#endif
    const int64_t P0 = (w / a.n_split) * kPixTile;
    const int64_t split = w % a.n_split;
    const int64_t kp = a.kp;
    const int n_stage = (int)(kp / kSlice);

    // running best per lane and pixel block over the entries this lane has
    // seen. A lane sees its entries in increasing order, so a later entry
    // replaces the best only with a strictly larger score (ties: lower index)
    float bs[2] = {-1.0f, -1.0f};
    int32_t bi[2] = {0x7fffffff, 0x7fffffff};

    // global -> LDS copy of a slice: kNC chunks of 16 bytes per row, kPer chunks
    // per thread and operand (chunk c = tid + 256 u: row c / kNC, part c % kNC)
    constexpr int kNC = kSlice / 8;
    constexpr int kPerA = kPixTile * kNC / kMatchWG, kPerB = kEntTile * kNC / kMatchWG;
    static_assert(kPerA * kMatchWG == kPixTile * kNC && kPerB * kMatchWG == kEntTile * kNC, "whole chunks per thread");
    const int cpart = tid % kNC;
    const int64_t t0 = split * a.tiles_per_split;
    const int64_t t1 = min(t0 + a.tiles_per_split, a.n_ent_tiles);
    for (int64_t et = t0; et < t1; ++et) {
        const int64_t E0 = et * kEntTile;
        float *wt = lw[(et - t0) & 1];
        // read after this tile's last barrier; the buffer was last read in
        // the epilogue of tile et - 2, before the barriers of tile et - 1
        if (tid < kEntTile) {
            const float v = a.inv_norm2[E0 + tid];
            wt[tid] = v < 0.0f ? -__builtin_inff() : v;
        }
        const u32x4 *ga[kPerA], *gb[kPerB];
        u32x4 ra[kPerA], rb[kPerB];
#pragma unroll
        for (int u = 0; u < kPerA; ++u) {
            ga[u] = reinterpret_cast<const u32x4 *>(a.xh + (P0 + (tid + kMatchWG * u) / kNC) * kp + 8 * cpart);
            ra[u] = ga[u][0];
        }
#pragma unroll
        for (int u = 0; u < kPerB; ++u) {  // binary16 bits
            gb[u] = reinterpret_cast<const u32x4 *>(a.dh + (E0 + (tid + kMatchWG * u) / kNC) * kp + 8 * cpart);
            rb[u] = gb[u][0];
        }
        f32x16 acc[2][2][2];  // [entry block][pixel block][re, im]
        for (int st = 0; st < n_stage; ++st) {
            const int buf = st & 1;
            _Float16 *la = ldsa[buf];
            _Float16 *lb = ldsb[buf];
#pragma unroll
            for (int u = 0; u < kPerA; ++u)
                *reinterpret_cast<u32x4 *>(la + ((tid + kMatchWG * u) / kNC) * kLdsRow + 8 * cpart) = ra[u];
#pragma unroll
            for (int u = 0; u < kPerB; ++u)
                *reinterpret_cast<u32x4 *>(lb + ((tid + kMatchWG * u) / kNC) * kLdsRow + 8 * cpart) = rb[u];
            __syncthreads();
            if (st + 1 < n_stage) {  // next slice in flight while this one is multiplied
                const int q = (st + 1) * kNC;
#pragma unroll
                for (int u = 0; u < kPerA; ++u) ra[u] = ga[u][q];
#pragma unroll
                for (int u = 0; u < kPerB; ++u) rb[u] = gb[u][q];
            }
            // the first stage starts the sums from an inline zero (no register clearing)
            if (st == 0)
                mma_slice<true>(acc, la, lb, wp, we, col, half);
            else
                mma_slice<false>(acc, la, lb, wp, we, col, half);
            // the other buffer is written next; one barrier per stage suffices
            // because stage st + 1 writes buffer buf ^ 1, last read in stage st - 1
        }
        __syncthreads();  // all reads of this tile done before the next tile's first write
        // score: this lane holds entries E0 + we + 32 i + 8 q + 4 half + t
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int eo = we + 32 * i + 8 * q + 4 * half;
                const float4 w4 = *reinterpret_cast<const float4 *>(wt + eo);
                const float ww[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int r = 4 * q + t;
                    const int32_t e = (int32_t)(E0 + eo + t);
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const float re = acc[i][j][0][r], im = acc[i][j][1][r];
                        const float sc = (re * re + im * im) * ww[t];
                        if (sc > bs[j]) {
                            bs[j] = sc;
                            bi[j] = e;
                        }
                    }
                }
            }
    }
    // the two half waves hold the same pixels (other entry rows); then one lane
    // per pixel writes the partial plane of (split, entry half of the tile)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const float os = __shfl_xor(bs[j], 32);
        const int32_t oi = __shfl_xor(bi[j], 32);
        if (better(os, oi, bs[j], bi[j])) {
            bs[j] = os;
            bi[j] = oi;
        }
    }
    if (half == 0) {
        const int64_t plane = split * kEntWaves + (wave / kPixWaves);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t o = plane * a.n_pix_pad + P0 + wp + 32 * j + col;
            a.part_score[o] = bs[j];
            a.part_idx[o] = bi[j];
        }
    }
}

// One wavefront per pixel: the best of the partial planes (any order: the
// order (score desc, index asc) is total), then <d, x> of the chosen entry
// recomputed in FP64 from the binary16 operands, in the caller's units.
__global__ __launch_bounds__(kMrfWG) void k_mrf_final(MrfArgs a, int32_t *best, double *proj) {
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * kMrfWaves + (threadIdx.x >> 6);
    if (p >= a.n_pix) return;  // uniform per wavefront
    float bsc = -1.0f;
    int32_t bid = 0x7fffffff;
    for (int64_t s = lane; s < a.n_planes; s += 64) {
        const int64_t o = s * a.n_pix_pad + p;
        if (better(a.part_score[o], a.part_idx[o], bsc, bid)) {
            bsc = a.part_score[o];
            bid = a.part_idx[o];
        }
    }
    for (int m = 1; m < 64; m <<= 1) {
        const float os = __shfl_xor(bsc, m);
        const int32_t oi = __shfl_xor(bid, m);
        if (better(os, oi, bsc, bid)) {
            bsc = os;
            bid = oi;
        }
    }
    if (bid == 0x7fffffff || bsc < 0.0f) {  // no valid entry
        if (lane == 0) {
            best[p] = -1;
            proj[2 * p] = 0.0;
            proj[2 * p + 1] = 0.0;
        }
        return;
    }
    const _Float16 *xr = reinterpret_cast<const _Float16 *>(a.xh) + p * a.kp;
    const _Float16 *dr = reinterpret_cast<const _Float16 *>(a.dh) + (int64_t)bid * a.kp;
    double sr = 0.0, si = 0.0;
    for (int64_t k = 2 * lane; k < a.kp; k += 128) {
        const double x0 = (double)xr[k], x1 = (double)xr[k + 1];
        const double d0 = (double)dr[k], d1 = (double)dr[k + 1];
        sr += d0 * x0 + d1 * x1;  // Re conj(d) x
        si += d0 * x1 - d1 * x0;  // Im conj(d) x
    }
    for (int m = 1; m < 64; m <<= 1) {
        sr += __shfl_xor(sr, m);
        si += __shfl_xor(si, m);
    }
    if (lane == 0) {
        best[p] = bid;
        const double f = sqrt((double)a.inv_norm2[bid]) * ldexp(1.0, -a.x_exp[p]);
        proj[2 * p] = sr * f;
        proj[2 * p + 1] = si * f;
    }
}

static int check_launch() { return hipGetLastError() == hipSuccess ? 0 : -1; }

int launch_mrf_pack(const float2 *src, int64_t n_rows, int64_t n_rows_pad, int64_t n_t, int64_t kp,
                    uint16_t *dst, int32_t *exps, float *inv_norm2, void *stream) {
    if (n_rows_pad <= 0) return 0;
    if (n_rows_pad > 0x7fffffff || kp < 2 * n_t || kp % 32) return -1;
    hipLaunchKernelGGL(k_mrf_pack, dim3((unsigned)n_rows_pad), dim3(kMrfWG), 0, (hipStream_t)stream, src, n_rows,
                       n_t, kp, reinterpret_cast<_Float16 *>(dst), exps, inv_norm2);
    return check_launch();
}

int launch_mrf_match(const MrfArgs &a, void *stream) {
    if (a.n_pix_pad % kPixTile || a.n_ent_tiles <= 0 || a.kp % kSlice || a.n_split <= 0 ||
        a.n_planes != kEntWaves * a.n_split)
        return -1;
    const int64_t n_wg = a.n_pix_pad / kPixTile * a.n_split;
    if (n_wg > 0x7fffffff) return -1;
    hipLaunchKernelGGL(k_mrf_match, dim3((unsigned)n_wg), dim3(kMatchWG), 0, (hipStream_t)stream, a);
    return check_launch();
}

int mrf_pix_tile() { return kPixTile; }
int mrf_ent_tile() { return kEntTile; }

int launch_mrf_final(const MrfArgs &a, int32_t *best, double *proj, void *stream) {
    if (a.n_pix <= 0) return 0;
    dim3 grid((unsigned)((a.n_pix + kMrfWaves - 1) / kMrfWaves));
    hipLaunchKernelGGL(k_mrf_final, grid, dim3(kMrfWG), 0, (hipStream_t)stream, a, best, proj);
    return check_launch();
}

}  // namespace koma
