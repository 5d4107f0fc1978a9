// Low-rank compression of an MRF dictionary (the paper's LRTV matching uses a
// dictionary of reduced rank 5): the leading right singular vectors of the
// dictionary D ([n_e][n_t] complex) by subspace iteration on D^H D, in FP64.
//
//   V <- orth(D^H (D V))      repeated `iters` times, p = rank + oversampling
//   T  = (D V)^H (D V)        p x p Hermitian
//   T  = U diag(lambda) U^H   cyclic complex Jacobi
//   basis = V U[:, :rank]     (descending lambda), singular values sqrt(lambda)
//
// Projection of rows onto a basis (coefficients c_j = sum_t x_t V[t][j], so
// that inner products of rows inside the span are preserved) shares the D V
// kernel. Every kernel is a plain FP64 reduction in a fixed order: results are
// reproducible run to run.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "komahip_lowrank.h"

namespace koma {

constexpr int kLrWG = 256;
constexpr int kLrMaxP = 32;

__device__ __forceinline__ double2 cmul_d(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc_d(double2 a, double2 b) {  // conj(a) b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Counter-based start block: splitmix64 of (t, j) mapped to [-1, 1).
__device__ __forceinline__ double hash_unit(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(kLrWG) void k_lr_init(double2 *v, int64_t n_t, int p) {
    const int64_t i = (int64_t)blockIdx.x * kLrWG + threadIdx.x;
    if (i >= n_t * p) return;
    v[i] = make_double2(hash_unit(2 * (uint64_t)i), hash_unit(2 * (uint64_t)i + 1));
}

// Y[r][j] = sum_t X[r][t] V[t][j]: one wavefront per row, lanes stride over t,
// a fixed butterfly over the lanes. Output FP64 (y) or complex float (yf).
template <int P>
__global__ __launch_bounds__(kLrWG) void k_lr_xv(const float2 *x, int64_t n_rows, int64_t n_t, const double2 *v,
                                                int p, double2 *y, float2 *yf) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (kLrWG / 64) + (threadIdx.x >> 6);
    if (r >= n_rows) return;  // uniform per wavefront
    double2 acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = make_double2(0.0, 0.0);
    for (int64_t t = lane; t < n_t; t += 64) {
        const float2 xf = x[r * n_t + t];
        const double2 xd = make_double2(xf.x, xf.y);
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (j < p) {
                const double2 w = v[t * p + j];
                acc[j].x += xd.x * w.x - xd.y * w.y;
                acc[j].y += xd.x * w.y + xd.y * w.x;
            }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double sx = acc[j].x, sy = acc[j].y;
        for (int m = 1; m < 64; m <<= 1) {
            sx += __shfl_xor(sx, m);
            sy += __shfl_xor(sy, m);
        }
        if (lane == 0 && j < p) {
            if (y) y[r * p + j] = make_double2(sx, sy);
            if (yf) yf[r * p + j] = make_float2((float)sx, (float)sy);
        }
    }
}

// Zpart[c][t][j] = sum over rows e of chunk c of conj(D[e][t]) Y[e][j]: one
// lane per t, rows of the chunk in order.
template <int P>
__global__ __launch_bounds__(64) void k_lr_dhy(const float2 *d, int64_t n_e, int64_t n_t, const double2 *y, int p,
                                              int64_t rows_per_chunk, double2 *zpart) {
    const int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t c = blockIdx.y;
    const int64_t e0 = c * rows_per_chunk, e1 = min(e0 + rows_per_chunk, n_e);
    double2 acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = make_double2(0.0, 0.0);
    if (t < n_t) {
        for (int64_t e = e0; e < e1; ++e) {
            const float2 df = d[e * n_t + t];
            const double2 dd = make_double2(df.x, df.y);
#pragma unroll
            for (int j = 0; j < P; ++j)
                if (j < p) {
                    const double2 yj = y[e * p + j];
                    acc[j].x += dd.x * yj.x + dd.y * yj.y;
                    acc[j].y += dd.x * yj.y - dd.y * yj.x;
                }
        }
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (j < p) zpart[(c * n_t + t) * p + j] = acc[j];
    }
}

// Z[t][j] = sum over chunks (in order) of Zpart.
__global__ __launch_bounds__(kLrWG) void k_lr_sum(const double2 *zpart, int64_t n_chunks, int64_t n, double2 *z) {
    const int64_t i = (int64_t)blockIdx.x * kLrWG + threadIdx.x;
    if (i >= n) return;
    double2 s = zpart[i];
    for (int64_t c = 1; c < n_chunks; ++c) {
        s.x += zpart[c * n + i].x;
        s.y += zpart[c * n + i].y;
    }
    z[i] = s;
}

// Sum of a value over the workgroup, every thread receives it (fixed order).
__device__ double block_sum(double v, double *red) {
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kLrWG / 64; ++i) s += red[i];
    return s;
}

// Modified Gram-Schmidt of the p columns of z ([n_t][p]) into v, one
// workgroup, each column orthogonalised twice against the earlier ones (one
// pass loses orthogonality when a column lies almost in their span, as the
// columns beyond the dictionary's numerical rank do); a column that vanishes
// is replaced by zero.
__global__ __launch_bounds__(kLrWG) void k_lr_orth(const double2 *z, int64_t n_t, int p, double2 *v) {
    __shared__ double red[kLrWG / 64];
    for (int64_t i = threadIdx.x; i < n_t * p; i += kLrWG) v[i] = z[i];
    __syncthreads();
    for (int j = 0; j < p; ++j) {
        for (int pass = 0; pass < 2; ++pass) {
            for (int i = 0; i < j; ++i) {
                double dr = 0.0, di = 0.0;
                for (int64_t t = threadIdx.x; t < n_t; t += kLrWG) {
                    const double2 pr = cmulc_d(v[t * p + i], v[t * p + j]);
                    dr += pr.x;
                    di += pr.y;
                }
                dr = block_sum(dr, red);
                di = block_sum(di, red);
                for (int64_t t = threadIdx.x; t < n_t; t += kLrWG) {
                    const double2 vi = v[t * p + i];
                    double2 &vj = v[t * p + j];
                    vj.x -= dr * vi.x - di * vi.y;
                    vj.y -= dr * vi.y + di * vi.x;
                }
                __syncthreads();
            }
        }
        double n2 = 0.0;
        for (int64_t t = threadIdx.x; t < n_t; t += kLrWG) {
            const double2 a = v[t * p + j];
            n2 += a.x * a.x + a.y * a.y;
        }
        n2 = block_sum(n2, red);
        const double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
        for (int64_t t = threadIdx.x; t < n_t; t += kLrWG) {
            double2 &a = v[t * p + j];
            a.x *= inv;
            a.y *= inv;
        }
        __syncthreads();
    }
}

// T = Y^H Y ([p][p]) and its eigen-decomposition by cyclic complex Jacobi
// (one workgroup; the Gram sums by the whole group, the rotations by one
// thread), then basis = V U[:, order] for the `rank` largest eigenvalues.
__global__ __launch_bounds__(kLrWG) void k_lr_ritz(const double2 *y, int64_t n_e, const double2 *v, int64_t n_t,
                                                  int p, int rank, int sweeps, double2 *basis, double *sv) {
    __shared__ double red[kLrWG / 64];
    __shared__ double2 T[kLrMaxP][kLrMaxP];
    __shared__ double2 U[kLrMaxP][kLrMaxP];
    __shared__ int order[kLrMaxP];
    for (int i = 0; i < p; ++i)
        for (int j = i; j < p; ++j) {
            double sr = 0.0, si = 0.0;
            for (int64_t e = threadIdx.x; e < n_e; e += kLrWG) {
                const double2 pr = cmulc_d(y[e * p + i], y[e * p + j]);
                sr += pr.x;
                si += pr.y;
            }
            sr = block_sum(sr, red);
            si = block_sum(si, red);
            if (threadIdx.x == 0) {
                T[i][j] = make_double2(sr, si);
                T[j][i] = make_double2(sr, -si);
            }
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < p; ++i)
            for (int j = 0; j < p; ++j) U[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
        for (int sw = 0; sw < sweeps; ++sw) {
            double off = 0.0;
            for (int i = 0; i < p; ++i)
                for (int j = i + 1; j < p; ++j) off += T[i][j].x * T[i][j].x + T[i][j].y * T[i][j].y;
            if (off == 0.0) break;
            for (int a = 0; a < p; ++a)
                for (int b = a + 1; b < p; ++b) {
                    const double2 tab = T[a][b];
                    const double mag = sqrt(tab.x * tab.x + tab.y * tab.y);
                    const double taa = T[a][a].x, tbb = T[b][b].x;
                    if (mag <= 1e-18 * (fabs(taa) + fabs(tbb))) {  // negligible: drop it
                        T[a][b] = make_double2(0.0, 0.0);
                        T[b][a] = make_double2(0.0, 0.0);
                        continue;
                    }
                    // unit phase e^{i phi} of T[a][b]; rotate in the plane (a, b)
                    const double er = tab.x / mag, ei = tab.y / mag;
                    const double th = 0.5 * atan2(2.0 * mag, tbb - taa);
                    const double cs = cos(th), sn = sin(th);
                    // columns: col_a' = cs col_a - sn e^{-i phi} col_b, col_b' = sn e^{i phi} col_a + cs col_b
                    for (int k = 0; k < p; ++k) {
                        const double2 ka = T[k][a], kb = T[k][b];
                        const double2 ekb = make_double2(er * kb.x + ei * kb.y, er * kb.y - ei * kb.x);  // e^{-i phi} kb
                        const double2 eka = make_double2(er * ka.x - ei * ka.y, er * ka.y + ei * ka.x);  // e^{i phi} ka
                        T[k][a] = make_double2(cs * ka.x - sn * ekb.x, cs * ka.y - sn * ekb.y);
                        T[k][b] = make_double2(sn * eka.x + cs * kb.x, sn * eka.y + cs * kb.y);
                        const double2 ua = U[k][a], ub = U[k][b];
                        const double2 eub = make_double2(er * ub.x + ei * ub.y, er * ub.y - ei * ub.x);
                        const double2 eua = make_double2(er * ua.x - ei * ua.y, er * ua.y + ei * ua.x);
                        U[k][a] = make_double2(cs * ua.x - sn * eub.x, cs * ua.y - sn * eub.y);
                        U[k][b] = make_double2(sn * eua.x + cs * ub.x, sn * eua.y + cs * ub.y);
                    }
                    // rows: the conjugate transpose of the same rotation
                    for (int k = 0; k < p; ++k) {
                        const double2 ak = T[a][k], bk = T[b][k];
                        const double2 ebk = make_double2(er * bk.x - ei * bk.y, er * bk.y + ei * bk.x);  // e^{i phi} bk
                        const double2 eak = make_double2(er * ak.x + ei * ak.y, er * ak.y - ei * ak.x);  // e^{-i phi} ak
                        T[a][k] = make_double2(cs * ak.x - sn * ebk.x, cs * ak.y - sn * ebk.y);
                        T[b][k] = make_double2(sn * eak.x + cs * bk.x, sn * eak.y + cs * bk.y);
                    }
                    T[a][b] = make_double2(0.0, 0.0);
                    T[b][a] = make_double2(0.0, 0.0);
                }
        }
        // order by descending eigenvalue (stable: lower index first on ties)
        for (int i = 0; i < p; ++i) order[i] = i;
        for (int i = 1; i < p; ++i)
            for (int j = i; j > 0 && T[order[j]][order[j]].x > T[order[j - 1]][order[j - 1]].x; --j) {
                const int tmp = order[j];
                order[j] = order[j - 1];
                order[j - 1] = tmp;
            }
        for (int k = 0; k < rank; ++k) {
            const double lam = T[order[k]][order[k]].x;
            sv[k] = lam > 0.0 ? sqrt(lam) : 0.0;
        }
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n_t * rank; i += kLrWG) {
        const int64_t t = i / rank;
        const int k = (int)(i % rank);
        const int c = order[k];
        double2 s = make_double2(0.0, 0.0);
        for (int j = 0; j < p; ++j) {
            const double2 pr = cmul_d(v[t * p + j], U[j][c]);
            s.x += pr.x;
            s.y += pr.y;
        }
        basis[t * rank + k] = s;
    }
}

static int check_launch() { return hipGetLastError() == hipSuccess ? 0 : -1; }

template <int P>
static void xv_launch(const float2 *x, int64_t n_rows, int64_t n_t, const double2 *v, int p, double2 *y, float2 *yf,
                      hipStream_t s) {
    dim3 grid((unsigned)((n_rows + 3) / 4));
    hipLaunchKernelGGL((k_lr_xv<P>), grid, dim3(kLrWG), 0, s, x, n_rows, n_t, v, p, y, yf);
}

int launch_lr_xv(const float2 *x, int64_t n_rows, int64_t n_t, const double2 *v, int p, double2 *y, float2 *yf,
                 void *stream) {
    if (n_rows <= 0) return 0;
    if (p < 1 || p > kLrMaxP || (n_rows + 3) / 4 > 0x7fffffff) return -1;
    hipStream_t s = (hipStream_t)stream;
    if (p <= 8)
        xv_launch<8>(x, n_rows, n_t, v, p, y, yf, s);
    else if (p <= 16)
        xv_launch<16>(x, n_rows, n_t, v, p, y, yf, s);
    else
        xv_launch<32>(x, n_rows, n_t, v, p, y, yf, s);
    return check_launch();
}

int launch_lr_iter(const float2 *d, int64_t n_e, int64_t n_t, int p, int iters, double2 *v, double2 *y,
                   double2 *zpart, int64_t n_chunks, double2 *z, void *stream) {
    if (p < 1 || p > kLrMaxP || n_chunks < 1 || n_chunks > 65535) return -1;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = n_t * p;
    hipLaunchKernelGGL(k_lr_init, dim3((unsigned)((n + kLrWG - 1) / kLrWG)), dim3(kLrWG), 0, s, z, n_t, p);
    hipLaunchKernelGGL(k_lr_orth, dim3(1), dim3(kLrWG), 0, s, z, n_t, p, v);
    const int64_t rpc = (n_e + n_chunks - 1) / n_chunks;
    dim3 gd((unsigned)((n_t + 63) / 64), (unsigned)n_chunks);
    for (int it = 0; it < iters; ++it) {
        if (launch_lr_xv(d, n_e, n_t, v, p, y, nullptr, stream) != 0) return -1;
        if (p <= 8)
            hipLaunchKernelGGL((k_lr_dhy<8>), gd, dim3(64), 0, s, d, n_e, n_t, y, p, rpc, zpart);
        else if (p <= 16)
            hipLaunchKernelGGL((k_lr_dhy<16>), gd, dim3(64), 0, s, d, n_e, n_t, y, p, rpc, zpart);
        else
            hipLaunchKernelGGL((k_lr_dhy<32>), gd, dim3(64), 0, s, d, n_e, n_t, y, p, rpc, zpart);
        hipLaunchKernelGGL(k_lr_sum, dim3((unsigned)((n + kLrWG - 1) / kLrWG)), dim3(kLrWG), 0, s, zpart, n_chunks, n,
                           z);
        hipLaunchKernelGGL(k_lr_orth, dim3(1), dim3(kLrWG), 0, s, z, n_t, p, v);
        if (check_launch() != 0) return -1;
    }
    return launch_lr_xv(d, n_e, n_t, v, p, y, nullptr, stream);
}

int launch_lr_ritz(const double2 *y, int64_t n_e, const double2 *v, int64_t n_t, int p, int rank, double2 *basis,
                   double *sv, void *stream) {
    if (p < 1 || p > kLrMaxP || rank < 1 || rank > p) return -1;
    hipLaunchKernelGGL(k_lr_ritz, dim3(1), dim3(kLrWG), 0, (hipStream_t)stream, y, n_e, v, n_t, p, rank, 30, basis,
                       sv);
    return check_launch();
}

}  // namespace koma
