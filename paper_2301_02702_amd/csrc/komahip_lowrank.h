// Internal launchers of the dictionary compression kernels
// (komahip_lowrank.hip). Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace koma {

// Y[r][j] = sum_t X[r][t] V[t][j] (X complex float [n_rows][n_t], V [n_t][p]);
// into y (FP64) and/or yf (complex float), either may be null. p <= 32.
int launch_lr_xv(const float2 *x, int64_t n_rows, int64_t n_t, const double2 *v, int p, double2 *y, float2 *yf,
                 void *stream);
// Subspace iteration: v <- orth(D^H D v) `iters` times from a fixed start
// block, then y = D v. Scratch: zpart [n_chunks][n_t][p], z [n_t][p].
int launch_lr_iter(const float2 *d, int64_t n_e, int64_t n_t, int p, int iters, double2 *v, double2 *y,
                   double2 *zpart, int64_t n_chunks, double2 *z, void *stream);
// Rayleigh-Ritz: eigen-pairs of y^H y, basis = v U[:, :rank] by descending
// eigenvalue, sv = sqrt(eigenvalues).
int launch_lr_ritz(const double2 *y, int64_t n_e, const double2 *v, int64_t n_t, int p, int rank, double2 *basis,
                   double *sv, void *stream);

}  // namespace koma
