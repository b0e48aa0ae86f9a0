// The least-squares step of Anderson acceleration (Walker & Ni 2011, type
// II): gamma = argmin |f - dF gamma|, solved through the normal equations
// (dF^T dF + ridge) gamma = dF^T f with the Gram matrix and right-hand side
// summed in double.  Shared by the adjoint iteration and the local/global
// iteration.
#pragma once

#include "device_common.h"

namespace gs {

constexpr int kAaSolveThreads = kAaMaxMem * kAaMaxMem;  // one thread per Gram entry

// Cholesky solve of the mk x mk system in A (LDS, overwritten by its factor)
// with right-hand side rhs (LDS), ridge 1e-10 times the largest diagonal
// entry: right-looking factorisation with one thread per entry, then the two
// triangular solves by wavefront 0 (one shuffle-reduced dot product per row).
// Every thread of a block of kAaSolveThreads calls it; lane j < mk of
// wavefront 0 returns gamma_j in *gj (0 when a pivot is not positive), and
// the function returns whether the factorisation succeeded (uniform).
__device__ __forceinline__ bool gram_solve(double (*A)[kAaMaxMem], const double* rhs, int mk, double* gj) {
  __shared__ int ok;
  __shared__ double ridge;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = mk > 0 ? tid / mk : 0, j = mk > 0 ? tid % mk : 0;
  const bool mine = tid < mk * mk;
  if (tid == 0) {
    double dmax = 0.0;
    for (int q = 0; q < mk; ++q) dmax = fmax(dmax, A[q][q]);
    ok = (mk > 0 && dmax > 0.0) ? 1 : 0;
    ridge = 1e-10 * dmax;
  }
  __syncthreads();
  if (mine && i == j) A[i][i] += ridge;
  __syncthreads();
  for (int kk = 0; kk < mk; ++kk) {
    if (tid == 0) {
      if (ok && A[kk][kk] > 0.0) A[kk][kk] = sqrt(A[kk][kk]);
      else ok = 0;
    }
    __syncthreads();
    if (!ok) break;
    if (tid > kk && tid < mk) A[tid][kk] /= A[kk][kk];
    __syncthreads();
    if (mine && i > kk && j > kk && j <= i) A[i][j] -= A[i][kk] * A[j][kk];
    __syncthreads();
  }
  *gj = 0.0;
  if (wave == 0 && ok) {
    // L y = rhs, then L^T gamma = y (lower triangle of A holds L); lane r
    // keeps y_r and gamma_r
    double yl = 0.0, gl = 0.0;
    for (int r = 0; r < mk; ++r) {
      double t = (lane < r) ? A[r][lane] * yl : 0.0;
      t = wave_sum(t);
      const double yr = (rhs[r] - t) / A[r][r];
      if (lane == r) yl = yr;
    }
    for (int r = mk - 1; r >= 0; --r) {
      double t = (lane > r && lane < mk) ? A[lane][r] * gl : 0.0;
      t = wave_sum(t);
      const double gr = (__shfl(yl, r, 64) - t) / A[r][r];
      if (lane == r) gl = gr;
    }
    *gj = gl;
  }
  const bool res = ok != 0;
  __syncthreads();
  return res;
}

}  // namespace gs
