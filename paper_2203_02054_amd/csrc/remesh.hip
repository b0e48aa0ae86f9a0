// Remesh checks of Section III-B (Algorithm 1's outer loop): after a stage
// of the progressive actuation, every chamber element is tested for a volume
// gain above alpha_max against its reference shape, and for a distortion
// norm(Sigma) above d_max, Sigma being the singular values of the affine map
// taking the deformed element back onto the reference one.  That map is the
// inverse of the deformation gradient F = D_x D_ref^-1 (D: the three edges
// from the first vertex), so norm(Sigma) (its 2-norm) is 1 / sigma_min(F).
//
// One thread per tet; both decisions are taken in FP64 from the positions as
// stored (FP32 positions are widened exactly).  sigma_min(F)^2 is the
// smallest eigenvalue of F^T F, found by cyclic Jacobi sweeps.  The kernel is
// a streaming gather: 16 B of vertex ids, 4 B of tag and 8 positions of 12 or
// 24 B per tet in, one byte out.
#include "tet_math.h"

namespace gs {

__global__ void k_zero_count(int* count) { *count = 0; }

template <typename R>
__global__ __launch_bounds__(kBlock) void k_remesh_flags(Dev<R> d, Consts c, const R* __restrict__ x,
                                                         const R* __restrict__ xref, double amax, double dmax,
                                                         uint8_t* __restrict__ flags, int* __restrict__ count) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  int f = 0;
  if (e < c.T) {
    if ((d.tag[e] & 7) != GS_BODY) {
      const size_t n = (size_t)c.n;
      int vi[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) vi[j] = d.tets[j * c.T + e];
      double Dx[3][3], Dr[3][3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double x0 = (double)x[k * n + vi[0]];
        const double r0 = xref ? (double)xref[k * n + vi[0]] : d.X0[k * n + vi[0]];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          Dx[k][j] = (double)x[k * n + vi[j + 1]] - x0;
          Dr[k][j] = (xref ? (double)xref[k * n + vi[j + 1]] : d.X0[k * n + vi[j + 1]]) - r0;
        }
      }
      const double dx = det3<double>(Dx), dr = det3<double>(Dr);
      const double ratio = dx / dr;
      // D_ref^-1 = adj(D_ref) / det(D_ref)
      double Ai[3][3];
      Ai[0][0] = Dr[1][1] * Dr[2][2] - Dr[1][2] * Dr[2][1];
      Ai[0][1] = Dr[0][2] * Dr[2][1] - Dr[0][1] * Dr[2][2];
      Ai[0][2] = Dr[0][1] * Dr[1][2] - Dr[0][2] * Dr[1][1];
      Ai[1][0] = Dr[1][2] * Dr[2][0] - Dr[1][0] * Dr[2][2];
      Ai[1][1] = Dr[0][0] * Dr[2][2] - Dr[0][2] * Dr[2][0];
      Ai[1][2] = Dr[0][2] * Dr[1][0] - Dr[0][0] * Dr[1][2];
      Ai[2][0] = Dr[1][0] * Dr[2][1] - Dr[1][1] * Dr[2][0];
      Ai[2][1] = Dr[0][1] * Dr[2][0] - Dr[0][0] * Dr[2][1];
      Ai[2][2] = Dr[0][0] * Dr[1][1] - Dr[0][1] * Dr[1][0];
      const double id = 1.0 / dr;
      double F[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) F[i][j] = (Dx[i][0] * Ai[0][j] + Dx[i][1] * Ai[1][j] + Dx[i][2] * Ai[2][j]) * id;
      double S[3][3], V[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          S[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
          V[i][j] = (i == j) ? 1.0 : 0.0;
        }
      for (int sw = 0; sw < 10; ++sw) {
        jacobi_rot<double, 0, 1>(S, V);
        jacobi_rot<double, 0, 2>(S, V);
        jacobi_rot<double, 1, 2>(S, V);
      }
      const double lmin = fmin(S[0][0], fmin(S[1][1], S[2][2]));
      const double dist = 1.0 / sqrt(fmax(lmin, 0.0));
      f = (ratio > amax ? 1 : 0) | (dist > dmax ? 2 : 0);
    }
    flags[e] = (uint8_t)f;
  }
  const int nb = __syncthreads_count(f != 0);
  if (threadIdx.x == 0 && nb) atomicAdd(count, nb);
}

template <typename R>
hipError_t launch_remesh_flags(const Dev<R>& d, const Consts& c, const R* x, const R* xref, double amax,
                               double dmax, uint8_t* flags, int* count, hipStream_t s) {
  k_zero_count<<<1, 1, 0, s>>>(count);
  k_remesh_flags<R><<<(c.T + kBlock - 1) / kBlock, kBlock, 0, s>>>(d, c, x, xref, amax, dmax, flags, count);
  return hipGetLastError();
}

template hipError_t launch_remesh_flags<float>(const Dev<float>&, const Consts&, const float*, const float*, double,
                                               double, uint8_t*, int*, hipStream_t);
template hipError_t launch_remesh_flags<double>(const Dev<double>&, const Consts&, const double*, const double*,
                                                double, double, uint8_t*, int*, hipStream_t);

}  // namespace gs
