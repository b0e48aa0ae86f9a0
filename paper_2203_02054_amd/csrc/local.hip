// Local step (Section III-A): per-tet target shapes and the element residual
// columns omega_e (T_e - D_e) of the correction system.
//
// One thread per tet.  Vertex data are gathered from SoA arrays (positions in
// double for the centring, then the 3x3 algebra in R = float or double).  The
// rotation is the Kabsch fit of the target's rest-frame shape Q to the current
// centred shape D (below Eq. 1): the signed SVD M = D Q^T = U S V^T with U, V
// proper rotations (the smallest singular value carries the sign of det M)
// gives R = U V^T.  V comes from cyclic Jacobi on M^T M, U from a Givens QR of
// M V with columns sorted by norm (the structure of McAdams et al. 2011, here
// with exact Jacobi angles and a fixed sweep count).
#include "tet_math.h"
#include "tet_query.h"

namespace gs {

// Local step of tet e: its residual columns, scattered to the incidence
// slots; returns its term of the elastic part of Eq. (9).
template <typename R>
__device__ __forceinline__ double local_one(const Dev<R>& d, const Consts& c, const R* __restrict__ alpha, int e) {
  const int m = d.tmesh[e];
  V4<R>* res = reinterpret_cast<V4<R>*>(d.res4);
  double eloc = 0.0;
  if (mesh_frozen(d, c.mask_done, m)) {
    // a converged mesh of a batch: no residual, so its correction stays zero
    V4<R> z;
    z.x = z.y = z.z = z.w = R(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) res[d.inc_pos[j * c.T + e]] = z;
  } else {
    int vi[4];
    R P[3][4], D[3][4], Dminv[3][3];
    double vol;
    load_tet<R, false>(d, c, e, nullptr, vi, P, D, Dminv, vol);
    const int tag = d.tag[e];
    const int mode = tag & 7, ch = tag >> 3;
    const R a = (mode != GS_BODY) ? alpha[ch] : R(1);
    R Tt[3][4];
    tet_target<R>(mode, a, P, D, Dminv, (R)vol, c, Tt);
    const R om = (R)(vol * d.mesh[m].inv_mean_vol);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const R r0 = Tt[0][j] - D[0][j], r1 = Tt[1][j] - D[1][j], r2 = Tt[2][j] - D[2][j];
      V4<R> v;
      v.x = om * r0;
      v.y = om * r1;
      v.z = om * r2;
      v.w = R(0);
      res[d.inc_pos[j * c.T + e]] = v;
      eloc += (double)om * ((double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2);
    }
  }
  return eloc;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_local(Dev<R> d, Consts c, const R* __restrict__ alpha) {
  __shared__ double lds[kBlock / 64];
  if (is_done(d.st)) return;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  const double eloc = e < c.T ? local_one(d, c, alpha, e) : 0.0;
  const double bs = block_sum<kBlock>(eloc, lds);
  if (threadIdx.x == 0) d.part_a[blockIdx.x] = bs;
}

// Local step and tet query in one launch for meshes below kTetQueryWide tets
// (both read only the iteration's positions).  A workgroup takes 64 tets;
// wavefronts 0-2 share their queries (wavefront w: the cells i = w mod 3),
// wavefront 3 runs their local steps, so the two kinds of work run side by
// side on the compute unit instead of one after the other in every lane.
// The energy partials are per workgroup.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_query_local(Dev<R> d, Consts c, const R* __restrict__ alpha) {
  static_assert(kBlock == 256, "four wavefronts per workgroup");
  __shared__ double lds[kBlock / 64];
  if (is_done(d.st)) return;
  const int wv = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + (int)(threadIdx.x & 63);
  double eloc = 0.0;
  if (wv == 3) {
    if (e < c.T) eloc = local_one(d, c, alpha, e);
  } else {
    tet_query_part<R, false, true>(d, c, e, wv, 3);
  }
  // the energy reduction after both kinds of work (a barrier before the
  // query would hold it behind the local steps)
  const double bs = block_sum<kBlock>(eloc, lds);
  if (threadIdx.x == 0) d.part_a[blockIdx.x] = bs;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_local_debug(Dev<R> d, Consts c, const R* __restrict__ alpha,
                                                         const R* __restrict__ xin, R* __restrict__ tout) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= c.T) return;
  int vi[4];
  R P[3][4], D[3][4], Dminv[3][3];
  double vol;
  load_tet<R, true>(d, c, e, xin, vi, P, D, Dminv, vol);
  const int tag = d.tag[e];
  const int mode = tag & 7, ch = tag >> 3;
  const R a = (mode != GS_BODY) ? alpha[ch] : R(1);
  R Tt[3][4];
  tet_target<R>(mode, a, P, D, Dminv, (R)vol, c, Tt);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) tout[(size_t)(k * 4 + j) * c.T + e] = Tt[k][j];
}

template <typename R>
hipError_t launch_local(const Dev<R>& d, const Consts& c, const R* alpha, hipStream_t s) {
  k_local<R><<<cdiv(c.T, kBlock), kBlock, 0, s>>>(d, c, alpha);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_query_local(const Dev<R>& d, const Consts& c, const R* alpha, hipStream_t s) {
  k_query_local<R><<<cdiv(c.T * TetQueryLanes<true>::n, kBlock), kBlock, 0, s>>>(d, c, alpha);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_local_debug(const Dev<R>& d, const Consts& c, const R* alpha, const R* x, R* targets,
                              hipStream_t s) {
  k_local_debug<R><<<cdiv(c.T, kBlock), kBlock, 0, s>>>(d, c, alpha, x, targets);
  return hipGetLastError();
}

template hipError_t launch_local<float>(const Dev<float>&, const Consts&, const float*, hipStream_t);
template hipError_t launch_local<double>(const Dev<double>&, const Consts&, const double*, hipStream_t);
template hipError_t launch_query_local<float>(const Dev<float>&, const Consts&, const float*, hipStream_t);
template hipError_t launch_query_local<double>(const Dev<double>&, const Consts&, const double*, hipStream_t);
template hipError_t launch_local_debug<float>(const Dev<float>&, const Consts&, const float*, const float*, float*,
                                              hipStream_t);
template hipError_t launch_local_debug<double>(const Dev<double>&, const Consts&, const double*, const double*,
                                               double*, hipStream_t);

}  // namespace gs
