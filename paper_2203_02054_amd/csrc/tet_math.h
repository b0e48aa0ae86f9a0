// Per-tet algebra of the local step (Section III-A), shared by the local-step
// kernels and their adjoint: the Kabsch rotation (signed SVD from cyclic
// Jacobi on M^T M and a sorted-column Givens QR, the structure of McAdams et
// al. 2011 with exact Jacobi angles and a fixed sweep count), the target of
// one tet, and the gather of a tet's rest and current shapes.
#pragma once

#include "device_common.h"

namespace gs {

template <typename R> struct Sweeps;
template <> struct Sweeps<float> { static constexpr int n = 5; };
template <> struct Sweeps<double> { static constexpr int n = 7; };

template <typename R> __device__ __forceinline__ R rsq(R v);
template <> __device__ __forceinline__ float rsq<float>(float v) { return sqrtf(v); }
template <> __device__ __forceinline__ double rsq<double>(double v) { return sqrt(v); }
template <typename R> __device__ __forceinline__ R cbrt_(R v);
template <> __device__ __forceinline__ float cbrt_<float>(float v) { return cbrtf(v); }
template <> __device__ __forceinline__ double cbrt_<double>(double v) { return cbrt(v); }

// One Jacobi rotation zeroing S[P][Q] of the symmetric S; V <- V J.
template <typename R, int P, int Q>
__device__ __forceinline__ void jacobi_rot(R (&S)[3][3], R (&V)[3][3]) {
  constexpr int K = 3 - P - Q;
  const R apq = S[P][Q];
  if (apq == R(0)) return;
  const R tau = (S[Q][Q] - S[P][P]) / (R(2) * apq);
  const R t = (tau >= R(0) ? R(1) : R(-1)) / (fabs(tau) + rsq<R>(R(1) + tau * tau));
  const R c = R(1) / rsq<R>(R(1) + t * t);
  const R s = t * c;
  const R skp = c * S[K][P] - s * S[K][Q];
  const R skq = s * S[K][P] + c * S[K][Q];
  S[P][P] = S[P][P] - t * apq;
  S[Q][Q] = S[Q][Q] + t * apq;
  S[P][Q] = S[Q][P] = R(0);
  S[K][P] = S[P][K] = skp;
  S[K][Q] = S[Q][K] = skq;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R vp = V[k][P], vq = V[k][Q];
    V[k][P] = c * vp - s * vq;
    V[k][Q] = s * vp + c * vq;
  }
}

template <typename R, int A, int B>
__device__ __forceinline__ void swap_cols_neg(R (&Bm)[3][3], R (&V)[3][3], R (&nrm)[3]) {
  // swap columns A and B and negate the new column B (keeps det V = +1)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R t = Bm[k][A];
    Bm[k][A] = Bm[k][B];
    Bm[k][B] = -t;
    t = V[k][A];
    V[k][A] = V[k][B];
    V[k][B] = -t;
  }
  R t = nrm[A];
  nrm[A] = nrm[B];
  nrm[B] = t;
}

// Givens rotation on rows I, J of Bm zeroing Bm[J][C]; Q <- Q G^T.
template <typename R, int I, int J, int C>
__device__ __forceinline__ void givens(R (&Bm)[3][3], R (&Q)[3][3]) {
  const R a = Bm[I][C], b = Bm[J][C];
  const R r = rsq<R>(a * a + b * b);
  if (r == R(0)) return;
  const R c = a / r, s = b / r;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R bi = Bm[I][k], bj = Bm[J][k];
    Bm[I][k] = c * bi + s * bj;
    Bm[J][k] = -s * bi + c * bj;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R qi = Q[k][I], qj = Q[k][J];
    Q[k][I] = c * qi + s * qj;
    Q[k][J] = -s * qi + c * qj;
  }
}

// Kabsch rotation maximising tr(Rot^T M).
template <typename R>
__device__ __forceinline__ void kabsch(const R (&M)[3][3], R (&Rot)[3][3]) {
  R S[3][3], V[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      S[i][j] = M[0][i] * M[0][j] + M[1][i] * M[1][j] + M[2][i] * M[2][j];
      V[i][j] = (i == j) ? R(1) : R(0);
    }
#pragma unroll
  for (int sw = 0; sw < Sweeps<R>::n; ++sw) {
    jacobi_rot<R, 0, 1>(S, V);
    jacobi_rot<R, 0, 2>(S, V);
    jacobi_rot<R, 1, 2>(S, V);
  }
  R Bm[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Bm[i][j] = M[i][0] * V[0][j] + M[i][1] * V[1][j] + M[i][2] * V[2][j];
  R nrm[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) nrm[j] = Bm[0][j] * Bm[0][j] + Bm[1][j] * Bm[1][j] + Bm[2][j] * Bm[2][j];
  if (nrm[0] < nrm[1]) swap_cols_neg<R, 0, 1>(Bm, V, nrm);
  if (nrm[0] < nrm[2]) swap_cols_neg<R, 0, 2>(Bm, V, nrm);
  if (nrm[1] < nrm[2]) swap_cols_neg<R, 1, 2>(Bm, V, nrm);
  R Q[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Q[i][j] = (i == j) ? R(1) : R(0);
  givens<R, 0, 1, 0>(Bm, Q);
  givens<R, 0, 2, 0>(Bm, Q);
  givens<R, 1, 2, 1>(Bm, Q);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Rot[i][j] = Q[i][0] * V[j][0] + Q[i][1] * V[j][1] + Q[i][2] * V[j][2];
}

template <typename R>
__device__ __forceinline__ R det3(const R (&A)[3][3]) {
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

template <typename R>
using V4 = W4<R>;

// Target shape of one tet.  P: centred rest shape, D: centred current shape,
// Dminv: inverse rest edge matrix, vol: rest volume.
template <typename R>
__device__ __forceinline__ void tet_target(int mode, R a, const R (&P)[3][4], const R (&D)[3][4],
                                           const R (&Dminv)[3][3], R vol, const Consts& c, R (&Tt)[3][4]) {
  R sc[3];
  const R s_iso = (mode == GS_CH_ISO) ? cbrt_<R>(a) : R(1);
  sc[0] = (mode == GS_CH_AX_X) ? a : s_iso;
  sc[1] = (mode == GS_CH_AX_Y) ? a : s_iso;
  sc[2] = (mode == GS_CH_AX_Z) ? a : s_iso;
  R Q[3][4];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) Q[k][j] = sc[k] * P[k][j];
  R M[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[i][k] = D[i][0] * Q[k][0] + D[i][1] * Q[k][1] + D[i][2] * Q[k][2] + D[i][3] * Q[k][3];
  R Rot[3][3];
  kabsch<R>(M, Rot);
  R RQ[3][4];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) RQ[i][j] = Rot[i][0] * Q[0][j] + Rot[i][1] * Q[1][j] + Rot[i][2] * Q[2][j];
  if (mode != GS_BODY) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) Tt[i][j] = RQ[i][j];
    return;
  }
  // body element: Mooney-Rivlin blend (Eq. 6) and volume scaling (Eq. 7)
  R Ds[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Ds[i][j] = D[i][j + 1] - D[i][0];
  R F[3][3];
  R I1 = R(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      F[i][j] = Ds[i][0] * Dminv[0][j] + Ds[i][1] * Dminv[1][j] + Ds[i][2] * Dminv[2][j];
      I1 += F[i][j] * F[i][j];
    }
  const R J = det3<R>(F);
  R w = R(1);
  if (c.hyper) {
    const R lam = (J > R(0)) ? rsq<R>(I1 / (R(3) * cbrt_<R>(J * J))) : R(1);
    const R il = R(1) / lam;
    const R c1 = (R)c.c1, c2 = (R)c.c2;
    w = (R(1) + il + il * il) * (c1 + c2 * il) / (R(3) * (c1 + c2));
  }
  R B[3][4];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) B[i][j] = (R(1) - w) * D[i][j] + w * RQ[i][j];
  R Be[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Be[i][j] = B[i][j + 1] - B[i][0];
  const R VB = det3<R>(Be) / R(6);
  if (VB > R(0)) {
    const R s = cbrt_<R>(vol / VB);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) Tt[i][j] = s * B[i][j];
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) Tt[i][j] = RQ[i][j];
  }
}

// Gather one tet: centred rest shape P, centred current shape D (both
// centred in double), inverse rest edge matrix and rest volume.
template <typename R, bool FROM_X>
__device__ __forceinline__ void load_tet(const Dev<R>& d, const Consts& c, int e, const R* __restrict__ xin,
                                         int (&vi)[4], R (&P)[3][4], R (&D)[3][4], R (&Dminv)[3][3], double& vol) {
  double X[3][4], x[3][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) vi[j] = d.tets[j * c.T + e];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      X[k][j] = d.X0[(size_t)k * c.n + vi[j]];
      if (FROM_X)
        x[k][j] = (double)xin[(size_t)k * c.n + vi[j]];
      else
        x[k][j] = X[k][j] + (double)d.u[(size_t)k * c.n + vi[j]];
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double mX = ((X[k][0] + X[k][1]) + (X[k][2] + X[k][3])) * 0.25;
    const double mx = ((x[k][0] + x[k][1]) + (x[k][2] + x[k][3])) * 0.25;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      P[k][j] = (R)(X[k][j] - mX);
      D[k][j] = (R)(x[k][j] - mx);
    }
  }
  double Dm[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j) Dm[k][j] = X[k][j + 1] - X[k][0];
  const double det = det3<double>(Dm);
  vol = det / 6.0;
  const double id = 1.0 / det;
  Dminv[0][0] = (R)((Dm[1][1] * Dm[2][2] - Dm[1][2] * Dm[2][1]) * id);
  Dminv[0][1] = (R)((Dm[0][2] * Dm[2][1] - Dm[0][1] * Dm[2][2]) * id);
  Dminv[0][2] = (R)((Dm[0][1] * Dm[1][2] - Dm[0][2] * Dm[1][1]) * id);
  Dminv[1][0] = (R)((Dm[1][2] * Dm[2][0] - Dm[1][0] * Dm[2][2]) * id);
  Dminv[1][1] = (R)((Dm[0][0] * Dm[2][2] - Dm[0][2] * Dm[2][0]) * id);
  Dminv[1][2] = (R)((Dm[0][2] * Dm[1][0] - Dm[0][0] * Dm[1][2]) * id);
  Dminv[2][0] = (R)((Dm[1][0] * Dm[2][1] - Dm[1][1] * Dm[2][0]) * id);
  Dminv[2][1] = (R)((Dm[0][1] * Dm[2][0] - Dm[0][0] * Dm[2][1]) * id);
  Dminv[2][2] = (R)((Dm[0][0] * Dm[1][1] - Dm[0][1] * Dm[1][0]) * id);
}

}  // namespace gs
