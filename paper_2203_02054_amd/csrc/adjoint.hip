// Implicit adjoint of the converged local/global iteration: the gradient of a
// loss L(x) w.r.t. the per-chamber volume ratios alpha.
//
// At a fixed point x of x = M^-1 b(x, alpha) (Section III-B, M = A_el +
// springs, b = element targets of Section III-A plus spring targets of
// Section II-C) with the contact set held fixed, the implicit function
// theorem gives dL/dalpha = (db/dalpha)^T mu with (M - db/dx)^T mu = dL/dx.
// mu is found by the fixed-point iteration mu <- M^-1 (g + (db/dx)^T mu),
// written in correction form exactly like the forward solve: each iteration
// gathers r = g + (db/dx)^T mu - M mu and solves M d = r with the same
// warm-started Jacobi-CG kernel (mu += d); a mesh is done once
// max|d| <= tol max|mu|.  The iteration contracts at the rate of the forward
// local/global map (the same operator, transposed).
//
// (db/dx)^T mu is assembled from per-tet vector-Jacobian products (one thread
// per tet, written in incidence order and gathered per vertex like the
// forward residual) and per-contact ones:
//   chamber tet   T = R Q                      (R: Kabsch fit of Q to D)
//   body tet      T = s B, B = (1 - w) D + w R P, s = (Vol / Vol(B))^(1/3),
//                 w = R_w(lambda(F)) (Eq. 6, Eq. 7)
//   rotation      polar derivative: with S = R^T M, dR = R [w]x where
//                 (tr(S) I - S) w = vee(R^T dM - dM^T R); its adjoint maps
//                 Rbar to Mbar = R [z]x, z = (tr(S) I - S)^-1 axial(R^T Rbar)
//   sphere/plane  closed-form targets (per vertex, in the gather)
//   self contact  given a new target this iteration: c = x_v + (t + eps) d,
//                 d = -n_v/|n_v|, t the Moller-Trumbore distance to the hit
//                 face (per contact, scattered as fixed-point integers, so the
//                 sums do not depend on the order of the atomic adds: the few
//                 such contacts touch the vertex, its boundary-face ring and
//                 the hit face's vertices); kept self contacts are constant.
#include "anderson.h"
#include "tet_math.h"

namespace gs {

// z = (tr(S) I - S)^-1 a for symmetric S (cofactor inverse; the matrix is
// positive definite for a proper polar factor, its eigenvalues being the
// sums of pairs of singular values).  For a reflected element the signed
// singular values make one eigenvalue sigma_2 - sigma_3, zero when the two
// smallest singular values are equal: the rotation is then not
// differentiable, and where |det| falls below a relative 1e-12 (1e-6 in
// FP32) of tr(S)^3 its derivative is taken as zero (Mbar = 0) rather than
// dividing by the vanishing determinant.
template <typename R>
__device__ __forceinline__ void polar_adjoint(const R (&Rot)[3][3], const R (&M)[3][3], const R (&Rbar)[3][3],
                                              R (&Mbar)[3][3]) {
  R S[3][3], A[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      S[i][j] = Rot[0][i] * M[0][j] + Rot[1][i] * M[1][j] + Rot[2][i] * M[2][j];
      A[i][j] = Rot[0][i] * Rbar[0][j] + Rot[1][i] * Rbar[1][j] + Rot[2][i] * Rbar[2][j];
    }
  const R tr = S[0][0] + S[1][1] + S[2][2];
  R K[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) K[i][j] = (i == j ? tr : R(0)) - R(0.5) * (S[i][j] + S[j][i]);
  const R a[3] = {A[2][1] - A[1][2], A[0][2] - A[2][0], A[1][0] - A[0][1]};
  const R c00 = K[1][1] * K[2][2] - K[1][2] * K[2][1], c01 = K[1][2] * K[2][0] - K[1][0] * K[2][2],
          c02 = K[1][0] * K[2][1] - K[1][1] * K[2][0];
  const R c11 = K[0][0] * K[2][2] - K[0][2] * K[2][0], c12 = K[0][1] * K[2][0] - K[0][0] * K[2][1];
  const R c22 = K[0][0] * K[1][1] - K[0][1] * K[1][0];
  const R det = K[0][0] * c00 + K[0][1] * c01 + K[0][2] * c02;
  const R guard = (sizeof(R) == 4 ? R(1e-6) : R(1e-12)) * fabs(tr * tr * tr);
  if (!(fabs(det) > guard)) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Mbar[i][j] = R(0);
    return;
  }
  const R id = R(1) / det;
  // K symmetric: its inverse is the symmetric cofactor matrix over det
  const R z0 = (c00 * a[0] + c01 * a[1] + c02 * a[2]) * id;
  const R z1 = (c01 * a[0] + c11 * a[1] + c12 * a[2]) * id;
  const R z2 = (c02 * a[0] + c12 * a[1] + c22 * a[2]) * id;
  // Mbar = Rot [z]x
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Mbar[i][0] = Rot[i][1] * z2 - Rot[i][2] * z1;
    Mbar[i][1] = -Rot[i][0] * z2 + Rot[i][2] * z0;
    Mbar[i][2] = Rot[i][0] * z1 - Rot[i][1] * z0;
  }
}

// Cofactor matrix of A (d det A = <cof A, dA>).
template <typename R>
__device__ __forceinline__ void cofactor(const R (&A)[3][3], R (&C)[3][3]) {
  C[0][0] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  C[0][1] = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  C[0][2] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  C[1][0] = A[0][2] * A[2][1] - A[0][1] * A[2][2];
  C[1][1] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
  C[1][2] = A[0][1] * A[2][0] - A[0][0] * A[2][1];
  C[2][0] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
  C[2][1] = A[0][2] * A[1][0] - A[0][0] * A[1][2];
  C[2][2] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
}

// Vector-Jacobian product of one tet's target: given Tbar = MU (3x4, centred),
// Xbar = (dT/dD)^T MU composed with the centring (3x4, centred) and, for a
// chamber tet, ga = <MU, dT/dalpha>.  Recomputes the forward quantities in
// the same order as tet_target.
template <typename R>
__device__ __forceinline__ void tet_vjp(int mode, R a, const R (&P)[3][4], const R (&D)[3][4],
                                        const R (&Dminv)[3][3], R vol, const Consts& c, const R (&MU)[3][4],
                                        R (&Xbar)[3][4], R& ga) {
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
  R Dbar[3][4], Rbar[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) Dbar[i][j] = R(0);
  ga = R(0);
  R direct[3] = {R(0), R(0), R(0)};  // chamber: <(R^T MU)[k,:], P[k,:]>
  if (mode != GS_BODY) {
    // T = R Q: Rbar = MU Q^T
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        Rbar[i][k] = MU[i][0] * Q[k][0] + MU[i][1] * Q[k][1] + MU[i][2] * Q[k][2] + MU[i][3] * Q[k][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R acc = R(0);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc += (Rot[0][k] * MU[0][j] + Rot[1][k] * MU[1][j] + Rot[2][k] * MU[2][j]) * P[k][j];
      direct[k] = acc;
    }
  } else {
    R RQ[3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) RQ[i][j] = Rot[i][0] * Q[0][j] + Rot[i][1] * Q[1][j] + Rot[i][2] * Q[2][j];
    R Ds[3][3], F[3][3];
    R I1 = R(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Ds[i][j] = D[i][j + 1] - D[i][0];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        F[i][j] = Ds[i][0] * Dminv[0][j] + Ds[i][1] * Dminv[1][j] + Ds[i][2] * Dminv[2][j];
        I1 += F[i][j] * F[i][j];
      }
    const R J = det3<R>(F);
    R w = R(1), lam = R(1);
    const bool dlam = c.hyper && J > R(0);
    if (c.hyper) {
      lam = (J > R(0)) ? rsq<R>(I1 / (R(3) * cbrt_<R>(J * J))) : R(1);
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
      // T = s B, s = (vol / VB)^(1/3): Bbar = s MU + <MU, B> ds/dB
      const R s = cbrt_<R>(vol / VB);
      R mb = R(0);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) mb += MU[i][j] * B[i][j];
      const R coef = -s * mb / (R(18) * VB);  // ds = -(s / (3 VB)) dVB, dVB = <cof Be, dBe> / 6
      R Cb[3][3];
      cofactor<R>(Be, Cb);
      R Bbar[3][4];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        R acc = R(0);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          Bbar[i][j + 1] = s * MU[i][j + 1] + coef * Cb[i][j];
          acc += coef * Cb[i][j];
        }
        Bbar[i][0] = s * MU[i][0] - acc;
      }
      // B = (1 - w) D + w R Q
      R wbar = R(0);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          Dbar[i][j] += (R(1) - w) * Bbar[i][j];
          wbar += Bbar[i][j] * (RQ[i][j] - D[i][j]);
        }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          Rbar[i][k] = w * (Bbar[i][0] * Q[k][0] + Bbar[i][1] * Q[k][1] + Bbar[i][2] * Q[k][2] + Bbar[i][3] * Q[k][3]);
      if (dlam) {
        // w(lambda), lambda = sqrt(I1 J^(-2/3) / 3)
        const R il = R(1) / lam;
        const R c1 = (R)c.c1, c2 = (R)c.c2;
        const R dw_dil = ((R(1) + R(2) * il) * (c1 + c2 * il) + (R(1) + il + il * il) * c2) / (R(3) * (c1 + c2));
        const R lbar = wbar * dw_dil * (-il * il);
        const R jm23 = R(1) / cbrt_<R>(J * J);
        const R cf = lbar * jm23 / (R(6) * lam);
        R Cf[3][3];
        cofactor<R>(F, Cf);
        const R t = R(2) * I1 / (R(3) * J);
        R Fbar[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) Fbar[i][j] = cf * (R(2) * F[i][j] - t * Cf[i][j]);
        // F = Ds Dm^-1: Dsbar = Fbar Dm^-T; Ds[:, j] = D[:, j+1] - D[:, 0]
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          R acc = R(0);
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const R v = Fbar[i][0] * Dminv[j][0] + Fbar[i][1] * Dminv[j][1] + Fbar[i][2] * Dminv[j][2];
            Dbar[i][j + 1] += v;
            acc += v;
          }
          Dbar[i][0] -= acc;
        }
      }
    } else {
      // inverted blend: T = R P
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          Rbar[i][k] = MU[i][0] * Q[k][0] + MU[i][1] * Q[k][1] + MU[i][2] * Q[k][2] + MU[i][3] * Q[k][3];
    }
  }
  // rotation: M = D Q^T, Dbar += Mbar Q
  R Mbar[3][3];
  polar_adjoint<R>(Rot, M, Rbar, Mbar);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) Dbar[i][j] += Mbar[i][0] * Q[0][j] + Mbar[i][1] * Q[1][j] + Mbar[i][2] * Q[2][j];
  if (mode != GS_BODY) {
    // dT/dalpha = dR Q + R dQ, dQ = diag(dsc) P: <MU, R dQ> + <dQ, Mbar^T D>
    R ds[3];
    const R diso = (mode == GS_CH_ISO) ? s_iso / (R(3) * a) : R(0);
    ds[0] = (mode == GS_CH_AX_X) ? R(1) : diso;
    ds[1] = (mode == GS_CH_AX_Y) ? R(1) : diso;
    ds[2] = (mode == GS_CH_AX_Z) ? R(1) : diso;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R acc = direct[k];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc += (Mbar[0][k] * D[0][j] + Mbar[1][k] * D[1][j] + Mbar[2][k] * D[2][j]) * P[k][j];
      ga += ds[k] * acc;
    }
  }
  // D = x_e N: Xbar = Dbar N
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const R m = R(0.25) * ((Dbar[i][0] + Dbar[i][1]) + (Dbar[i][2] + Dbar[i][3]));
#pragma unroll
    for (int j = 0; j < 4; ++j) Xbar[i][j] = Dbar[i][j] - m;
  }
}

// Start of an adjoint solve: mu = 0, warm start 0, cleared accumulators and
// the adjoint's status block.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_adj_init(Dev<R> d, Consts c) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  const size_t n = (size_t)c.n;
  if (v < c.n) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      d.mu[k * n + v] = R(0);
      d.acc3[k * n + v] = 0.0;
      d.dl[4 * (size_t)v + k] = R(0);  // the CG start and its history: none yet
      d.dlp[4 * (size_t)v + k] = R(0);
      d.dlpp[4 * (size_t)v + k] = R(0);
    }
  }
  const int stride = gridDim.x * kBlock;
  for (int i = v; i < c.M; i += stride) {
    d.mdone[i] = 0;
    d.mres[i] = 0ull;
    d.mmax[i] = 0ull;
    d.mbar[i] = 0u;
  }
  if (v == 0 && c.aa_m > 0) d.aa_k[0] = 0;
  if (v == 0) {
    DevStatus* st = d.st;
    st->n_active = c.M;
    st->iters = 0;
    st->done = RUNNING;
    st->changed = 0;
    st->pcg_total = 0;
    st->ray_miss = 0;
    st->ray_miss_last = 0;
    st->n_pen = 0;
    st->n_over = 0;
    st->ticket = 0;
    st->n_contacts = 0;
    st->n_contacts_last = 0;
    st->cand_tet = 0;
    st->cand_tri = 0;
    st->pcg_last = 0;
    st->changed_last = 0;
    st->residual = INFINITY;
    st->energy = 0.0;
    st->bar_count = 0;
    st->mb_last = 0u;
    for (int i = 0; i <= kBarGroups; ++i) d.bar2[64 * i] = 0u;
  }
}

__device__ __forceinline__ void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
// The scatter of the new self-contact targets' adjoint is deterministic: its
// contributions are added as 64-bit fixed-point integers (integer addition
// is associative), on a scale set by the largest contribution magnitude M of
// the iteration (found by a first pass): scale = 2^(41 - ilogb(M)), so one
// contribution stays below 2^42 and up to 2^20 of them can meet at a vertex
// without overflow; the quantum is below 2^-41 M.
__device__ __forceinline__ double acc_scale(unsigned long long mbits) {
  const double M = __longlong_as_double((long long)mbits);
  return M > 0.0 ? ldexp(1.0, 41 - ilogb(M)) : 0.0;
}

template <int PASS>
struct AccAdd {
  unsigned long long* acc;
  size_t n;
  double scale;  // PASS 1
  double mx;     // PASS 0: largest magnitude seen by this thread
  __device__ __forceinline__ void operator()(int v, const double* g, double sgn) {
    if (PASS == 0) {
      mx = fmax(mx, fmax(fabs(g[0]), fmax(fabs(g[1]), fabs(g[2]))));
      if (!(g[0] == g[0] && g[1] == g[1] && g[2] == g[2])) mx = INFINITY;
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k)
        atomicAdd(&acc[k * n + v], (unsigned long long)llrint(sgn * g[k] * scale));
    }
  }
};

__global__ void k_acc_reset(unsigned long long* acc_max) { *acc_max = 0ull; }

// Adjoint of the new self-contact targets (one thread per query vertex with
// such a contact): the spring adds k c(x) to b_v, so the adjoint input is
// cbar = k mu_v; the products with dc/dx are scattered into acc3 (pass 0:
// their largest magnitude only; pass 1: the fixed-point sums).
template <typename R, int PASS>
__global__ __launch_bounds__(kBlock) void k_adj_springs(Dev<R> d, Consts c) {
  if (is_done(d.st)) return;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= c.S || !c.self_col) return;
  const int base = s * c.slots;
  if (d.cact[base] != 2) return;
  const int v = d.qverts[s];
  const int m = d.vmesh[v];
  if (mesh_frozen(d, c.mask_done, m)) return;
  const size_t n = (size_t)c.n;
  AccAdd<PASS> add_to{reinterpret_cast<unsigned long long*>(d.acc3), n, PASS ? acc_scale(*d.acc_max) : 0.0, 0.0};
  const double eps = d.mesh[m].eps;
  const double k = d.kq[s];
  const double cbar[3] = {k * (double)d.mu[v], k * (double)d.mu[n + v], k * (double)d.mu[2 * n + v]};
  double o[3];
  load3(d.xc, n, v, o);
  // forward: vertex normal, ray direction, Moller-Trumbore distance
  double nv[3] = {0.0, 0.0, 0.0};
  const int q0 = d.qf_start[s], q1 = d.qf_start[s + 1];
  for (int q = q0; q < q1; ++q) {
    const int f = d.qf_list[q];
    double xi[3], xj[3], xk[3], e1[3], e2[3], cr[3];
    load3(d.xc, n, d.faces[f], xi);
    load3(d.xc, n, d.faces[c.F + f], xj);
    load3(d.xc, n, d.faces[2 * c.F + f], xk);
    sub3(xj, xi, e1);
    sub3(xk, xi, e2);
    cross3(e1, e2, cr);
    nv[0] += cr[0];
    nv[1] += cr[1];
    nv[2] += cr[2];
  }
  const double ln = sqrt(dot3(nv, nv));
  if (!(ln > 0.0)) return;
  const double nh[3] = {nv[0] / ln, nv[1] / ln, nv[2] / ln};
  const double dd[3] = {-nh[0], -nh[1], -nh[2]};
  const int hf = d.cprim[base];
  const int h0 = d.faces[hf], h1 = d.faces[c.F + hf], h2 = d.faces[2 * c.F + hf];
  double a0[3], a1[3], a2[3], e1[3], e2[3], pv[3], tv[3], qv[3];
  load3(d.xc, n, h0, a0);
  load3(d.xc, n, h1, a1);
  load3(d.xc, n, h2, a2);
  sub3(a1, a0, e1);
  sub3(a2, a0, e2);
  cross3(dd, e2, pv);
  const double det = dot3(e1, pv);
  if (det == 0.0) return;
  sub3(o, a0, tv);
  cross3(tv, e1, qv);
  const double t = dot3(e2, qv) / det;
  // backward: c = o + (t + eps) d
  double obar[3] = {cbar[0], cbar[1], cbar[2]};
  double dbar[3] = {(t + eps) * cbar[0], (t + eps) * cbar[1], (t + eps) * cbar[2]};
  const double tbar = dot3(cbar, dd);
  // t = (e2 . q) / det, q = tv x e1, det = e1 . (d x e2)
  double e2bar[3] = {tbar * qv[0] / det, tbar * qv[1] / det, tbar * qv[2] / det};
  const double qbar[3] = {tbar * e2[0] / det, tbar * e2[1] / det, tbar * e2[2] / det};
  const double detbar = -tbar * t / det;
  double tvbar[3], e1bar[3], tmp[3];
  cross3(e1, qbar, tvbar);
  cross3(qbar, tv, e1bar);
  e1bar[0] += detbar * pv[0];
  e1bar[1] += detbar * pv[1];
  e1bar[2] += detbar * pv[2];
  const double pbar[3] = {detbar * e1[0], detbar * e1[1], detbar * e1[2]};
  cross3(e2, pbar, tmp);
  dbar[0] += tmp[0];
  dbar[1] += tmp[1];
  dbar[2] += tmp[2];
  cross3(pbar, dd, tmp);
  e2bar[0] += tmp[0];
  e2bar[1] += tmp[1];
  e2bar[2] += tmp[2];
  obar[0] += tvbar[0];
  obar[1] += tvbar[1];
  obar[2] += tvbar[2];
  const double a0bar[3] = {-tvbar[0] - e1bar[0] - e2bar[0], -tvbar[1] - e1bar[1] - e2bar[1],
                           -tvbar[2] - e1bar[2] - e2bar[2]};
  add_to(v, obar, 1.0);
  add_to(h0, a0bar, 1.0);
  add_to(h1, e1bar, 1.0);
  add_to(h2, e2bar, 1.0);
  // d = -n / |n|: nbar = -(dbar - (dbar . nh) nh) / |n|
  const double dn = dot3(dbar, nh);
  const double nbar[3] = {-(dbar[0] - dn * nh[0]) / ln, -(dbar[1] - dn * nh[1]) / ln, -(dbar[2] - dn * nh[2]) / ln};
  // n = sum_f (x_j - x_i) x (x_k - x_i)
  for (int q = q0; q < q1; ++q) {
    const int f = d.qf_list[q];
    const int i0 = d.faces[f], i1 = d.faces[c.F + f], i2 = d.faces[2 * c.F + f];
    double xi[3], xj[3], xk[3], E1[3], E2[3], E1b[3], E2b[3];
    load3(d.xc, n, i0, xi);
    load3(d.xc, n, i1, xj);
    load3(d.xc, n, i2, xk);
    sub3(xj, xi, E1);
    sub3(xk, xi, E2);
    cross3(E2, nbar, E1b);
    cross3(nbar, E1, E2b);
    const double sb[3] = {E1b[0] + E2b[0], E1b[1] + E2b[1], E1b[2] + E2b[2]};
    add_to(i1, E1b, 1.0);
    add_to(i2, E2b, 1.0);
    add_to(i0, sb, -1.0);
  }
  if (PASS == 0) atomicMax(d.acc_max, (unsigned long long)__double_as_longlong(add_to.mx));
}

// Per-tet adjoint columns omega_e ((dT_e/dx_e)^T mu_e - mu_e N) in incidence
// order; with alpha_grad, the per-tet term of dL/dalpha instead (all meshes).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_adj_local(Dev<R> d, Consts c, int mode_out) {
  const bool alpha_grad = mode_out == ADJ_ALPHA, jt_only = mode_out == ADJ_JT;
  if (!alpha_grad && is_done(d.st)) return;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= c.T) return;
  const int m = d.tmesh[e];
  const size_t n = (size_t)c.n;
  V4<R>* res = reinterpret_cast<V4<R>*>(d.res4);
  const int tag = d.tag[e];
  const int mode = tag & 7, ch = tag >> 3;
  if (!alpha_grad && mesh_frozen(d, c.mask_done, m)) {
    V4<R> z;
    z.x = z.y = z.z = z.w = R(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) res[d.inc_pos[j * c.T + e]] = z;
    return;
  }
  if (alpha_grad && mode == GS_BODY) {
    d.ga[e] = 0.0;
    return;
  }
  int vi[4];
  R P[3][4], D[3][4], Dminv[3][3];
  double vol;
  load_tet<R, false>(d, c, e, nullptr, vi, P, D, Dminv, vol);
  R MU[3][4];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R mu4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) mu4[j] = d.mu[k * n + vi[j]];
    const R mm = R(0.25) * ((mu4[0] + mu4[1]) + (mu4[2] + mu4[3]));
#pragma unroll
    for (int j = 0; j < 4; ++j) MU[k][j] = mu4[j] - mm;
  }
  const R a = (mode != GS_BODY) ? d.alpha_last[ch] : R(1);
  R Xbar[3][4], ga;
  tet_vjp<R>(mode, a, P, D, Dminv, (R)vol, c, MU, Xbar, ga);
  const R om = (R)(vol * d.mesh[m].inv_mean_vol);
  if (alpha_grad) {
    d.ga[e] = (double)om * (double)ga;
    return;
  }
  const R keep = jt_only ? R(0) : R(1);  // the residual form also subtracts A_el mu
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    V4<R> v;
    v.x = om * (Xbar[0][j] - keep * MU[0][j]);
    v.y = om * (Xbar[1][j] - keep * MU[1][j]);
    v.z = om * (Xbar[2][j] - keep * MU[2][j]);
    v.w = R(0);
    res[d.inc_pos[j * c.T + e]] = v;
  }
}

template <typename R>
struct alignas(4 * sizeof(R)) A4 {
  R x, y, z, w;
};

// Right-hand side of the adjoint correction system per vertex:
// g + (db/dx)^T mu - M mu = gathered element columns + scattered self-contact
// terms + obstacle-spring terms - spring diagonal * mu + g; the Jacobi
// diagonal of M for the frozen contact set.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_adj_gather(Dev<R> d, Consts c) {
  if (is_done(d.st)) return;
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= c.n) return;
  const size_t n = (size_t)c.n;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  sum_columns(reinterpret_cast<const W4<R>*>(d.res4), d.inc_start[v], d.inc_start[v + 1], r0, r1, r2);
  {
    // fixed-point sums of the self-contact scatter (see acc_scale)
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(d.acc3);
    const double M = __longlong_as_double((long long)*d.acc_max);
    if (M > 0.0 && M < INFINITY) {
      const double inv = 1.0 / acc_scale(*d.acc_max);
      r0 += (double)(long long)acc[v] * inv;
      r1 += (double)(long long)acc[n + v] * inv;
      r2 += (double)(long long)acc[2 * n + v] * inv;
    } else if (!(M == 0.0)) {
      r0 = r1 = r2 = NAN;  // a non-finite contribution: the CG reports the breakdown
    }
    acc[v] = 0ull;
    acc[n + v] = 0ull;
    acc[2 * n + v] = 0ull;
  }
  double ds = 0.0;
  const bool frozen = mesh_frozen(d, c.mask_done, d.vmesh[v]);
  if (!d.freem[v] || frozen) {
    r0 = r1 = r2 = 0.0;
  } else {
    const double mu[3] = {(double)d.mu[v], (double)d.mu[n + v], (double)d.mu[2 * n + v]};
    const int s = d.vq[v];
    if (s >= 0) {
      const double k = d.kq[s];
      double x[3];
      load3(d.xc, n, v, x);
      for (int sl = 0; sl < c.slots; ++sl) {
        const int b = s * c.slots + sl;
        if (!d.cact[b]) continue;
        ds += k;
        if (sl == 0) continue;  // self contacts: scattered terms only
        double jt[3];
        if (sl <= c.ns) {
          // c = c0 + (r + eps) u, u = (x - c0)/|x - c0|: dc/dx = (r + eps)/|x - c0| (I - u u^T)
          const double* sp = d.obst + 4 * (sl - 1);
          const double dx[3] = {x[0] - sp[0], x[1] - sp[1], x[2] - sp[2]};
          const double dist = sqrt(dot3(dx, dx));
          if (!(dist > 0.0)) continue;
          const double u[3] = {dx[0] / dist, dx[1] / dist, dx[2] / dist};
          const double rho = (sp[3] + d.mesh[d.vmesh[v]].eps) / dist;
          const double um = dot3(u, mu);
          jt[0] = rho * (mu[0] - um * u[0]);
          jt[1] = rho * (mu[1] - um * u[1]);
          jt[2] = rho * (mu[2] - um * u[2]);
        } else {
          // c = x - (n.(x - p) - eps) n: dc/dx = I - n n^T
          const double* pl = d.obst + 4 * c.ns + 6 * (sl - 1 - c.ns);
          const double nm = (pl[3] * mu[0] + pl[4] * mu[1]) + pl[5] * mu[2];
          jt[0] = mu[0] - nm * pl[3];
          jt[1] = mu[1] - nm * pl[4];
          jt[2] = mu[2] - nm * pl[5];
        }
        r0 += k * jt[0];
        r1 += k * jt[1];
        r2 += k * jt[2];
      }
    }
    if (!c.adj_jt) {
      r0 += (double)d.gL[v] - ds * mu[0];
      r1 += (double)d.gL[n + v] - ds * mu[1];
      r2 += (double)d.gL[2 * n + v] - ds * mu[2];
    }
  }
  if (c.adj_jt) {
    d.lam[v] = (R)r0;
    d.lam[n + v] = (R)r1;
    d.lam[2 * n + v] = (R)r2;
    return;
  }
  A4<R> rb;
  rb.x = (R)r0;
  rb.y = (R)r1;
  rb.z = (R)r2;
  rb.w = R(0);
  reinterpret_cast<A4<R>*>(d.cg)[c.cg_soa ? (size_t)v : 3 * (size_t)v] = rb;
  d.dg[v] = d.freem[v] ? (R)((double)d.adiag[v] + ds) : R(1);
}

// dL/dalpha_c = sum of the chamber's per-tet terms (one block per chamber,
// fixed order: strided per-thread sums, then the block tree).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_adj_chamber_sum(Dev<R> d, Consts c, R* __restrict__ out) {
  __shared__ double lds[kBlock / 64];
  const int ch = blockIdx.x;
  if (ch >= c.nch) return;
  double acc = 0.0;
  const int b = d.ch_start[ch], e = d.ch_start[ch + 1];
  for (int i = b + threadIdx.x; i < e; i += kBlock) acc += d.ga[d.ch_tets[i]];
  const double t = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) out[ch] = (R)t;
}

// ---------------------------------------------------------------------------
// Anderson acceleration of the adjoint iteration (Walker & Ni 2011, type II,
// memory m): with f_k = G(mu_k) - mu_k the correction the CG kernel left in
// dl, and the last m differences dX_j = mu_{j+1} - mu_j, dF_j = f_{j+1} - f_j,
//   gamma = argmin |f_k - dF gamma|,   mu_{k+1} = mu_k + f_k - (dX + dF) gamma.
// For a linear fixed-point map this is a Krylov method on (I - G') (it
// matches GMRES in exact arithmetic with full memory), so the slow modes of
// the iteration no longer set the iteration count.  The normal equations
// (dF^T dF + ridge) gamma = dF^T f are solved in double by one thread; the
// dot products are block partials summed in a fixed order.

constexpr int kAaMax = kAaMaxMem;
constexpr int kAaBlock = 256;

// New difference column (k >= 1), previous iterate / residual, and the
// block partials of dF_j . dF_new and dF_j . f_k.
template <typename R>
__global__ __launch_bounds__(kAaBlock) void k_aa_diff_dots(Dev<R> d, Consts c) {
  __shared__ double lds[kAaBlock / 64];
  if (is_done(d.st)) return;
  const int k = d.aa_k[0];
  const int m = c.aa_m;
  const int mk = min(k, m);
  const int col = (k - 1 + m) % m;
  const size_t n3 = 3 * (size_t)c.n;
  const size_t n = (size_t)c.n;
  double a[kAaMax], b[kAaMax];
#pragma unroll
  for (int j = 0; j < kAaMax; ++j) a[j] = b[j] = 0.0;
  for (size_t e = (size_t)blockIdx.x * kAaBlock + threadIdx.x; e < n3; e += (size_t)gridDim.x * kAaBlock) {
    const size_t v = e % n, kc = e / n;
    const R f = d.dl[4 * v + kc];
    const R mu = d.mu[e];
    if (k >= 1) {
      const R df = f - d.aa_fp[e];
      d.aa_df[col * n3 + e] = df;
      d.aa_dx[col * n3 + e] = mu - d.aa_xp[e];
#pragma unroll
      for (int j = 0; j < kAaMax; ++j) {
        if (j < mk) {
          const double dj = (j == col) ? (double)df : (double)d.aa_df[j * n3 + e];
          a[j] += dj * (double)df;
          b[j] += dj * (double)f;
        }
      }
    }
    d.aa_xp[e] = mu;
    d.aa_fp[e] = f;
  }
  if (k < 1) return;
#pragma unroll
  for (int j = 0; j < kAaMax; ++j) {
    if (j < mk) {  // uniform over the block
      const double ta = block_sum<kAaBlock>(a[j], lds);
      const double tb = block_sum<kAaBlock>(b[j], lds);
      if (threadIdx.x == 0) {
        d.aa_part[(2 * j) * (size_t)gridDim.x + blockIdx.x] = ta;
        d.aa_part[(2 * j + 1) * (size_t)gridDim.x + blockIdx.x] = tb;
      }
    }
  }
}

// Sum the partials (one wavefront per value), update the Gram matrix, and
// solve for gamma (gram_solve: Cholesky with a relative ridge; a
// non-positive pivot gives gamma = 0, a plain step).  Counts the iteration.
constexpr int kAaSolveBlock = kAaSolveThreads;

template <typename R>
__global__ __launch_bounds__(kAaSolveBlock) void k_aa_solve(Dev<R> d, Consts c, int G) {
  __shared__ double val[2 * kAaMax];
  __shared__ double A[kAaMax][kAaMax];
  __shared__ double y[kAaMax];
  if (is_done(d.st)) return;
  const int k = d.aa_k[0];
  const int m = c.aa_m;
  const int mk = min(k, m);
  const int col = (k - 1 + m) % m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int nw = kAaSolveBlock / 64;
  for (int q = wave; q < 2 * mk; q += nw) {
    double t = 0.0;
    for (int b = lane; b < G; b += 64) t += d.aa_part[(size_t)q * G + b];
    t = wave_sum(t);
    if (lane == 0) val[q] = t;
  }
  __syncthreads();
  const int i = mk > 0 ? tid / mk : 0, j = mk > 0 ? tid % mk : 0;
  if (tid < mk * mk) {
    // Gram matrix: the new column from the partial sums, the rest as stored
    double h;
    if (i == col) h = val[2 * j];
    else if (j == col) h = val[2 * i];
    else h = d.aa_h[i * m + j];
    d.aa_h[i * m + j] = h;
    A[i][j] = h;
  }
  if (tid < mk) y[tid] = val[2 * tid + 1];
  __syncthreads();
  double gj;
  gram_solve(A, y, mk, &gj);
  if (wave == 0 && lane < mk) d.aa_gamma[lane] = gj;
  if (tid == 0) d.aa_k[0] = k + 1;
}

// mu_{k+1} = mu_k + f_k - sum_j gamma_j (dX_j + dF_j)
template <typename R>
__global__ __launch_bounds__(kAaBlock) void k_aa_update(Dev<R> d, Consts c) {
  if (is_done(d.st)) return;
  const int k = d.aa_k[0] - 1;  // k_aa_solve counted this iteration already
  const int mk = min(k, c.aa_m);
  const size_t n3 = 3 * (size_t)c.n;
  const size_t n = (size_t)c.n;
  double g[kAaMax];
#pragma unroll
  for (int j = 0; j < kAaMax; ++j) g[j] = j < mk ? d.aa_gamma[j] : 0.0;
  for (size_t e = (size_t)blockIdx.x * kAaBlock + threadIdx.x; e < n3; e += (size_t)gridDim.x * kAaBlock) {
    const size_t v = e % n, kc = e / n;
    double x = (double)d.mu[e] + (double)d.dl[4 * v + kc];
#pragma unroll
    for (int j = 0; j < kAaMax; ++j)
      if (j < mk) x -= g[j] * ((double)d.aa_dx[j * n3 + e] + (double)d.aa_df[j * n3 + e]);
    d.mu[e] = (R)x;
  }
}

template <typename R>
hipError_t launch_adj_anderson(const Dev<R>& d, const Consts& c, hipStream_t s) {
  if (c.aa_m <= 0) return hipSuccess;
  const int G = max(1, min(cdiv(3L * c.n, kAaBlock), min(c.nparts, 1024)));
  k_aa_diff_dots<R><<<G, kAaBlock, 0, s>>>(d, c);
  k_aa_solve<R><<<1, kAaSolveBlock, 0, s>>>(d, c, G);
  k_aa_update<R><<<G, kAaBlock, 0, s>>>(d, c);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Unrolled adjoint (reverse sweep over recorded iterations)
//
// For K iterations x_{k+1} = M_k^-1 b_k(x_k, alpha) (contact set A_k as the
// forward found it): lambda_K = g; for k = K-1 ... 0, nu = M_k^-1 lambda_{k+1}
// (the CG kernel on right-hand side lambda from a zero start, mu = nu),
// dL/dalpha += (db_k/dalpha)^T nu, lambda_k = (db_k/dx_k)^T nu.

// State x_k restored from u: collision positions, and the status block of
// the recomputed forward iterations set running.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_unr_restore(Dev<R> d, Consts c, DevStatus* run) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  const size_t n = (size_t)c.n;
  if (v < c.n) {
#pragma unroll
    for (int k = 0; k < 3; ++k) d.xc[k * n + v] = d.X0[k * n + v] + (double)d.u[k * n + v];
  }
  // the spatial hash held other positions: cleared, refilled before the next
  // iteration's tet query
  for (int i = v; i < c.H; i += gridDim.x * kBlock) d.hcount[i] = 0;
  if (v == 0) {
    DevStatus* st = d.st;
    st->done = RUNNING;
    st->changed = 0;
    st->ray_miss = 0;
    st->n_pen = 0;
    st->n_over = 0;
    st->ticket = 0;
    st->n_contacts = 0;
    st->bar_count = 0;
    st->mb_last = 0u;
    for (int i = 0; i <= kBarGroups; ++i) d.bar2[64 * i] = 0u;
    run->done = RUNNING;
  }
}

// Right-hand side lambda_{k+1} of the reverse CG solve (zero rows for fixed
// vertices), the Jacobi diagonal of M_k for the restored contact set, a zero
// start, and a fresh status block for the solve.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_unr_rhs(Dev<R> d, Consts c) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  const size_t n = (size_t)c.n;
  if (v < c.n) {
    const bool fr = d.freem[v] != 0;
    double ds = 0.0;
    const int s = d.vq[v];
    if (fr && s >= 0)
      for (int sl = 0; sl < c.slots; ++sl)
        if (d.cact[s * c.slots + sl]) ds += d.kq[s];
    A4<R> rb;
    rb.x = fr ? d.lam[v] : R(0);
    rb.y = fr ? d.lam[n + v] : R(0);
    rb.z = fr ? d.lam[2 * n + v] : R(0);
    rb.w = R(0);
    reinterpret_cast<A4<R>*>(d.cg)[c.cg_soa ? (size_t)v : 3 * (size_t)v] = rb;
    d.dg[v] = fr ? (R)((double)d.adiag[v] + ds) : R(1);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      d.mu[k * n + v] = R(0);
      // each reverse solve starts from zero, with no history (its system
      // differs from the previous one's)
      d.dl[4 * (size_t)v + k] = R(0);
      d.dlp[4 * (size_t)v + k] = R(0);
      d.dlpp[4 * (size_t)v + k] = R(0);
    }
  }
  for (int i = v; i < c.M; i += gridDim.x * kBlock) {
    d.mdone[i] = 0;
    d.mres[i] = 0ull;
    d.mmax[i] = 0ull;
  }
  if (v == 0) {
    DevStatus* st = d.st;
    st->iters = 0;
    st->done = RUNNING;
    st->ticket = 0;
    st->bar_count = 0;
    st->mb_last = 0u;
    for (int i = 0; i <= kBarGroups; ++i) d.bar2[64 * i] = 0u;
    st->pcg_last = 0;
  }
}

// dL/dalpha += this step's per-chamber sums (one block per chamber, fixed order).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_unr_accumulate(Dev<R> d, Consts c) {
  __shared__ double lds[kBlock / 64];
  const int ch = blockIdx.x;
  if (ch >= c.nch) return;
  double acc = 0.0;
  const int b = d.ch_start[ch], e = d.ch_start[ch + 1];
  for (int i = b + threadIdx.x; i < e; i += kBlock) acc += d.ga[d.ch_tets[i]];
  const double t = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) d.ga_acc[ch] += t;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_unr_finish(Dev<R> d, Consts c, R* dalpha, R* dx0) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (dalpha && i < c.nch) dalpha[i] = (R)d.ga_acc[i];
  if (dx0 && i < 3 * c.n) dx0[i] = d.lam[i];
}

template <typename R>
hipError_t launch_adj_init(const Dev<R>& d, const Consts& c, hipStream_t s) {
  k_adj_init<R><<<max(1, cdiv(c.n, kBlock)), kBlock, 0, s>>>(d, c);
  return hipGetLastError();
}
template <typename R>
hipError_t launch_adj_springs(const Dev<R>& d, const Consts& c, hipStream_t s) {
  k_acc_reset<<<1, 1, 0, s>>>(d.acc_max);
  if (!c.self_col || c.S == 0) return hipGetLastError();
  k_adj_springs<R, 0><<<max(1, cdiv(c.S, kBlock)), kBlock, 0, s>>>(d, c);
  k_adj_springs<R, 1><<<max(1, cdiv(c.S, kBlock)), kBlock, 0, s>>>(d, c);
  return hipGetLastError();
}
template <typename R>
hipError_t launch_adj_local(const Dev<R>& d, const Consts& c, bool alpha_grad, hipStream_t s) {
  k_adj_local<R><<<cdiv(c.T, kBlock), kBlock, 0, s>>>(d, c, alpha_grad ? ADJ_ALPHA : ADJ_RESIDUAL);
  return hipGetLastError();
}
template <typename R>
hipError_t launch_adj_local_mode(const Dev<R>& d, const Consts& c, int mode, hipStream_t s) {
  k_adj_local<R><<<cdiv(c.T, kBlock), kBlock, 0, s>>>(d, c, mode);
  return hipGetLastError();
}
template <typename R>
hipError_t launch_adj_gather(const Dev<R>& d, const Consts& c, hipStream_t s) {
  k_adj_gather<R><<<cdiv(c.n, kBlock), kBlock, 0, s>>>(d, c);
  return hipGetLastError();
}
template <typename R>
hipError_t launch_adj_chamber_sum(const Dev<R>& d, const Consts& c, R* out, hipStream_t s) {
  if (c.nch == 0) return hipSuccess;
  k_adj_chamber_sum<R><<<max(1, c.nch), kBlock, 0, s>>>(d, c, out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_unr_restore(const Dev<R>& d, const Consts& c, DevStatus* run, hipStream_t s) {
  k_unr_restore<R><<<max(1, cdiv(c.n, kBlock)), kBlock, 0, s>>>(d, c, run);
  return hipGetLastError();
}
template <typename R>
hipError_t launch_unr_rhs(const Dev<R>& d, const Consts& c, hipStream_t s) {
  k_unr_rhs<R><<<max(1, cdiv(c.n, kBlock)), kBlock, 0, s>>>(d, c);
  return hipGetLastError();
}
template <typename R>
hipError_t launch_unr_accumulate(const Dev<R>& d, const Consts& c, hipStream_t s) {
  if (c.nch == 0) return hipSuccess;
  k_unr_accumulate<R><<<max(1, c.nch), kBlock, 0, s>>>(d, c);
  return hipGetLastError();
}
template <typename R>
hipError_t launch_unr_finish(const Dev<R>& d, const Consts& c, R* dalpha, R* dx0, hipStream_t s) {
  k_unr_finish<R><<<max(1, cdiv(max(3 * c.n, c.nch), kBlock)), kBlock, 0, s>>>(d, c, dalpha, dx0);
  return hipGetLastError();
}

#define INST(R)                                                                                  \
  template hipError_t launch_adj_init<R>(const Dev<R>&, const Consts&, hipStream_t);             \
  template hipError_t launch_adj_springs<R>(const Dev<R>&, const Consts&, hipStream_t);          \
  template hipError_t launch_adj_local<R>(const Dev<R>&, const Consts&, bool, hipStream_t);      \
  template hipError_t launch_adj_gather<R>(const Dev<R>&, const Consts&, hipStream_t);           \
  template hipError_t launch_adj_chamber_sum<R>(const Dev<R>&, const Consts&, R*, hipStream_t); \
  template hipError_t launch_adj_anderson<R>(const Dev<R>&, const Consts&, hipStream_t);       \
  template hipError_t launch_adj_local_mode<R>(const Dev<R>&, const Consts&, int, hipStream_t);  \
  template hipError_t launch_unr_restore<R>(const Dev<R>&, const Consts&, DevStatus*, hipStream_t); \
  template hipError_t launch_unr_rhs<R>(const Dev<R>&, const Consts&, hipStream_t);             \
  template hipError_t launch_unr_accumulate<R>(const Dev<R>&, const Consts&, hipStream_t);      \
  template hipError_t launch_unr_finish<R>(const Dev<R>&, const Consts&, R*, R*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace gs
