// Global step (Section III-B) in correction form and the outer-iteration
// bookkeeping.
//
// With targets fixed, Eq. (9) is minimised by M x = b, M = A_el + diag(k)
// (springs), fixed vertices held at X0.  The iterate is the displacement
// u = x - X0; each outer iteration solves M d = b - M x_k for the correction d
// with a Jacobi-preconditioned conjugate gradient warm-started from the
// previous corrections (the Galerkin projection onto d_{k-1} and its first and
// second differences) and stopped once sqrt(r'z) <= eta sqrt(b'D^-1 b), b the
// right-hand side (relative to b, not to the warm-started residual).  The
// slow modes of the local/global map are smooth bending modes, where both the
// outer iteration and Jacobi-CG converge slowly; the warm start carries the
// slow part of the correction across iterations.  The right-hand side b - M x_k is
// the gathered element residual sum_e omega_e (T_e - D_e) plus the spring
// pulls k (c - x): it vanishes exactly at the fixed point, so an inexact inner
// solve changes the path, not the answer.
//
// The CG runs as one persistent kernel on a small grid (every block resident:
// an ordinary launch when the grid is at most half the resident capacity, a
// cooperative launch otherwise): the per-barrier cost on this GPU grows with the number of
// participating blocks, so the solve uses few, wide blocks.  Dot products are
// accumulated in double; block partials are summed in block order by every
// block, so all blocks take identical decisions.
#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>

#include "contacts.h"
#include "gather.h"

namespace gs {

// Start of a solve: u from the warm start (fixed vertices reset), collision
// positions, cleared hash counters and status.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_init(Dev<R> d, Consts c, const R* __restrict__ xin) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  const size_t n = (size_t)c.n;
  if (v < c.n) {
    const bool fr = d.freem[v] != 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double X = d.X0[k * n + v];
      const R uu = fr ? (R)((double)xin[k * n + v] - X) : R(0);
      d.u[k * n + v] = uu;
      d.xc[k * n + v] = X + (double)uu;
      d.dl[4 * (size_t)v + k] = R(0);
      d.dlp[4 * (size_t)v + k] = R(0);
      d.dlpp[4 * (size_t)v + k] = R(0);
    }
  }
  const int stride = gridDim.x * kBlock;
  for (int i = v; i < c.H; i += stride) d.hcount[i] = 0;
  for (int i = v; i < c.S; i += stride) d.pen[i] = 0;
  for (int i = v; i < c.M; i += stride) {
    d.mdone[i] = 0;
    d.mres[i] = 0ull;
    d.mchanged[i] = 0;
    d.mbar[i] = 0u;
    AaMesh a{};
    a.act = AA_NONE;
    a.r_acc = INFINITY;
    a.e_acc = INFINITY;
    d.faa[i] = a;
  }
  if (v == 0) {
    DevStatus* st = d.st;
    st->aa_pending = 0;
    st->aa_ticket = 0;
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

// Collision positions straight from a caller's array (collision check alone).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_set_positions(Dev<R> d, Consts c, const R* __restrict__ xin) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  const size_t n = (size_t)c.n;
  if (v < c.n) {
#pragma unroll
    for (int k = 0; k < 3; ++k) d.xc[k * n + v] = (double)xin[k * n + v];
  }
  const int stride = gridDim.x * kBlock;
  for (int i = v; i < c.H; i += stride) d.hcount[i] = 0;
  for (int i = v; i < c.S; i += stride) d.pen[i] = 0;
  for (int i = v; i < c.M; i += stride) {
    d.mdone[i] = 0;
    d.mchanged[i] = 0;
  }
  if (v == 0) {
    DevStatus* st = d.st;
    st->done = RUNNING;
    st->changed = 0;
    st->ray_miss = 0;
    st->n_pen = 0;
    st->n_over = 0;
    st->n_contacts = 0;
    st->cand_tet = 0;
    st->cand_tri = 0;
  }
}

// The spatial hash cleared for the CG kernel's final insertions, before a
// per-mesh CG launch (the whole-grid kernel clears it itself).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_hash_clear(Dev<R> d, Consts c) {
  if (is_done(d.st)) return;
  const int v = blockIdx.x * kBlock + threadIdx.x;
  for (int i = v; i < c.H; i += gridDim.x * kBlock) d.hcount[i] = 0;
  if (v == 0) d.st->n_over = 0;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_output(Dev<R> d, Consts c, R* __restrict__ xout) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= c.n) return;
  const size_t n = (size_t)c.n;
#pragma unroll
  for (int k = 0; k < 3; ++k) xout[k * n + v] = (R)(d.X0[k * n + v] + (double)d.u[k * n + v]);
}


constexpr int kPcgBlock = kPcgThreads;

// Sums of the G <= kMaxPcgGrid block partials of two arrays in one round
// trip: wave 0 reduces `a`, wave 1 reduces `b`; lane l first adds entries
// l, l+64, l+128, ... in that order, then a fixed shuffle tree combines the
// lanes (every block obtains the same bits).
template <bool SYNC_AFTER = true>
__device__ __forceinline__ void grid_sum2(const double* a, const double* b, int G, double* sh, double& ra,
                                          double& rb) {
  if (threadIdx.x < 128) {
    const double* src = threadIdx.x < 64 ? a : b;
    const int l = threadIdx.x & 63;
    double t = (l < G) ? src[l] : 0.0;
    for (int k = l + 64; k < G; k += 64) t += src[k];
    t = wave_sum(t);
    if (l == 0) sh[threadIdx.x >> 6] = t;
  }
  __syncthreads();
  ra = sh[0];
  rb = sh[1];
  if (SYNC_AFTER) __syncthreads();
}

// Block sums of two values, stored by thread 0 to out_a and out_b (the
// per-wave order and the fixed tree of block_sum).  No closing
// __syncthreads: the caller's next step (a grid barrier) starts with one
// before `lds` is written again.
__device__ __forceinline__ void block_sum2_store(double a, double b, double (*lds)[kPcgBlock / 64], double* out_a,
                                                 double* out_b) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    lds[0][w] = a;
    lds[1][w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int i = 0; i < kPcgBlock / 64; ++i) {
      ta += lds[0][i];
      tb += lds[1][i];
    }
    st_wt(out_a, ta);
    st_wt(out_b, tb);
  }
}

// Block sums of K values in one LDS round; thread i stores sum i to
// base[i * stride] (the per-wave order and fixed tree of block_sum; no
// closing __syncthreads, the caller's grid barrier starts with one).
template <int K>
__device__ __forceinline__ void block_sums_store(const double (&v)[K], double (*lds)[kPcgBlock / 64], double* base,
                                                 int stride) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const double t = wave_sum(v[i]);
    if (lane == 0) lds[i][w] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < K) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < kPcgBlock / 64; ++j) t += lds[threadIdx.x][j];
    st_wt(base + (size_t)threadIdx.x * stride, t);
  }
}

// Sums of the G block partials of K arrays base + i * stride in one round:
// wavefront w reduces arrays w, w + 8, ... in grid_sum2's order, all of its
// loads issued before the first reduction; every block obtains the same bits.
template <int K>
__device__ __forceinline__ void grid_sums(const double* base, int stride, int G, double* sh, double (&out)[K]) {
  constexpr int NW = kPcgBlock / 64;
  constexpr int PER = (K + NW - 1) / NW;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  double t[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = w + j * NW;
    t[j] = 0.0;
    if (i < K) {
      const double* a = base + (size_t)i * stride;
      t[j] = (l < G) ? a[l] : 0.0;
      for (int k = l + 64; k < G; k += 64) t[j] += a[k];
    }
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = w + j * NW;
    if (i < K) {
      const double r = wave_sum(t[j]);
      if (l == 0) sh[i] = r;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < K; ++i) out[i] = sh[i];
}

// A double every lane of the wavefront holds equally, moved to scalar
// registers (the CG scalars: they then take no vector registers in the loop).
__device__ __forceinline__ double uniform_d(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The x, y, z lanes of a padded vector (the padding lane is not loaded: a
// 12-byte load, three registers instead of four).
template <typename R>
__device__ __forceinline__ W4<R> ld3(const W4<R>* p) {
  W4<R> o;
  o.x = p->x;
  o.y = p->y;
  o.z = p->z;
  o.w = R(0);
  return o;
}

template <typename R>
__device__ __forceinline__ W4<R> w4(R x, R y, R z) {
  W4<R> o;
  o.x = x;
  o.y = y;
  o.z = z;
  o.w = R(0);
  return o;
}

// Weights (g1, g2) of the warm start g1 w1 + g2 w2 that minimise the A-norm
// error of M d = b over span{w1, w2}: the 2x2 system H g = e with
// H_ij = w_i' A w_j, e_i = w_i' b.  The start's residual is formed as
// b - g1 A w1 - g2 A w2, so large weights of opposite sign (w1, w2 close to
// parallel, as when the iteration contracts along one mode) would leave a
// rounding error in it that the CG stopping test cannot see: the pair is
// taken only when |g1| |w1|_A + |g2| |w2|_A stays within 16 |g1 w1 + g2 w2|_A
// (about one decimal digit of cancellation), else the projection onto w1
// alone; an empty w1 gives the zero start.
__device__ __forceinline__ void galerkin_weights(double e1, double e2, double h11, double h12, double h22,
                                                 double& g1, double& g2) {
  g1 = 0.0;
  g2 = 0.0;
  if (!(h11 > 0.0) || isinf(h11)) return;
  const double det = h11 * h22 - h12 * h12;
  if (h22 > 0.0 && det > 0.0) {
    const double a = (e1 * h22 - e2 * h12) / det, c = (e2 * h11 - e1 * h12) / det;
    const double nn = a * a * h11 + 2.0 * a * c * h12 + c * c * h22;  // |g1 w1 + g2 w2|_A^2
    const double sum = fabs(a) * sqrt(h11) + fabs(c) * sqrt(h22);
    if (nn > 0.0 && sum * sum <= 256.0 * nn) {
      g1 = a;
      g2 = c;
    }
  }
  if (g1 == 0.0 && g2 == 0.0) g1 = e1 / h11;
  if (!(g1 == g1) || !(g2 == g2) || isinf(g1) || isinf(g2)) g1 = g2 = 0.0;
}

// Three-vector version: the 3x3 system over span{w1, w2, w3} by Cholesky,
// accepted under the same cancellation bound (sum of |g_i| |w_i|_A within 16
// |x_0|_A), else the two-vector weights of (w1, w2).
__device__ __forceinline__ void galerkin_weights3(double e1, double e2, double e3, double h11, double h12,
                                                  double h13, double h22, double h23, double h33, double& g1,
                                                  double& g2, double& g3) {
  g3 = 0.0;
  if (h11 > 0.0 && h22 > 0.0 && h33 > 0.0 && !isinf(h11) && !isinf(h22) && !isinf(h33)) {
    const double l11 = sqrt(h11), l21 = h12 / l11, l31 = h13 / l11;
    const double p2 = h22 - l21 * l21;
    if (p2 > 1e-12 * h22) {
      const double l22 = sqrt(p2), l32 = (h23 - l31 * l21) / l22;
      const double p3 = h33 - l31 * l31 - l32 * l32;
      if (p3 > 1e-12 * h33) {
        const double l33 = sqrt(p3);
        const double y1 = e1 / l11, y2 = (e2 - l21 * y1) / l22, y3 = (e3 - l31 * y1 - l32 * y2) / l33;
        const double c = y3 / l33, b = (y2 - l32 * c) / l22, a = (y1 - l21 * b - l31 * c) / l11;
        const double nn = a * (a * h11 + b * h12 + c * h13) + b * (a * h12 + b * h22 + c * h23) +
                          c * (a * h13 + b * h23 + c * h33);  // |g1 w1 + g2 w2 + g3 w3|_A^2
        const double sum = fabs(a) * sqrt(h11) + fabs(b) * sqrt(h22) + fabs(c) * sqrt(h33);
        if (nn > 0.0 && sum * sum <= 256.0 * nn && !isinf(a) && !isinf(b) && !isinf(c) && a == a && b == b &&
            c == c) {
          g1 = a;
          g2 = b;
          g3 = c;
          return;
        }
      }
    }
  }
  galerkin_weights(e1, e2, h11, h12, h22, g1, g2);
}

// Preconditioned conjugate gradient in the Chronopoulos-Gear arrangement:
// both inner products of an iteration are taken after its single
// matrix-vector product, so one grid-wide reduction (one barrier) per
// iteration suffices.  The product w_{i+1} = A M^-1 r_{i+1} needs r_{i+1} at
// neighbouring rows; each block rebuilds those values from the neighbours'
// previous state (r_i, w_i, s_{i-1}: one 16-byte vector per row in each of
// three arrays, in the other half of a double buffer) instead of waiting for
// a second barrier.
//
//   p_i = u_i + b_i p_{i-1}        s_i = w_i + b_i s_{i-1}      (s_i = A p_i)
//   x_{i+1} = x_i + a_i p_i        r_{i+1} = r_i - a_i s_i      u = M^-1 r
//   w_{i+1} = A u_{i+1}            g = (r, u), d = (w, u)
//   b_{i+1} = g_{i+1} / g_i        a_{i+1} = g_{i+1} / (d_{i+1} - b_{i+1} g_{i+1} / a_i)
//
// The matrix is A_el (fixed rows removed) plus the spring diagonal: its
// diagonal is the Jacobi diagonal dg, its off-diagonal part is stored as a
// fixed-width ELL array (padded with the row itself and value 0) so every
// neighbour load of a row is issued at once.
// End of an outer iteration, run by the CG kernel after its last reduction:
// u += d on the rows each block owns, collision positions refreshed and, with
// self-collision, the query vertices inserted into the spatial hash (cleared
// by the contact/gather pass) for the next iteration's tet query;
// r_k = max|d| / diag and the convergence decision are taken by the last
// block to arrive (ticket).
// In the adjoint iteration (ADJ) the update is mu += d and a mesh is done once
// max|d| <= tol max|mu| over its vertices.
// MB (one workgroup per mesh): a workgroup whose CG broke down (skip) leaves
// its mesh as it is but still takes its ticket, so the last block's decisions
// see every block; the breakdown it flagged becomes the solve's status.
template <typename R, bool ADJ, bool MB>
__device__ __forceinline__ void finish_tail(const Dev<R>& d, const Consts& c, int row0, int row1, double* lds,
                                            bool skip) {
  __shared__ int last;
  const size_t n = (size_t)c.n;
  const W4<R>* x = reinterpret_cast<const W4<R>*>(d.dl);
  double dmax = 0.0;
  if (MB && skip) row1 = row0;
  for (int v0 = row0 + (int)(threadIdx.x & ~63u); v0 < row1; v0 += kPcgBlock) {
    // one wavefront handles 64 consecutive rows: the per-mesh maximum of |d|
    // is reduced in the wavefront when all its rows share a mesh
    const int v = v0 + (int)(threadIdx.x & 63);
    double dm = 0.0, um = 0.0;
    int m = -1;
    if (v < row1) {
      m = d.vmesh[v];
      if (!ADJ && mesh_frozen(d, c.mask_done, m)) {
        // a converged mesh of a batch: its positions stay as they are and its
        // CG rows start (and so stay) at zero
        W4<R>* dlw = reinterpret_cast<W4<R>*>(d.dl);
        W4<R>* dlp = reinterpret_cast<W4<R>*>(d.dlp);
        dlw[v] = w4<R>(R(0), R(0), R(0));
        dlp[v] = w4<R>(R(0), R(0), R(0));
        reinterpret_cast<W4<R>*>(d.dlpp)[v] = w4<R>(R(0), R(0), R(0));
      } else if (d.freem[v]) {
        const W4<R> dv = x[v];
        const R dd[3] = {dv.x, dv.y, dv.z};
        double uq = 0.0, xn[3] = {0.0, 0.0, 0.0};
        // accelerated local/global iteration: u stays at x_k, the update
        // (plain, accelerated or the fallback) is taken by k_faa_update
        const bool move = ADJ || !c.faa_m;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if (ADJ) {
            // with Anderson acceleration the update is taken by its own kernels
            const R mm = d.mu[k * n + v] + dd[k];
            if (!c.aa_m) d.mu[k * n + v] = mm;
            uq += (double)mm * (double)mm;
          } else if (move) {
            const R uu = d.u[k * n + v] + dd[k];
            d.u[k * n + v] = uu;
            xn[k] = d.X0[k * n + v] + (double)uu;
            d.xc[k * n + v] = xn[k];
          }
        }
        if (!ADJ && move && c.self_col && d.vq[v] >= 0) hash_insert_entry(d, c, d.vq[v], v, m, xn[0], xn[1], xn[2]);
        dm = sqrt(((double)dv.x * dv.x + (double)dv.y * dv.y) + (double)dv.z * dv.z);
        um = sqrt(uq);
      }
    }
    dmax = fmax(dmax, dm);
    const int m0 = __shfl(m, 0, 64);
    const bool uniform = __all(m == m0 || m < 0);
    if (uniform) {
      const double wm = wave_max(dm);
      if ((threadIdx.x & 63) == 0 && m0 >= 0 && wm > 0.0)
        atomicMax(&d.mres[m0], (unsigned long long)__double_as_longlong(wm));
      if (ADJ) {
        const double wu = wave_max(um);
        if ((threadIdx.x & 63) == 0 && m0 >= 0 && wu > 0.0)
          atomicMax(&d.mmax[m0], (unsigned long long)__double_as_longlong(wu));
      }
    } else if (m >= 0) {
      if (dm > 0.0) atomicMax(&d.mres[m], (unsigned long long)__double_as_longlong(dm));
      if (ADJ && um > 0.0) atomicMax(&d.mmax[m], (unsigned long long)__double_as_longlong(um));
    }
  }
  const double bm = block_max<kPcgBlock>(dmax, lds);
  if (threadIdx.x == 0) {
    d.part_f[blockIdx.x] = bm;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const int t = __hip_atomic_fetch_add(&d.st->ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = (t == (int)gridDim.x - 1);
    if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (!last) return;
  // read by every thread before thread 0 clears it below
  const unsigned mbl = MB ? d.st->mb_last : 0u;
  // the last block: the per-mesh convergence decisions (r = max|d| / diag,
  // active set unchanged), then, when the iteration is the last or traced,
  // the energy (fixed order per thread, then a fixed tree); the energy is
  // reported only, so the other iterations skip its partial sums
  DevStatus* st = d.st;
  const int it = st->iters + 1;
  double rloc = 0.0, active = 0.0, bad = 0.0;
  for (int mi = threadIdx.x; mi < c.M; mi += kPcgBlock) {
    const double dmx = __longlong_as_double((long long)d.mres[mi]);
    double r;
    if (ADJ) {
      const double umx = __longlong_as_double((long long)d.mmax[mi]);
      r = umx > 0.0 ? dmx / umx : (dmx > 0.0 ? INFINITY : 0.0);
      d.mmax[mi] = 0ull;
    } else {
      r = dmx * d.mesh[mi].inv_diag;
    }
    const bool was_running = d.mdone[mi] == 0;
    if (!(r == r) || (isinf(r) && !ADJ)) bad = 1.0;
    if (was_running) {
      rloc = fmax(rloc, r);
      if (c.fixed_iters <= 0 && r <= c.tol && (ADJ || !d.mchanged[mi])) d.mdone[mi] = it;
      if (d.mdone[mi] == 0) active += 1.0;
    }
    if (!ADJ && c.faa_m > 0) {
      // the accelerated iteration's decision for the point x_k just
      // evaluated (a mesh that converged now, or was frozen, takes none):
      // an accelerated point whose residual grew past (1 + slack) times the
      // last accepted one's is rejected and the history cleared; an
      // accepted point clears the history when its active set changed (the
      // map changed with it).  The energy guard decides below, after the
      // energy sum.
      AaMesh* a = d.faa + mi;
      int act = AA_NONE;
      if (was_running && d.mdone[mi] == 0) {
        act = AA_ACCEPT;
        if (a->cand && (c.faa_guard & 3) == GS_AA_GUARD_RESIDUAL && !(r <= (1.0 + c.faa_slack) * a->r_acc))
          act = AA_REJECT;
        if (a->cand && (c.faa_guard & GS_AA_GUARD_SET) && d.mchanged[mi]) act = AA_REJECT;
        if (act == AA_REJECT) {
          a->rejected += 1;
          a->cand = 0;
        } else {
          a->r_acc = r;
        }
        if (act == AA_REJECT || d.mchanged[mi]) {
          a->k = 0;
          a->head = 0;
          a->has_prev = 0;
        }
      }
      a->act = act;
    }
    d.mres[mi] = 0ull;
    if (!ADJ) d.mchanged[mi] = 0;
    if (MB) d.mbar[mi] = 0u;  // every block is past its mesh's last barrier
  }
  // the three block reductions in one LDS round (per-wave order and fixed
  // tree of block_sum / block_max); every thread reads the results
  __shared__ double lds4[4][kPcgBlock / 64];
  {
    const double b0 = wave_max(rloc), e0 = wave_sum(active), f0 = wave_sum(bad);
    if ((threadIdx.x & 63) == 0) {
      const int w = threadIdx.x >> 6;
      lds4[1][w] = b0;
      lds4[2][w] = e0;
      lds4[3][w] = f0;
    }
  }
  __syncthreads();
  double res = 0.0, n_act = 0.0, nbad = 0.0;
#pragma unroll
  for (int i = 0; i < kPcgBlock / 64; ++i) {
    res = fmax(res, lds4[1][i]);
    n_act += lds4[2][i];
    nbad += lds4[3][i];
  }
  int code = RUNNING;
  if (MB && (mbl >> 31)) nbad = 1.0;
  if (nbad > 0.0)
    code = BREAKDOWN;
  else if (c.fixed_iters > 0)
    code = (it >= c.fixed_iters) ? FIXED_DONE : RUNNING;
  else if (n_act == 0.0)
    code = CONVERGED;
  else if (it >= c.max_iter)
    code = MAXITER;
  double E = st->energy;
  const bool eguard = !ADJ && c.faa_m > 0 && (c.faa_guard & 3) == GS_AA_GUARD_ENERGY;
  if (!ADJ && (code != RUNNING || it <= c.trace_len || eguard)) {  // the same for every thread
    double eloc = 0.0;
    const int gl = c.a_parts, gg = gridDim.x;  // spring-energy partials: one per CG block
    for (int b = threadIdx.x; b < gl; b += kPcgBlock) eloc += d.part_a[b];
    for (int b = threadIdx.x; b < gg; b += kPcgBlock) eloc += d.part_b[b];
    const double a0 = wave_sum(eloc);
    if ((threadIdx.x & 63) == 0) lds4[0][threadIdx.x >> 6] = a0;
    __syncthreads();
    E = 0.0;
#pragma unroll
    for (int i = 0; i < kPcgBlock / 64; ++i) E += lds4[0][i];
    if (!(E == E)) code = BREAKDOWN;
  }
  if (threadIdx.x != 0) return;
  if constexpr (MB) {
    st->pcg_last = (int)(mbl & 0x7fffffffu);
    st->mb_last = 0u;
  }
  if (eguard) {
    // one mesh (thread 0 took its decision above): an accelerated point whose
    // energy exceeds the last accepted one's by more than the slack is rejected
    AaMesh* a = d.faa;
    if (a->act == AA_ACCEPT) {
      if (a->cand && !(E <= a->e_acc + c.faa_slack * fabs(a->e_acc))) {
        a->act = AA_REJECT;
        a->rejected += 1;
        a->cand = 0;
        a->k = 0;
        a->head = 0;
        a->has_prev = 0;
      } else {
        a->e_acc = E;
      }
    }
  }
  if (!ADJ && c.faa_m > 0) st->aa_pending = 1;
  st->residual = res;
  st->energy = E;
  st->iters = it;
  st->n_active = (int)n_act;
  const int changed = st->changed;
  if (it <= c.trace_len) {
    double* row = d.trace + 6 * (size_t)(it - 1);
    row[0] = res;
    row[1] = E;
    row[2] = (double)st->n_contacts;
    row[3] = (double)changed;
    row[4] = (double)st->pcg_last;
    row[5] = (double)st->ray_miss;
  }
  st->changed_last = changed;
  st->changed = 0;
  st->ray_miss_last = st->ray_miss;
  st->ray_miss = 0;
  st->n_contacts_last = st->n_contacts;
  st->n_contacts = 0;
  st->n_pen = 0;
  st->ticket = 0;
  st->bar_count = 0u;  // every block is past its last barrier
  if (c.bar2)
    for (int i = 0; i <= kBarGroups; ++i) d.bar2[64 * i] = 0u;
  __hip_atomic_store(&st->done, code, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Neighbour gathers are issued in chunks of CH rows of 16-byte vectors, all
// loads of a chunk in flight together.  In FP32 one chunk covers a 16-wide row
// (one dependent round of neighbour loads per row: faster than two rounds at
// twice the occupancy); FP64 rows use chunks of 4 to stay within registers.
template <typename R> struct Chunk { static constexpr int n = 16; };
template <> struct Chunk<double> { static constexpr int n = 4; };

template <typename R, int MW, bool ADJ, bool PAIR, bool CZ, bool MB, bool WB = false>
__global__ __launch_bounds__(kPcgBlock) void k_pcg(Dev<R> d, Consts c) {
  static_assert(!PAIR || (std::is_same<R, float>::value && MW == 16), "paired lanes: FP32, ELL width 16");
  constexpr int CH = Chunk<R>::n;
  __shared__ double lds[kPcgBlock / 64];
  __shared__ double lds2[12][kPcgBlock / 64];
  __shared__ double sh[16];
  // coarse correction (unpaired kernels): the coarse residual c = R0 r of
  // every row range, and the coarse solution y = A0^-1 c of the ranges this
  // workgroup's rows reach, in two buffers (iteration i's and i+1's)
  static_assert(!(PAIR && CZ), "the coarse correction runs in the unpaired kernels");
  static_assert(!(MB && (PAIR || CZ)), "one workgroup per mesh: the unpaired kernel, Jacobi");
  static_assert(!(WB && (PAIR || CZ || MB)), "write-back state: the unpaired whole-grid kernel");
  constexpr int CZG = CZ ? kCoarseMaxG : 1;
  __shared__ double cz_c[3][CZG];
  __shared__ double cz_y[2][3][CZG];
  if (is_done(d.st)) return;
  const int G = gridDim.x;
  const int stride = G * kPcgBlock;
  const int tid0 = blockIdx.x * kPcgBlock + threadIdx.x;
  const size_t n = (size_t)c.n;
  // CG state layout: element q (r, w, s) of row v at q * qs + v * vs in each
  // half.  The paired variant keeps three arrays of rows, so a wavefront's
  // (write-through) store covers whole cache lines; the others keep rows of
  // three vectors, one neighbour's state in one 48- or 96-byte record, which
  // suits their bandwidth-bound gathers.
  constexpr bool SOA = PAIR;
  const size_t qs = SOA ? n : 1, vs = SOA ? 1 : 3;
  // state that other blocks read after a barrier is written through (sc1):
  // the barrier's release then has little left to write back from L2.  In
  // the row-record layout a wavefront's 16-byte stores at a 48-byte stride
  // cover lines only partly, yet writing them through still beat assembling
  // the lines in L2 (about 10% per CG iteration on the 378,666-tet gripper at
  // 128 blocks)
  // (WB: ordinary write-back stores instead, for state far larger than the
  // caches, where merging a row record's three vectors in L2 saves HBM
  // writes)
  auto st_state = [&](W4<R>* base, unsigned i, const W4<R>& v) {
    if constexpr (WB)
      st_wb(base, i, v);
    else
      st_wt(base, i, v);
  };
  // each block owns one contiguous range of rows (a multiple of 64 long), so
  // the rows spread over all G blocks however many rows a thread gets
  const int chunk = ((c.n + G - 1) / G + 63) & ~63;
  // MB (a batch, per-mesh CG): the k workgroups of a mesh split its rows as
  // k workgroups split the rows of that mesh alone, and run its CG with its
  // own scalars and stopping test: their reductions are over the mesh's k
  // partials, their barriers wait for the mesh's workgroups only (a block
  // barrier when k = 1)
  const int4 sg = MB ? d.seg[blockIdx.x] : make_int4(0, 0, 0, 0);
  int row0, row1;
  if constexpr (MB) {
    const int vb = d.mesh[sg.x].vbeg, ve = d.mesh[sg.x].vend;
    const int ch = ((ve - vb + sg.z - 1) / sg.z + 63) & ~63;
    row0 = min(ve, vb + sg.y * ch);
    row1 = min(ve, row0 + ch);
  } else {
    row0 = min(c.n, (int)blockIdx.x * chunk);
    row1 = min(c.n, row0 + chunk);
  }
  const int Gr = MB ? sg.z : G;   // partials a reduction sums
  const int pg0 = MB ? sg.w : 0;  // and where they start
  // coarse correction: u = D^-1 r + R0^T y, y = A0^-1 R0 r, with R0 summing
  // the free rows of each workgroup's range.  Every workgroup holds the whole
  // coarse residual (thread t that of range t) and forms y for the ranges its
  // rows reach, one wavefront per range, in the same order in every
  // workgroup (so a row's u is the same wherever it is formed).
  constexpr bool cz = CZ;
  R czq[9];  // coarse: this thread's sums of r, w and s over its free rows
#pragma unroll
  for (int i = 0; i < 9; ++i) czq[i] = R(0);
  auto coarse_solve = [&](int buf) {
    if constexpr (CZ) {
      const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
      if (wv < kCoarseNb) {
        const int bb = d.cz_nb[blockIdx.x * kCoarseNb + wv];
        if (bb >= 0) {
          const double* Ar = d.cz_inv + (size_t)bb * G;
          double t0 = 0.0, t1 = 0.0, t2 = 0.0;
          for (int k = l; k < G; k += 64) {
            const double a = Ar[k];
            t0 += a * cz_c[0][k];
            t1 += a * cz_c[1][k];
            t2 += a * cz_c[2][k];
          }
          t0 = wave_sum(t0);
          t1 = wave_sum(t1);
          t2 = wave_sum(t2);
          if (l == 0) {
            cz_y[buf][0][bb] = t0;
            cz_y[buf][1][bb] = t1;
            cz_y[buf][2][bb] = t2;
          }
        }
      }
      __syncthreads();
    }
  };
  // block sums of gamma, delta and the range's sums of r, w and s (free rows)
  // in one LDS round, stored write-through by threads 0-10 (the order of
  // block_sum2_store): the next iteration forms the coarse residual
  // R0 r_{i+1} = R0 r_i - alpha (R0 w_i + beta R0 s_{i-1}) from these exact
  // sums, so it never drifts from the stored residual by more than one
  // step's rounding
  auto store11 = [&](double ag, double ad, double* og, double* od, double* oq) {
    double q[11];
    q[0] = ag;
    q[1] = ad;
#pragma unroll
    for (int i = 0; i < 9; ++i) q[2 + i] = (double)czq[i];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 11; ++i) {
      const double t = wave_sum(q[i]);
      if (lane == 0) lds2[i][wv] = t;
    }
    __syncthreads();
    if (threadIdx.x < 11) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < kPcgBlock / 64; ++i) t += lds2[threadIdx.x][i];
      double* dst = threadIdx.x == 0 ? og : (threadIdx.x == 1 ? od : oq + (size_t)(threadIdx.x - 2) * G);
      st_wt(dst, t);
    }
  };
  if (PAIR && 2 * chunk > kPcgBlock) {
    // launched for a grid with more rows per block than lane pairs (the host
    // chooses the variant from the same formula): refuse, uniformly
    if (blockIdx.x == 0 && threadIdx.x == 0)
      __hip_atomic_store(&d.st->done, (int)BREAKDOWN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  unsigned* bc = &d.st->bar_count;
  unsigned bar_target = 0;  // arrivals the next grid barrier waits for
  unsigned bar_inst = 0;    // barriers of this launch (two-level barrier)
  // the whole-grid barrier: flat, or (c.bar2) two-level for larger grids
  auto wbar = [&]() -> bool {
    if (c.bar2)
      return grid_barrier2(d.bar2, d.bar2 + 64 * kBarGroups, bar_inst, G, kBarGroups, &d.st->done, c.bar_timeout);
    return grid_barrier(bc, bar_target, G, &d.st->done, c.bar_timeout);
  };
  // the barrier that publishes the partials: grid-wide, or (MB) the block's
  auto gbar = [&]() -> bool {
    if constexpr (MB) {
      if (sg.z == 1) {
        __syncthreads();
        return true;
      }
      return grid_barrier(d.mbar + sg.x, bar_target, sg.z, &d.st->done, c.bar_timeout);
    } else {
      return wbar();
    }
  };
  W4<R>* __restrict__ x = reinterpret_cast<W4<R>*>(d.dl);
  W4<R>* __restrict__ p = reinterpret_cast<W4<R>*>(d.p);
  W4<R>* const cg0 = reinterpret_cast<W4<R>*>(d.cg);
  const R* __restrict__ dg = d.dg;
  const int32_t* __restrict__ ecol = d.ell_col;
  const R* __restrict__ evl = d.ell_val;
  R* __restrict__ evs = d.ell_scaled;

  // (A) r_0 = b - A x_0 from the warm start x_0; p_{-1} = s_{-1} = 0;
  //     right-hand-side norm b' M^-1 b; a_vj / dg_j.  Every solve starts from
  //     the A-norm-best combination of the previous correction and its first
  //     and second differences (a Galerkin projection of M d = b onto their
  //     span: never a worse start, in the A-norm, than the previous correction
  //     alone).  The forward solve first forms its right-hand side (phase 0);
  //     the adjoint kernels have formed theirs before the launch.
  double acc_b = 0.0, acc_g = 0.0, acc_d = 0.0;
  double rhs1 = 0.0;  // paired kernel, one mesh: b' M^-1 b, summed after the first barrier
  int cur = 0;  // half of the double-buffered CG state holding (r_0, w_0, s_0)
  // PAIR: lanes 2i and 2i+1 share row row0 + i from the start-up on, each
  // taking 8 of the row's 16 neighbour slots; the row's state passes from
  // phase to phase in registers
  const int pv_row = row0 + (int)(threadIdx.x >> 1), pv_half = (int)(threadIdx.x & 1);
  const bool pv_has = PAIR && pv_row < row1;
  int pj[8];
  R pa[8];
  W4<R> prc, pwc, psc, ppv, pxv;
  R pidg = R(0);
  W4<R> pb, pw1, pwp, pwpp, paw1, paw2, paw3;  // b, the history and its products
  R pdv = R(0);
  // sum of a row's own term and its two lanes' partial neighbour sums, in the
  // same order on both lanes: own, slots 0-7, slots 8-15
  auto pair_sum = [&](R own, R part) {
    const R o = __shfl_xor(part, 1, 64);
    return pv_half == 0 ? (own + part) + o : (own + o) + part;
  };
  {
    // (0) the outer iteration's contact update and right-hand side for the
    //     block's rows, each by the thread that then runs the row's first
    //     warm-start pass (which reads only the row's own b and diagonal);
    //     with self-collision the spatial hash is cleared for the final
    //     update's insertions (the iteration's tet query has run)
    if constexpr (!ADJ) {
      double esp = 0.0;
      if constexpr (PAIR) {
        if (pv_has) {
          if (pv_half == 0 && (c.self_col || c.obst_col || c.mo)) {
            const int s = d.vq[pv_row];
            if (s >= 0) contacts_one(d, c, s);
          }
          esp = gather_row_pair<SOA>(d, c, pv_row, pv_half, pb, pdv);
        }
      } else {
        for (int v = row0 + (int)threadIdx.x; v < row1; v += kPcgBlock) {
          if (c.self_col || c.obst_col || c.mo) {
            const int s = d.vq[v];
            if (s >= 0) contacts_one(d, c, s);
          }
          esp += gather_row<SOA>(d, c, v);
        }
      }
      // (MB: workgroups do not wait for each other, so one could clear what
      // another has already inserted; the host clears the hash before the
      // launch instead)
      if (c.self_col && !MB) {
        for (int i = tid0; i < c.H; i += stride) d.hcount[i] = 0;
        if (tid0 == 0) d.st->n_over = 0;
      }
      const double bs = block_sum<kPcgBlock>(esp, lds);
      if (threadIdx.x == 0) d.part_b[blockIdx.x] = bs;
    }
    // history: w1 = d_k, w2 = d_k - d_{k-1}, w3 = d_k - 2 d_{k-1} + d_{k-2}
    // (the last correction, its change and the change's change)
    W4<R>* __restrict__ xp = reinterpret_cast<W4<R>*>(d.dlp);
    W4<R>* __restrict__ xpp = reinterpret_cast<W4<R>*>(d.dlpp);
    double tq[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // e1 e2 e3 h11 h12 h13 h22 h23 h33
    double czb[12] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // unpaired kernels: 8 neighbour slots per gather round (the CG loop sets
    // their registers); the paired kernel's lanes take 8 slots each
    constexpr int CH1 = CH < 8 ? CH : 8;
    if constexpr (PAIR) {
      if (pv_has) {
        const int v = pv_row;
        if constexpr (ADJ) {  // the adjoint kernels formed b and the diagonal
          pb = cg0[v * vs];
          pdv = dg[v];
        }
        const R dv = pdv, idg = R(1) / dv;
        pw1 = x[v];
        pwp = xp[v];
        pwpp = xpp[v];
        const W4<R> w1 = pw1, wp = pwp, wpp = pwpp;
        const W4<R> w2 = w4<R>(w1.x - wp.x, w1.y - wp.y, w1.z - wp.z);
        const W4<R> w3 = w4<R>(w2.x - (wp.x - wpp.x), w2.y - (wp.y - wpp.y), w2.z - (wp.z - wpp.z));
        R s10 = R(0), s11 = R(0), s12 = R(0), s20 = R(0), s21 = R(0), s22 = R(0), s30 = R(0), s31 = R(0), s32 = R(0);
        W4<R> xn[8], pn[8], qn[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          pj[k] = ecol[(size_t)(8 * pv_half + k) * n + v];
          pa[k] = evl[(size_t)(8 * pv_half + k) * n + v];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          xn[k] = ld3(x + pj[k]);
          pn[k] = ld3(xp + pj[k]);
          qn[k] = ld3(xpp + pj[k]);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const R d0 = xn[k].x - pn[k].x, d1 = xn[k].y - pn[k].y, d2 = xn[k].z - pn[k].z;
          s10 += pa[k] * xn[k].x;
          s11 += pa[k] * xn[k].y;
          s12 += pa[k] * xn[k].z;
          s20 += pa[k] * d0;
          s21 += pa[k] * d1;
          s22 += pa[k] * d2;
          s30 += pa[k] * (d0 - (pn[k].x - qn[k].x));
          s31 += pa[k] * (d1 - (pn[k].y - qn[k].y));
          s32 += pa[k] * (d2 - (pn[k].z - qn[k].z));
        }
        const R a10 = pair_sum(dv * w1.x, s10), a11 = pair_sum(dv * w1.y, s11), a12 = pair_sum(dv * w1.z, s12);
        const R a20 = pair_sum(dv * w2.x, s20), a21 = pair_sum(dv * w2.y, s21), a22 = pair_sum(dv * w2.z, s22);
        const R a30 = pair_sum(dv * w3.x, s30), a31 = pair_sum(dv * w3.y, s31), a32 = pair_sum(dv * w3.z, s32);
        paw1 = w4<R>(a10, a11, a12);
        paw2 = w4<R>(a20, a21, a22);
        paw3 = w4<R>(a30, a31, a32);
        if (pv_half == 0) {
          const W4<R> b = pb;
          acc_b += ((double)b.x * (double)(b.x * idg) + (double)b.y * (double)(b.y * idg)) + (double)b.z * (double)(b.z * idg);
          const double t[9] = {((double)w1.x * b.x + (double)w1.y * b.y) + (double)w1.z * b.z,
                               ((double)w2.x * b.x + (double)w2.y * b.y) + (double)w2.z * b.z,
                               ((double)w3.x * b.x + (double)w3.y * b.y) + (double)w3.z * b.z,
                               ((double)w1.x * a10 + (double)w1.y * a11) + (double)w1.z * a12,
                               ((double)w1.x * a20 + (double)w1.y * a21) + (double)w1.z * a22,
                               ((double)w1.x * a30 + (double)w1.y * a31) + (double)w1.z * a32,
                               ((double)w2.x * a20 + (double)w2.y * a21) + (double)w2.z * a22,
                               ((double)w2.x * a30 + (double)w2.y * a31) + (double)w2.z * a32,
                               ((double)w3.x * a30 + (double)w3.y * a31) + (double)w3.z * a32};
          // A w1, A w2, A w3 for the neighbours' second pass
          st_state(cg0 + qs + row0 * vs, (unsigned)((v - row0) * vs), paw1);
          st_state(cg0 + 2 * qs + row0 * vs, (unsigned)((v - row0) * vs), paw2);
          st_state(p + row0, (unsigned)(v - row0), paw3);
          if (c.M > 1 && !MB) {
            double* q = reinterpret_cast<double*>(cg0 + 3 * n);
            q[v] = t[0];
            q[n + v] = t[1];
            q[2 * n + v] = t[3];
            q[3 * n + v] = t[4];
            q[4 * n + v] = t[6];
          } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) tq[i] += t[i];
          }
        }
      }
    } else {
      for (int v = row0 + (int)threadIdx.x; v < row1; v += kPcgBlock) {
        const R dv = dg[v], idg = R(1) / dv;
        const W4<R> w1 = x[v], wp = xp[v], wpp = xpp[v];
        const W4<R> w2 = w4<R>(w1.x - wp.x, w1.y - wp.y, w1.z - wp.z);
        const W4<R> w3 = w4<R>(w2.x - (wp.x - wpp.x), w2.y - (wp.y - wpp.y), w2.z - (wp.z - wpp.z));
        R a10 = dv * w1.x, a11 = dv * w1.y, a12 = dv * w1.z;
        R a20 = dv * w2.x, a21 = dv * w2.y, a22 = dv * w2.z;
        R a30 = dv * w3.x, a31 = dv * w3.y, a32 = dv * w3.z;
  #pragma unroll 1
        for (int k0 = 0; k0 < MW; k0 += CH1) {
          int jj[CH1];
          R aa[CH1];
          W4<R> xn[CH1], pn[CH1], qn[CH1];
  #pragma unroll
          for (int k = 0; k < CH1; ++k) {
            jj[k] = ecol[(size_t)(k0 + k) * n + v];
            aa[k] = evl[(size_t)(k0 + k) * n + v];
          }
  #pragma unroll
          for (int k = 0; k < CH1; ++k) {
            xn[k] = ld3(x + jj[k]);
            pn[k] = ld3(xp + jj[k]);
            qn[k] = ld3(xpp + jj[k]);
          }
  #pragma unroll
          for (int k = 0; k < CH1; ++k) {
            const R d0 = xn[k].x - pn[k].x, d1 = xn[k].y - pn[k].y, d2 = xn[k].z - pn[k].z;
            a10 += aa[k] * xn[k].x;
            a11 += aa[k] * xn[k].y;
            a12 += aa[k] * xn[k].z;
            a20 += aa[k] * d0;
            a21 += aa[k] * d1;
            a22 += aa[k] * d2;
            a30 += aa[k] * (d0 - (pn[k].x - qn[k].x));
            a31 += aa[k] * (d1 - (pn[k].y - qn[k].y));
            a32 += aa[k] * (d2 - (pn[k].z - qn[k].z));
          }
        }
        const W4<R> b = cg0[v * vs];
        acc_b += ((double)b.x * (double)(b.x * idg) + (double)b.y * (double)(b.y * idg)) + (double)b.z * (double)(b.z * idg);
        if constexpr (cz) if (d.freem[v]) {
          // range sums of b, A w1, A w2, A w3: the coarse residual of the start
          czb[0] += b.x, czb[1] += b.y, czb[2] += b.z;
          czb[3] += a10, czb[4] += a11, czb[5] += a12;
          czb[6] += a20, czb[7] += a21, czb[8] += a22;
          czb[9] += a30, czb[10] += a31, czb[11] += a32;
        }
        const double t[9] = {((double)w1.x * b.x + (double)w1.y * b.y) + (double)w1.z * b.z,
                             ((double)w2.x * b.x + (double)w2.y * b.y) + (double)w2.z * b.z,
                             ((double)w3.x * b.x + (double)w3.y * b.y) + (double)w3.z * b.z,
                             ((double)w1.x * a10 + (double)w1.y * a11) + (double)w1.z * a12,
                             ((double)w1.x * a20 + (double)w1.y * a21) + (double)w1.z * a22,
                             ((double)w1.x * a30 + (double)w1.y * a31) + (double)w1.z * a32,
                             ((double)w2.x * a20 + (double)w2.y * a21) + (double)w2.z * a22,
                             ((double)w2.x * a30 + (double)w2.y * a31) + (double)w2.z * a32,
                             ((double)w3.x * a30 + (double)w3.y * a31) + (double)w3.z * a32};
        // A w1, A w2, A w3 until the second pass (p is free until the first CG
        // iteration, which takes p_{-1} = 0 without reading it)
        // read by neighbouring rows of other blocks after the barrier
        st_state(cg0 + qs + row0 * vs, (unsigned)((v - row0) * vs), w4<R>(a10, a11, a12));
        st_state(cg0 + 2 * qs + row0 * vs, (unsigned)((v - row0) * vs), w4<R>(a20, a21, a22));
        st_state(p + row0, (unsigned)(v - row0), w4<R>(a30, a31, a32));
        if (c.M > 1 && !MB) {
          // a batch projects on (w1, w2): per-row terms, summed per mesh below,
          // in the half of the CG state the first iteration has yet to write
          double* q = reinterpret_cast<double*>(cg0 + 3 * n);
          q[v] = t[0];
          q[n + v] = t[1];
          q[2 * n + v] = t[3];
          q[3 * n + v] = t[4];
          q[4 * n + v] = t[6];
        } else {
  #pragma unroll
          for (int i = 0; i < 9; ++i) tq[i] += t[i];
        }
      }
    }
    double g1 = 0.0, g2 = 0.0, g3 = 0.0;
    if (c.M == 1 || MB) {
      // partials at part_c[(2 + i) G + block]: the nine terms, then b' M^-1 b
      // (also in part_d).  The paired kernel reads the ten grid sums in one
      // round after the barrier; the unpaired kernels, whose registers the CG
      // loop fills, read the nine terms in two and b' M^-1 b after the next
      // barrier.
      const double q[10] = {tq[0], tq[1], tq[2], tq[3], tq[4], tq[5], tq[6], tq[7], tq[8], acc_b};
      block_sums_store<10>(q, lds2, d.part_c + 2 * G + blockIdx.x, G);
      if (!PAIR && threadIdx.x == 9) d.part_d[blockIdx.x] = d.part_c[11 * G + blockIdx.x];
      if constexpr (cz) {
        __syncthreads();  // lds2 is read above before it is written again
        block_sums_store<12>(czb, lds2, d.part_f + 18 * G + blockIdx.x, G);
      }
      if (!gbar()) return;
      double S[10];
      if constexpr (PAIR) {
        grid_sums<10>(d.part_c + 2 * G + pg0, G, Gr, sh, S);
        rhs1 = S[9];
      } else {
        double S1[5], S2[4];
        grid_sums<5>(d.part_c + 2 * G + pg0, G, Gr, sh, S1);
        grid_sums<4>(d.part_c + 7 * G + pg0, G, Gr, sh + 8, S2);
#pragma unroll
        for (int i = 0; i < 5; ++i) S[i] = S1[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) S[5 + i] = S2[i];
      }
      // every block takes the same decision from the same sums
      galerkin_weights3(S[0], S[1], S[2], S[3], S[4], S[5], S[6], S[7], S[8], g1, g2, g3);
      if constexpr (cz) {
        // c_0 = R0 (b - g1 A w1 - g2 A w2 - g3 A w3), every range's by its thread
        for (int t = threadIdx.x; t < G; t += kPcgBlock)
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const double* P = d.part_f + 18 * G + t;
            cz_c[k][t] = ((P[k * G] - g1 * P[(3 + k) * G]) - g2 * P[(6 + k) * G]) - g3 * P[(9 + k) * G];
          }
        __syncthreads();
        coarse_solve(0);
      }
    } else {
      const double bs = block_sum<kPcgBlock>(acc_b, lds);
      if (threadIdx.x == 0) d.part_d[blockIdx.x] = bs;
      // a batch: each mesh gets its own weights (the meshes' systems are
      // independent), its sums taken by one block in a fixed order
      if (!wbar()) return;
      const double* q = reinterpret_cast<const double*>(cg0 + 3 * n);
      for (int m = blockIdx.x; m < c.M; m += G) {
        const int v0 = d.mesh[m].vbeg, v1 = d.mesh[m].vend;
        double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int v = v0 + (int)threadIdx.x; v < v1; v += kPcgBlock)
#pragma unroll
          for (int i = 0; i < 5; ++i) t[i] += q[i * n + v];
        double S[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) S[i] = block_sum<kPcgBlock>(t[i], lds);
        if (threadIdx.x == 0) {
          double m1, m2;
          galerkin_weights(S[0], S[1], S[2], S[3], S[4], m1, m2);
          d.mgam[2 * m] = m1;
          d.mgam[2 * m + 1] = m2;
        }
      }
      if (!wbar()) return;
    }
    // x_0, r_0 = b - g1 A w1 - g2 A w2 - g3 A w3 and, in the same pass,
    // w_0 = A u_0: the neighbours' r_0 are rebuilt from their
    // (b, A w1, A w2, A w3) as the CG iterations rebuild r_{i+1}, so no barrier
    // separates the two.  A row's neighbours belong to its mesh and share its
    // weights.  The start goes to the other half of the CG state, whose
    // (b, A w1, A w2) other blocks are still reading; the history moves on.
    constexpr int CH2 = CH < 4 ? CH : 4;
    W4<R>* __restrict__ ns = cg0 + 3 * n;
    if constexpr (PAIR) {
      if (pv_has) {
        const int v = pv_row;
        R r1 = (R)g1, r2 = (R)g2, r3 = (R)g3;
        if (c.M > 1 && !MB) {
          const int m = d.vmesh[v];
          r1 = (R)d.mgam[2 * m];
          r2 = (R)d.mgam[2 * m + 1];
          r3 = R(0);
        }
        const R idg = R(1) / pdv;
        const W4<R> b = pb, aw1 = paw1, aw2 = paw2, aw3 = paw3;
        const W4<R> rv = w4<R>(b.x - r1 * aw1.x - r2 * aw2.x - r3 * aw3.x, b.y - r1 * aw1.y - r2 * aw2.y - r3 * aw3.y,
                               b.z - r1 * aw1.z - r2 * aw2.z - r3 * aw3.z);
        W4<R> nb[8], n1[8], n2[8], n3[8];
        R dgn[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          nb[k] = ld3(cg0 + pj[k] * vs);
          n1[k] = ld3(cg0 + qs + pj[k] * vs);
          n2[k] = ld3(cg0 + 2 * qs + pj[k] * vs);
          n3[k] = ld3(p + pj[k]);
          dgn[k] = dg[pj[k]];
        }
        R s0 = R(0), s1 = R(0), s2 = R(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          // a_vj / dg_j, kept for the CG iterations
          pa[k] = pa[k] / dgn[k];
          evs[(size_t)(8 * pv_half + k) * n + v] = pa[k];
          s0 += pa[k] * (nb[k].x - r1 * n1[k].x - r2 * n2[k].x - r3 * n3[k].x);
          s1 += pa[k] * (nb[k].y - r1 * n1[k].y - r2 * n2[k].y - r3 * n3[k].y);
          s2 += pa[k] * (nb[k].z - r1 * n1[k].z - r2 * n2[k].z - r3 * n3[k].z);
        }
        const R a0 = pair_sum(rv.x, s0), a1 = pair_sum(rv.y, s1), a2 = pair_sum(rv.z, s2);
        const W4<R> w1 = pw1, wp = pwp, wpp = pwpp;
        const W4<R> w2 = w4<R>(w1.x - wp.x, w1.y - wp.y, w1.z - wp.z);
        const W4<R> w3 = w4<R>(w2.x - (wp.x - wpp.x), w2.y - (wp.y - wpp.y), w2.z - (wp.z - wpp.z));
        const W4<R> x0 = w4<R>(r1 * w1.x + r2 * w2.x + r3 * w3.x, r1 * w1.y + r2 * w2.y + r3 * w3.y,
                               r1 * w1.z + r2 * w2.z + r3 * w3.z);
        if (pv_half == 0) {
          const unsigned vi = (unsigned)(v - row0);
          st_state(x + row0, vi, x0);
          st_state(xpp + row0, vi, wp);
          st_state(xp + row0, vi, w1);
          st_state(ns + row0 * vs, (unsigned)(vi * vs), rv);
          st_state(ns + qs + row0 * vs, (unsigned)(vi * vs), w4<R>(a0, a1, a2));
          st_state(ns + 2 * qs + row0 * vs, (unsigned)(vi * vs), w4<R>(R(0), R(0), R(0)));
          const R u0 = rv.x * idg, u1 = rv.y * idg, u2 = rv.z * idg;
          acc_g += ((double)rv.x * u0 + (double)rv.y * u1) + (double)rv.z * u2;
          acc_d += ((double)a0 * u0 + (double)a1 * u1) + (double)a2 * u2;
        }
        // the row's state for the CG iterations
        prc = rv;
        pwc = w4<R>(a0, a1, a2);
        psc = w4<R>(R(0), R(0), R(0));
        ppv = w4<R>(R(0), R(0), R(0));  // p_{-1} = 0
        pxv = x0;
        pidg = idg;
      }
    } else {
      for (int v = row0 + (int)threadIdx.x; v < row1; v += kPcgBlock) {
        R r1 = (R)g1, r2 = (R)g2, r3 = (R)g3;
        if (c.M > 1 && !MB) {
          const int m = d.vmesh[v];
          r1 = (R)d.mgam[2 * m];
          r2 = (R)d.mgam[2 * m + 1];
          r3 = R(0);
        }
        const R idg = R(1) / dg[v];
        const W4<R> w1 = x[v], wp = xp[v], wpp = xpp[v];
        const W4<R> b = cg0[v * vs], aw1 = cg0[qs + v * vs], aw2 = cg0[2 * qs + v * vs], aw3 = p[v];
        const W4<R> rv = w4<R>(b.x - r1 * aw1.x - r2 * aw2.x - r3 * aw3.x, b.y - r1 * aw1.y - r2 * aw2.y - r3 * aw3.y,
                               b.z - r1 * aw1.z - r2 * aw2.z - r3 * aw3.z);
        R a0 = rv.x, a1 = rv.y, a2 = rv.z;  // dg_v * (r_v / dg_v)
  #pragma unroll 1
        for (int k0 = 0; k0 < MW; k0 += CH2) {
          int jj[CH2];
          R aa[CH2], dgn[CH2];
  #pragma unroll
          for (int k = 0; k < CH2; ++k) {
            jj[k] = ecol[(size_t)(k0 + k) * n + v];
            aa[k] = evl[(size_t)(k0 + k) * n + v];
          }

          W4<R> nb[CH2], n1[CH2], n2[CH2], n3[CH2];
  #pragma unroll
          for (int k = 0; k < CH2; ++k) {
            nb[k] = ld3(cg0 + jj[k] * vs);
            n1[k] = ld3(cg0 + qs + jj[k] * vs);
            n2[k] = ld3(cg0 + 2 * qs + jj[k] * vs);
            n3[k] = ld3(p + jj[k]);
            dgn[k] = dg[jj[k]];
          }
          // a_vj / dg_j for the CG iterations (the neighbours' diagonals of
          // this outer iteration are visible past the barrier above)
  #pragma unroll
          for (int k = 0; k < CH2; ++k) {
            aa[k] = aa[k] / dgn[k];
            evs[(size_t)(k0 + k) * n + v] = aa[k];
          }
  #pragma unroll
          for (int k = 0; k < CH2; ++k) {
            a0 += aa[k] * (nb[k].x - r1 * n1[k].x - r2 * n2[k].x - r3 * n3[k].x);
            a1 += aa[k] * (nb[k].y - r1 * n1[k].y - r2 * n2[k].y - r3 * n3[k].y);
            a2 += aa[k] * (nb[k].z - r1 * n1[k].z - r2 * n2[k].z - r3 * n3[k].z);
          }
        }
        const W4<R> w2 = w4<R>(w1.x - wp.x, w1.y - wp.y, w1.z - wp.z);
        const W4<R> w3 = w4<R>(w2.x - (wp.x - wpp.x), w2.y - (wp.y - wpp.y), w2.z - (wp.z - wpp.z));
        const unsigned vi = (unsigned)(v - row0);
        st_state(x + row0, vi,
              w4<R>(r1 * w1.x + r2 * w2.x + r3 * w3.x, r1 * w1.y + r2 * w2.y + r3 * w3.y,
                    r1 * w1.z + r2 * w2.z + r3 * w3.z));
        R u0 = rv.x * idg, u1 = rv.y * idg, u2 = rv.z * idg;
        if constexpr (cz) {
          // w_0 = A u_0 with u_0 = D^-1 r_0 + R0^T y_0: the row's own range
          // (its diagonal and its neighbours there) and the other ranges
          const R fr = d.freem[v] ? R(1) : R(0);
          const W4<R> q = reinterpret_cast<const W4<R>*>(d.cz_rho)[v];
          const int i1 = d.cz_ri[v] & 0xffff, i2 = d.cz_ri[v] >> 16;
          const R cf = dg[v] * fr + q.x;
          const R y0 = (R)cz_y[0][0][blockIdx.x], y1 = (R)cz_y[0][1][blockIdx.x], y2 = (R)cz_y[0][2][blockIdx.x];
          a0 += (cf * y0 + q.y * (R)cz_y[0][0][i1]) + q.z * (R)cz_y[0][0][i2];
          a1 += (cf * y1 + q.y * (R)cz_y[0][1][i1]) + q.z * (R)cz_y[0][1][i2];
          a2 += (cf * y2 + q.y * (R)cz_y[0][2][i1]) + q.z * (R)cz_y[0][2][i2];
          u0 += fr * y0;
          u1 += fr * y1;
          u2 += fr * y2;
          czq[0] += fr * rv.x;
          czq[1] += fr * rv.y;
          czq[2] += fr * rv.z;
          czq[3] += fr * a0;
          czq[4] += fr * a1;
          czq[5] += fr * a2;  // s_{-1} = 0: czq[6..8] stay 0
        }
        st_state(xpp + row0, vi, wp);
        st_state(xp + row0, vi, w1);
        st_state(ns + row0 * vs, (unsigned)(vi * vs), rv);
        st_state(ns + qs + row0 * vs, (unsigned)(vi * vs), w4<R>(a0, a1, a2));
        st_state(ns + 2 * qs + row0 * vs, (unsigned)(vi * vs), w4<R>(R(0), R(0), R(0)));
        acc_g += ((double)rv.x * u0 + (double)rv.y * u1) + (double)rv.z * u2;
        acc_d += ((double)a0 * u0 + (double)a1 * u1) + (double)a2 * u2;
      }
    }
    cur = 1;
  }
  if constexpr (cz)
    store11(acc_g, acc_d, d.part_c + blockIdx.x, d.part_e + blockIdx.x, d.part_f + blockIdx.x);
  else
    block_sum2_store(acc_g, acc_d, lds2, d.part_c + blockIdx.x, d.part_e + blockIdx.x);
  if (!gbar()) return;
  // PAIR: the lane pair's first neighbour gather, issued before the grid
  // sums so the round trips overlap
  // the neighbours' (r, w, s) of the coming iteration, loaded right after the
  // barrier that publishes them, while the partial sums are read
  W4<R> nr[8], nw[8], nsv[8];
  auto gather = [&](const W4<R>* cs) {
    if (pv_has) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        nr[k] = ld3(cs + pj[k] * vs);
        nw[k] = ld3(cs + qs + pj[k] * vs);
        nsv[k] = ld3(cs + 2 * qs + pj[k] * vs);
      }
    }
  };
  if constexpr (PAIR) {
    gather(cg0 + cur * 3 * n);
  }
  double gam, del, rhs = rhs1, dummy;
  grid_sum2(d.part_c + pg0, d.part_e + pg0, Gr, sh, gam, del);
  if (!PAIR || c.M > 1) grid_sum2(d.part_d + pg0, d.part_d + pg0, Gr, sh, rhs, dummy);
  gam = uniform_d(gam);
  del = uniform_d(del);
  rhs = uniform_d(rhs);
  // inner tolerance: fixed, or (pcg_eta_min > 0) the last outer residual
  // (the forward r_k, or the adjoint's relative change of mu) clamped to
  // [pcg_eta_min, pcg_eta]
  double eta = c.pcg_eta;
  if (c.pcg_eta_min > 0.0) eta = fmin(c.pcg_eta, fmax(c.pcg_eta_min, d.st->residual));
  const double stop = uniform_d(eta * eta * rhs);
  int it = 0;
  bool broke = !(rhs >= 0.0) || isinf(rhs) || !(gam >= 0.0) || isinf(gam);
  bool run = !broke && gam > stop;
  if (run && !(del > 0.0 && !isinf(del))) {
    broke = true;
    run = false;
  }
  double al = run ? gam / del : 0.0, be = 0.0;
  // End of an iteration after its row work: block partials, the grid
  // barrier, the grid sums and the next step lengths; false ends the solve.
  // publish: the iteration's block partials, then the grid barrier (partial
  // sums alternate halves so a slow block still reading the previous
  // iteration's sums is never overwritten)
  // (false: the barrier gave up, and the kernel must end at once)
  auto publish = [&](double ag, double ad) -> bool {
    const int half = (it & 1) ? 0 : G;
    if constexpr (cz)
      store11(ag, ad, d.part_c + half + blockIdx.x, d.part_e + half + blockIdx.x,
              d.part_f + ((it & 1) ? 0 : 9 * G) + blockIdx.x);
    else
      block_sum2_store(ag, ad, lds2, d.part_c + half + blockIdx.x, d.part_e + half + blockIdx.x);
    return gbar();
  };
  // coarse: at the top of iteration i, c_{i+1} = R0 r_i - alpha (R0 w_i +
  // beta R0 s_{i-1}) for every range (thread t: range t) from the sums
  // published with the last barrier (the start-up's at offset 0, iteration
  // i-1's at its half), then y_{i+1} into the other buffer
  int ycur = 0;
  auto coarse_advance = [&]() {
    const int src = it == 0 ? 0 : (((it - 1) & 1) ? 0 : 9 * G);
    for (int t = threadIdx.x; t < G; t += kPcgBlock) {
      const double* P = d.part_f + src + t;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        cz_c[k][t] = P[(size_t)k * G] - al * (P[(size_t)(3 + k) * G] + be * P[(size_t)(6 + k) * G]);
    }
    __syncthreads();
    coarse_solve(ycur ^ 1);
  };
  // advance: the grid sums of the published partials and the next step
  // lengths; false ends the solve
  auto advance = [&]() -> bool {
    const int half = (it & 1) ? 0 : G;
    double gn, dn;
    grid_sum2<false>(d.part_c + half + pg0, d.part_e + half + pg0, Gr, sh + 2 * (it & 1), gn, dn);
    gn = uniform_d(gn);
    dn = uniform_d(dn);
    ++it;
    cur ^= 1;
    if (!(gn >= 0.0) || isinf(gn) || !(dn == dn) || isinf(dn)) {
      broke = true;
      return false;
    }
    if (gn <= stop) return false;
    const double bn = gn / gam;
    const double den = dn - bn * gn / al;
    if (!(den > 0.0)) {
      broke = true;
      return false;
    }
    al = uniform_d(gn / den);
    be = uniform_d(bn);
    gam = gn;
    return true;
  };
  bool stalled = false;
  auto next_step = [&](double ag, double ad) -> bool {
    if (!publish(ag, ad)) {
      stalled = true;
      return false;
    }
    return advance();
  };
  // PAIR (FP32, ELL width 16, at most kPcgBlock / 2 rows per block):
  // lanes 2i and 2i+1 share row row0 + i, each gathering 8 of its 16
  // neighbour slots, and the row's own state (r, w, s, p, x, 1/dg) and its
  // lane's ELL columns and scaled values stay in registers through the
  // iterations.  An iteration then has one level of dependent memory reads
  // (the neighbours' r, w, s) instead of two.
  if constexpr (PAIR) {
    {
      while (run && it < c.pcg_max) {
        W4<R>* ns = cg0 + (cur ^ 1) * 3 * n;
        const R ra = (R)al, rb = (R)be;
        acc_g = 0.0;
        acc_d = 0.0;
        if (pv_has) {
          const W4<R> pv = w4<R>(prc.x * pidg + rb * ppv.x, prc.y * pidg + rb * ppv.y, prc.z * pidg + rb * ppv.z);
          const W4<R> sv = w4<R>(pwc.x + rb * psc.x, pwc.y + rb * psc.y, pwc.z + rb * psc.z);
          const W4<R> rv = w4<R>(prc.x - ra * sv.x, prc.y - ra * sv.y, prc.z - ra * sv.z);
          ppv = pv;
          pxv = w4<R>(pxv.x + ra * pv.x, pxv.y + ra * pv.y, pxv.z + ra * pv.z);
          R a0 = R(0), a1 = R(0), a2 = R(0);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            a0 += pa[k] * (nr[k].x - ra * (nw[k].x + rb * nsv[k].x));
            a1 += pa[k] * (nr[k].y - ra * (nw[k].y + rb * nsv[k].y));
            a2 += pa[k] * (nr[k].z - ra * (nw[k].z + rb * nsv[k].z));
          }
          // both lanes form (own term) + (slots 0-7) + (slots 8-15) in that order
          const R b0 = __shfl_xor(a0, 1, 64), b1 = __shfl_xor(a1, 1, 64), b2 = __shfl_xor(a2, 1, 64);
          const W4<R> wn = pv_half == 0 ? w4<R>(rv.x + a0 + b0, rv.y + a1 + b1, rv.z + a2 + b2)
                                        : w4<R>(rv.x + b0 + a0, rv.y + b1 + a1, rv.z + b2 + a2);
          if (pv_half == 0) {
            const unsigned vi = (unsigned)(pv_row - row0);
            st_state(ns + row0 * vs, (unsigned)(vi * vs), rv);
            st_state(ns + qs + row0 * vs, (unsigned)(vi * vs), wn);
            st_state(ns + 2 * qs + row0 * vs, (unsigned)(vi * vs), sv);
            const R u0 = rv.x * pidg, u1 = rv.y * pidg, u2 = rv.z * pidg;
            acc_g = ((double)rv.x * u0 + (double)rv.y * u1) + (double)rv.z * u2;
            acc_d = ((double)wn.x * u0 + (double)wn.y * u1) + (double)wn.z * u2;
          }
          prc = rv;
          pwc = wn;
          psc = sv;
        }
        if (!publish(acc_g, acc_d)) return;
        gather(ns);
        if (!advance()) break;
      }
      if (pv_has && pv_half == 0) x[pv_row] = pxv;
      // the final update reads x with one row per thread, other wavefronts
      // than the lane pairs that wrote it
      __syncthreads();
    }
  }
  if constexpr (!PAIR)
  while (run && it < c.pcg_max) {
    const W4<R>* cs = cg0 + cur * 3 * n;
    W4<R>* ns = cg0 + (cur ^ 1) * 3 * n;
    const R ra = (R)al, rb = (R)be;
    acc_g = 0.0;
    acc_d = 0.0;
    R yc0 = R(0), yc1 = R(0), yc2 = R(0), yn0 = R(0), yn1 = R(0), yn2 = R(0);
    if constexpr (cz) {
      coarse_advance();
#pragma unroll
      for (int i = 0; i < 9; ++i) czq[i] = R(0);
      yc0 = (R)cz_y[ycur][0][blockIdx.x];
      yc1 = (R)cz_y[ycur][1][blockIdx.x];
      yc2 = (R)cz_y[ycur][2][blockIdx.x];
      yn0 = (R)cz_y[ycur ^ 1][0][blockIdx.x];
      yn1 = (R)cz_y[ycur ^ 1][1][blockIdx.x];
      yn2 = (R)cz_y[ycur ^ 1][2][blockIdx.x];
    }
    for (int v = row0 + (int)threadIdx.x; v < row1; v += kPcgBlock) {
      const R idg = R(1) / dg[v];
      const W4<R> rc = cs[v * vs], wc = cs[qs + v * vs], sc = cs[2 * qs + v * vs];
      const W4<R> pv0 = p[v];  // at i = 0 b_0 = 0: p_{-1} enters as 0 * (finite start-up data)
      const W4<R> xv = x[v];
      // u_i = D^-1 r_i (+ R0^T y_i with the coarse correction)
      const R fr = (cz && d.freem[v]) ? R(1) : R(0);
      const W4<R> pv = cz ? w4<R>((rc.x * idg + fr * yc0) + rb * pv0.x, (rc.y * idg + fr * yc1) + rb * pv0.y,
                                  (rc.z * idg + fr * yc2) + rb * pv0.z)
                          : w4<R>(rc.x * idg + rb * pv0.x, rc.y * idg + rb * pv0.y, rc.z * idg + rb * pv0.z);
      const W4<R> sv = w4<R>(wc.x + rb * sc.x, wc.y + rb * sc.y, wc.z + rb * sc.z);
      const W4<R> rv = w4<R>(rc.x - ra * sv.x, rc.y - ra * sv.y, rc.z - ra * sv.z);
      const unsigned vi = (unsigned)(v - row0);
      st_state(p + row0, vi, pv);
      st_state(x + row0, vi, w4<R>(xv.x + ra * pv.x, xv.y + ra * pv.y, xv.z + ra * pv.z));
      R a0 = rv.x, a1 = rv.y, a2 = rv.z;  // dg_v * (r_v / dg_v)
#pragma unroll 1
      for (int k0 = 0; k0 < MW; k0 += CH) {
        int jj[CH];
        R aa[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          if constexpr (WB) {
            // streamed once per iteration: kept from displacing the
            // neighbours' state lines in L2
            jj[k] = __builtin_nontemporal_load(&ecol[(size_t)(k0 + k) * n + v]);
            aa[k] = __builtin_nontemporal_load(&evs[(size_t)(k0 + k) * n + v]);
          } else {
            jj[k] = ecol[(size_t)(k0 + k) * n + v];
            aa[k] = evs[(size_t)(k0 + k) * n + v];
          }
        }

        W4<R> nr[CH], nw[CH], nsv[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          nr[k] = ld3(cs + jj[k] * vs);
          nw[k] = ld3(cs + qs + jj[k] * vs);
          nsv[k] = ld3(cs + 2 * qs + jj[k] * vs);
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          a0 += aa[k] * (nr[k].x - ra * (nw[k].x + rb * nsv[k].x));
          a1 += aa[k] * (nr[k].y - ra * (nw[k].y + rb * nsv[k].y));
          a2 += aa[k] * (nr[k].z - ra * (nw[k].z + rb * nsv[k].z));
        }
      }
      R u0 = rv.x * idg, u1 = rv.y * idg, u2 = rv.z * idg;
      if constexpr (cz) {
        // w_{i+1} = A u_{i+1}: A R0^T y_{i+1} from the row's couplings to its
        // own range (with the diagonal) and to at most two others
        const W4<R> q = reinterpret_cast<const W4<R>*>(d.cz_rho)[v];
        const int i1 = d.cz_ri[v] & 0xffff, i2 = d.cz_ri[v] >> 16;
        const R cf = dg[v] * fr + q.x;
        const int nb = ycur ^ 1;
        a0 += (cf * yn0 + q.y * (R)cz_y[nb][0][i1]) + q.z * (R)cz_y[nb][0][i2];
        a1 += (cf * yn1 + q.y * (R)cz_y[nb][1][i1]) + q.z * (R)cz_y[nb][1][i2];
        a2 += (cf * yn2 + q.y * (R)cz_y[nb][2][i1]) + q.z * (R)cz_y[nb][2][i2];
        u0 += fr * yn0;
        u1 += fr * yn1;
        u2 += fr * yn2;
        czq[0] += fr * rv.x;
        czq[1] += fr * rv.y;
        czq[2] += fr * rv.z;
        czq[3] += fr * a0;
        czq[4] += fr * a1;
        czq[5] += fr * a2;
        czq[6] += fr * sv.x;
        czq[7] += fr * sv.y;
        czq[8] += fr * sv.z;
      }
      st_state(ns + row0 * vs, (unsigned)(vi * vs), rv);
      st_state(ns + qs + row0 * vs, (unsigned)(vi * vs), w4<R>(a0, a1, a2));
      st_state(ns + 2 * qs + row0 * vs, (unsigned)(vi * vs), sv);
      acc_g += ((double)rv.x * u0 + (double)rv.y * u1) + (double)rv.z * u2;
      acc_d += ((double)a0 * u0 + (double)a1 * u1) + (double)a2 * u2;
    }
    ycur ^= 1;
    if (!next_step(acc_g, acc_d)) break;
  }
  if (stalled) return;
  if (MB && threadIdx.x == 0 && sg.y == 0) {
    // each mesh's CG iterations summed over the batch; the longest one, and a
    // breakdown, for the last block (the status is stored only there, so a
    // workgroup that starts late still runs)
    atomicAdd(&d.st->pcg_total, it);
    atomicMax(&d.st->mb_last, (unsigned)it | (broke ? 0x80000000u : 0u));
  } else if (!MB && blockIdx.x == 0 && threadIdx.x == 0) {
    d.st->pcg_total += it;
    d.st->pcg_last = it;
    if (broke) __hip_atomic_store(&d.st->done, (int)BREAKDOWN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!broke || MB) {
    finish_tail<R, ADJ, MB>(d, c, row0, row1, lds, broke);
  } else if (threadIdx.x == 0) {
    // every block leaves after the same barrier; the last one out clears the
    // barrier counter for the next launch
    const int t = __hip_atomic_fetch_add(&d.st->ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t == G - 1) {
      d.st->ticket = 0;
      d.st->bar_count = 0u;
      if (c.bar2)
        for (int i = 0; i <= kBarGroups; ++i) d.bar2[64 * i] = 0u;
    }
  }
}

template <typename R>
hipError_t launch_hash_clear(const Dev<R>& d, const Consts& c, hipStream_t s) {
  k_hash_clear<R><<<max(1, min(cdiv(c.H, kBlock), 1024)), kBlock, 0, s>>>(d, c);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_init(const Dev<R>& d, const Consts& c, const R* xin, hipStream_t s) {
  k_init<R><<<max(1, cdiv(c.n, kBlock)), kBlock, 0, s>>>(d, c, xin);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_set_positions(const Dev<R>& d, const Consts& c, const R* x, hipStream_t s) {
  k_set_positions<R><<<max(1, cdiv(c.n, kBlock)), kBlock, 0, s>>>(d, c, x);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_output(const Dev<R>& d, const Consts& c, R* xout, hipStream_t s) {
  k_output<R><<<max(1, cdiv(c.n, kBlock)), kBlock, 0, s>>>(d, c, xout);
  return hipGetLastError();
}



// The CG kernel for a matrix of ELL width ell_w; pair selects the
// paired-lane variant (FP32, width 16 only), cz the unpaired variant with the
// coarse correction, mb the unpaired variant that runs per mesh, wb the
// unpaired whole-grid variant with write-back state stores.
template <typename R>
const void* pcg_kernel(int ell_w, bool adjoint, bool pair, bool cz, bool mb = false, bool wb = false) {
  if (mb) {
    if (adjoint)
      return ell_w <= 16 ? (const void*)k_pcg<R, 16, true, false, false, true>
                         : ell_w <= 32 ? (const void*)k_pcg<R, 32, true, false, false, true>
                                       : (const void*)k_pcg<R, 64, true, false, false, true>;
    return ell_w <= 16 ? (const void*)k_pcg<R, 16, false, false, false, true>
                       : ell_w <= 32 ? (const void*)k_pcg<R, 32, false, false, false, true>
                                     : (const void*)k_pcg<R, 64, false, false, false, true>;
  }
  if constexpr (std::is_same<R, float>::value) {
    if (pair && ell_w <= 16)
      return adjoint ? (const void*)k_pcg<R, 16, true, true, false, false> : (const void*)k_pcg<R, 16, false, true, false, false>;
  }
  if (cz) {
    if (adjoint)
      return ell_w <= 16 ? (const void*)k_pcg<R, 16, true, false, true, false>
                         : ell_w <= 32 ? (const void*)k_pcg<R, 32, true, false, true, false>
                                       : (const void*)k_pcg<R, 64, true, false, true, false>;
    return ell_w <= 16 ? (const void*)k_pcg<R, 16, false, false, true, false>
                       : ell_w <= 32 ? (const void*)k_pcg<R, 32, false, false, true, false>
                                     : (const void*)k_pcg<R, 64, false, false, true, false>;
  }
  if (wb) {
    if (adjoint)
      return ell_w <= 16 ? (const void*)k_pcg<R, 16, true, false, false, false, true>
                         : ell_w <= 32 ? (const void*)k_pcg<R, 32, true, false, false, false, true>
                                       : (const void*)k_pcg<R, 64, true, false, false, false, true>;
    return ell_w <= 16 ? (const void*)k_pcg<R, 16, false, false, false, false, true>
                       : ell_w <= 32 ? (const void*)k_pcg<R, 32, false, false, false, false, true>
                                     : (const void*)k_pcg<R, 64, false, false, false, false, true>;
  }
  if (adjoint)
    return ell_w <= 16 ? (const void*)k_pcg<R, 16, true, false, false, false>
                       : ell_w <= 32 ? (const void*)k_pcg<R, 32, true, false, false, false>
                                     : (const void*)k_pcg<R, 64, true, false, false, false>;
  return ell_w <= 16 ? (const void*)k_pcg<R, 16, false, false, false, false>
                     : ell_w <= 32 ? (const void*)k_pcg<R, 32, false, false, false, false>
                                   : (const void*)k_pcg<R, 64, false, false, false, false>;
}

template <typename R>
hipError_t launch_pcg(const Dev<R>& d, const Consts& c, int grid, hipStream_t s, bool adjoint, bool cooperative,
                      hipEvent_t ev_start, hipEvent_t ev_stop) {
  void* args[] = {(void*)&d, (void*)&c};
  // per-mesh CG: the grid is the plan's workgroups, at least one per mesh
  const bool mb = c.per_mesh && c.M > 1;
  if (mb && (grid < c.M || c.coarse)) return hipErrorInvalidValue;
  const bool pair = !mb && pcg_paired((int)sizeof(R), c.ell_w, c.n, grid);
  // the adjoint kernels wrote the right-hand side in the layout of the grid
  // the constants were made for
  if (adjoint && c.cg_soa != (pair ? 1 : 0)) return hipErrorInvalidValue;
  const bool cz = c.coarse && !pair;
  const void* f = pcg_kernel<R>(c.ell_w, adjoint, pair, cz, mb, c.cg_wb && !pair && !cz && !mb);
  if (cooperative) return hipLaunchCooperativeKernel(f, dim3(grid), dim3(kPcgBlock), args, 0, s);
  if (ev_start || ev_stop)  // the events take the kernel's own start and end times
    return hipExtLaunchKernel(f, dim3(grid), dim3(kPcgBlock), args, 0, s, ev_start, ev_stop, 0);
  return hipLaunchKernel(f, dim3(grid), dim3(kPcgBlock), args, 0, s);
}


// Workgroups of the CG kernel that can be resident at once for a matrix of
// ELL width ell_w: the smallest occupancy of its variants (forward and
// adjoint; unpaired, paired, with the coarse correction, per mesh and with
// write-back stores) times the compute units (0 on a runtime error).
template <typename R>
int pcg_max_grid(int ell_w) {
  int occ = 1 << 30, dev = 0, cus = 0;
  for (int v = 0; v < 10; ++v) {
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, pcg_kernel<R>(ell_w, v & 1, (v >> 1) == 1, (v >> 1) == 2,
                                                                      (v >> 1) == 3, (v >> 1) == 4),
                                                     kPcgBlock, 0) != hipSuccess)
      return 0;
    occ = std::min(occ, o);
  }
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return occ * cus;
}

#define INST(R)                                                                                  \
  template hipError_t launch_init<R>(const Dev<R>&, const Consts&, const R*, hipStream_t);      \
  template hipError_t launch_set_positions<R>(const Dev<R>&, const Consts&, const R*, hipStream_t); \
  template hipError_t launch_output<R>(const Dev<R>&, const Consts&, R*, hipStream_t);          \
  template hipError_t launch_hash_clear<R>(const Dev<R>&, const Consts&, hipStream_t);          \
  template hipError_t launch_pcg<R>(const Dev<R>&, const Consts&, int, hipStream_t, bool, bool, hipEvent_t, hipEvent_t); \
  template int pcg_max_grid<R>(int);
INST(float)
INST(double)
#undef INST

}  // namespace gs
