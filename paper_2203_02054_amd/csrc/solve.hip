// Global step (Section III-B) in correction form and the outer-iteration
// bookkeeping.
//
// With targets fixed, Eq. (9) is minimised by M x = b, M = A_el + diag(k)
// (springs), fixed vertices held at X0.  The iterate is the displacement
// u = x - X0; each outer iteration solves M d = b - M x_k for the correction d
// with a Jacobi-preconditioned conjugate gradient warm-started at the previous
// correction d_{k-1} and stopped once sqrt(r'z) <= eta sqrt(b'D^-1 b), b the
// right-hand side (relative to b, not to the warm-started residual).  The
// slow modes of the local/global map are smooth bending modes, where both the
// outer iteration and Jacobi-CG converge slowly; the warm start carries the
// slow part of the correction across iterations.  The right-hand side b - M x_k is
// the gathered element residual sum_e omega_e (T_e - D_e) plus the spring
// pulls k (c - x): it vanishes exactly at the fixed point, so an inexact inner
// solve changes the path, not the answer.
//
// The CG runs as one cooperative kernel on a small grid (every block
// resident): the per-barrier cost on this GPU grows with the number of
// participating blocks, so the solve uses few, wide blocks.  Dot products are
// accumulated in double; block partials are summed in block order by every
// block, so all blocks take identical decisions.
#include "device_common.h"

namespace gs {

template <typename R>
struct alignas(4 * sizeof(R)) W4 {
  R x, y, z, w;
};

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
      d.dl[k * n + v] = R(0);
    }
  }
  const int stride = gridDim.x * kBlock;
  for (int i = v; i < c.H; i += stride) d.hcount[i] = 0;
  for (int i = v; i < c.S; i += stride) d.pen[i] = 0;
  if (v == 0) {
    DevStatus* st = d.st;
    st->iters = 0;
    st->done = RUNNING;
    st->changed = 0;
    st->pcg_total = 0;
    st->ray_miss = 0;
    st->ray_miss_last = 0;
    st->n_pen = 0;
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
    st->bar_gen = 0;
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
  if (v == 0) {
    DevStatus* st = d.st;
    st->done = RUNNING;
    st->changed = 0;
    st->ray_miss = 0;
    st->n_pen = 0;
    st->n_contacts = 0;
    st->cand_tet = 0;
    st->cand_tri = 0;
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_output(Dev<R> d, Consts c, R* __restrict__ xout) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= c.n) return;
  const size_t n = (size_t)c.n;
#pragma unroll
  for (int k = 0; k < 3; ++k) xout[k * n + v] = (R)(d.X0[k * n + v] + (double)d.u[k * n + v]);
}

// Right-hand side of the correction system per vertex: the element residual
// columns (deterministic gather in incidence order) plus spring pulls; the
// Jacobi diagonal; the spring part of Eq. (9).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_gather(Dev<R> d, Consts c) {
  __shared__ double lds[kBlock / 64];
  if (is_done(d.st)) return;
  const int v = blockIdx.x * kBlock + threadIdx.x;
  const size_t n = (size_t)c.n;
  double esp = 0.0;
  if (v < c.n) {
    double r0 = 0.0, r1 = 0.0, r2 = 0.0;
    const W4<R>* res = reinterpret_cast<const W4<R>*>(d.res4);
    const int i1 = d.inc_start[v + 1];
    for (int i = d.inc_start[v]; i < i1; ++i) {
      const W4<R> t = res[i];
      r0 += (double)t.x;
      r1 += (double)t.y;
      r2 += (double)t.z;
    }
    double ds = 0.0;
    if (!d.freem[v]) {
      r0 = r1 = r2 = 0.0;
    } else {
      const int s = d.vq[v];
      if (s >= 0) {
        const double x0 = d.xc[v], x1 = d.xc[n + v], x2 = d.xc[2 * n + v];
        const double k = d.kq[s];
        for (int sl = 0; sl < c.slots; ++sl) {
          const int b = s * c.slots + sl;
          if (!d.cact[b]) continue;
          const double e0 = d.ctgt[3 * b] - x0, e1 = d.ctgt[3 * b + 1] - x1, e2 = d.ctgt[3 * b + 2] - x2;
          ds += k;
          r0 += k * e0;
          r1 += k * e1;
          r2 += k * e2;
          esp += k * (e0 * e0 + e1 * e1 + e2 * e2);
        }
      }
    }
    d.r[v] = (R)r0;
    d.r[n + v] = (R)r1;
    d.r[2 * n + v] = (R)r2;
    d.dsp[v] = (R)ds;
    d.dg[v] = d.freem[v] ? (R)((double)d.adiag[v] + ds) : R(1);
  }
  const double bs = block_sum<kBlock>(esp, lds);
  if (threadIdx.x == 0) d.part_b[blockIdx.x] = bs;
}

constexpr int kPcgBlock = kPcgThreads;

// Sum of the G <= 64 block partials: one wavefront, fixed shuffle tree (every
// block obtains the same bits).
__device__ __forceinline__ double grid_sum(const double* part, int G, double* sh) {
  if (threadIdx.x < 64) {
    double t = (threadIdx.x < G) ? part[threadIdx.x] : 0.0;
    t = wave_sum(t);
    if (threadIdx.x == 0) sh[0] = t;
  }
  __syncthreads();
  const double t = sh[0];
  __syncthreads();
  return t;
}

// Preconditioned conjugate gradient in the Chronopoulos-Gear arrangement:
// both inner products of an iteration are taken after its single
// matrix-vector product, so one grid-wide reduction (one barrier) per
// iteration suffices.  The product w_{i+1} = A M^-1 r_{i+1} needs
// r_{i+1} at neighbouring rows; each block recomputes those values from the
// neighbours' previous state (r_i, w_i, s_{i-1}, kept in the other half of a
// double buffer) instead of waiting for a second barrier.
//
//   p_i = u_i + b_i p_{i-1}        s_i = w_i + b_i s_{i-1}      (s_i = A p_i)
//   x_{i+1} = x_i + a_i p_i        r_{i+1} = r_i - a_i s_i      u = M^-1 r
//   w_{i+1} = A u_{i+1}            g = (r, u), d = (w, u)
//   b_{i+1} = g_{i+1} / g_i        a_{i+1} = g_{i+1} / (d_{i+1} - b_{i+1} g_{i+1} / a_i)
template <typename R, int MW>
__global__ __launch_bounds__(kPcgBlock) void k_pcg(Dev<R> d, Consts c) {
  __shared__ double lds[kPcgBlock / 64];
  __shared__ double sh[1];
  if (is_done(d.st)) return;
  const int G = gridDim.x;
  const int stride = G * kPcgBlock;
  const int tid0 = blockIdx.x * kPcgBlock + threadIdx.x;
  const size_t n = (size_t)c.n;
  const size_t n3 = 3 * n;
  unsigned* bc = &d.st->bar_count;
  unsigned* bg = &d.st->bar_gen;
  R* __restrict__ x = d.dl;
  R* __restrict__ p = d.p;
  const R* __restrict__ dg = d.dg;
  const int32_t* __restrict__ ecol = d.ell_col;
  const R* __restrict__ evl = d.ell_val;

  // (A) r_0 = b - A x_0 with the warm start x_0 = previous correction;
  //     p_{-1} = s_{-1} = 0; right-hand-side norm b' M^-1 b
  double acc_b = 0.0;
  {
    R* r0 = d.r;
    R* s0 = d.s;
    R* __restrict__ evs = d.ell_scaled;
    for (int v = tid0; v < c.n; v += stride) {
      const R dv = dg[v], idg = R(1) / dv;
      int jj[MW];
      R aa[MW];
#pragma unroll
      for (int k = 0; k < MW; ++k) {
        jj[k] = ecol[(size_t)k * n + v];
        aa[k] = evl[(size_t)k * n + v];
      }
      R ax0 = dv * x[v], ax1 = dv * x[n + v], ax2 = dv * x[2 * n + v];
#pragma unroll
      for (int k = 0; k < MW; ++k) {
        const int j = jj[k];
        ax0 += aa[k] * x[j];
        ax1 += aa[k] * x[n + j];
        ax2 += aa[k] * x[2 * n + j];
        evs[(size_t)k * n + v] = aa[k] / dg[j];  // a_vj / dg_j, fixed during this solve
      }
      const R ax[3] = {ax0, ax1, ax2};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const R b = r0[k * n + v];
        acc_b += (double)b * (double)(b * idg);
        r0[k * n + v] = b - ax[k];
        p[k * n + v] = R(0);
        s0[k * n + v] = R(0);
      }
    }
  }
  double bs = block_sum<kPcgBlock>(acc_b, lds);
  if (threadIdx.x == 0) d.part_d[blockIdx.x] = bs;
  grid_barrier(bc, bg, G);
  // (B) w_0 = A u_0, g_0 = (r_0, u_0), d_0 = (w_0, u_0)
  double acc_g = 0.0, acc_d = 0.0;
  {
    const R* r0 = d.r;
    R* w0 = d.w;
    for (int v = tid0; v < c.n; v += stride) {
      const R dv = dg[v], idg = R(1) / dv;
      const R u0 = r0[v] * idg, u1 = r0[n + v] * idg, u2 = r0[2 * n + v] * idg;
      R a0 = dv * u0, a1 = dv * u1, a2 = dv * u2;
      int jj[MW];
      R aa[MW];
#pragma unroll
      for (int k = 0; k < MW; ++k) {
        jj[k] = ecol[(size_t)k * n + v];
        aa[k] = d.ell_scaled[(size_t)k * n + v];
      }
#pragma unroll
      for (int k = 0; k < MW; ++k) {
        const int j = jj[k];
        a0 += aa[k] * r0[j];
        a1 += aa[k] * r0[n + j];
        a2 += aa[k] * r0[2 * n + j];
      }
      w0[v] = a0;
      w0[n + v] = a1;
      w0[2 * n + v] = a2;
      acc_g += (double)r0[v] * u0 + (double)r0[n + v] * u1 + (double)r0[2 * n + v] * u2;
      acc_d += (double)a0 * u0 + (double)a1 * u1 + (double)a2 * u2;
    }
  }
  bs = block_sum<kPcgBlock>(acc_g, lds);
  if (threadIdx.x == 0) d.part_c[blockIdx.x] = bs;
  bs = block_sum<kPcgBlock>(acc_d, lds);
  if (threadIdx.x == 0) d.part_e[blockIdx.x] = bs;
  grid_barrier(bc, bg, G);
  const double rhs = grid_sum(d.part_d, G, sh);
  double gam = grid_sum(d.part_c, G, sh);
  const double del = grid_sum(d.part_e, G, sh);
  const double stop = c.pcg_eta * c.pcg_eta * rhs;
  int it = 0;
  bool broke = !(rhs >= 0.0) || isinf(rhs) || !(gam >= 0.0) || isinf(gam);
  bool run = !broke && gam > stop;
  if (run && !(del > 0.0 && !isinf(del))) {
    broke = true;
    run = false;
  }
  double al = run ? gam / del : 0.0, be = 0.0;
  int cur = 0;
  while (run && it < c.pcg_max) {
    const R* rc = d.r + cur * n3;
    const R* wc = d.w + cur * n3;
    const R* sc = d.s + cur * n3;
    R* rn = d.r + (cur ^ 1) * n3;
    R* wn = d.w + (cur ^ 1) * n3;
    R* sn = d.s + (cur ^ 1) * n3;
    const R ra = (R)al, rb = (R)be;
    acc_g = 0.0;
    acc_d = 0.0;
    for (int v = tid0; v < c.n; v += stride) {
      const R dv = dg[v], idg = R(1) / dv;
      R rv[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const size_t o = k * n + v;
        const R pv = rc[o] * idg + rb * p[o];
        p[o] = pv;
        const R sv = wc[o] + rb * sc[o];
        sn[o] = sv;
        x[o] += ra * pv;
        rv[k] = rc[o] - ra * sv;
        rn[o] = rv[k];
      }
      // w_{i+1} at this row from neighbours' r_{i+1}, rebuilt from their state
      R a0 = rv[0], a1 = rv[1], a2 = rv[2];  // dg_v * (r_v / dg_v)
      int jj[MW];
      R aa[MW];
#pragma unroll
      for (int k = 0; k < MW; ++k) {
        jj[k] = ecol[(size_t)k * n + v];
        aa[k] = d.ell_scaled[(size_t)k * n + v];
      }
#pragma unroll
      for (int k = 0; k < MW; ++k) {
        const int j = jj[k];
        a0 += aa[k] * (rc[j] - ra * (wc[j] + rb * sc[j]));
        a1 += aa[k] * (rc[n + j] - ra * (wc[n + j] + rb * sc[n + j]));
        a2 += aa[k] * (rc[2 * n + j] - ra * (wc[2 * n + j] + rb * sc[2 * n + j]));
      }
      wn[v] = a0;
      wn[n + v] = a1;
      wn[2 * n + v] = a2;
      const R u0 = rv[0] * idg, u1 = rv[1] * idg, u2 = rv[2] * idg;
      acc_g += (double)rv[0] * u0 + (double)rv[1] * u1 + (double)rv[2] * u2;
      acc_d += (double)a0 * u0 + (double)a1 * u1 + (double)a2 * u2;
    }
    // partial sums alternate halves so a slow block still reading the previous
    // iteration's sums is never overwritten
    const int half = (it & 1) ? 0 : G;
    bs = block_sum<kPcgBlock>(acc_g, lds);
    if (threadIdx.x == 0) d.part_c[half + blockIdx.x] = bs;
    bs = block_sum<kPcgBlock>(acc_d, lds);
    if (threadIdx.x == 0) d.part_e[half + blockIdx.x] = bs;
    grid_barrier(bc, bg, G);
    const double gn = grid_sum(d.part_c + half, G, sh);
    const double dn = grid_sum(d.part_e + half, G, sh);
    ++it;
    cur ^= 1;
    if (!(gn >= 0.0) || isinf(gn) || !(dn == dn) || isinf(dn)) {
      broke = true;
      break;
    }
    if (gn <= stop) break;
    const double bn = gn / gam;
    const double den = dn - bn * gn / al;
    if (!(den > 0.0)) {
      broke = true;
      break;
    }
    al = gn / den;
    be = bn;
    gam = gn;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.st->pcg_total += it;
    d.st->pcg_last = it;
    if (broke) __hip_atomic_store(&d.st->done, (int)BREAKDOWN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// u += d on free vertices, collision positions refreshed, r_k = max|d|/diag,
// convergence decision by the last block to finish.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_finish(Dev<R> d, Consts c) {
  __shared__ double lds[kBlock / 64];
  __shared__ int last;
  if (is_done(d.st)) return;
  const int v = blockIdx.x * kBlock + threadIdx.x;
  const size_t n = (size_t)c.n;
  double dm = 0.0;
  if (v < c.n && d.freem[v]) {
    double dd[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R dk = d.dl[k * n + v];
      const R uu = d.u[k * n + v] + dk;
      d.u[k * n + v] = uu;
      d.xc[k * n + v] = d.X0[k * n + v] + (double)uu;
      dd[k] = (double)dk;
    }
    dm = sqrt((dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]);
  }
  const int stride = gridDim.x * kBlock;
  for (int i = v; i < c.H; i += stride) d.hcount[i] = 0;
  const double bm = block_max<kBlock>(dm, lds);
  if (threadIdx.x == 0) {
    d.part_d[blockIdx.x] = bm;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const int t = __hip_atomic_fetch_add(&d.st->ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = (t == (int)gridDim.x - 1);
    if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (!last) return;
  // the last block reduces every block's partials (fixed order per thread,
  // then a fixed tree: deterministic)
  double mloc = 0.0, eloc = 0.0;
  const int gl = cdiv(c.T, kBlock), gg = cdiv(c.n, kBlock);
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) mloc = fmax(mloc, d.part_d[b]);
  for (int b = threadIdx.x; b < gl; b += kBlock) eloc += d.part_a[b];
  for (int b = threadIdx.x; b < gg; b += kBlock) eloc += d.part_b[b];
  const double m = block_max<kBlock>(mloc, lds);
  const double E = block_sum<kBlock>(eloc, lds);
  if (threadIdx.x != 0) return;
  DevStatus* st = d.st;
  const double res = m / c.diag;
  st->residual = res;
  st->energy = E;
  const int it = st->iters + 1;
  st->iters = it;
  const int changed = st->changed;
  int code = RUNNING;
  if (!(res == res) || isinf(res) || !(E == E))
    code = BREAKDOWN;
  else if (c.fixed_iters > 0)
    code = (it >= c.fixed_iters) ? FIXED_DONE : RUNNING;
  else if (res <= c.tol && !changed)
    code = CONVERGED;
  else if (it >= c.max_iter)
    code = MAXITER;
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
  __hip_atomic_store(&st->done, code, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
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

template <typename R>
hipError_t launch_gather(const Dev<R>& d, const Consts& c, hipStream_t s) {
  k_gather<R><<<cdiv(c.n, kBlock), kBlock, 0, s>>>(d, c);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_pcg(const Dev<R>& d, const Consts& c, int grid, hipStream_t s) {
  void* args[] = {(void*)&d, (void*)&c};
  const void* f = c.ell_w <= 16 ? (const void*)k_pcg<R, 16> : c.ell_w <= 32 ? (const void*)k_pcg<R, 32>
                                                                             : (const void*)k_pcg<R, 64>;
  return hipLaunchCooperativeKernel(f, dim3(grid), dim3(kPcgBlock), args, 0, s);
}

template <typename R>
hipError_t launch_finish(const Dev<R>& d, const Consts& c, hipStream_t s) {
  k_finish<R><<<cdiv(c.n, kBlock), kBlock, 0, s>>>(d, c);
  return hipGetLastError();
}

template <typename R>
int pcg_max_grid(int block) {
  int occ = 0;
  int o16 = 0, o32 = 0, o64 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o16, k_pcg<R, 16>, kPcgBlock, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&o32, k_pcg<R, 32>, kPcgBlock, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&o64, k_pcg<R, 64>, kPcgBlock, 0) != hipSuccess)
    return 0;
  occ = std::min(o16, std::min(o32, o64));
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  (void)block;
  return occ * cus;
}

#define INST(R)                                                                                  \
  template hipError_t launch_init<R>(const Dev<R>&, const Consts&, const R*, hipStream_t);      \
  template hipError_t launch_set_positions<R>(const Dev<R>&, const Consts&, const R*, hipStream_t); \
  template hipError_t launch_output<R>(const Dev<R>&, const Consts&, R*, hipStream_t);          \
  template hipError_t launch_gather<R>(const Dev<R>&, const Consts&, hipStream_t);              \
  template hipError_t launch_pcg<R>(const Dev<R>&, const Consts&, int, hipStream_t);            \
  template hipError_t launch_finish<R>(const Dev<R>&, const Consts&, hipStream_t);              \
  template int pcg_max_grid<R>(int);
INST(float)
INST(double)
#undef INST

}  // namespace gs
