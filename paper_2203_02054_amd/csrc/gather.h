// Right-hand side of the correction system for one vertex: the element
// residual columns (summed in incidence order) plus spring pulls; the Jacobi
// diagonal; the vertex's term of the spring part of Eq. (9), returned.  Run
// by the CG kernel's first phase, right after the row's contact update.
#pragma once

#include "device_common.h"

namespace gs {

// The row's spring pulls added to its summed columns (r0, r1, r2); b, the
// spring diagonal and the Jacobi diagonal stored (SOA: the CG state's layout,
// three arrays of rows, else rows of three vectors); b and the diagonal
// returned in `b` and `diag`, the vertex's spring energy term as the value.
template <bool SOA, typename R>
__device__ __forceinline__ double finish_row(const Dev<R>& d, const Consts& c, int v, double r0, double r1,
                                             double r2, W4<R>& b, R& diag) {
  const size_t n = (size_t)c.n;
  double esp = 0.0;
  double ds = 0.0;
  const bool frozen = mesh_frozen(d, c.mask_done, d.vmesh[v]);
  if (!d.freem[v] || frozen) {
    r0 = r1 = r2 = 0.0;
  } else {
    const int s = d.vq[v];
    if (s >= 0) {
      const double x0 = d.xc[v], x1 = d.xc[n + v], x2 = d.xc[2 * n + v];
      const double k = d.kq[s];
      for (int sl = 0; sl < c.slots; ++sl) {
        const int sb = s * c.slots + sl;
        if (!d.cact[sb]) continue;
        const double e0 = d.ctgt[3 * sb] - x0, e1 = d.ctgt[3 * sb + 1] - x1, e2 = d.ctgt[3 * sb + 2] - x2;
        ds += k;
        r0 += k * e0;
        r1 += k * e1;
        r2 += k * e2;
        esp += k * (e0 * e0 + e1 * e1 + e2 * e2);
      }
    }
  }
  b.x = (R)r0;
  b.y = (R)r1;
  b.z = (R)r2;
  b.w = R(0);
  diag = d.freem[v] ? (R)((double)d.adiag[v] + ds) : R(1);
  reinterpret_cast<W4<R>*>(d.cg)[SOA ? (size_t)v : 3 * (size_t)v] = b;
  d.dsp[v] = (R)ds;
  d.dg[v] = diag;
  return esp;
}

// One thread per row: the incidence columns summed in index order.
template <bool SOA, typename R>
__device__ __forceinline__ double gather_row(const Dev<R>& d, const Consts& c, int v) {
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  sum_columns(reinterpret_cast<const W4<R>*>(d.res4), d.inc_start[v], d.inc_start[v + 1], r0, r1, r2);
  W4<R> b;
  R diag;
  return finish_row<SOA>(d, c, v, r0, r1, r2, b, diag);
}

// A lane pair per row (half = 0 or 1, adjacent lanes): each lane sums half of
// the row's incidence columns, the two halves are added in index order, and
// the first lane adds the springs and stores.  Both lanes receive b and the
// diagonal through the pair's registers (the second lane reads nothing the
// first has just written); the energy term comes from the first lane only.
template <bool SOA, typename R>
__device__ __forceinline__ double gather_row_pair(const Dev<R>& d, const Consts& c, int v, int half, W4<R>& b,
                                                  R& diag) {
  const int i0 = d.inc_start[v], i1 = d.inc_start[v + 1], im = i0 + ((i1 - i0 + 1) >> 1);
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  sum_columns(reinterpret_cast<const W4<R>*>(d.res4), half ? im : i0, half ? i1 : im, r0, r1, r2);
  const double o0 = __shfl_xor(r0, 1, 64), o1 = __shfl_xor(r1, 1, 64), o2 = __shfl_xor(r2, 1, 64);
  double esp = 0.0;
  W4<R> bb = {R(0), R(0), R(0), R(0)};
  R dd = R(0);
  if (half == 0) esp = finish_row<SOA>(d, c, v, r0 + o0, r1 + o1, r2 + o2, bb, dd);
  const int src = (int)(threadIdx.x & 63) & ~1;
  b.x = __shfl(bb.x, src, 64);
  b.y = __shfl(bb.y, src, 64);
  b.z = __shfl(bb.z, src, 64);
  b.w = R(0);
  diag = __shfl(dd, src, 64);
  return esp;
}

}  // namespace gs
