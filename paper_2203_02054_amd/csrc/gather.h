// Right-hand side of the correction system for one vertex: the element
// residual columns (summed in incidence order) plus spring pulls; the Jacobi
// diagonal; the vertex's term of the spring part of Eq. (9), returned.  Shared
// by the stand-alone gather kernel and the kernel that fuses it with the
// contact update.
#pragma once

#include "device_common.h"

namespace gs {

// SOA: the CG state's layout (three arrays of rows, else rows of three vectors).
template <bool SOA, typename R>
__device__ __forceinline__ double gather_row(const Dev<R>& d, const Consts& c, int v) {
  const size_t n = (size_t)c.n;
  double esp = 0.0;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  sum_columns(reinterpret_cast<const W4<R>*>(d.res4), d.inc_start[v], d.inc_start[v + 1], r0, r1, r2);
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
  W4<R> rb;
  rb.x = (R)r0;
  rb.y = (R)r1;
  rb.z = (R)r2;
  rb.w = R(0);
  reinterpret_cast<W4<R>*>(d.cg)[SOA ? (size_t)v : 3 * (size_t)v] = rb;
  d.dsp[v] = (R)ds;
  d.dg[v] = d.freem[v] ? (R)((double)d.adiag[v] + ds) : R(1);
  return esp;
}

}  // namespace gs
