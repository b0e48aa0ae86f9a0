// Broadphase and exact narrowphase of the tet query (Sections II-B, III-A.3),
// shared by the stand-alone tet-query kernel and the kernel that fuses it
// with the local step.  Every floating-point step here is either a single
// operation (a product, a comparison) or an orientation predicate evaluated
// without contraction, so the candidate and penetration sets do not depend on
// the contraction setting of the including file.
#pragma once

#include "device_common.h"

namespace gs {

// Lanes per tet of the tet query: with few tets (latency-bound) a tet's cells
// are shared by 4 consecutive lanes, so each lane's chain of dependent bucket
// reads covers a few cells; with many tets one lane each.
template <bool PREFETCH>
struct TetQueryLanes { static constexpr int n = PREFETCH ? 4 : 1; };

template <typename R, bool DEBUG>
__device__ __forceinline__ void test_point(const Dev<R>& d, const double4& en, int e, int vbeg, int vend, const int (&vi)[4],
                                          const double (&p)[4][3], const double (&lo)[3], const double (&hi)[3]) {
  const double q[3] = {en.x, en.y, en.z};
  if (!(lo[0] <= q[0] && q[0] <= hi[0] && lo[1] <= q[1] && q[1] <= hi[1] && lo[2] <= q[2] && q[2] <= hi[2])) return;
  const unsigned long long bits = (unsigned long long)__double_as_longlong(en.w);
  const int s = (int)(unsigned)(bits & 0xffffffffull);
  const int v = (int)(unsigned)(bits >> 32);
  if (v == vi[0] || v == vi[1] || v == vi[2] || v == vi[3] || v < vbeg || v >= vend) return;
  if (DEBUG) {
    const int k = atomicAdd(&d.st->cand_tet, 1);
    if (k < d.dbg_cap) {
      d.dbg_tet[k] = v;
      d.dbg_tet[d.dbg_cap + k] = e;
    }
  }
  if (point_in_tet(q, p[0], p[1], p[2], p[3])) {
    // the first tet to find the vertex inside lists it for the ray cast
    if (atomicOr(&d.pen[s], 1) == 0) d.penlist[atomicAdd(&d.st->n_pen, 1)] = s;
  }
}

// Tests the entries of up to 8 buckets (key < 0: none).  PREFETCH (few
// tets, latency-bound): the entries are loaded in rounds, round i taking the
// i-th entry of every bucket that has one, so a round costs one memory round
// trip; otherwise one by one, with fewer registers.
template <typename R, bool DEBUG, bool PREFETCH>
__device__ __forceinline__ void test_buckets(const Dev<R>& d, const double4* slots, const int (&keys)[8], int e,
                                             int vbeg, int vend, const int (&vi)[4], const double (&p)[4][3],
                                             const double (&lo)[3], const double (&hi)[3]) {
  int cnt[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) cnt[k] = (keys[k] >= 0) ? min(d.hcount[keys[k]], kHashCap) : 0;
  if (PREFETCH) {
    double4 e0[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (cnt[k] > 0) e0[k] = slots[(size_t)keys[k] * kHashCap];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (cnt[k] > 0) test_point<R, DEBUG>(d, e0[k], e, vbeg, vend, vi, p, lo, hi);
  } else {
#pragma unroll 1
    for (int k = 0; k < 8; ++k)
      if (cnt[k] > 0) test_point<R, DEBUG>(d, slots[(size_t)keys[k] * kHashCap], e, vbeg, vend, vi, p, lo, hi);
  }
  if (PREFETCH) {
    int cmax = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) cmax = max(cmax, cnt[k]);
    for (int i = 1; i < cmax; ++i) {
      double4 ei[8];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (cnt[k] > i) ei[k] = slots[(size_t)keys[k] * kHashCap + i];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (cnt[k] > i) test_point<R, DEBUG>(d, ei[k], e, vbeg, vend, vi, p, lo, hi);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      for (int i = 1; i < cnt[k]; ++i)
        test_point<R, DEBUG>(d, slots[(size_t)keys[k] * kHashCap + i], e, vbeg, vend, vi, p, lo, hi);
  }
}

// Part sub of nsub of the query of tet e: cells sub, sub + nsub, ... (and the
// same share of the brute-force and overflow scans).
template <typename R, bool DEBUG, bool PREFETCH>
__device__ __forceinline__ void tet_query_part(const Dev<R>& d, const Consts& c, int e, int sub, int nsub) {
  if (e >= c.T) return;
  const int m = d.tmesh[e];
  if (mesh_frozen(d, c.mask_done, m)) return;
  const double ic = d.mesh[m].inv_cell;
  const int vbeg = d.mesh[m].vbeg, vend = d.mesh[m].vend;
  int vi[4];
  double p[4][3];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    vi[j] = d.tets[j * c.T + e];
#pragma unroll
    for (int k = 0; k < 3; ++k) p[j][k] = d.xc[(size_t)k * c.n + vi[j]];
  }
  double lo[3], hi[3];
  int clo[3], chi[3];
  long ncell = 1;
  bool finite = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = fmin(fmin(p[0][k], p[1][k]), fmin(p[2][k], p[3][k]));
    hi[k] = fmax(fmax(p[0][k], p[1][k]), fmax(p[2][k], p[3][k]));
    finite = finite && isfinite(lo[k]) && isfinite(hi[k]) && fabs(lo[k] * ic) < 1e9 && fabs(hi[k] * ic) < 1e9;
  }
  if (!finite) return;  // a diverged iterate: no candidates (the CG reports the breakdown)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    clo[k] = cell_of(lo[k], ic);
    chi[k] = cell_of(hi[k], ic);
    const long ext = (long)chi[k] - (long)clo[k] + 1;
    ncell = (ext > kCellCap || ncell > kCellCap) ? (long)kCellCap + 1 : ncell * ext;
  }
  const double4* slots = reinterpret_cast<const double4*>(d.hslot);
  if (ncell > kCellCap) {
    // a tet stretched over many cells: test every query vertex of its mesh (still exact)
    for (int s = d.mesh[m].sbeg + sub; s < d.mesh[m].send; s += nsub) {
      const int v = d.qverts[s];
      double4 en;
      en.x = d.xc[v];
      en.y = d.xc[(size_t)c.n + v];
      en.z = d.xc[2 * (size_t)c.n + v];
      en.w = __longlong_as_double((long long)(((unsigned long long)(unsigned)v << 32) | (unsigned)s));
      test_point<R, DEBUG>(d, en, e, vbeg, vend, vi, p, lo, hi);
    }
    return;
  }
  // the covered cells (x fastest), cell i taken by part i mod nsub, each part
  // taking its cells in groups of 8: one round trip fetches a group's bucket
  // counts, the next the first entries of its non-empty buckets (the common
  // tet covers at most 2 cells per axis, 8 cells: shared by the parts)
  const int nx = chi[0] - clo[0] + 1, ny = chi[1] - clo[1] + 1;
  const int nc = (int)ncell;
  for (int c0 = sub; c0 < nc; c0 += 8 * nsub) {
    int keys[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = c0 + k * nsub;
      keys[k] = i < nc ? hash_cell(clo[0] + i % nx, clo[1] + (i / nx) % ny, clo[2] + i / (nx * ny), m, c.H) : -1;
    }
    test_buckets<R, DEBUG, PREFETCH>(d, slots, keys, e, vbeg, vend, vi, p, lo, hi);
  }
  const int nover = min(__hip_atomic_load(&d.st->n_over, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), c.S);
  for (int i = sub; i < nover; i += nsub)
    test_point<R, DEBUG>(d, reinterpret_cast<const double4*>(d.hover)[i], e, vbeg, vend, vi, p, lo, hi);
}

// One lane of the stand-alone tet query: tet gid / L, part gid mod L of L.
template <typename R, bool DEBUG, bool PREFETCH>
__device__ __forceinline__ void tet_query_lane(const Dev<R>& d, const Consts& c, int gid) {
  constexpr int L = TetQueryLanes<PREFETCH>::n;
  tet_query_part<R, DEBUG, PREFETCH>(d, c, gid / L, gid % L, L);
}

}  // namespace gs
