// Self-collision broadphase by a refit-only AABB tree over the tets (Section
// II-B: the tree's structure is kept through the deformation and only its
// boxes follow the positions).  The topology comes from the host (median
// splits of the rest centroids, nodes in breadth-first order so that every
// depth is one contiguous range); each use refits the boxes bottom-up, one
// launch per depth, and then every query vertex walks the tree.
//
// The candidate set is the broadphase's definition, C_tet = {(v, e): v not a
// vertex of e, lo_e <= x_v <= hi_e on every axis} with exact min/max boxes
// of the FP64 collision positions: the same set the spatial hash of the
// solver produces, so either broadphase feeds the same exact tests.
#include "internal.h"
#include "device_common.h"

namespace gs {

// Refit the nodes [begin, end) of one depth: a leaf takes the union of its
// tets' boxes (computed here and kept for the query), an inner node the union
// of its children's (one depth deeper, already refit).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_tree_refit(Dev<R> d, Consts c, MoNode* __restrict__ nodes,
                                                       const int32_t* __restrict__ order, double* __restrict__ tbox,
                                                       int begin, int end) {
  const int i = begin + blockIdx.x * kBlock + threadIdx.x;
  if (i >= end) return;
  MoNode nd = nodes[i];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (nd.count > 0) {
    for (int j = nd.first; j < nd.first + nd.count; ++j) {
      const int e = order[j];
      double bl[3] = {INFINITY, INFINITY, INFINITY}, bh[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int q = 0; q < 4; ++q) {
        const int v = d.tets[q * c.T + e];
        for (int k = 0; k < 3; ++k) {
          const double x = d.xc[(size_t)k * c.n + v];
          bl[k] = fmin(bl[k], x);
          bh[k] = fmax(bh[k], x);
        }
      }
      for (int k = 0; k < 3; ++k) {
        tbox[6 * (size_t)j + k] = bl[k];
        tbox[6 * (size_t)j + 3 + k] = bh[k];
        lo[k] = fmin(lo[k], bl[k]);
        hi[k] = fmax(hi[k], bh[k]);
      }
    }
  } else {
    const MoNode a = nodes[nd.left], b = nodes[nd.right];
    for (int k = 0; k < 3; ++k) {
      lo[k] = fmin(a.lo[k], b.lo[k]);
      hi[k] = fmax(a.hi[k], b.hi[k]);
    }
  }
  for (int k = 0; k < 3; ++k) {
    nodes[i].lo[k] = lo[k];
    nodes[i].hi[k] = hi[k];
  }
}

__device__ __forceinline__ bool in_box(const double* p, const double* lo, const double* hi) {
  return p[0] >= lo[0] && p[0] <= hi[0] && p[1] >= lo[1] && p[1] <= hi[1] && p[2] >= lo[2] && p[2] <= hi[2];
}

// One query vertex per thread: every (v, e) of C_tet, appended to pairs
// [2][cap] (the count may exceed cap; pairs beyond it are not written).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_tree_query(Dev<R> d, Consts c, const MoNode* __restrict__ nodes,
                                                       const int32_t* __restrict__ order,
                                                       const double* __restrict__ tbox, int32_t* __restrict__ pairs,
                                                       int cap, int* __restrict__ count) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= c.S) return;
  const int v = d.qverts[s];
  double p[3];
  load3(d.xc, (size_t)c.n, v, p);
  int stack[64];
  int top = 0;
  stack[top++] = 0;
  while (top > 0) {
    const MoNode nd = nodes[stack[--top]];
    if (!in_box(p, nd.lo, nd.hi)) continue;
    if (nd.count > 0) {
      for (int j = nd.first; j < nd.first + nd.count; ++j) {
        if (!in_box(p, tbox + 6 * (size_t)j, tbox + 6 * (size_t)j + 3)) continue;
        const int e = order[j];
        if (d.tets[e] == v || d.tets[c.T + e] == v || d.tets[2 * c.T + e] == v || d.tets[3 * c.T + e] == v)
          continue;
        const int k = atomicAdd(count, 1);
        if (k < cap) {
          pairs[k] = v;
          pairs[cap + k] = e;
        }
      }
    } else if (top + 2 <= 64) {  // the host builds trees shallower than 60
      stack[top++] = nd.left;
      stack[top++] = nd.right;
    }
  }
}

__global__ void k_tree_zero(int* count) { *count = 0; }

template <typename R>
hipError_t launch_tree_refit(const Dev<R>& d, const Consts& c, MoNode* nodes, const int32_t* order, double* tbox,
                             const int* level_start, int levels, hipStream_t s) {
  for (int l = levels - 1; l >= 0; --l) {
    const int b = level_start[l], e = level_start[l + 1];
    if (e > b) k_tree_refit<R><<<(e - b + kBlock - 1) / kBlock, kBlock, 0, s>>>(d, c, nodes, order, tbox, b, e);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_tree_query(const Dev<R>& d, const Consts& c, const MoNode* nodes, const int32_t* order,
                             const double* tbox, int32_t* pairs, int cap, int* count, hipStream_t s) {
  k_tree_zero<<<1, 1, 0, s>>>(count);
  if (c.S > 0) k_tree_query<R><<<(c.S + kBlock - 1) / kBlock, kBlock, 0, s>>>(d, c, nodes, order, tbox, pairs, cap, count);
  return hipGetLastError();
}

template hipError_t launch_tree_refit<float>(const Dev<float>&, const Consts&, MoNode*, const int32_t*, double*,
                                             const int*, int, hipStream_t);
template hipError_t launch_tree_refit<double>(const Dev<double>&, const Consts&, MoNode*, const int32_t*, double*,
                                              const int*, int, hipStream_t);
template hipError_t launch_tree_query<float>(const Dev<float>&, const Consts&, const MoNode*, const int32_t*,
                                             const double*, int32_t*, int, int*, hipStream_t);
template hipError_t launch_tree_query<double>(const Dev<double>&, const Consts&, const MoNode*, const int32_t*,
                                              const double*, int32_t*, int, int*, hipStream_t);

}  // namespace gs
