// Triangle-mesh obstacles (Section II-B, the obstacle term; Section II-C,
// the target on the collided boundary): for every query vertex inside the
// obstacle's box, or holding a contact with it, the closest point c on the
// closed, outward-oriented mesh, whether the vertex is inside it, and the
// spring target c + eps u with u the outward unit direction at the vertex.
//
// * Closest point on a triangle: the Voronoi-region walk of Ericson,
//   Real-Time Collision Detection (2005), Section 5.1.5, in a fixed order of
//   operations with contraction off, so the squared distances (and the
//   choice among equal ones: the lowest triangle id) are reproducible bit for
//   bit.
// * Over the mesh: a static bounding-volume hierarchy over the triangles
//   (built once on the host), searched depth first, nearer child first,
//   pruning a subtree only when its box is strictly farther than the best
//   distance so far (a tie may still hold a lower id).
// * Inside: (p - c) . psi < 0, psi the angle-weighted pseudonormal of the
//   feature c lies on (Baerentzen and Aanaes, 2005), precomputed per
//   triangle for its face, three edges and three vertices.
//
// One thread per query vertex; the tree and the triangle records (30 doubles
// each) stay in L2 for any obstacle of practical size.
#include "internal.h"
#include "device_common.h"

namespace gs {

namespace {

// closest point of p on triangle (a, b, c); kind 0 face, 1 edge, 2 vertex;
// loc: vertex 0/1/2 or edge 0 = ab, 1 = ac, 2 = bc
__device__ __forceinline__ void closest_tri(const double* p, const double* a, const double* b, const double* c,
                                            double* q, int& kind, int& loc) {
#pragma clang fp contract(off)
  double ab[3], ac[3], ap[3], bp[3], cp[3];
  for (int k = 0; k < 3; ++k) {
    ab[k] = b[k] - a[k];
    ac[k] = c[k] - a[k];
    ap[k] = p[k] - a[k];
    bp[k] = p[k] - b[k];
    cp[k] = p[k] - c[k];
  }
  const double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  const double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  const double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  const double vc = d1 * d4 - d3 * d2;
  const double vb = d5 * d2 - d1 * d6;
  const double va = d3 * d6 - d5 * d4;
  if (d1 <= 0.0 && d2 <= 0.0) {
    for (int k = 0; k < 3; ++k) q[k] = a[k];
    kind = 2, loc = 0;
    return;
  }
  if (d3 >= 0.0 && d4 <= d3) {
    for (int k = 0; k < 3; ++k) q[k] = b[k];
    kind = 2, loc = 1;
    return;
  }
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
    const double t = d1 / (d1 - d3);
    for (int k = 0; k < 3; ++k) q[k] = a[k] + t * ab[k];
    kind = 1, loc = 0;
    return;
  }
  if (d6 >= 0.0 && d5 <= d6) {
    for (int k = 0; k < 3; ++k) q[k] = c[k];
    kind = 2, loc = 2;
    return;
  }
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
    const double t = d2 / (d2 - d6);
    for (int k = 0; k < 3; ++k) q[k] = a[k] + t * ac[k];
    kind = 1, loc = 1;
    return;
  }
  const double e43 = d4 - d3, e56 = d5 - d6;
  if (va <= 0.0 && e43 >= 0.0 && e56 >= 0.0) {
    const double t = e43 / (e43 + e56);
    for (int k = 0; k < 3; ++k) q[k] = b[k] + t * (c[k] - b[k]);
    kind = 1, loc = 2;
    return;
  }
  const double den = 1.0 / ((va + vb) + vc);
  const double v = vb * den, w = vc * den;
  for (int k = 0; k < 3; ++k) q[k] = (a[k] + ab[k] * v) + ac[k] * w;
  kind = 0, loc = 0;
}

// squared distance from p to the box of a node (0 inside)
__device__ __forceinline__ double box_d2(const double* p, const MoNode& nd) {
#pragma clang fp contract(off)
  double s = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double g = p[k] < nd.lo[k] ? nd.lo[k] - p[k] : (p[k] > nd.hi[k] ? p[k] - nd.hi[k] : 0.0);
    s = s + g * g;
  }
  return s;
}

}  // namespace

template <typename R>
__global__ __launch_bounds__(kBlock) void k_mesh_obstacle(Dev<R> d, Consts c) {
#pragma clang fp contract(off)
  if (is_done(d.st)) return;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= c.S) return;
  const int v = d.qverts[s];
  const int m = d.vmesh[v];
  if (mesh_frozen(d, c.mask_done, m)) return;
  double p[3];
  load3(d.xc, (size_t)c.n, v, p);
  const MoNode root = d.mo_node[0];
  const bool inbox = p[0] >= root.lo[0] && p[0] <= root.hi[0] && p[1] >= root.lo[1] && p[1] <= root.hi[1] &&
                     p[2] >= root.lo[2] && p[2] <= root.hi[2];
  const bool old = d.cact[s * c.slots + 1 + c.ns + c.np] != 0;
  if (!inbox && !old) {
    d.mo_flag[s] = 0;
    return;
  }
  double best = INFINITY, bq[3] = {0.0, 0.0, 0.0};
  int bt = 0x7fffffff, bslot = 0, bkind = 0, bloc = 0;
  int stack[64];
  int top = 0;
  stack[top++] = 0;
  while (top > 0) {
    const MoNode nd = d.mo_node[stack[--top]];
    if (box_d2(p, nd) > best) continue;
    if (nd.count > 0) {
      for (int i = nd.first; i < nd.first + nd.count; ++i) {
        const double* tr = d.mo_tri + (size_t)30 * i;
        double q[3];
        int kind, loc;
        closest_tri(p, tr, tr + 3, tr + 6, q, kind, loc);
        const double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        const int id = d.mo_id[i];
        if (d2 < best || (d2 == best && id < bt)) {
          best = d2, bt = id, bslot = i, bkind = kind, bloc = loc;
          bq[0] = q[0], bq[1] = q[1], bq[2] = q[2];
        }
      }
    } else {
      // nearer child last on the stack, so it is searched first
      const MoNode l = d.mo_node[nd.left], r = d.mo_node[nd.right];
      const double dl = box_d2(p, l), dr = box_d2(p, r);
      if (top + 2 > 64) {
        // deeper than the host ever builds; cannot happen for a tree it made
        d.mo_flag[s] = 0;
        return;
      }
      if (dl <= dr) {
        stack[top++] = nd.right;
        stack[top++] = nd.left;
      } else {
        stack[top++] = nd.left;
        stack[top++] = nd.right;
      }
    }
  }
  // pseudonormal of the feature: face, edge (ab, ac, bc) or vertex (a, b, c)
  const double* tr = d.mo_tri + (size_t)30 * bslot;
  const double* psi = tr + 9 + 3 * (bkind == 0 ? 0 : (bkind == 1 ? 1 + bloc : 4 + bloc));
  const double g[3] = {p[0] - bq[0], p[1] - bq[1], p[2] - bq[2]};
  const bool inside = dot3(g, psi) < 0.0;
  double u[3];
  if (best > 0.0) {
    const double dist = sqrt(best);
    for (int k = 0; k < 3; ++k) u[k] = inside ? -g[k] / dist : g[k] / dist;
  } else {
    for (int k = 0; k < 3; ++k) u[k] = psi[k];
  }
  const double eps = d.mesh[m].eps;
  for (int k = 0; k < 3; ++k) {
    d.mo_tgt[3 * s + k] = bq[k] + eps * u[k];
    d.mo_nrm[3 * s + k] = u[k];
  }
  d.mo_prim[s] = bt;
  d.mo_flag[s] = inside ? 2 : 1;
}

template <typename R>
hipError_t launch_mesh_obstacle(const Dev<R>& d, const Consts& c, hipStream_t s) {
  if (c.S == 0) return hipSuccess;
  k_mesh_obstacle<R><<<(c.S + kBlock - 1) / kBlock, kBlock, 0, s>>>(d, c);
  return hipGetLastError();
}

template hipError_t launch_mesh_obstacle<float>(const Dev<float>&, const Consts&, hipStream_t);
template hipError_t launch_mesh_obstacle<double>(const Dev<double>&, const Consts&, hipStream_t);

}  // namespace gs
