// Collision detection and response (Sections II-B, II-C, III-A.3).
//
// Broadphase: a spatial hash of the query vertices (non-fixed boundary
// vertices), one cell per vertex, rebuilt every iteration (Teschner et al.
// 2003) into fixed-capacity buckets with an overflow list.  Each tet visits the cells its min/max box covers and
// tests the vertices found there exactly: the candidate set is
// C_tet = {(v, e): v not in e, lo_e <= x_v <= hi_e}, the same set a brute-force
// or BVH search yields, because the cell map is monotone in x.
// Narrowphase: exact point-in-tet by four FP64 orientation signs (Eq. 3).
// Response: the inverse-normal ray of every penetrating vertex is cast against
// the boundary triangles (one wavefront per vertex, Moller-Trumbore), giving
// the spring target an offset eps past the first hit (Section II-C); obstacle
// targets are closed form; the active set follows the release rule of Eq. 8.
// All decisions are made in double precision in the operation order written
// here, and this file is compiled without floating-point contraction, so
// identical inputs give identical sets on any conforming implementation.
#include <climits>
#include <mutex>

#include "contacts.h"
#include "tet_query.h"

namespace gs {

// Candidate-list staging of the allocation-free collision check
// (gs_collide_debug_static): the two candidate lists of at most
// kStaticCandCap pairs each, [2][cap] tet pairs then [2][cap] triangle pairs,
// exactly the layout gs_collide_debug takes from its caller's scratch (with
// the 256 bytes of slack its size rule adds).  Each
// device holds its own copy for the life of the process; calls on one device
// share it, so overlapping calls on a device race.
static __device__ __align__(256) int32_t scratch[4 * kStaticCandCap + 64];

// Address of this device's copy of `scratch`, resolved once per device with
// that device current (the array's name is not a device address in host
// code).
hipError_t static_candidate_scratch(void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = a;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

// Insert every query vertex into the bucket of its cell (the first iteration
// after positions were set; later iterations insert in the CG kernel's final
// update).  A bucket keeps its first kHashCap entries; further entries go to
// an overflow list that every tet scans, so no candidate is ever lost.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_hash_insert(Dev<R> d, Consts c) {
  if (is_done(d.st)) return;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= c.S) return;
  const int v = d.qverts[s];
  const int m = d.vmesh[v];
  if (mesh_frozen(d, c.mask_done, m)) return;
  hash_insert_entry(d, c, s, v, m, d.xc[v], d.xc[(size_t)c.n + v], d.xc[2 * (size_t)c.n + v]);
}

template <typename R, bool DEBUG, bool PREFETCH>
__global__ __launch_bounds__(kBlock) void k_tet_query(Dev<R> d, Consts c) {
  if (is_done(d.st)) return;
  tet_query_lane<R, DEBUG, PREFETCH>(d, c, blockIdx.x * kBlock + threadIdx.x);
}

// One workgroup per penetrating vertex: vertex normal, then the first hit of
// [x_v, x_v - L_ray n_v] on a boundary face of its mesh not containing v, the
// faces split over the workgroup's lanes and the first hit (smallest t, ties
// to the lowest face id) reduced through the wavefronts and LDS.
template <typename R, bool DEBUG>
__global__ __launch_bounds__(kBlock) void k_ray(Dev<R> d, Consts c) {
  __shared__ double sh_t[kBlock / 64];
  __shared__ int sh_f[kBlock / 64];
  if (is_done(d.st)) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int npen = __hip_atomic_load(&d.st->n_pen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const size_t n = (size_t)c.n;
  const int F = c.F;
  for (int i = blockIdx.x; i < npen; i += gridDim.x) {
    const int s = d.penlist[i];
    const int v = d.qverts[s];
    const MeshConst mc = d.mesh[d.vmesh[v]];
    // area-weighted normal: sum over incident faces in ascending id
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = d.qf_start[s]; j < d.qf_start[s + 1]; ++j) {
      const int f = d.qf_list[j];
      double a0[3], a1[3], a2[3], e1[3], e2[3], cr[3];
      load3(d.xc, n, d.faces[f], a0);
      load3(d.xc, n, d.faces[F + f], a1);
      load3(d.xc, n, d.faces[2 * F + f], a2);
      for (int k = 0; k < 3; ++k) {
        e1[k] = a1[k] - a0[k];
        e2[k] = a2[k] - a0[k];
      }
      cross3(e1, e2, cr);
      acc[0] = acc[0] + cr[0];
      acc[1] = acc[1] + cr[1];
      acc[2] = acc[2] + cr[2];
    }
    double len;
    {
      len = sqrt((acc[0] * acc[0] + acc[1] * acc[1]) + acc[2] * acc[2]);
    }
    if (!(len > 0.0)) {  // the same for every thread of the block
      if (threadIdx.x == 0) d.fhit[s] = -1;
      continue;
    }
    double o[3], dir[3], end[3], slo[3], shi[3];
    load3(d.xc, n, v, o);
    {
      for (int k = 0; k < 3; ++k) {
        dir[k] = -(acc[k] / len);
        end[k] = o[k] + mc.Lray * dir[k];
        slo[k] = fmin(o[k], end[k]);
        shi[k] = fmax(o[k], end[k]);
      }
    }
    double best_t = INFINITY;
    int best_f = INT_MAX;
    for (int f = mc.fbeg + (int)threadIdx.x; f < mc.fend; f += kBlock) {
      const int i0 = d.faces[f], i1 = d.faces[F + f], i2 = d.faces[2 * F + f];
      if (i0 == v || i1 == v || i2 == v) continue;
      double a0[3], a1[3], a2[3];
      load3(d.xc, n, i0, a0);
      load3(d.xc, n, i1, a1);
      load3(d.xc, n, i2, a2);
      bool ov = true;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double flo = fmin(fmin(a0[k], a1[k]), a2[k]);
        const double fhi = fmax(fmax(a0[k], a1[k]), a2[k]);
        ov = ov && (flo <= shi[k]) && (slo[k] <= fhi);
      }
      if (!ov) continue;
      if (DEBUG) {
        const int k = atomicAdd(&d.st->cand_tri, 1);
        if (k < d.dbg_cap) {
          d.dbg_tri[k] = v;
          d.dbg_tri[d.dbg_cap + k] = f;
        }
      }
      double t;
      if (moller_trumbore(o, dir, a0, a1, a2, mc.Lray, &t)) {
        if (t < best_t || (t == best_t && f < best_f)) {
          best_t = t;
          best_f = f;
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ot = __shfl_xor(best_t, off, 64);
      const int of = __shfl_xor(best_f, off, 64);
      if (ot < best_t || (ot == best_t && of < best_f)) {
        best_t = ot;
        best_f = of;
      }
    }
    if (lane == 0) {
      sh_t[wv] = best_t;
      sh_f[wv] = best_f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < kBlock / 64; ++w)
        if (sh_t[w] < best_t || (sh_t[w] == best_t && sh_f[w] < best_f)) {
          best_t = sh_t[w];
          best_f = sh_f[w];
        }
      if (best_f == INT_MAX) {
        d.fhit[s] = -1;
      } else {
        d.fhit[s] = best_f;
        double a0[3], a1[3], a2[3], e1[3], e2[3], cr[3];
        load3(d.xc, n, d.faces[best_f], a0);
        load3(d.xc, n, d.faces[F + best_f], a1);
        load3(d.xc, n, d.faces[2 * F + best_f], a2);
        const double te = best_t + mc.eps;
        for (int k = 0; k < 3; ++k) {
          d.fc[3 * s + k] = o[k] + te * dir[k];
          e1[k] = a1[k] - a0[k];
          e2[k] = a2[k] - a0[k];
        }
        cross3(e1, e2, cr);
        const double ln = sqrt((cr[0] * cr[0] + cr[1] * cr[1]) + cr[2] * cr[2]);
        for (int k = 0; k < 3; ++k) d.fn[3 * s + k] = cr[k] / ln;
      }
    }
    __syncthreads();  // sh_t / sh_f are reused by the next vertex
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_contacts(Dev<R> d, Consts c) {
  if (is_done(d.st)) return;
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s < c.S) contacts_one(d, c, s);
}


template <typename R>
hipError_t launch_collide_stage(const Dev<R>& d, const Consts& c, int stage, bool debug, hipStream_t s) {
  // grids of at least one block: a mesh may have no query vertex (all fixed)
  const int gs = max(1, cdiv(c.S, kBlock)), gt = cdiv(c.T, kBlock);
  const int gt4 = cdiv(c.T * TetQueryLanes<true>::n, kBlock);
  switch (stage) {
    case STAGE_HASH_INSERT:
      k_hash_insert<R><<<gs, kBlock, 0, s>>>(d, c);
      break;
    case STAGE_TET_QUERY:
      if (debug)
        k_tet_query<R, true, true><<<gt4, kBlock, 0, s>>>(d, c);
      else if (c.T < kTetQueryWide)
        k_tet_query<R, false, true><<<gt4, kBlock, 0, s>>>(d, c);
      else
        k_tet_query<R, false, false><<<gt, kBlock, 0, s>>>(d, c);
      break;
    case STAGE_RAY: {
      // one workgroup per penetrating vertex on the first pass (up to 2048)
      const int gr = max(1, min(c.S, 2048));
      if (debug)
        k_ray<R, true><<<gr, kBlock, 0, s>>>(d, c);
      else
        k_ray<R, false><<<gr, kBlock, 0, s>>>(d, c);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_contacts(const Dev<R>& d, const Consts& c, hipStream_t s) {
  k_contacts<R><<<max(1, cdiv(c.S, kBlock)), kBlock, 0, s>>>(d, c);
  return hipGetLastError();
}


template hipError_t launch_collide_stage<float>(const Dev<float>&, const Consts&, int, bool, hipStream_t);
template hipError_t launch_collide_stage<double>(const Dev<double>&, const Consts&, int, bool, hipStream_t);
template hipError_t launch_contacts<float>(const Dev<float>&, const Consts&, hipStream_t);
template hipError_t launch_contacts<double>(const Dev<double>&, const Consts&, hipStream_t);

}  // namespace gs
