// Device helpers: wavefront/block reductions, a grid barrier for persistent
// launches, and the exact (FP64, fixed order, no contraction) predicates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace gs {

// Three reals padded to 16 (float) or 32 (double) bytes: one vector load.
template <typename R>
struct alignas(4 * sizeof(R)) W4 {
  R x, y, z, w;
};

// Store of a W4 with the sc1 cache policy: written through to the device's
// coherence point instead of left dirty in the XCD's L2.  The grid barrier's
// agent-scope release writes back every dirty L2 line, which costs time in
// proportion to what is dirty; state that other workgroups read after a
// barrier is stored this way, so that write-back finds little to do.  The
// release and acquire fences stay as they are.  `base` must be the same for
// the whole wavefront (it forms the buffer descriptor) and `i` is an element
// index from it with i * sizeof(W4) < 2^31.
// POL is the buffer store's cache-policy operand: 16 (sc1) writes through,
// 0 is the ordinary write-back store (st_wb below).
template <int POL, typename R>
__device__ __forceinline__ void st_buf(W4<R>* base, unsigned i, const W4<R>& v) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  constexpr int kRawDword3 = 0x00020000;    // raw buffer descriptor word 3 (32-bit data format)
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, 0x7fffffff, kRawDword3);
  if constexpr (sizeof(R) == 4) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, v), r, i * 16u, 0, POL);
  } else {
    struct Half {
      R a, b;
    };
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, Half{v.x, v.y}), r, i * 32u, 0, POL);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, Half{v.z, v.w}), r, i * 32u + 16u, 0, POL);
  }
}
template <typename R>
__device__ __forceinline__ void st_wt(W4<R>* base, unsigned i, const W4<R>& v) {
  st_buf<16>(base, i, v);
}
// The same store through L2 (write-back): the three 16-byte vectors of a row
// record merge into whole lines there before they reach memory, which pays
// when the CG state is far larger than the caches and the iteration is bound
// by memory traffic rather than by the barrier.
template <typename R>
__device__ __forceinline__ void st_wb(W4<R>* base, unsigned i, const W4<R>& v) {
  st_buf<0>(base, i, v);
}

// A double partial sum stored the same way (an agent-scope relaxed store).
__device__ __forceinline__ void st_wt(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the incidence columns res[i0, i1) into double accumulators, in index
// order; the loads are issued 8 at a time so their latencies overlap.
template <typename R>
__device__ __forceinline__ void sum_columns(const W4<R>* __restrict__ res, int i0, int i1, double& r0, double& r1,
                                            double& r2) {
  int i = i0;
  for (; i + 8 <= i1; i += 8) {
    W4<R> t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = res[i + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      r0 += (double)t[k].x;
      r1 += (double)t[k].y;
      r2 += (double)t[k].z;
    }
  }
  for (; i < i1; ++i) {
    const W4<R> t = res[i];
    r0 += (double)t.x;
    r1 += (double)t.y;
    r2 += (double)t.z;
  }
}

// ---- reductions (64-wide wavefronts) ---------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over the block; the result is valid in thread 0.  `lds` holds one
// double per wavefront.  Fixed association order (deterministic).
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < BLOCK / 64; ++i) t += lds[i];
  }
  __syncthreads();
  return t;
}
template <int BLOCK>
__device__ __forceinline__ double block_max(double v, double* lds) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < BLOCK / 64; ++i) t = fmax(t, lds[i]);
  }
  __syncthreads();
  return t;
}

// ---- grid barrier (every block resident: an ordinary launch of a grid that
// fits in half the resident capacity, or a cooperative launch) ---------------
// One arrival counter that only grows during a launch: barrier j of the launch
// is complete once it reads (j + 1) * nblocks, so the last arrival has nothing
// more to write and no generation word has to be reset and re-published.
// Thread 0 of each block releases the block's writes at agent scope, arrives,
// waits for the count (wrap-safe comparison) and acquires.  The release writes
// back the XCD's dirty L2 lines, so state that other blocks read afterwards
// is stored write-through (st_wt) to leave it little to do.  `target` is the
// block's own count of arrivals expected so far.  The launch's last block
// clears the counter once every block is past its last barrier.
//
// The wait is bounded: a block that has waited `timeout` ticks of the
// constant-rate wall clock (a workgroup that never arrives: the grid was not
// co-resident), or that finds the status word `done` already set to STALLED
// by another block, stores STALLED there (only over RUNNING) and returns
// false without the acquire; every caller then leaves the kernel at once,
// so all blocks end normally and the host reads the code instead of the GPU
// spinning.  A block launched after the others gave up finds the word set
// at its start and returns.  timeout = 0 gives up at the first unfinished
// poll (the host's way to exercise this path).
__device__ __forceinline__ bool grid_barrier(unsigned* count, unsigned& target, unsigned nblocks, int* done,
                                             unsigned long long timeout) {
  __shared__ int ok_sh;
  target += nblocks;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    const unsigned long long t0 = wall_clock64();
    while ((int)(__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      if (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == STALLED ||
          wall_clock64() - t0 >= timeout) {
        int expect = RUNNING;
        __hip_atomic_compare_exchange_strong(done, &expect, (int)STALLED, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok_sh = ok;
  }
  __syncthreads();
  return ok_sh != 0;
}

// Two-level grid barrier for larger grids: workgroup b arrives at the
// counter of group b mod NG (NG = 8: one group per XCD, as consecutive
// workgroups are placed round-robin over the XCDs), the group's last arrival
// passes one arrival on to the top counter, and every workgroup waits on the
// top counter.  G arrivals on one word become at most G/NG per group word
// plus NG on the top word.  `inst` counts this launch's barriers (the
// counters are monotonic within a launch and cleared after it); the give-up
// rule is grid_barrier's.  grp[64 g] is group g's counter (a cache line
// apart), top the top counter.
__device__ __forceinline__ bool grid_barrier2(unsigned* grp, unsigned* top, unsigned& inst, unsigned nblocks,
                                              unsigned NG, int* done, unsigned long long timeout) {
  __shared__ int ok_sh2;
  inst += 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g = blockIdx.x % NG;
    const unsigned members = (nblocks - g + NG - 1) / NG;  // workgroups b < nblocks with b mod NG = g
    const unsigned groups = nblocks < NG ? nblocks : NG;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned t = __hip_atomic_fetch_add(grp + 64 * g, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t + 1 == inst * members) {
      // the group's last arrival: what the group published happens before
      // the top arrival that the waiting workgroups observe
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const unsigned target = inst * groups;
    int ok = 1;
    const unsigned long long t0 = wall_clock64();
    while ((int)(__hip_atomic_load(top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      if (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == STALLED ||
          wall_clock64() - t0 >= timeout) {
        int expect = RUNNING;
        __hip_atomic_compare_exchange_strong(done, &expect, (int)STALLED, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok_sh2 = ok;
  }
  __syncthreads();
  return ok_sh2 != 0;
}

// ---- exact predicates -------------------------------------------------------
// Six times the signed volume det[p1-p0, p2-p0, p3-p0], evaluated in the
// order written (contraction off), FP64.
__device__ __forceinline__ double orient(const double* p0, const double* p1, const double* p2, const double* p3) {
#pragma clang fp contract(off)
  const double ax = p1[0] - p0[0], ay = p1[1] - p0[1], az = p1[2] - p0[2];
  const double bx = p2[0] - p0[0], by = p2[1] - p0[1], bz = p2[2] - p0[2];
  const double cx = p3[0] - p0[0], cy = p3[1] - p0[1], cz = p3[2] - p0[2];
  return ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx);
}

// Strictly inside a positively oriented tet (a,b,c,d): all four sub-volumes
// with one vertex replaced by q are positive (ties are outside).
__device__ __forceinline__ bool point_in_tet(const double* q, const double* a, const double* b, const double* c,
                                             const double* d) {
  return orient(q, b, c, d) > 0.0 && orient(a, q, c, d) > 0.0 && orient(a, b, q, d) > 0.0 &&
         orient(a, b, c, q) > 0.0;
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* o) {
#pragma clang fp contract(off)
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dot3(const double* a, const double* b) {
#pragma clang fp contract(off)
  return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

// Segment o + t d (0 < t <= L) against triangle (a0, a1, a2): Moller-Trumbore.
__device__ __forceinline__ bool moller_trumbore(const double* o, const double* d, const double* a0, const double* a1,
                                                const double* a2, double L, double* t_out) {
#pragma clang fp contract(off)
  double e1[3] = {a1[0] - a0[0], a1[1] - a0[1], a1[2] - a0[2]};
  double e2[3] = {a2[0] - a0[0], a2[1] - a0[1], a2[2] - a0[2]};
  double pv[3];
  cross3(d, e2, pv);
  const double det = dot3(e1, pv);
  if (det == 0.0) return false;
  double tv[3] = {o[0] - a0[0], o[1] - a0[1], o[2] - a0[2]};
  const double u = dot3(tv, pv) / det;
  double qv[3];
  cross3(tv, e1, qv);
  const double w = dot3(d, qv) / det;
  const double t = dot3(e2, qv) / det;
  *t_out = t;
  return (u >= 0.0) && (w >= 0.0) && (u + w <= 1.0) && (t > 0.0) && (t <= L);
}

// Vertex v of an SoA [3][n] double array.
__device__ __forceinline__ void load3(const double* xc, size_t n, int v, double* o) {
  o[0] = xc[v];
  o[1] = xc[n + v];
  o[2] = xc[2 * n + v];
}

// Spatial-hash cell of a coordinate (monotone in x, so a point inside a box
// lies in a cell of the box's cell range).
__device__ __forceinline__ int cell_of(double x, double inv_cell) { return (int)floor(x * inv_cell); }

// Bucket of cell (ix, iy, iz) of mesh m (meshes of a batch share the table).
__device__ __forceinline__ int hash_cell(int ix, int iy, int iz, int m, int H) {
  const uint32_t h = ((uint32_t)ix * 73856093u) ^ ((uint32_t)iy * 19349663u) ^ ((uint32_t)iz * 83492791u) ^
                     ((uint32_t)m * 2654435761u);
  return (int)(h & (uint32_t)(H - 1));
}

// Inserts query vertex s (vertex v of mesh m, collision position x) into the
// bucket of its cell; a full bucket's entry goes to the overflow list, which
// holds S entries (one insertion per query vertex between clears).  Entries
// carry the position, so a candidate costs one 32-byte read.  A diverged
// position is not inserted.
template <typename DevT>
__device__ __forceinline__ void hash_insert_entry(const DevT& d, const Consts& c, int s, int v, int m, double x0,
                                                  double x1, double x2) {
  const double ic = d.mesh[m].inv_cell;
  if (!(fabs(x0 * ic) < 1e9 && fabs(x1 * ic) < 1e9 && fabs(x2 * ic) < 1e9)) return;
  double4 e;
  e.x = x0;
  e.y = x1;
  e.z = x2;
  e.w = __longlong_as_double((long long)(((unsigned long long)(unsigned)v << 32) | (unsigned)s));
  const int key = hash_cell(cell_of(x0, ic), cell_of(x1, ic), cell_of(x2, ic), m, c.H);
  const int slot = atomicAdd(&d.hcount[key], 1);
  if (slot < kHashCap) {
    reinterpret_cast<double4*>(d.hslot)[(size_t)key * kHashCap + slot] = e;
  } else {
    const int o = atomicAdd(&d.st->n_over, 1);
    if (o < c.S) reinterpret_cast<double4*>(d.hover)[o] = e;
  }
}

// Mesh of a vertex / tet is frozen once it has converged (batched solves).
template <typename DevT>
__device__ __forceinline__ bool mesh_frozen(const DevT& d, int mask, int m) {
  return mask && d.mdone[m] != 0;
}

__device__ __forceinline__ bool is_done(const DevStatus* st) {
  return __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != RUNNING;
}

}  // namespace gs
