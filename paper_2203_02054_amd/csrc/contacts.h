// Collision response per query vertex (Sections II-C, III-A.3, Eq. 5, Eq. 8):
// the active set A_k from A_{k-1}, fresh ray hits and obstacle closest points,
// with the release rule of Eq. 8.  Shared by the stand-alone contact kernels
// and the CG kernel's first phase; every function here evaluates its
// arithmetic in the order written, without contraction, whatever the
// including file's setting, so the decisions match the oracle bit for bit.
#pragma once

#include "device_common.h"

namespace gs {

__device__ __forceinline__ bool released(const double* x, const double* tc, const double* nc, double eps) {
#pragma clang fp contract(off)
  const double g = (nc[0] * (x[0] - tc[0]) + nc[1] * (x[1] - tc[1])) + nc[2] * (x[2] - tc[2]);
  return fabs(g) > eps;
}

// Active set A_k from A_{k-1} (stored in place), per query vertex.
template <typename R>
__device__ __forceinline__ void contacts_one(const Dev<R>& d, const Consts& c, int s) {
#pragma clang fp contract(off)
  const int v = d.qverts[s];
  const int m = d.vmesh[v];
  if (mesh_frozen(d, c.mask_done, m)) return;
  const double eps = d.mesh[m].eps;
  double x[3];
  load3(d.xc, (size_t)c.n, v, x);
  const int base = s * c.slots;
  bool changed = false;
  int nact = 0;
  if (c.self_col) {
    const bool old = d.cact[base] != 0;
    const bool pen = d.pen[s] != 0;
    const int hit = pen ? d.fhit[s] : -1;
    bool now = false;
    if (pen && hit >= 0) {
      now = true;
      for (int k = 0; k < 3; ++k) {
        d.ctgt[3 * base + k] = d.fc[3 * s + k];
        d.cnrm[3 * base + k] = d.fn[3 * s + k];
      }
      d.cprim[base] = hit;
    } else if (old) {
      now = pen ? true : !released(x, d.ctgt + 3 * base, d.cnrm + 3 * base, eps);
    }
    if (pen && hit < 0) atomicAdd(&d.st->ray_miss, 1);
    d.cact[base] = now ? ((pen && hit >= 0) ? 2 : 1) : 0;
    changed |= (now != old);
    nact += now;
    d.pen[s] = 0;
  }
  if (c.obst_col) {
    for (int j = 0; j < c.ns; ++j) {
      const double* sp = d.obst + 4 * j;
      const int slot = base + 1 + j;
      const bool old = d.cact[slot] != 0;
      const double dx = x[0] - sp[0], dy = x[1] - sp[1], dz = x[2] - sp[2];
      const double q = (dx * dx + dy * dy) + dz * dz;
      const bool inside = q < sp[3] * sp[3];
      bool now = false;
      if (inside || old) {
        const double dist = sqrt(q);
        double nc[3];
        if (dist > 0.0) {
          nc[0] = dx / dist;
          nc[1] = dy / dist;
          nc[2] = dz / dist;
        } else {
          nc[0] = 0.0;
          nc[1] = 0.0;
          nc[2] = 1.0;
        }
        const double rr = sp[3] + eps;
        const double tc[3] = {sp[0] + rr * nc[0], sp[1] + rr * nc[1], sp[2] + rr * nc[2]};
        now = inside || !released(x, tc, nc, eps);
        if (now) {
          for (int k = 0; k < 3; ++k) {
            d.ctgt[3 * slot + k] = tc[k];
            d.cnrm[3 * slot + k] = nc[k];
          }
          d.cprim[slot] = j;
        }
      }
      d.cact[slot] = now ? 1 : 0;
      changed |= (now != old);
      nact += now;
    }
    for (int j = 0; j < c.np; ++j) {
      const double* pl = d.obst + 4 * c.ns + 6 * j;
      const int slot = base + 1 + c.ns + j;
      const bool old = d.cact[slot] != 0;
      const double sd = (pl[3] * (x[0] - pl[0]) + pl[4] * (x[1] - pl[1])) + pl[5] * (x[2] - pl[2]);
      const bool inside = sd < 0.0;
      bool now = false;
      if (inside || old) {
        const double se = sd - eps;
        const double nc[3] = {pl[3], pl[4], pl[5]};
        const double tc[3] = {x[0] - se * nc[0], x[1] - se * nc[1], x[2] - se * nc[2]};
        now = inside || !released(x, tc, nc, eps);
        if (now) {
          for (int k = 0; k < 3; ++k) {
            d.ctgt[3 * slot + k] = tc[k];
            d.cnrm[3 * slot + k] = nc[k];
          }
          d.cprim[slot] = j;
        }
      }
      d.cact[slot] = now ? 1 : 0;
      changed |= (now != old);
      nact += now;
    }
  }
  if (c.mo) {
    // the triangle-mesh obstacle: its kernel tested the vertices inside the
    // obstacle's box and those holding a contact with it
    const int slot = base + 1 + c.ns + c.np;
    const bool old = d.cact[slot] != 0;
    const int fl = d.mo_flag[s];
    bool now = false;
    if (fl) {
      const double* tc = d.mo_tgt + 3 * s;
      const double* nc = d.mo_nrm + 3 * s;
      now = fl == 2 || (old && !released(x, tc, nc, eps));
      if (now) {
        for (int k = 0; k < 3; ++k) {
          d.ctgt[3 * slot + k] = tc[k];
          d.cnrm[3 * slot + k] = nc[k];
        }
        d.cprim[slot] = d.mo_prim[s];
      }
    }
    d.cact[slot] = now ? 1 : 0;
    changed |= (now != old);
    nact += now;
  }
  if (changed) {
    atomicOr(&d.st->changed, 1);
    d.mchanged[m] = 1;
  }
  if (nact) atomicAdd(&d.st->n_contacts, nact);
}

}  // namespace gs
