// Anderson acceleration of the local/global iteration (the acceleration the
// paper applies to its solver, end of Section III-B; Walker & Ni 2011, type
// II, memory m; safeguarded after Peng et al. 2018).
//
// Every outer iteration evaluates the plain map at the current point x_k
// (collision, local step, global step): the CG kernel leaves the correction
// f_k = G(x_k) - x_k in dl, the residual r_k, the energy E_k, and, per mesh,
// the decision on x_k (AaMesh::act, taken by its last block).  Then, per mesh:
//   accepted   the history gains dX = x_k - x_acc, dF = f_k - f_acc (x_acc,
//              f_acc: the last accepted point and residual) and keeps its
//              last m columns; gamma = argmin |f_k - dF gamma| and
//              x_{k+1} = x_k + f_k - (dX + dF) gamma   (x_k + f_k = G(x_k));
//   rejected   x_{k+1} = x_acc + f_acc = G(x_acc), the plain step from the
//              last accepted point, with that point's active set restored
//              (history cleared by the decision);
//   converged  x_{k+1} = G(x_k), as in the plain iteration.
// When the solve ends (converged, max_iter or fixed_iters) the result is
// G(x_k), so the stopping rule and the result are the plain iteration's.
// The iterate is the displacement u = x - X0 ([3][n]).  The dot products of a
// mesh are summed over a fixed list of blocks that never straddle meshes, in
// a fixed order, so every decision is deterministic.
#include "anderson.h"

namespace gs {

constexpr int kFaaBlock = 256;

// The new difference column of each accepted mesh, the stored point and
// residual, and the block partials of dF_j . dF_new and dF_j . f_k.
template <typename R>
__global__ __launch_bounds__(kFaaBlock) void k_faa_dots(Dev<R> d, Consts c) {
  __shared__ double lds[kFaaBlock / 64];
  if (is_done(d.st)) return;
  const AaBlock B = d.faa_blk[blockIdx.x];
  const AaMesh* a = d.faa + B.m;
  if (a->act != AA_ACCEPT) return;  // uniform: the block's rows share the mesh
  const int m = c.faa_m;
  const bool push = a->has_prev != 0;
  const int col = a->head;
  const int mk = push ? min(a->k + 1, m) : 0;
  const size_t n = (size_t)c.n, n3 = 3 * n;
  const W4<R>* dl = reinterpret_cast<const W4<R>*>(d.dl);
  double pa[kAaMaxMem], pb[kAaMaxMem];
#pragma unroll
  for (int j = 0; j < kAaMaxMem; ++j) pa[j] = pb[j] = 0.0;
  for (int v = B.v0 + (int)threadIdx.x; v < B.v1; v += kFaaBlock) {
    const W4<R> fv = dl[v];
    const R f3[3] = {fv.x, fv.y, fv.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const size_t e = k * n + v;
      const R f = f3[k], x = d.u[e];
      if (push) {
        const R df = f - d.aa_fp[e];
        d.aa_df[col * n3 + e] = df;
        d.aa_dx[col * n3 + e] = x - d.aa_xp[e];
#pragma unroll
        for (int j = 0; j < kAaMaxMem; ++j) {
          if (j < mk) {
            const double dj = (j == col) ? (double)df : (double)d.aa_df[j * n3 + e];
            pa[j] += dj * (double)df;
            pb[j] += dj * (double)f;
          }
        }
      }
      d.aa_xp[e] = x;
      d.aa_fp[e] = f;
    }
  }
  if (!push) return;
  const int NB = c.faa_nblk;
#pragma unroll
  for (int j = 0; j < kAaMaxMem; ++j) {
    if (j < mk) {  // uniform over the block
      const double ta = block_sum<kFaaBlock>(pa[j], lds);
      const double tb = block_sum<kFaaBlock>(pb[j], lds);
      if (threadIdx.x == 0) {
        d.aa_part[(size_t)(2 * j) * NB + blockIdx.x] = ta;
        d.aa_part[(size_t)(2 * j + 1) * NB + blockIdx.x] = tb;
      }
    }
  }
}

// One block per mesh: its partials summed over its blocks in order, the
// Gram matrix updated in the new column, gamma solved (gram_solve), and the
// mesh's history bookkeeping.
template <typename R>
__global__ __launch_bounds__(kAaSolveThreads) void k_faa_solve(Dev<R> d, Consts c) {
  __shared__ double val[2 * kAaMaxMem];
  __shared__ double A[kAaMaxMem][kAaMaxMem];
  __shared__ double y[kAaMaxMem];
  if (is_done(d.st)) return;
  const int mi = blockIdx.x;
  AaMesh* a = d.faa + mi;
  if (a->act != AA_ACCEPT) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (!a->has_prev) {
    // first accepted point after a reset: stored by k_faa_dots, plain step
    __syncthreads();
    if (tid == 0) {
      a->has_prev = 1;
      a->cand = 0;
      a->ok = 0;
    }
    return;
  }
  const int m = c.faa_m;
  const int col = a->head;
  const int mk = min(a->k + 1, m);
  const int b0 = d.faa_mblk[mi], b1 = d.faa_mblk[mi + 1], NB = c.faa_nblk;
  constexpr int nw = kAaSolveThreads / 64;
  for (int q = wave; q < 2 * mk; q += nw) {
    double t = 0.0;
    for (int b = b0 + lane; b < b1; b += 64) t += d.aa_part[(size_t)q * NB + b];
    t = wave_sum(t);
    if (lane == 0) val[q] = t;
  }
  __syncthreads();
  double* H = d.faa_h + (size_t)mi * kAaMaxMem * kAaMaxMem;
  const int i = tid / mk, j = tid % mk;
  if (tid < mk * mk) {
    double h;
    if (i == col) h = val[2 * j];
    else if (j == col) h = val[2 * i];
    else h = H[i * kAaMaxMem + j];
    H[i * kAaMaxMem + j] = h;
    A[i][j] = h;
  }
  if (tid < mk) y[tid] = val[2 * tid + 1];
  __syncthreads();
  double gj;
  const bool ok = gram_solve(A, y, mk, &gj);
  if (wave == 0 && lane < mk) d.faa_gam[(size_t)mi * kAaMaxMem + lane] = gj;
  if (tid == 0) {
    a->k = mk;
    a->head = (col + 1) % m;
    a->cand = ok ? 1 : 0;
    a->ok = ok ? 1 : 0;
  }
}

// The position update of the iteration just evaluated, per row (its mesh's
// decision), then the collision positions and, while the solve runs, the
// spatial-hash entries of the query vertices for the next tet query (the
// CG kernel's first phase cleared the table).  Runs once per finished
// iteration: the CG kernel's last block raises aa_pending, the last block
// here lowers it, so launches after the solve has ended change nothing.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_faa_update(Dev<R> d, Consts c) {
  __shared__ int last;
  DevStatus* st = d.st;
  if (__hip_atomic_load(&st->aa_pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  const int code = __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int it = st->iters;
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v < c.n && code != BREAKDOWN && code != STALLED) {
    const int m = d.vmesh[v];
    const AaMesh* a = d.faa + m;
    const int act = a->act;
    // a mesh with no decision was frozen earlier, or converged now (then
    // the plain step is due); a finished solve ends on the plain step
    const bool plain = (act == AA_NONE && d.mdone[m] == it) || (act != AA_NONE && code != RUNNING);
    if (plain || act != AA_NONE) {
      const size_t n = (size_t)c.n, n3 = 3 * n;
      const W4<R> fv = reinterpret_cast<const W4<R>*>(d.dl)[v];
      const R f3[3] = {fv.x, fv.y, fv.z};
      const int mk = (!plain && act == AA_ACCEPT && a->ok) ? a->k : 0;
      double g[kAaMaxMem];
#pragma unroll
      for (int j = 0; j < kAaMaxMem; ++j) g[j] = j < mk ? d.faa_gam[(size_t)m * kAaMaxMem + j] : 0.0;
      double xn[3];
      R pr[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const size_t e = k * n + v;
        R u;
        pr[k] = f3[k];
        if (!plain && act == AA_REJECT) {
          u = d.aa_xp[e] + d.aa_fp[e];
        } else {
          double t = (double)d.u[e] + (double)f3[k], q = (double)f3[k];
#pragma unroll
          for (int j = 0; j < kAaMaxMem; ++j)
            if (j < mk) {
              const double df = (double)d.aa_df[j * n3 + e];
              t -= g[j] * ((double)d.aa_dx[j * n3 + e] + df);
              q -= g[j] * df;
            }
          u = (R)t;
          pr[k] = (R)q;
        }
        d.u[e] = u;
        xn[k] = d.X0[e] + (double)u;
        d.xc[e] = xn[k];
      }
      if (mk > 0 && code == RUNNING) {
        // warm start of the next global step: the least-squares model's
        // prediction of the next correction, f_k - dF gamma, with f_k kept
        // as the history's last correction (the CG start is the Galerkin
        // projection onto the prediction and the last two corrections)
        W4<R>* dl = reinterpret_cast<W4<R>*>(d.dl);
        W4<R>* dlp = reinterpret_cast<W4<R>*>(d.dlp);
        dlp[v] = fv;
        W4<R> q;
        q.x = pr[0];
        q.y = pr[1];
        q.z = pr[2];
        q.w = R(0);
        dl[v] = q;
      }
      const int sq = d.vq[v];
      if (code == RUNNING && act != AA_NONE && sq >= 0) {
        // the active set of an accepted point is kept; a rejected point's is
        // replaced by it, so the plain step from the accepted point starts
        // from the set the plain iteration would have had
        const int b0 = sq * c.slots;
        for (int sl = 0; sl < c.slots; ++sl) {
          const int b = b0 + sl;
          if (act == AA_ACCEPT) {
            d.cact_s[b] = d.cact[b];
            d.cprim_s[b] = d.cprim[b];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              d.ctgt_s[3 * b + q] = d.ctgt[3 * b + q];
              d.cnrm_s[3 * b + q] = d.cnrm[3 * b + q];
            }
          } else {
            d.cact[b] = d.cact_s[b];
            d.cprim[b] = d.cprim_s[b];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              d.ctgt[3 * b + q] = d.ctgt_s[3 * b + q];
              d.cnrm[3 * b + q] = d.cnrm_s[3 * b + q];
            }
          }
        }
        if (c.self_col) hash_insert_entry(d, c, sq, v, m, xn[0], xn[1], xn[2]);
      }
    }
  }
  // the last block out lowers the flag (every block has read it)
  __syncthreads();
  if (threadIdx.x == 0) {
    const int t = __hip_atomic_fetch_add(&st->aa_ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = (t == (int)gridDim.x - 1);
    if (last) {
      st->aa_ticket = 0;
      __hip_atomic_store(&st->aa_pending, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <typename R>
hipError_t launch_fwd_anderson(const Dev<R>& d, const Consts& c, hipStream_t s) {
  if (c.faa_m <= 0) return hipSuccess;
  k_faa_dots<R><<<max(1, c.faa_nblk), kFaaBlock, 0, s>>>(d, c);
  k_faa_solve<R><<<max(1, c.M), kAaSolveThreads, 0, s>>>(d, c);
  k_faa_update<R><<<max(1, cdiv(c.n, kBlock)), kBlock, 0, s>>>(d, c);
  return hipGetLastError();
}

template hipError_t launch_fwd_anderson<float>(const Dev<float>&, const Consts&, hipStream_t);
template hipError_t launch_fwd_anderson<double>(const Dev<double>&, const Consts&, hipStream_t);

}  // namespace gs
