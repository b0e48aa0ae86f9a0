// Host layer of the C ABI: input validation, the once-per-mesh set-up, the
// device workspace layout, and the outer-iteration driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <stdexcept>
#include <string>
#include <functional>
#include <map>
#include <vector>

#include "geosim.h"
#include "internal.h"

using namespace gs;

namespace {

thread_local std::string g_err;

gs_status fail(gs_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                             \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return fail(GS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// outward faces of a positively oriented tet: the face opposite each slot
constexpr int kFaceSlots[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};

// six times the signed volume det[p1-p0, p2-p0, p3-p0] (same evaluation order
// as the device predicate; this file is compiled without contraction)
double orient_h(const double* p0, const double* p1, const double* p2, const double* p3) {
  const double ax = p1[0] - p0[0], ay = p1[1] - p0[1], az = p1[2] - p0[2];
  const double bx = p2[0] - p0[0], by = p2[1] - p0[1], bz = p2[2] - p0[2];
  const double cx = p3[0] - p0[0], cy = p3[1] - p0[1], cz = p3[2] - p0[2];
  return ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Offsets of every device array inside the workspace.
struct Layout {
  size_t X0, tets, tag, inc_start, inc_pos, ell_col, ell_val, ell_scaled, adiag, freem, faces, qverts, vq, qf_start, qf_list, kq,
      obst;
  size_t u, xc, res4, cg, dl, dlp, dlpp, p, dg, dsp, pen, hcount, hslot, hover, penlist, fhit, fc, fn, cact, ctgt, cnrm,
      cprim, part_a, part_b, part_c, part_d, part_e, part_f, st, trace, mesh, vmesh, tmesh, mres, mchanged, mdone;
  size_t mu, acc3, ga, ch_start, ch_tets, mmax, mdone2, st2, alpha_last, mgam;
  size_t aa_dx, aa_df, aa_xp, aa_fp, aa_h, aa_gamma, aa_part, aa_k;
  size_t lam, ga_acc, st3, st4;
  size_t faa, faa_h, faa_gam, faa_blk, faa_mblk, cact_s, ctgt_s, cnrm_s, cprim_s;
  size_t rcount, alpha_stage, acc_max;
  size_t cz_inv, cz_nb, cz_rho, cz_ri;
  size_t mo_tri, mo_id, mo_node, mo_flag, mo_tgt, mo_nrm, mo_prim;
  size_t seg, mbar, bar2;
  size_t total;
};

constexpr int kNKernels = 14;
const char* const kKernelNames[kNKernels] = {"hash_insert", "tet_query",  "ray_cast",     "contacts",   "local",
                                             "gather",      "pcg",        "adj_springs",  "adj_local",  "adj_gather",
                                             "adj_pcg",     "anderson",   "remesh_flags", "mesh_obstacle"};
enum { K_CONTACTS = 3, K_LOCAL = 4, K_GATHER = 5, K_PCG = 6, K_ADJ_SPRINGS = 7, K_ADJ_LOCAL = 8, K_ADJ_GATHER = 9,
       K_ADJ_PCG = 10, K_ANDERSON = 11, K_REMESH = 12, K_MESH_OBST = 13 };

// Optional per-kernel timing: each launch is bracketed by two events on the
// bound stream; elapsed times are collected whenever the driver synchronises.
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<int> fam;  // kernel id of each recorded pair
  double ms[kNKernels] = {};
  long long cnt[kNKernels] = {};

  hipError_t mark(hipStream_t s, int f, bool start) {
    const size_t i = 2 * fam.size() + (start ? 0 : 1);
    while (pool.size() <= i) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      pool.push_back(e);
    }
    if (!start) fam.push_back(f);
    return hipEventRecord(pool[i], s);
  }
  // an event pair for a launch that records the kernel's own start and end
  hipError_t pair(int f, hipEvent_t& a, hipEvent_t& b) {
    const size_t i = 2 * fam.size();
    while (pool.size() <= i + 1) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      pool.push_back(e);
    }
    fam.push_back(f);
    a = pool[i];
    b = pool[i + 1];
    return hipSuccess;
  }
  void drop_last() { fam.pop_back(); }
  hipError_t flush() {
    for (size_t k = 0; k < fam.size(); ++k) {
      float t = 0.f;
      hipError_t r = hipEventElapsedTime(&t, pool[2 * k], pool[2 * k + 1]);
      if (r != hipSuccess) return r;
      ms[fam[k]] += t;
      cnt[fam[k]] += 1;
    }
    fam.clear();
    return hipSuccess;
  }
  void reset() {
    fam.clear();
    for (int k = 0; k < kNKernels; ++k) {
      ms[k] = 0;
      cnt[k] = 0;
    }
  }
  ~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct gs_problem {
  int prec = 4;
  int n = 0, T = 0, nch = 0, S = 0, F = 0, slots = 1, H = 0, nnz = 0, nparts = 0;
  int ns = 0, np = 0;
  // triangle-mesh obstacle: leaf-ordered records, ids and tree (empty: none)
  std::vector<double> mo_tri;
  std::vector<int32_t> mo_id;
  std::vector<MoNode> mo_node;
  int mo_k = 0;
  // coarse correction: built for this CG grid (0: none yet), and whether it applies
  int coarse_G = 0;
  bool coarse_ok = false;
  // refit-only AABB tree over the tets (built on first use): nodes in
  // breadth-first order, leaf tet order, first node of every depth
  std::vector<MoNode> tree_node;
  std::vector<int32_t> tree_order;
  std::vector<int> tree_level;
  gs_params prm{};
  std::vector<double> X0;
  std::vector<int32_t> tets, tag, inc_start, inc_pos, rowptr, col, faces, qverts, vq, qf_start, qf_list, ell_col;
  std::vector<double> val, adiag, kq, obst, ell_val;
  int ell_w = 0;
  std::vector<uint8_t> freem;
  int n_surf_verts = 0;
  double h_ref = 0, eps = 0, Lray = 0, diag = 0, cell = 0, inv_mean_vol = 0;  // of a single mesh (mesh 0)
  // meshes (a single mesh is a batch of one)
  int M = 1;
  std::vector<double> mh_ref, mdiag, mcell, minv_mean_vol;
  std::vector<int32_t> vbeg, tbeg, chbeg, fbeg, sbeg;  // [M+1] offsets
  std::vector<int32_t> vmesh, tmesh;
  std::vector<int32_t> ch_start, ch_tets;  // chamber -> tets (ascending)
  std::vector<AaBlock> faa_blk;            // blocks of the acceleration's dot-product kernel
  std::vector<int32_t> faa_mblk;           // [M+1] first block of each mesh
  std::vector<int4> seg;                   // per-mesh CG: {mesh, index, workgroups, first} per workgroup
  std::vector<int32_t> seg_k;              // per-mesh CG: workgroups of each mesh
  // device binding
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  bool bound = false;
  Layout lay{};
  int pcg_grid = 1;
  int pcg_maxg = 0;  // CG workgroups that can be resident at once
  bool hash_ready = false;  // the device hash holds the current collision positions
  int trace_len = 0;
  int last_iters = 0;
  bool solved = false;  // a solve has run since gs_bind (the adjoint's state exists)
  int aa_cap = 0;       // Anderson memory the workspace holds (max(aa_m, adj_aa_m) at gs_create)
  int wclk_khz = 0;     // rate of the device's constant wall clock (grid-barrier time limit)
  Profiler prof;
  // pinned host copies of the device status, one per chunk in flight, and
  // the events that mark their copies (created at gs_bind)
  DevStatus* hstat = nullptr;
  hipEvent_t hev[2] = {nullptr, nullptr};
  // a chunk of outer iterations captured as a HIP graph, and what it was
  // captured for (the kernels' arguments); replaced when they change
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::string gkey;
  hipStream_t cap_stream = nullptr;  // the capture's own stream (the caller's may be the null stream)
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    gkey.clear();
  }
  ~gs_problem() {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (hstat) (void)hipHostFree(hstat);
    for (hipEvent_t e : hev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

gs_status check_params(const gs_params* p);

// The energy guard compares one mesh's energy: not for a batch.
gs_status check_batch_params(const gs_params* p, int M) {
  if (M > 1 && p->aa_m > 0 && (p->aa_guard & 3) == GS_AA_GUARD_ENERGY)
    return fail(GS_EINVAL, "the energy guard of the accelerated iteration needs a single mesh");
  return GS_OK;
}

gs_status check_params(const gs_params* p) {
  if (!p) return fail(GS_EINVAL, "null params");
  if (!(p->c1 > 0) || !(p->c2 >= 0) || !std::isfinite(p->c1) || !std::isfinite(p->c2))
    return fail(GS_EINVAL, "Mooney-Rivlin constants must be c1 > 0, c2 >= 0");
  if (!(p->kappa_col > 0) || !(p->eps_rel > 0) || !(p->ray_rel > 0))
    return fail(GS_EINVAL, "kappa_col, eps_rel and ray_rel must be positive");
  if (!(p->tol >= 0) || p->max_iter < 1 || p->fixed_iters < 0) return fail(GS_EINVAL, "bad tol/max_iter/fixed_iters");
  if (!(p->pcg_eta > 0 && p->pcg_eta < 1) || p->pcg_max < 1) return fail(GS_EINVAL, "bad pcg_eta/pcg_max");
  if (p->check_every < 1) return fail(GS_EINVAL, "check_every must be >= 1");
  if (p->trace_len < 0) return fail(GS_EINVAL, "trace_len must be >= 0");
  if (!(p->adj_tol >= 0) || p->adj_max_iter < 1) return fail(GS_EINVAL, "bad adj_tol/adj_max_iter");
  if (p->adj_aa_m < 0 || p->adj_aa_m > kAaMaxMem) return fail(GS_EINVAL, "adj_aa_m must be in [0, 16]");
  if (p->aa_m < 0 || p->aa_m > kAaMaxMem) return fail(GS_EINVAL, "aa_m must be in [0, 16]");
  if ((p->aa_guard & ~7) != 0 || (p->aa_guard & 3) == 3) return fail(GS_EINVAL, "bad aa_guard");
  if (!(p->aa_slack >= 0) || !std::isfinite(p->aa_slack)) return fail(GS_EINVAL, "aa_slack must be >= 0");
  if (!(p->barrier_timeout_ms >= 0) || !std::isfinite(p->barrier_timeout_ms))
    return fail(GS_EINVAL, "barrier_timeout_ms must be >= 0");
  if (!(p->pcg_eta_min >= 0) || !std::isfinite(p->pcg_eta_min)) return fail(GS_EINVAL, "pcg_eta_min must be >= 0");
  if (p->pcg_coarse != 0 && p->pcg_coarse != 1) return fail(GS_EINVAL, "pcg_coarse must be 0 or 1");
  if (p->pcg_per_mesh < 0 || p->pcg_per_mesh > 2) return fail(GS_EINVAL, "pcg_per_mesh must be 0, 1 or 2");
  if (p->graph != 0 && p->graph != 1) return fail(GS_EINVAL, "graph must be 0 or 1");
  if (p->pcg_store < 0 || p->pcg_store > 2) return fail(GS_EINVAL, "pcg_store must be 0, 1 or 2");
  return GS_OK;
}

Layout make_layout(const gs_problem* p) {
  Layout L{};
  size_t off = 0;
  const size_t W = (size_t)p->prec;
  auto take = [&](size_t bytes) {
    off = align256(off);
    const size_t o = off;
    off += std::max<size_t>(bytes, 1);
    return o;
  };
  const size_t n = p->n, T = p->T, S = p->S, F = p->F, sl = p->slots, H = p->H;
  L.X0 = take(3 * n * 8);
  L.tets = take(4 * T * 4);
  L.tag = take(T * 4);
  L.inc_start = take((n + 1) * 4);
  L.inc_pos = take(4 * T * 4);
  L.ell_col = take((size_t)p->ell_w * n * 4);
  L.ell_val = take((size_t)p->ell_w * n * W);
  L.ell_scaled = take((size_t)p->ell_w * n * W);
  L.adiag = take(n * W);
  L.freem = take(n);
  L.faces = take(3 * F * 4);
  L.qverts = take(S * 4);
  L.vq = take(n * 4);
  L.qf_start = take((S + 1) * 4);
  L.qf_list = take(p->qf_list.size() * 4);
  L.kq = take(S * 8);
  L.obst = take((4 * (size_t)p->ns + 6 * (size_t)p->np) * 8);
  L.u = take(3 * n * W);
  L.xc = take(3 * n * 8);
  L.res4 = take(4 * T * 4 * W);
  L.cg = take(24 * n * W);
  L.dl = take(4 * n * W);
  L.dlp = take(4 * n * W);
  L.dlpp = take(4 * n * W);
  L.p = take(4 * n * W);
  L.dg = take(n * W);
  L.dsp = take(n * W);
  L.pen = take(S * 4);
  L.hcount = take(H * 4);
  L.hslot = take(H * kHashCap * 32);
  L.hover = take(S * 32);
  L.penlist = take(S * 4);
  L.fhit = take(S * 4);
  L.fc = take(3 * S * 8);
  L.fn = take(3 * S * 8);
  L.cact = take(S * sl);
  L.ctgt = take(3 * S * sl * 8);
  L.cnrm = take(3 * S * sl * 8);
  L.cprim = take(S * sl * 4);
  L.part_a = take((size_t)p->nparts * 8);
  L.part_b = take((size_t)p->nparts * 8);
  L.part_c = take((size_t)p->nparts * 8);
  L.part_d = take((size_t)p->nparts * 8);
  L.part_e = take((size_t)p->nparts * 8);
  L.part_f = take((size_t)p->nparts * 8);
  L.st = take(sizeof(DevStatus));
  L.trace = take((size_t)p->trace_len * 6 * 8);
  L.mesh = take((size_t)p->M * sizeof(MeshConst));
  L.vmesh = take(n * 4);
  L.tmesh = take(T * 4);
  L.mres = take((size_t)p->M * 8);
  L.mchanged = take((size_t)p->M * 4);
  L.mdone = take((size_t)p->M * 4);
  L.mu = take(3 * n * W);
  L.acc3 = take(3 * n * 8);
  L.ga = take(T * 8);
  L.ch_start = take(((size_t)p->nch + 1) * 4);
  L.ch_tets = take(p->ch_tets.size() * 4);
  L.mmax = take((size_t)p->M * 8);
  L.mgam = take((size_t)p->M * 16);
  L.mdone2 = take((size_t)p->M * 4);
  L.st2 = take(sizeof(DevStatus));
  L.alpha_last = take((size_t)p->nch * W);
  const size_t am = (size_t)p->aa_cap;
  L.aa_dx = take(am * 3 * n * W);
  L.aa_df = take(am * 3 * n * W);
  L.aa_xp = take(am ? 3 * n * W : 0);
  L.aa_fp = take(am ? 3 * n * W : 0);
  L.aa_h = take(am * am * 8);
  L.aa_gamma = take(am * 8);
  L.aa_part = take(2 * am * (size_t)p->nparts * 8);
  L.aa_k = take(4);
  L.lam = take(3 * n * W);
  L.ga_acc = take((size_t)p->nch * 8);
  L.st3 = take(sizeof(DevStatus));
  L.st4 = take(sizeof(DevStatus));
  L.faa = take((size_t)p->M * sizeof(AaMesh));
  L.faa_h = take((size_t)p->M * kAaMaxMem * kAaMaxMem * 8);
  L.faa_gam = take((size_t)p->M * kAaMaxMem * 8);
  L.faa_blk = take(p->faa_blk.size() * sizeof(AaBlock));
  L.faa_mblk = take(p->faa_mblk.size() * 4);
  L.cact_s = take(S * sl);
  L.ctgt_s = take(3 * S * sl * 8);
  L.cnrm_s = take(3 * S * sl * 8);
  L.cprim_s = take(S * sl * 4);
  L.mo_tri = take(p->mo_tri.size() * 8);
  L.mo_id = take(p->mo_id.size() * 4);
  L.mo_node = take(p->mo_node.size() * sizeof(MoNode));
  L.mo_flag = take(p->mo_k ? S : 0);
  L.mo_tgt = take(p->mo_k ? 3 * S * 8 : 0);
  L.mo_nrm = take(p->mo_k ? 3 * S * 8 : 0);
  L.mo_prim = take(p->mo_k ? S * 4 : 0);
  L.rcount = take(4);
  L.acc_max = take(8);
  L.cz_inv = take(p->M == 1 ? (size_t)kCoarseMaxG * kCoarseMaxG * 8 : 0);
  L.cz_nb = take(p->M == 1 ? (size_t)kCoarseMaxG * kCoarseNb * 4 : 0);
  L.cz_rho = take(p->M == 1 ? 4 * n * W : 0);
  L.cz_ri = take(p->M == 1 ? n * 4 : 0);
  L.alpha_stage = take((size_t)p->nch * W);
  L.seg = take((size_t)std::max(p->M, kMaxPcgGrid) * sizeof(int4));
  L.mbar = take((size_t)p->M * 4);
  L.bar2 = take((size_t)kBarWords * 4);
  L.total = align256(off);
  return L;
}

template <typename R>
Dev<R> make_dev(const gs_problem* p) {
  const Layout& L = p->lay;
  char* b = p->ws;
  Dev<R> d{};
  d.X0 = (const double*)(b + L.X0);
  d.tets = (const int32_t*)(b + L.tets);
  d.tag = (const int32_t*)(b + L.tag);
  d.inc_start = (const int32_t*)(b + L.inc_start);
  d.inc_pos = (const int32_t*)(b + L.inc_pos);
  d.ell_col = (const int32_t*)(b + L.ell_col);
  d.ell_val = (const R*)(b + L.ell_val);
  d.ell_scaled = (R*)(b + L.ell_scaled);
  d.adiag = (const R*)(b + L.adiag);
  d.freem = (const uint8_t*)(b + L.freem);
  d.faces = (const int32_t*)(b + L.faces);
  d.qverts = (const int32_t*)(b + L.qverts);
  d.vq = (const int32_t*)(b + L.vq);
  d.qf_start = (const int32_t*)(b + L.qf_start);
  d.qf_list = (const int32_t*)(b + L.qf_list);
  d.kq = (const double*)(b + L.kq);
  d.obst = (const double*)(b + L.obst);
  d.u = (R*)(b + L.u);
  d.xc = (double*)(b + L.xc);
  d.res4 = (R*)(b + L.res4);
  d.cg = (R*)(b + L.cg);
  d.dl = (R*)(b + L.dl);
  d.dlp = (R*)(b + L.dlp);
  d.dlpp = (R*)(b + L.dlpp);
  d.p = (R*)(b + L.p);
  d.dg = (R*)(b + L.dg);
  d.dsp = (R*)(b + L.dsp);
  d.pen = (int32_t*)(b + L.pen);
  d.hcount = (int32_t*)(b + L.hcount);
  d.hslot = (double*)(b + L.hslot);
  d.hover = (double*)(b + L.hover);
  d.penlist = (int32_t*)(b + L.penlist);
  d.fhit = (int32_t*)(b + L.fhit);
  d.fc = (double*)(b + L.fc);
  d.fn = (double*)(b + L.fn);
  d.cact = (uint8_t*)(b + L.cact);
  d.ctgt = (double*)(b + L.ctgt);
  d.cnrm = (double*)(b + L.cnrm);
  d.cprim = (int32_t*)(b + L.cprim);
  d.part_a = (double*)(b + L.part_a);
  d.part_b = (double*)(b + L.part_b);
  d.part_c = (double*)(b + L.part_c);
  d.part_d = (double*)(b + L.part_d);
  d.part_e = (double*)(b + L.part_e);
  d.part_f = (double*)(b + L.part_f);
  d.st = (DevStatus*)(b + L.st);
  d.trace = (double*)(b + L.trace);
  d.mesh = (const MeshConst*)(b + L.mesh);
  d.vmesh = (const int32_t*)(b + L.vmesh);
  d.tmesh = (const int32_t*)(b + L.tmesh);
  d.mres = (unsigned long long*)(b + L.mres);
  d.mchanged = (int32_t*)(b + L.mchanged);
  d.mdone = (int32_t*)(b + L.mdone);
  d.mu = (R*)(b + L.mu);
  d.gL = nullptr;
  d.acc3 = (double*)(b + L.acc3);
  d.ga = (double*)(b + L.ga);
  d.ch_start = (const int32_t*)(b + L.ch_start);
  d.ch_tets = (const int32_t*)(b + L.ch_tets);
  d.mmax = (unsigned long long*)(b + L.mmax);
  d.mgam = (double*)(b + L.mgam);
  d.alpha_last = (R*)(b + L.alpha_last);
  d.aa_dx = (R*)(b + L.aa_dx);
  d.aa_df = (R*)(b + L.aa_df);
  d.aa_xp = (R*)(b + L.aa_xp);
  d.aa_fp = (R*)(b + L.aa_fp);
  d.aa_h = (double*)(b + L.aa_h);
  d.aa_gamma = (double*)(b + L.aa_gamma);
  d.aa_part = (double*)(b + L.aa_part);
  d.aa_k = (int32_t*)(b + L.aa_k);
  d.lam = (R*)(b + L.lam);
  d.ga_acc = (double*)(b + L.ga_acc);
  d.faa = (AaMesh*)(b + L.faa);
  d.faa_h = (double*)(b + L.faa_h);
  d.faa_gam = (double*)(b + L.faa_gam);
  d.faa_blk = (const AaBlock*)(b + L.faa_blk);
  d.faa_mblk = (const int32_t*)(b + L.faa_mblk);
  d.cact_s = (uint8_t*)(b + L.cact_s);
  d.ctgt_s = (double*)(b + L.ctgt_s);
  d.cnrm_s = (double*)(b + L.cnrm_s);
  d.cprim_s = (int32_t*)(b + L.cprim_s);
  d.dbg_tet = nullptr;
  d.dbg_tri = nullptr;
  d.acc_max = (unsigned long long*)(b + L.acc_max);
  d.cz_inv = (const double*)(b + L.cz_inv);
  d.cz_nb = (const int32_t*)(b + L.cz_nb);
  d.cz_rho = (const R*)(b + L.cz_rho);
  d.cz_ri = (const int32_t*)(b + L.cz_ri);
  d.mo_tri = (const double*)(b + L.mo_tri);
  d.mo_id = (const int32_t*)(b + L.mo_id);
  d.mo_node = (const MoNode*)(b + L.mo_node);
  d.mo_flag = (uint8_t*)(b + L.mo_flag);
  d.mo_tgt = (double*)(b + L.mo_tgt);
  d.mo_nrm = (double*)(b + L.mo_nrm);
  d.mo_prim = (int32_t*)(b + L.mo_prim);
  d.dbg_cap = 0;
  d.seg = (const int4*)(b + L.seg);
  d.mbar = (unsigned*)(b + L.mbar);
  d.bar2 = (unsigned*)(b + L.bar2);
  return d;
}

// The coarse correction applies to one-mesh problems whose CG grid runs the
// rows-of-three-vectors kernel variant on at most kCoarseMaxG workgroups.
template <typename T>
hipError_t upload(char* base, size_t off, const std::vector<T>& v, hipStream_t s) {
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(base + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

constexpr int kWbRows = 700000;
constexpr int kBar2Grid = 128;

// The CG state stored write-back: forced, or by default above kWbRows rows
// (state far beyond the caches, the iteration bound by memory traffic).
bool store_wb(const gs_problem* p) {
  return p->prm.pcg_store == 2 || (p->prm.pcg_store == 0 && p->n > kWbRows);
}

// A batch's CG with its own workgroups per mesh.
bool per_mesh_cg(const gs_problem* p) { return p->prm.pcg_per_mesh && p->M > 1; }

// The per-mesh CG plan: mesh m gets k_m consecutive workgroups, one plus its
// share, by rows, of the budget beyond one per mesh (pcg_blocks, else what
// can be resident), and at most one per kSegMinRows rows, so its rows split
// as the rows of that mesh alone split over k_m workgroups of the unpaired
// kernel.  Uploaded on the problem's stream.
constexpr int kSegMinRows = 512;
// The longest-processing-time plan (pcg_per_mesh = 2): the budget B
// (pcg_blocks, else the workgroups that can be resident at once) is read as
// the workgroups one pass of the device runs, and every workgroup should get
// about (all rows) / B rows: mesh m gets ceil(n_m / that) workgroups (at most
// one per kSegMinRows rows), so a large mesh is split and a small one keeps
// one.  The grid may then exceed what can be resident, which only a
// single-workgroup mesh may wait out: the meshes with several workgroups,
// whose workgroups wait for each other, come first in block order (placed
// first by an ordinary launch) and together take at most half the resident
// capacity, the split of the mesh that loses least being undone until they
// do; the single-workgroup meshes follow, largest first, so the smallest
// ones queue for the workgroups that finish first.
void plan_lpt(gs_problem* p, int maxg, std::vector<int>& order) {
  const int M = p->M;
  const long B = std::max(1, std::min(p->prm.pcg_blocks > 0 ? p->prm.pcg_blocks : maxg, kMaxPcgGrid));
  std::vector<long> nm(M);
  long tot = 0;
  for (int m = 0; m < M; ++m) tot += (nm[m] = p->vbeg[m + 1] - p->vbeg[m]);
  const long tgt = std::max(1L, (tot + B - 1) / B);
  long multi = 0, all = 0;
  for (int m = 0; m < M; ++m) {
    const long cap = std::max(1L, nm[m] / kSegMinRows);
    p->seg_k[m] = (int)std::max(1L, std::min((nm[m] + tgt - 1) / tgt, cap));
    all += p->seg_k[m];
    if (p->seg_k[m] > 1) multi += p->seg_k[m];
  }
  const long multi_cap = std::max(0, maxg / 2), all_cap = std::max(M, kMaxPcgGrid);
  while (multi > multi_cap || all > all_cap) {
    // undo one workgroup of the split mesh whose rows per workgroup grow least
    int best = -1;
    double best_rows = 0.0;
    for (int m = 0; m < M; ++m)
      if (p->seg_k[m] > 1) {
        const double r = (double)nm[m] / (p->seg_k[m] - 1);
        if (best < 0 || r < best_rows) {
          best = m;
          best_rows = r;
        }
      }
    if (best < 0) break;
    multi -= p->seg_k[best];
    p->seg_k[best] -= 1;
    all -= 1;
    if (p->seg_k[best] > 1) multi += p->seg_k[best];
  }
  order.resize(M);
  for (int m = 0; m < M; ++m) order[m] = m;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const bool sa = p->seg_k[a] > 1, sb = p->seg_k[b] > 1;
    if (sa != sb) return sa;
    return (double)nm[a] / p->seg_k[a] > (double)nm[b] / p->seg_k[b];
  });
}

gs_status plan_segments(gs_problem* p, int maxg) {
  p->seg_k.assign(p->M, 1);
  p->seg.clear();
  if (!per_mesh_cg(p)) return GS_OK;
  if (p->prm.pcg_per_mesh == 2) {
    std::vector<int> order;
    plan_lpt(p, maxg, order);
    for (int m : order) {
      const int k = p->seg_k[m], b0 = (int)p->seg.size();
      for (int j = 0; j < k; ++j) p->seg.push_back(make_int4(m, j, k, b0));
    }
    HIPCHK(upload(p->ws, p->lay.seg, p->seg, p->stream));
    return GS_OK;
  }
  const int budget = std::min({p->prm.pcg_blocks > 0 ? p->prm.pcg_blocks : maxg, maxg, kMaxPcgGrid});
  const long extra = std::max(0L, (long)budget - p->M);
  for (int m = 0; m < p->M; ++m) {
    const long nm = p->vbeg[m + 1] - p->vbeg[m];
    const int k = (int)std::min(1 + extra * nm / std::max(1, p->n), std::max(1L, nm / kSegMinRows));
    p->seg_k[m] = k;
    const int b0 = (int)p->seg.size();
    for (int j = 0; j < k; ++j) p->seg.push_back(make_int4(m, j, k, b0));
  }
  HIPCHK(upload(p->ws, p->lay.seg, p->seg, p->stream));
  return GS_OK;
}

bool coarse_wanted(const gs_problem* p) {
  const int G = p->pcg_grid;
  return p->prm.pcg_coarse && p->M == 1 && G >= 2 && G <= kCoarseMaxG && !pcg_paired(p->prec, p->ell_w, p->n, G);
}

// Two-level preconditioner D^-1 + R0^T A0^-1 R0 of the CG kernel (an
// additive coarse correction, Nicolaides-style aggregation): R0 sums
// the free rows of each workgroup's row range (the ranges the kernel uses:
// 64-aligned chunks of ceil(n / G) rows), A0 = R0 A_el R0^T from the elastic
// matrix (the springs of the current contact set stay in D only; the
// preconditioner need not match the matrix, only stay symmetric positive
// definite and fixed during a solve).  Built on the host in FP64 (Cholesky,
// then the explicit inverse, which the kernel applies as matrix-vector
// products); also each workgroup's list of the ranges its rows reach and
// each row's couplings (its off-diagonal sums per range: its own and at most
// two others, else the correction is not used).  Rebuilt when the grid
// changes.
gs_status ensure_coarse(gs_problem* p) {
  if (!coarse_wanted(p) || p->coarse_G == p->pcg_grid) return GS_OK;
  const int G = p->pcg_grid, n = p->n, w = p->ell_w;
  const int chunk = ((n + G - 1) / G + 63) & ~63;
  std::vector<double> A0((size_t)G * G, 0.0), rho(4 * (size_t)n, 0.0);
  std::vector<int32_t> ri(n, 0);
  std::vector<std::vector<int>> reach(G);
  for (int b = 0; b < G; ++b) reach[b].push_back(b);
  bool ok = true;
  for (int v = 0; v < n; ++v) {
    const int b = v / chunk;
    int oth[2] = {b, b};  // the other ranges the row couples to (at most two)
    ri[v] = b | (b << 16);
    if (!p->freem[v]) continue;
    A0[(size_t)b * G + b] += p->adiag[v];
    for (int k = 0; k < w; ++k) {
      const int j = p->ell_col[(size_t)k * n + v];
      const double a = p->ell_val[(size_t)k * n + v];
      if (a == 0.0) continue;  // padding
      const int bj = j / chunk;
      A0[(size_t)b * G + bj] += a;
      if (bj == b) {
        rho[4 * (size_t)v] += a;
        continue;
      }
      int slot = bj == oth[0] && oth[0] != b ? 0 : (bj == oth[1] && oth[1] != b ? 1 : -1);
      if (slot < 0) {
        if (oth[0] == b) slot = 0;
        else if (oth[1] == b) slot = 1;
        else {
          ok = false;  // a third other range: the per-row record cannot hold it
          continue;
        }
        oth[slot] = bj;
      }
      rho[4 * (size_t)v + 1 + slot] += a;
      if (std::find(reach[b].begin(), reach[b].end(), bj) == reach[b].end()) reach[b].push_back(bj);
    }
    ri[v] = oth[0] | (oth[1] << 16);
  }
  for (int b = 0; b < G; ++b) {
    if ((int)reach[b].size() > kCoarseNb) ok = false;
    if (A0[(size_t)b * G + b] == 0.0) A0[(size_t)b * G + b] = 1.0;  // a range of fixed rows only
  }
  // Cholesky A0 = L L^T, then A0^-1 column by column
  std::vector<double> L(A0);
  for (int j = 0; j < G && ok; ++j) {
    double d = L[(size_t)j * G + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * G + k] * L[(size_t)j * G + k];
    if (!(d > 0.0)) {
      ok = false;
      break;
    }
    d = std::sqrt(d);
    L[(size_t)j * G + j] = d;
    for (int i = j + 1; i < G; ++i) {
      double t = L[(size_t)i * G + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * G + k] * L[(size_t)j * G + k];
      L[(size_t)i * G + j] = t / d;
    }
  }
  std::vector<double> inv((size_t)G * G, 0.0);
  if (ok) {
    std::vector<double> y(G);
    for (int c = 0; c < G; ++c) {
      for (int i = 0; i < G; ++i) {
        double t = (i == c) ? 1.0 : 0.0;
        for (int k = 0; k < i; ++k) t -= L[(size_t)i * G + k] * y[k];
        y[i] = t / L[(size_t)i * G + i];
      }
      for (int i = G - 1; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < G; ++k) t -= L[(size_t)k * G + i] * inv[(size_t)k * G + c];
        inv[(size_t)i * G + c] = t / L[(size_t)i * G + i];
      }
    }
    // exactly symmetric, so every workgroup applies the same operator
    for (int i = 0; i < G; ++i)
      for (int j = i + 1; j < G; ++j) {
        const double m = 0.5 * (inv[(size_t)i * G + j] + inv[(size_t)j * G + i]);
        inv[(size_t)i * G + j] = inv[(size_t)j * G + i] = m;
      }
  }
  p->coarse_G = G;
  p->coarse_ok = ok;
  if (!ok) return GS_OK;
  std::vector<int32_t> nb((size_t)G * kCoarseNb, -1);
  for (int b = 0; b < G; ++b)
    for (size_t i = 0; i < reach[b].size(); ++i) nb[(size_t)b * kCoarseNb + i] = reach[b][i];
  hipStream_t s = p->stream;
  char* base = p->ws;
  HIPCHK(hipMemcpyAsync(base + p->lay.cz_inv, inv.data(), inv.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(base + p->lay.cz_nb, nb.data(), nb.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(base + p->lay.cz_ri, ri.data(), ri.size() * 4, hipMemcpyHostToDevice, s));
  if (p->prec == 4) {
    std::vector<float> r(rho.begin(), rho.end());
    HIPCHK(hipMemcpyAsync(base + p->lay.cz_rho, r.data(), r.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  } else {
    HIPCHK(hipMemcpyAsync(base + p->lay.cz_rho, rho.data(), rho.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return GS_OK;
}

Consts make_consts(const gs_problem* p) {
  Consts c{};
  c.n = p->n;
  c.T = p->T;
  c.S = p->S;
  c.F = p->F;
  c.nch = p->nch;
  c.slots = p->slots;
  c.H = p->H;
  c.ns = p->ns;
  c.np = p->np;
  c.self_col = p->prm.self_collision ? 1 : 0;
  c.obst_col = (p->prm.obstacle_collision && (p->ns + p->np) > 0) ? 1 : 0;
  c.mo = (p->prm.obstacle_collision && p->mo_k > 0) ? 1 : 0;
  c.coarse = (coarse_wanted(p) && p->coarse_G == p->pcg_grid && p->coarse_ok) ? 1 : 0;
  c.hyper = p->prm.hyperelastic ? 1 : 0;
  c.max_iter = p->prm.max_iter;
  c.fixed_iters = p->prm.fixed_iters;
  c.pcg_max = p->prm.pcg_max;
  c.nparts = p->nparts;
  // the local step runs in the tet-query launch (four lanes per tet) below
  // kTetQueryWide tets with self-collision, else on its own (one per tet)
  c.a_parts = (p->prm.self_collision && p->T < kTetQueryWide) ? cdiv(4L * p->T, kBlock) : cdiv(p->T, kBlock);
  c.ell_w = p->ell_w;
  c.per_mesh = per_mesh_cg(p) ? 1 : 0;
  c.cg_wb = store_wb(p) ? 1 : 0;
  // the two-level grid barrier above kBar2Grid workgroups (one counter takes
  // every arrival below that, and it measured as fast there)
  c.bar2 = (!c.per_mesh && p->pcg_grid > kBar2Grid) ? 1 : 0;
  c.cg_soa = (!c.per_mesh && pcg_paired(p->prec, p->ell_w, p->n, p->pcg_grid)) ? 1 : 0;
  c.trace_len = p->trace_len;
  c.c1 = p->prm.c1;
  c.c2 = p->prm.c2;
  c.kappa = p->prm.kappa_col;
  c.tol = p->prm.tol;
  c.pcg_eta = p->prm.pcg_eta;
  c.pcg_eta_min = p->prm.pcg_eta_min;
  c.M = p->M;
  c.mask_done = p->prm.fixed_iters > 0 ? 0 : 1;
  c.faa_m = std::min(p->prm.aa_m, p->aa_cap);
  c.faa_guard = p->prm.aa_guard;
  c.faa_slack = p->prm.aa_slack;
  c.faa_nblk = (int)p->faa_blk.size();
  c.bar_timeout = (unsigned long long)(p->prm.barrier_timeout_ms * (double)p->wclk_khz);
  return c;
}

template <typename R>
std::vector<R> cast_vec(const std::vector<double>& v) {
  return std::vector<R>(v.begin(), v.end());
}

// Workgroups of the cooperative CG kernel: about kPcgRowsPerBlock rows per
// block (half a block's threads on a small mesh, so twice the compute units
// share its neighbour gathers), within what can be resident and what the
// partial-sum arrays hold.
int pcg_grid_for(const gs_problem* p, int maxg) {
  int g = p->prm.pcg_blocks > 0 ? p->prm.pcg_blocks : cdiv(p->n, kPcgRowsPerBlock);
  return std::max(1, std::min({g, maxg, kMaxPcgGrid, p->nparts / 2}));
}

std::vector<MeshConst> mesh_table(const gs_problem* p) {
  std::vector<MeshConst> t(p->M);
  for (int m = 0; m < p->M; ++m) {
    t[m].eps = p->prm.eps_rel * p->mh_ref[m];
    t[m].Lray = p->prm.ray_rel * p->mh_ref[m];
    t[m].inv_cell = 1.0 / p->mcell[m];
    t[m].inv_diag = 1.0 / p->mdiag[m];
    t[m].inv_mean_vol = p->minv_mean_vol[m];
    t[m].fbeg = p->fbeg[m];
    t[m].fend = p->fbeg[m + 1];
    t[m].sbeg = p->sbeg[m];
    t[m].send = p->sbeg[m + 1];
    t[m].vbeg = p->vbeg[m];
    t[m].vend = p->vbeg[m + 1];
  }
  return t;
}

template <typename R>
gs_status bind_impl(gs_problem* p) {
  char* b = p->ws;
  const Layout& L = p->lay;
  hipStream_t s = p->stream;
  HIPCHK(upload(b, L.X0, p->X0, s));
  HIPCHK(upload(b, L.tets, p->tets, s));
  HIPCHK(upload(b, L.tag, p->tag, s));
  HIPCHK(upload(b, L.inc_start, p->inc_start, s));
  HIPCHK(upload(b, L.inc_pos, p->inc_pos, s));
  HIPCHK(upload(b, L.ell_col, p->ell_col, s));
  const std::vector<R> ell_val = cast_vec<R>(p->ell_val), adiag = cast_vec<R>(p->adiag);
  HIPCHK(upload(b, L.ell_val, ell_val, s));
  HIPCHK(upload(b, L.adiag, adiag, s));
  HIPCHK(upload(b, L.freem, p->freem, s));
  HIPCHK(upload(b, L.faces, p->faces, s));
  HIPCHK(upload(b, L.qverts, p->qverts, s));
  HIPCHK(upload(b, L.vq, p->vq, s));
  HIPCHK(upload(b, L.qf_start, p->qf_start, s));
  HIPCHK(upload(b, L.qf_list, p->qf_list, s));
  HIPCHK(upload(b, L.kq, p->kq, s));
  HIPCHK(upload(b, L.obst, p->obst, s));
  HIPCHK(upload(b, L.mo_tri, p->mo_tri, s));
  HIPCHK(upload(b, L.mo_id, p->mo_id, s));
  HIPCHK(upload(b, L.mo_node, p->mo_node, s));
  const std::vector<MeshConst> mt = mesh_table(p);
  HIPCHK(upload(b, L.mesh, mt, s));
  HIPCHK(upload(b, L.vmesh, p->vmesh, s));
  HIPCHK(upload(b, L.tmesh, p->tmesh, s));
  HIPCHK(upload(b, L.ch_start, p->ch_start, s));
  HIPCHK(upload(b, L.ch_tets, p->ch_tets, s));
  HIPCHK(upload(b, L.faa_blk, p->faa_blk, s));
  HIPCHK(upload(b, L.faa_mblk, p->faa_mblk, s));
  HIPCHK(hipMemsetAsync(b + L.mres, 0, (size_t)p->M * 8, s));
  HIPCHK(hipMemsetAsync(b + L.mchanged, 0, (size_t)p->M * 4, s));
  HIPCHK(hipMemsetAsync(b + L.mdone, 0, (size_t)p->M * 4, s));
  HIPCHK(hipMemsetAsync(b + L.mbar, 0, (size_t)p->M * 4, s));
  HIPCHK(hipMemsetAsync(b + L.bar2, 0, (size_t)kBarWords * 4, s));
  HIPCHK(hipMemsetAsync(b + L.cact, 0, (size_t)p->S * p->slots, s));
  HIPCHK(hipMemsetAsync(b + L.st, 0, sizeof(DevStatus), s));
  HIPCHK(hipMemsetAsync(b + L.hcount, 0, (size_t)p->H * 4, s));
  HIPCHK(hipMemsetAsync(b + L.pen, 0, (size_t)std::max(p->S, 1) * 4, s));
  HIPCHK(hipStreamSynchronize(s));
  const int maxg = pcg_max_grid<R>(p->ell_w);
  if (maxg < 1) return fail(GS_EHIP, "cannot size the cooperative CG grid");
  p->pcg_maxg = maxg;
  p->pcg_grid = pcg_grid_for(p, maxg);
  {
    const gs_status r = plan_segments(p, maxg);
    if (r != GS_OK) return r;
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&p->wclk_khz, hipDeviceAttributeWallClockRate, dev));
  if (p->wclk_khz <= 0) return fail(GS_EHIP, "device reports no wall-clock rate");
  return GS_OK;
}

// The CG kernel's grid barrier needs every workgroup resident at once.  A
// grid of at most half of what can be resident gets an ordinary launch (on
// an otherwise idle device every workgroup is placed at once, and work of
// other streams only delays some of them, it cannot hold them off for
// good); a larger one the cooperative launch, which guarantees it.
// Per-mesh CG: workgroups of a mesh wait for each other only, so a plan of
// one workgroup per mesh needs no co-residency at all; otherwise the plan
// fits what can be resident and the same rule applies.
bool pcg_cooperative(const gs_problem* p) {
  // (the longest-processing-time plan keeps its split meshes within half the
  // resident capacity and at the front, and takes an ordinary launch)
  if (per_mesh_cg(p)) return p->prm.pcg_per_mesh != 2 && (int)p->seg.size() > p->M && 2 * (int)p->seg.size() > p->pcg_maxg;
  return 2 * p->pcg_grid > p->pcg_maxg;
}
int pcg_launch_grid(const gs_problem* p) { return per_mesh_cg(p) ? (int)p->seg.size() : p->pcg_grid; }

// Launch one kernel, bracketed by timing events when profiling is on.
template <typename F>
hipError_t timed(gs_problem* p, int k, F&& launch) {
  hipError_t e;
  if (p->prof.on && (e = p->prof.mark(p->stream, k, true)) != hipSuccess) return e;
  if ((e = launch()) != hipSuccess) return e;
  if (p->prof.on) return p->prof.mark(p->stream, k, false);
  return hipSuccess;
}

// The CG launch, profiled: an ordinary launch carries the events itself, so
// they bracket the kernel alone (events recorded on the stream around it would
// add the dispatch gap); a cooperative launch is bracketed as the others.
template <typename R>
hipError_t timed_pcg(gs_problem* p, int k, const Dev<R>& d, const Consts& c, bool adjoint) {
  const bool coop = pcg_cooperative(p);
  if (!p->prof.on || coop)
    return timed(p, k, [&] { return launch_pcg<R>(d, c, pcg_launch_grid(p), p->stream, adjoint, coop); });
  hipEvent_t a, b;
  hipError_t e = p->prof.pair(k, a, b);
  if (e != hipSuccess) return e;
  if ((e = launch_pcg<R>(d, c, pcg_launch_grid(p), p->stream, adjoint, false, a, b)) != hipSuccess)
    p->prof.drop_last();
  return e;
}

// Iteration driver: enqueue `check_every` iterations at a time until the
// device status says done.  The status after each chunk is copied to pinned
// host memory behind an event, and the next chunk is enqueued before waiting
// for it, so the GPU never idles while the host enqueues; a chunk enqueued
// after the solve finished runs as no-ops (every kernel checks the done flag).
// With per-kernel profiling on, each chunk is waited for (its events must be
// complete before they are read).  `h` receives the final status.
template <typename F>
gs_status drive(gs_problem* p, const DevStatus* dstat, int limit, F&& enqueue_one, DevStatus& h,
                const std::string& gkey = std::string()) {
  hipStream_t s = p->stream;
  const int ce = p->prm.check_every;
  int enq = 0, c = 0;
  bool pending = false;
  while (true) {
    const int chunk = std::min(ce, std::max(1, limit - enq));
    if (!gkey.empty() && enq > 0 && chunk == ce) {
      // a full chunk after the first (which may build the hash): one graph
      // launch of the chunk's kernels, captured on first use
      if (!p->gexec || p->gkey != gkey) {
        // captured on a stream of its own (the kernels take p->stream, which
        // points there meanwhile); nothing runs until the graph is launched
        p->drop_graph();
        if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        p->stream = p->cap_stream;
        hipError_t e = hipSuccess;
        for (int i = 0; i < ce && e == hipSuccess; ++i) e = enqueue_one();
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(p->cap_stream, &g);
        p->stream = s;
        if (e != hipSuccess || e2 != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          return fail(GS_EHIP, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        }
        p->graph = g;
        HIPCHK(hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0));
        p->gkey = gkey;
      }
      HIPCHK(hipGraphLaunch(p->gexec, s));
    } else {
      for (int i = 0; i < chunk; ++i) HIPCHK(enqueue_one());
    }
    enq += chunk;
    HIPCHK(hipMemcpyAsync(&p->hstat[c & 1], dstat, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(p->hev[c & 1], s));
    if (p->prof.on) {
      HIPCHK(hipEventSynchronize(p->hev[c & 1]));
      HIPCHK(p->prof.flush());
      if (p->hstat[c & 1].done != RUNNING) break;
    } else if (pending) {
      HIPCHK(hipEventSynchronize(p->hev[(c - 1) & 1]));
      if (p->hstat[(c - 1) & 1].done != RUNNING) break;
    }
    pending = true;
    ++c;
    if (enq >= limit + 2 * ce) return fail(GS_EHIP, "iteration driver out of step with the device");
  }
  HIPCHK(hipMemcpyAsync(&p->hstat[0], dstat, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  h = p->hstat[0];
  return GS_OK;
}

// One outer iteration.  Below kTetQueryWide tets the local step rides in the
// tet-query launch (both read only the iteration's positions); the CG kernel
// updates the contacts, gathers the right-hand side, clears the spatial hash
// and refills it with the new positions: 3 launches per iteration with
// self-collision (tet query + local step, ray cast, CG) instead of 7.
template <typename R>
hipError_t enqueue_iteration(gs_problem* p, const Dev<R>& d, const Consts& c, const R* alpha) {
  hipError_t e;
  hipStream_t s = p->stream;
  const bool fused_local = c.self_col && c.T < kTetQueryWide;
  if (c.self_col) {
    // after positions were set the hash is built here; afterwards the CG
    // kernel's final update refills it (the contact/gather pass clears it)
    if (!p->hash_ready) {
      if ((e = timed(p, STAGE_HASH_INSERT,
                     [&] { return launch_collide_stage<R>(d, c, STAGE_HASH_INSERT, false, s); })) != hipSuccess)
        return e;
      p->hash_ready = true;
    }
    if (fused_local)
      e = timed(p, STAGE_TET_QUERY, [&] { return launch_query_local<R>(d, c, alpha, s); });
    else
      e = timed(p, STAGE_TET_QUERY, [&] { return launch_collide_stage<R>(d, c, STAGE_TET_QUERY, false, s); });
    if (e != hipSuccess) return e;
    if ((e = timed(p, STAGE_RAY, [&] { return launch_collide_stage<R>(d, c, STAGE_RAY, false, s); })) != hipSuccess)
      return e;
  }
  if (!fused_local)
    if ((e = timed(p, K_LOCAL, [&] { return launch_local<R>(d, c, alpha, s); })) != hipSuccess) return e;
  if (c.mo)
    if ((e = timed(p, K_MESH_OBST, [&] { return launch_mesh_obstacle<R>(d, c, s); })) != hipSuccess) return e;
  // the CG kernel first updates the contacts and gathers the right-hand side
  // (the per-mesh kernel finds the spatial hash already cleared)
  if (c.self_col && c.per_mesh)
    if ((e = launch_hash_clear<R>(d, c, s)) != hipSuccess) return e;
  if ((e = timed_pcg<R>(p, K_PCG, d, c, false)) != hipSuccess) return e;
  if (c.faa_m > 0) return timed(p, K_ANDERSON, [&] { return launch_fwd_anderson<R>(d, c, s); });
  return hipSuccess;
}

// Accelerated points rejected in the last solve (summed over the meshes).
gs_status aa_rejections(gs_problem* p, int& total) {
  total = 0;
  std::vector<AaMesh> a(p->M);
  HIPCHK(hipMemcpyAsync(a.data(), p->ws + p->lay.faa, a.size() * sizeof(AaMesh), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  for (const AaMesh& q : a) total += q.rejected;
  return GS_OK;
}

const char* kStalledMsg =
    "a grid barrier of the CG kernel gave up waiting (workgroups not co-resident, or barrier_timeout_ms too short)";

template <typename R>
gs_status solve_impl(gs_problem* p, const R* alpha, R* x, gs_stats* stats) {
  {
    const gs_status r = ensure_coarse(p);
    if (r != GS_OK) return r;
  }
  const Dev<R> d = make_dev<R>(p);
  const Consts c = make_consts(p);
  hipStream_t s = p->stream;
  if (p->nch > 0)
    HIPCHK(hipMemcpyAsync(d.alpha_last, alpha, (size_t)p->nch * sizeof(R), hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_init<R>(d, c, x, s));
  p->hash_ready = false;
  DevStatus h{};
  const int limit = p->prm.fixed_iters > 0 ? p->prm.fixed_iters : p->prm.max_iter;
  // a graph of a chunk of iterations is keyed by everything its kernels take
  std::string gkey;
  if (p->prm.graph && !p->prof.on && !pcg_cooperative(p)) {
    gkey.assign(1, (char)sizeof(R));
    gkey.append(reinterpret_cast<const char*>(&d), sizeof(d));
    gkey.append(reinterpret_cast<const char*>(&c), sizeof(c));
    gkey.append(reinterpret_cast<const char*>(&alpha), sizeof(alpha));
  }
  const gs_status ds = drive(p, d.st, limit, [&] { return enqueue_iteration<R>(p, d, c, alpha); }, h, gkey);
  if (ds != GS_OK) return ds;
  HIPCHK(launch_output<R>(d, c, x, s));
  HIPCHK(hipStreamSynchronize(s));
  p->last_iters = h.iters;
  p->solved = h.done != STALLED;
  int rej = 0;
  if (c.faa_m > 0) {
    const gs_status r = aa_rejections(p, rej);
    if (r != GS_OK) return r;
  }
  if (stats) {
    stats->iters = h.iters;
    stats->pcg_iters_total = h.pcg_total;
    stats->n_contacts = h.n_contacts_last;
    stats->ray_miss = h.ray_miss_last;
    stats->residual = h.residual;
    stats->energy = h.energy;
    stats->aa_rejected = rej;
    stats->pad = 0;
  }
  if (h.done == STALLED) return fail(GS_EHIP, kStalledMsg);
  if (h.done == BREAKDOWN) return fail(GS_EBREAKDOWN, "non-finite value or CG curvature p'Ap <= 0");
  if (h.done == MAXITER) {
    g_err = "max_iter reached";
    return GS_NOT_CONVERGED;
  }
  if (h.done == FIXED_DONE && !(h.residual <= p->prm.tol && !h.changed_last)) {
    g_err = "fixed iteration count reached above tolerance";
    return GS_NOT_CONVERGED;
  }
  return GS_OK;
}

// Implicit adjoint: mu <- M^-1 (g + (db/dx)^T mu) in correction form with its
// own status block and per-mesh done flags, then dL/dalpha per chamber.
template <typename R>
gs_status adjoint_impl(gs_problem* p, const R* gL, R* dalpha, R* mu_out, gs_stats* stats) {
  Dev<R> d = make_dev<R>(p);
  d.st = (DevStatus*)(p->ws + p->lay.st2);
  d.mdone = (int32_t*)(p->ws + p->lay.mdone2);
  d.gL = gL;
  Consts c = make_consts(p);
  c.fixed_iters = 0;
  c.mask_done = 1;
  c.tol = p->prm.adj_tol;
  c.max_iter = p->prm.adj_max_iter;
  c.trace_len = 0;
  c.aa_m = std::min(p->prm.adj_aa_m, p->aa_cap);
  c.faa_m = 0;  // the forward acceleration's kernels are not part of the adjoint iteration
  if (c.aa_m > 0) c.mask_done = 0;  // the accelerated update mixes meshes: converge all at once
  hipStream_t s = p->stream;
  HIPCHK(launch_adj_init<R>(d, c, s));
  DevStatus h{};
  auto one = [&]() -> hipError_t {
    hipError_t e;
    if ((e = timed(p, K_ADJ_SPRINGS, [&] { return launch_adj_springs<R>(d, c, s); })) != hipSuccess) return e;
    if ((e = timed(p, K_ADJ_LOCAL, [&] { return launch_adj_local<R>(d, c, false, s); })) != hipSuccess) return e;
    if ((e = timed(p, K_ADJ_GATHER, [&] { return launch_adj_gather<R>(d, c, s); })) != hipSuccess) return e;
    if ((e = timed_pcg<R>(p, K_ADJ_PCG, d, c, true)) != hipSuccess) return e;
    return launch_adj_anderson<R>(d, c, s);
  };
  const gs_status ds = drive(p, d.st, c.max_iter, one, h);
  if (ds != GS_OK) return ds;
  HIPCHK(launch_adj_local<R>(d, c, true, s));
  HIPCHK(launch_adj_chamber_sum<R>(d, c, dalpha, s));
  if (mu_out) HIPCHK(hipMemcpyAsync(mu_out, d.mu, 3 * (size_t)p->n * sizeof(R), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  if (stats) {
    stats->iters = h.iters;
    stats->pcg_iters_total = h.pcg_total;
    stats->n_contacts = 0;
    stats->ray_miss = 0;
    stats->residual = h.residual;
    stats->energy = 0.0;
    stats->aa_rejected = 0;
    stats->pad = 0;
  }
  if (h.done == STALLED) return fail(GS_EHIP, kStalledMsg);
  if (h.done == BREAKDOWN) return fail(GS_EBREAKDOWN, "non-finite value or CG curvature p'Ap <= 0 in the adjoint");
  if (h.done == MAXITER) {
    g_err = "adj_max_iter reached";
    return GS_NOT_CONVERGED;
  }
  return GS_OK;
}

// ---------------------------------------------------------------------------
// set-up

gs_status setup(gs_problem* p, const gs_mesh_desc* m) {
  const int n = m->n_verts, T = m->n_tets;
  p->n = n;
  p->T = T;
  p->nch = m->n_chambers;
  p->prec = m->precision;
  p->X0.assign(m->rest_xyz, m->rest_xyz + 3 * (size_t)n);
  for (double v : p->X0)
    if (!std::isfinite(v)) return fail(GS_EINVAL, "non-finite rest position");
  p->tets.assign(m->tets, m->tets + 4 * (size_t)T);
  for (int32_t v : p->tets)
    if (v < 0 || v >= n) return fail(GS_EINVAL, "tet vertex index out of range");
  p->tag.resize(T);
  for (int e = 0; e < T; ++e) {
    const int mode = m->tet_mode[e], ch = m->tet_chamber[e];
    if (mode < GS_BODY || mode > GS_CH_AX_Z) return fail(GS_EINVAL, "bad tet_mode");
    if (mode != GS_BODY && (ch < 0 || ch >= p->nch)) return fail(GS_EINVAL, "chamber element without a valid chamber");
    p->tag[e] = mode | ((mode != GS_BODY ? ch : 0) << 3);
  }
  p->freem.resize(n);
  for (int v = 0; v < n; ++v) p->freem[v] = m->fixed[v] ? 0 : 1;
  auto X = [&](int v, int k) { return p->X0[(size_t)k * n + v]; };

  // h_ref: mean rest length of the unique edges
  {
    std::vector<uint64_t> ek;
    ek.reserve(6 * (size_t)T);
    for (int e = 0; e < T; ++e)
      for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b) {
          uint64_t i = (uint32_t)p->tets[a * (size_t)T + e], j = (uint32_t)p->tets[b * (size_t)T + e];
          if (i > j) std::swap(i, j);
          ek.push_back((i << 32) | j);
        }
    std::sort(ek.begin(), ek.end());
    ek.erase(std::unique(ek.begin(), ek.end()), ek.end());
    double sum = 0.0;
    for (uint64_t k : ek) {
      const int i = (int)(k >> 32), j = (int)(k & 0xffffffffu);
      const double dx = X(i, 0) - X(j, 0), dy = X(i, 1) - X(j, 1), dz = X(i, 2) - X(j, 2);
      sum += std::sqrt((dx * dx + dy * dy) + dz * dz);
    }
    p->h_ref = sum / (double)ek.size();
  }

  // orientation (swap slots 2 and 3 of negative tets), volumes, cell size
  std::vector<double> vol(T);
  double vsum = 0.0, cell = 0.0;
  for (int e = 0; e < T; ++e) {
    int32_t* t[4];
    for (int j = 0; j < 4; ++j) t[j] = &p->tets[j * (size_t)T + e];
    double P[4][3];
    for (int j = 0; j < 4; ++j)
      for (int k = 0; k < 3; ++k) P[j][k] = X(*t[j], k);
    const double v6 = orient_h(P[0], P[1], P[2], P[3]);
    if (std::fabs(v6) / 6.0 <= 1e-12 * p->h_ref * p->h_ref * p->h_ref)
      return fail(GS_EDEGENERATE, "degenerate rest tet " + std::to_string(e));
    if (v6 < 0) std::swap(*t[2], *t[3]);
    vol[e] = std::fabs(v6) / 6.0;
    vsum += vol[e];
    for (int k = 0; k < 3; ++k) {
      const double lo = std::min(std::min(P[0][k], P[1][k]), std::min(P[2][k], P[3][k]));
      const double hi = std::max(std::max(P[0][k], P[1][k]), std::max(P[2][k], P[3][k]));
      cell = std::max(cell, hi - lo);
    }
  }
  const double mean_vol = vsum / T;
  p->inv_mean_vol = 1.0 / mean_vol;
  p->cell = cell;

  // bounding box, offsets
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int v = 0; v < n; ++v)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], X(v, k));
      hi[k] = std::max(hi[k], X(v, k));
    }
  p->diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                      (hi[2] - lo[2]) * (hi[2] - lo[2]));
  p->eps = p->prm.eps_rel * p->h_ref;
  p->Lray = p->prm.ray_rel * p->h_ref;

  // incidence: vertex -> (tet, slot) in (tet, slot) order
  p->inc_start.assign(n + 1, 0);
  for (size_t i = 0; i < 4 * (size_t)T; ++i) p->inc_start[p->tets[i] + 1]++;
  for (int v = 0; v < n; ++v) p->inc_start[v + 1] += p->inc_start[v];
  {
    std::vector<int32_t> cur(p->inc_start.begin(), p->inc_start.end() - 1);
    p->inc_pos.resize(4 * (size_t)T);
    for (int e = 0; e < T; ++e)
      for (int j = 0; j < 4; ++j) p->inc_pos[j * (size_t)T + e] = cur[p->tets[j * (size_t)T + e]]++;
  }

  // A_el = sum_e omega_e S_e^T N S_e, N = I - 11^T/4; Dirichlet rows/cols removed
  std::vector<double> full_diag(n, 0.0);
  {
    std::vector<std::pair<uint64_t, double>> trip;
    trip.reserve(16 * (size_t)T);
    for (int e = 0; e < T; ++e) {
      const double om = vol[e] / mean_vol;
      for (int a = 0; a < 4; ++a) {
        const uint64_t i = (uint32_t)p->tets[a * (size_t)T + e];
        full_diag[i] += 0.75 * om;
        for (int b = 0; b < 4; ++b) {
          const uint64_t j = (uint32_t)p->tets[b * (size_t)T + e];
          trip.emplace_back((i << 32) | j, (a == b ? 0.75 : -0.25) * om);
        }
      }
    }
    std::sort(trip.begin(), trip.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    p->rowptr.assign(n + 1, 0);
    p->col.clear();
    p->val.clear();
    size_t i = 0;
    for (int r = 0; r < n; ++r) {
      if (!p->freem[r]) {
        p->col.push_back(r);
        p->val.push_back(1.0);
        while (i < trip.size() && (int)(trip[i].first >> 32) == r) ++i;
      } else {
        while (i < trip.size() && (int)(trip[i].first >> 32) == r) {
          const int cj = (int)(trip[i].first & 0xffffffffu);
          double s = 0.0;
          while (i < trip.size() && trip[i].first == (((uint64_t)r << 32) | (uint32_t)cj)) s += trip[i++].second;
          if (p->freem[cj]) {
            p->col.push_back(cj);
            p->val.push_back(s);
          }
        }
      }
      p->rowptr[r + 1] = (int32_t)p->col.size();
    }
    p->nnz = (int)p->col.size();
    p->adiag.resize(n);
    for (int v = 0; v < n; ++v) p->adiag[v] = p->freem[v] ? full_diag[v] : 1.0;
  }

  // boundary faces: faces of exactly one tet, outward, in (tet, slot) order
  {
    struct FK {
      int32_t a, b, c;
      int32_t idx;
    };
    std::vector<FK> fk(4 * (size_t)T);
    for (int e = 0; e < T; ++e)
      for (int m2 = 0; m2 < 4; ++m2) {
        int32_t v[3];
        for (int k = 0; k < 3; ++k) v[k] = p->tets[kFaceSlots[m2][k] * (size_t)T + e];
        std::sort(v, v + 3);
        fk[4 * (size_t)e + m2] = {v[0], v[1], v[2], (int32_t)(4 * e + m2)};
      }
    std::sort(fk.begin(), fk.end(), [](const FK& x, const FK& y) {
      if (x.a != y.a) return x.a < y.a;
      if (x.b != y.b) return x.b < y.b;
      if (x.c != y.c) return x.c < y.c;
      return x.idx < y.idx;
    });
    std::vector<uint8_t> on(4 * (size_t)T, 0);
    for (size_t i = 0; i < fk.size();) {
      size_t j = i + 1;
      while (j < fk.size() && fk[j].a == fk[i].a && fk[j].b == fk[i].b && fk[j].c == fk[i].c) ++j;
      if (j - i == 1) on[fk[i].idx] = 1;
      i = j;
    }
    std::vector<int32_t> f0, f1, f2;
    for (size_t i = 0; i < on.size(); ++i)
      if (on[i]) {
        const int e = (int)(i / 4), m2 = (int)(i % 4);
        f0.push_back(p->tets[kFaceSlots[m2][0] * (size_t)T + e]);
        f1.push_back(p->tets[kFaceSlots[m2][1] * (size_t)T + e]);
        f2.push_back(p->tets[kFaceSlots[m2][2] * (size_t)T + e]);
      }
    p->F = (int)f0.size();
    p->faces.clear();
    p->faces.insert(p->faces.end(), f0.begin(), f0.end());
    p->faces.insert(p->faces.end(), f1.begin(), f1.end());
    p->faces.insert(p->faces.end(), f2.begin(), f2.end());
  }

  // query vertices: non-fixed boundary vertices, ascending; incident faces ascending
  {
    const int F = p->F;
    std::vector<uint8_t> surf(n, 0);
    for (int32_t v : p->faces) surf[v] = 1;
    p->n_surf_verts = 0;
    p->qverts.clear();
    p->vq.assign(n, -1);
    for (int v = 0; v < n; ++v) {
      p->n_surf_verts += surf[v];
      if (surf[v] && p->freem[v]) {
        p->vq[v] = (int32_t)p->qverts.size();
        p->qverts.push_back(v);
      }
    }
    p->S = (int)p->qverts.size();
    p->qf_start.assign(p->S + 1, 0);
    for (int f = 0; f < F; ++f)
      for (int k = 0; k < 3; ++k) {
        const int s = p->vq[p->faces[k * (size_t)F + f]];
        if (s >= 0) p->qf_start[s + 1]++;
      }
    for (int s = 0; s < p->S; ++s) p->qf_start[s + 1] += p->qf_start[s];
    std::vector<int32_t> cur(p->qf_start.begin(), p->qf_start.end() - 1);
    p->qf_list.assign(p->qf_start[p->S], 0);
    for (int f = 0; f < F; ++f)
      for (int k = 0; k < 3; ++k) {
        const int s = p->vq[p->faces[k * (size_t)F + f]];
        if (s >= 0) p->qf_list[cur[s]++] = f;
      }
    p->kq.resize(p->S);
    // spring stiffness k_v = kappa_col * A_el[v, v]
    for (int s = 0; s < p->S; ++s) p->kq[s] = p->prm.kappa_col * full_diag[p->qverts[s]];
  }

  // a single mesh: one entry in the per-mesh tables
  p->M = 1;
  p->mh_ref = {p->h_ref};
  p->mdiag = {p->diag};
  p->mcell = {p->cell};
  p->minv_mean_vol = {p->inv_mean_vol};
  p->vbeg = {0, n};
  p->tbeg = {0, T};
  p->chbeg = {0, p->nch};
  p->fbeg = {0, p->F};
  p->sbeg = {0, p->S};
  p->vmesh.assign(n, 0);
  p->tmesh.assign(T, 0);
  return GS_OK;
}

// Sizes and structures derived from the (possibly merged) arrays: the ELL
// copy of the off-diagonal entries (slot-major, padded with the row itself
// and value 0; the diagonal lives in the Jacobi diagonal), hash table size,
// partial-sum slots.
void finalize(gs_problem* p) {
  const int n = p->n;
  int wmax = 0;
  for (int r = 0; r < n; ++r) {
    int cnt = 0;
    if (p->freem[r])
      for (int j = p->rowptr[r]; j < p->rowptr[r + 1]; ++j) cnt += (p->col[j] != r);
    wmax = std::max(wmax, cnt);
  }
  if (wmax > 64) throw std::runtime_error("a vertex has more than 64 neighbours");
  p->ell_w = wmax <= 16 ? 16 : (wmax <= 32 ? 32 : 64);
  p->ell_col.assign((size_t)p->ell_w * n, 0);
  p->ell_val.assign((size_t)p->ell_w * n, 0.0);
  for (int r = 0; r < n; ++r) {
    int k = 0;
    if (p->freem[r])
      for (int j = p->rowptr[r]; j < p->rowptr[r + 1]; ++j)
        if (p->col[j] != r) {
          p->ell_col[(size_t)k * n + r] = p->col[j];
          p->ell_val[(size_t)k * n + r] = p->val[j];
          ++k;
        }
    for (; k < p->ell_w; ++k) p->ell_col[(size_t)k * n + r] = r;
  }
  int H = 1024;
  while (H < 2 * p->S) H <<= 1;
  p->H = H;
  // the CG's partial sums: 12 per workgroup, one workgroup per mesh at most
  p->nparts = std::max({cdiv(p->T, kBlock), cdiv(n, kBlock), 12 * kMaxPcgGrid, 12 * p->M});
  p->slots = 1 + p->ns + p->np + (p->mo_k > 0 ? 1 : 0);
  // chamber -> tets, ascending tet id within a chamber
  p->ch_start.assign(p->nch + 1, 0);
  for (int e = 0; e < p->T; ++e)
    if ((p->tag[e] & 7) != GS_BODY) p->ch_start[(p->tag[e] >> 3) + 1]++;
  for (int c = 0; c < p->nch; ++c) p->ch_start[c + 1] += p->ch_start[c];
  p->ch_tets.assign(p->ch_start[p->nch], 0);
  std::vector<int32_t> cur(p->ch_start.begin(), p->ch_start.end() - 1);
  for (int e = 0; e < p->T; ++e)
    if ((p->tag[e] & 7) != GS_BODY) p->ch_tets[cur[p->tag[e] >> 3]++] = e;
  // blocks of the acceleration's dot products: kFaaRows rows each, never
  // straddling meshes (a mesh's sums are taken over its own blocks)
  p->faa_blk.clear();
  p->faa_mblk.assign(1, 0);
  for (int m = 0; m < p->M; ++m) {
    for (int v0 = p->vbeg[m]; v0 < p->vbeg[m + 1]; v0 += kFaaRows)
      p->faa_blk.push_back({m, v0, std::min(v0 + kFaaRows, p->vbeg[m + 1]), 0});
    p->faa_mblk.push_back((int32_t)p->faa_blk.size());
  }
  if ((int)p->faa_blk.size() > p->nparts) throw std::runtime_error("too many blocks for the partial-sum arrays");
}

// Concatenate single-mesh set-ups into one problem: vertex, tet, chamber,
// face and query-vertex ids are offset; the system matrix is block diagonal.
void merge(gs_problem* p, const std::vector<gs_problem*>& parts) {
  const int M = (int)parts.size();
  int n = 0, T = 0, nch = 0, F = 0, S = 0, inc = 0, qf = 0;
  for (auto* q : parts) {
    n += q->n;
    T += q->T;
    nch += q->nch;
    F += q->F;
    S += q->S;
    inc += q->inc_start[q->n];
    qf += (int)q->qf_list.size();
  }
  p->M = M;
  p->n = n;
  p->T = T;
  p->nch = nch;
  p->F = F;
  p->S = S;
  p->X0.assign(3 * (size_t)n, 0.0);
  p->tets.assign(4 * (size_t)T, 0);
  p->inc_pos.assign(4 * (size_t)T, 0);
  p->faces.assign(3 * (size_t)F, 0);
  p->tag.clear();
  p->freem.clear();
  p->adiag.clear();
  p->kq.clear();
  p->qverts.clear();
  p->vq.assign(n, -1);
  p->inc_start.assign(1, 0);
  p->rowptr.assign(1, 0);
  p->col.clear();
  p->val.clear();
  p->qf_start.assign(1, 0);
  p->qf_list.clear();
  p->vmesh.clear();
  p->tmesh.clear();
  p->mh_ref.clear();
  p->mdiag.clear();
  p->mcell.clear();
  p->minv_mean_vol.clear();
  p->vbeg.assign(1, 0);
  p->tbeg.assign(1, 0);
  p->chbeg.assign(1, 0);
  p->fbeg.assign(1, 0);
  p->sbeg.assign(1, 0);
  p->n_surf_verts = 0;
  p->nnz = 0;
  int vo = 0, to = 0, co = 0, fo = 0, so = 0, io = 0;
  for (int m = 0; m < M; ++m) {
    const gs_problem* q = parts[m];
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < q->n; ++i) p->X0[(size_t)k * n + vo + i] = q->X0[(size_t)k * q->n + i];
    for (int j = 0; j < 4; ++j)
      for (int e = 0; e < q->T; ++e) {
        p->tets[(size_t)j * T + to + e] = q->tets[(size_t)j * q->T + e] + vo;
        p->inc_pos[(size_t)j * T + to + e] = q->inc_pos[(size_t)j * q->T + e] + io;
      }
    for (int e = 0; e < q->T; ++e) {
      const int tg = q->tag[e], mode = tg & 7;
      p->tag.push_back(mode == GS_BODY ? tg : (mode | (((tg >> 3) + co) << 3)));
      p->tmesh.push_back(m);
    }
    for (int k = 0; k < 3; ++k)
      for (int f = 0; f < q->F; ++f) p->faces[(size_t)k * F + fo + f] = q->faces[(size_t)k * q->F + f] + vo;
    for (int i = 0; i < q->n; ++i) {
      p->freem.push_back(q->freem[i]);
      p->adiag.push_back(q->adiag[i]);
      p->vmesh.push_back(m);
      p->inc_start.push_back(q->inc_start[i + 1] + io);
      for (int j = q->rowptr[i]; j < q->rowptr[i + 1]; ++j) {
        p->col.push_back(q->col[j] + vo);
        p->val.push_back(q->val[j]);
      }
      p->rowptr.push_back((int32_t)p->col.size());
      if (q->vq[i] >= 0) p->vq[vo + i] = q->vq[i] + so;
    }
    const int qbase = (int)p->qf_list.size();
    for (int s2 = 0; s2 < q->S; ++s2) {
      p->qverts.push_back(q->qverts[s2] + vo);
      p->kq.push_back(q->kq[s2]);
      p->qf_start.push_back(q->qf_start[s2 + 1] + qbase);
    }
    for (int32_t f : q->qf_list) p->qf_list.push_back(f + fo);
    p->n_surf_verts += q->n_surf_verts;
    p->mh_ref.push_back(q->h_ref);
    p->mdiag.push_back(q->diag);
    p->mcell.push_back(q->cell);
    p->minv_mean_vol.push_back(q->inv_mean_vol);
    vo += q->n;
    to += q->T;
    co += q->nch;
    fo += q->F;
    so += q->S;
    io += q->inc_start[q->n];
    p->vbeg.push_back(vo);
    p->tbeg.push_back(to);
    p->chbeg.push_back(co);
    p->fbeg.push_back(fo);
    p->sbeg.push_back(so);
  }
  p->nnz = (int)p->col.size();
  p->h_ref = p->mh_ref[0];
  p->diag = p->mdiag[0];
  p->cell = p->mcell[0];
  p->inv_mean_vol = p->minv_mean_vol[0];
  p->eps = p->prm.eps_rel * p->h_ref;
  p->Lray = p->prm.ray_rel * p->h_ref;
  (void)inc;
  (void)qf;
}

}  // namespace

// ---------------------------------------------------------------------------
// Unrolled adjoint with checkpoints
//
// A record is the state before iteration k: displacement u_k, CG warm start
// and the previous correction it is extrapolated from, and the contact set A_{k-1} (flags, targets, normals, prims).  Checkpoints
// are kept every C = ceil(sqrt(K)) iterations; each segment is recomputed
// from its checkpoint into C + 1 segment records before its reverse steps.

namespace {

struct RecordLayout {
  size_t u, dl, dlp, dlpp, cact, ctgt, cnrm, cprim, bytes;
};

RecordLayout record_layout(const gs_problem* p) {
  RecordLayout r{};
  size_t off = 0;
  auto take = [&](size_t b) {
    off = align256(off);
    const size_t o = off;
    off += std::max<size_t>(b, 1);
    return o;
  };
  const size_t W = (size_t)p->prec, n = p->n, m = (size_t)p->S * p->slots;
  r.u = take(3 * n * W);
  r.dl = take(4 * n * W);
  r.dlp = take(4 * n * W);
  r.dlpp = take(4 * n * W);
  r.cact = take(m);
  r.ctgt = take(3 * m * 8);
  r.cnrm = take(3 * m * 8);
  r.cprim = take(m * 4);
  r.bytes = align256(off);
  return r;
}

int ckpt_stride(int K) {
  int c = 1;
  while ((long)c * c < K) ++c;
  return c;
}

size_t unrolled_records(int K) {
  const int C = ckpt_stride(K);
  return (size_t)cdiv(K, C) + (size_t)C + 2;  // checkpoints, segment records, final contact set
}

hipError_t copy_record(gs_problem* p, char* rec, bool save, bool state, bool contacts) {
  const RecordLayout R = record_layout(p);
  const size_t W = (size_t)p->prec, n = p->n, m = (size_t)p->S * p->slots;
  char* ws = p->ws;
  const Layout& L = p->lay;
  struct Item {
    size_t ws_off, rec_off, bytes;
    bool is_state;
  } items[] = {{L.u, R.u, 3 * n * W, true},       {L.dl, R.dl, 4 * n * W, true},
               {L.dlp, R.dlp, 4 * n * W, true},         {L.dlpp, R.dlpp, 4 * n * W, true},
               {L.cact, R.cact, m, false},        {L.ctgt, R.ctgt, 3 * m * 8, false},
               {L.cnrm, R.cnrm, 3 * m * 8, false}, {L.cprim, R.cprim, m * 4, false}};
  for (const Item& it : items) {
    if ((it.is_state && !state) || (!it.is_state && !contacts)) continue;
    char* a = ws + it.ws_off;
    char* b = rec + it.rec_off;
    hipError_t e = save ? hipMemcpyAsync(b, a, it.bytes, hipMemcpyDeviceToDevice, p->stream)
                        : hipMemcpyAsync(a, b, it.bytes, hipMemcpyDeviceToDevice, p->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename R>
gs_status unrolled_impl(gs_problem* p, const R* alpha, const R* x0, int K, const R* gL, R* dalpha, R* dx0, R* xK,
                        char* scratch, gs_stats* stats) {
  hipStream_t s = p->stream;
  const RecordLayout RL = record_layout(p);
  const int C = ckpt_stride(K);
  const int nck = cdiv(K, C);
  char* ck = scratch;                                  // nck checkpoint records
  char* seg = scratch + (size_t)nck * RL.bytes;        // C + 1 segment records
  char* fin = seg + (size_t)(C + 1) * RL.bytes;        // final contact set
  const Dev<R> d = make_dev<R>(p);
  Consts cf = make_consts(p);                          // forward iterations: never stop early
  cf.fixed_iters = 1 << 30;
  cf.mask_done = 0;
  cf.faa_m = 0;                                        // the plain map is what the sweep differentiates
  if (p->nch > 0)
    HIPCHK(hipMemcpyAsync(d.alpha_last, alpha, (size_t)p->nch * sizeof(R), hipMemcpyDeviceToDevice, s));
  // forward sweep with checkpoints
  HIPCHK(launch_init<R>(d, cf, x0, s));
  p->hash_ready = false;
  for (int k = 0; k < K; ++k) {
    if (k % C == 0) HIPCHK(copy_record(p, ck + (size_t)(k / C) * RL.bytes, true, true, true));
    HIPCHK(enqueue_iteration<R>(p, d, cf, alpha));
  }
  DevStatus h{};
  HIPCHK(hipMemcpyAsync(&h, d.st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h.done == STALLED) return fail(GS_EHIP, kStalledMsg);
  if (h.done == BREAKDOWN) return fail(GS_EBREAKDOWN, "non-finite value or CG curvature p'Ap <= 0");
  if (xK) HIPCHK(launch_output<R>(d, cf, xK, s));
  HIPCHK(copy_record(p, fin, true, false, true));
  const int fwd_iters = h.iters, fwd_pcg = h.pcg_total;
  // reverse sweep
  DevStatus* run = (DevStatus*)(p->ws + p->lay.st4);
  Dev<R> dv = d;                                       // VJP kernels: never "done", no frozen meshes
  dv.st = run;
  dv.mdone = (int32_t*)(p->ws + p->lay.mdone2);
  Dev<R> dc = d;                                       // reverse CG solves: their own status block
  dc.st = (DevStatus*)(p->ws + p->lay.st3);
  dc.mdone = (int32_t*)(p->ws + p->lay.mdone2);
  Consts cv = make_consts(p);
  cv.mask_done = 0;
  cv.adj_jt = 1;
  cv.aa_m = 0;
  cv.faa_m = 0;
  Consts cc = make_consts(p);
  cc.faa_m = 0;
  cc.pcg_eta_min = 0.0;  // each reverse solve is one CG to pcg_eta
  cc.mask_done = 0;
  cc.fixed_iters = 0;
  cc.max_iter = 1;
  cc.tol = 0.0;
  cc.aa_m = 0;
  cc.trace_len = 0;
  HIPCHK(hipMemsetAsync(d.ga_acc, 0, (size_t)std::max(p->nch, 1) * 8, s));
  HIPCHK(hipMemcpyAsync(d.lam, gL, 3 * (size_t)p->n * sizeof(R), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemsetAsync(d.acc3, 0, 3 * (size_t)p->n * 8, s));
  int rev_pcg = 0;
  for (int sg = nck - 1; sg >= 0; --sg) {
    const int k0 = sg * C, k1 = std::min(k0 + C, K);
    // recompute the segment from its checkpoint
    HIPCHK(copy_record(p, ck + (size_t)sg * RL.bytes, false, true, true));
    HIPCHK(launch_unr_restore<R>(d, cf, run, s));
    p->hash_ready = false;
    for (int k = k0; k < k1; ++k) {
      HIPCHK(copy_record(p, seg + (size_t)(k - k0) * RL.bytes, true, true, true));
      HIPCHK(enqueue_iteration<R>(p, d, cf, alpha));
    }
    HIPCHK(copy_record(p, seg + (size_t)(k1 - k0) * RL.bytes, true, true, true));
    for (int k = k1 - 1; k >= k0; --k) {
      // x_k from record k, A_k from record k + 1
      HIPCHK(copy_record(p, seg + (size_t)(k - k0) * RL.bytes, false, true, false));
      HIPCHK(copy_record(p, seg + (size_t)(k + 1 - k0) * RL.bytes, false, false, true));
      HIPCHK(launch_unr_restore<R>(d, cf, run, s));
      p->hash_ready = false;
      HIPCHK(launch_unr_rhs<R>(dc, cc, s));
      HIPCHK(timed_pcg<R>(p, K_ADJ_PCG, dc, cc, true));
      HIPCHK(timed(p, K_ADJ_SPRINGS, [&] { return launch_adj_springs<R>(dv, cv, s); }));
      HIPCHK(timed(p, K_ADJ_LOCAL, [&] { return launch_adj_local_mode<R>(dv, cv, ADJ_JT, s); }));
      HIPCHK(timed(p, K_ADJ_GATHER, [&] { return launch_adj_gather<R>(dv, cv, s); }));
      HIPCHK(launch_adj_local_mode<R>(dv, cv, ADJ_ALPHA, s));
      HIPCHK(launch_unr_accumulate<R>(dv, cv, s));
    }
    DevStatus hc{};
    HIPCHK(hipMemcpyAsync(&hc, dc.st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (p->prof.on) HIPCHK(p->prof.flush());
    if (hc.done == STALLED) return fail(GS_EHIP, kStalledMsg);
    if (hc.done == BREAKDOWN) return fail(GS_EBREAKDOWN, "breakdown in a reverse CG solve");
    rev_pcg += hc.pcg_total;
  }
  HIPCHK(launch_unr_finish<R>(d, cf, dalpha, dx0, s));
  // leave the contact set the forward sweep ended with
  HIPCHK(copy_record(p, fin, false, false, true));
  HIPCHK(hipStreamSynchronize(s));
  p->solved = false;
  if (stats) {
    stats->iters = fwd_iters;
    stats->pcg_iters_total = fwd_pcg + rev_pcg;
    stats->n_contacts = h.n_contacts_last;
    stats->ray_miss = h.ray_miss_last;
    stats->residual = h.residual;
    stats->energy = h.energy;
    stats->aa_rejected = 0;
    stats->pad = 0;
  }
  return GS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int32_t gs_version(void) { return GEOSIM_VERSION; }

const char* gs_last_error(void) { return g_err.c_str(); }

void gs_default_params(gs_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->c1 = 0.0418;
  p->c2 = 0.0106;
  p->hyperelastic = 1;
  p->kappa_col = 1.0;
  p->eps_rel = 0.05;
  p->ray_rel = 4.0;
  p->self_collision = 0;
  p->obstacle_collision = 0;
  p->tol = 1e-6;
  p->max_iter = 20000;
  p->fixed_iters = 0;
  p->pcg_eta = 1e-3;
  p->pcg_max = 200;
  p->check_every = 16;
  p->pcg_blocks = 0;
  p->trace_len = 0;
  p->adj_tol = 1e-6;
  p->adj_max_iter = 20000;
  p->adj_aa_m = 16;
  p->aa_m = 8;
  p->aa_guard = GS_AA_GUARD_RESIDUAL | GS_AA_GUARD_SET;
  p->aa_slack = 0.5;
  p->barrier_timeout_ms = 2000.0;
  p->pcg_eta_min = 0.0;
  p->pcg_coarse = 0;
  p->pcg_per_mesh = 0;
  p->graph = 0;
  p->pcg_store = 0;
}

gs_status gs_create(const gs_mesh_desc* m, const gs_params* prm, gs_problem** out) {
  if (!out) return fail(GS_EINVAL, "null output handle");
  *out = nullptr;
  if (!m || !m->rest_xyz || !m->tets || !m->tet_mode || !m->tet_chamber || !m->fixed)
    return fail(GS_EINVAL, "null mesh array");
  if (m->n_verts <= 0 || m->n_tets <= 0 || m->n_chambers < 0) return fail(GS_EINVAL, "empty mesh");
  if (m->precision != 4 && m->precision != 8) return fail(GS_EINVAL, "precision must be 4 or 8");
  if ((long)m->n_tets * 4 >= (1L << 31)) return fail(GS_EINVAL, "mesh too large");
  gs_status st = check_params(prm);
  if (st != GS_OK) return st;
  gs_problem* p = new (std::nothrow) gs_problem();
  if (!p) return fail(GS_EINVAL, "out of host memory");
  p->prm = *prm;
  p->trace_len = prm->trace_len;
  p->aa_cap = std::max(prm->adj_aa_m, prm->aa_m);
  try {
    st = setup(p, m);
    if (st == GS_OK) finalize(p);
  } catch (const std::exception& ex) {
    st = fail(GS_EINVAL, std::string("set-up failed: ") + ex.what());
  }
  if (st != GS_OK) {
    delete p;
    return st;
  }
  *out = p;
  return GS_OK;
}

gs_status gs_create_batch(int32_t n_mesh, const gs_mesh_desc* meshes, const gs_params* prm, gs_problem** out) {
  if (!out) return fail(GS_EINVAL, "null output handle");
  *out = nullptr;
  if (n_mesh < 1 || !meshes) return fail(GS_EINVAL, "need at least one mesh");
  gs_status st = check_params(prm);
  if (st != GS_OK) return st;
  if ((st = check_batch_params(prm, n_mesh)) != GS_OK) return st;
  long nt = 0, nv = 0;
  for (int m = 0; m < n_mesh; ++m) {
    const gs_mesh_desc* d = &meshes[m];
    if (!d->rest_xyz || !d->tets || !d->tet_mode || !d->tet_chamber || !d->fixed)
      return fail(GS_EINVAL, "null mesh array in mesh " + std::to_string(m));
    if (d->n_verts <= 0 || d->n_tets <= 0 || d->n_chambers < 0)
      return fail(GS_EINVAL, "empty mesh " + std::to_string(m));
    if (d->precision != meshes[0].precision || (d->precision != 4 && d->precision != 8))
      return fail(GS_EINVAL, "meshes of a batch share one precision (4 or 8)");
    nt += d->n_tets;
    nv += d->n_verts;
  }
  if (nt * 4 >= (1L << 31) || nv * 64 >= (1L << 31)) return fail(GS_EINVAL, "batch too large");
  std::vector<gs_problem*> parts;
  gs_problem* p = nullptr;
  try {
    for (int m = 0; m < n_mesh && st == GS_OK; ++m) {
      gs_problem* q = new gs_problem();
      q->prm = *prm;
      parts.push_back(q);
      st = setup(q, &meshes[m]);
      if (st != GS_OK) g_err = "mesh " + std::to_string(m) + ": " + g_err;
    }
    if (st == GS_OK) {
      p = new gs_problem();
      p->prm = *prm;
      p->prec = meshes[0].precision;
      p->trace_len = prm->trace_len;
      p->aa_cap = std::max(prm->adj_aa_m, prm->aa_m);
      merge(p, parts);
      finalize(p);
    }
  } catch (const std::exception& ex) {
    st = fail(GS_EINVAL, std::string("set-up failed: ") + ex.what());
  }
  for (auto* q : parts) delete q;
  if (st != GS_OK) {
    delete p;
    return st;
  }
  *out = p;
  return GS_OK;
}

gs_status gs_batch_layout(const gs_problem* p, int32_t cap, int32_t* vert_offset, int32_t* tet_offset,
                          int32_t* chamber_offset, int32_t* n_mesh) {
  if (!p || !n_mesh) return fail(GS_EINVAL, "null argument");
  *n_mesh = p->M;
  if (cap < p->M + 1) return fail(GS_ECAPACITY, "offset arrays need n_mesh + 1 entries");
  for (int m = 0; m <= p->M; ++m) {
    if (vert_offset) vert_offset[m] = p->vbeg[m];
    if (tet_offset) tet_offset[m] = p->tbeg[m];
    if (chamber_offset) chamber_offset[m] = p->chbeg[m];
  }
  return GS_OK;
}

gs_status gs_mesh_iters(gs_problem* p, int32_t cap, int32_t* iters) {
  if (!p || !iters) return fail(GS_EINVAL, "null argument");
  if (!p->bound) return fail(GS_ESTATE, "not bound");
  if (cap < p->M) return fail(GS_ECAPACITY, "iteration array needs n_mesh entries");
  HIPCHK(hipMemcpyAsync(iters, p->ws + p->lay.mdone, (size_t)p->M * 4, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return GS_OK;
}

gs_status gs_set_obstacles(gs_problem* p, int32_t n_sph, const double* sph, int32_t n_pln, const double* pln) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (p->bound) return fail(GS_ESTATE, "obstacles must be set before gs_bind");
  if (n_sph < 0 || n_pln < 0 || n_sph > 8 || n_pln > 8) return fail(GS_EINVAL, "at most 8 spheres and 8 planes");
  if ((n_sph && !sph) || (n_pln && !pln)) return fail(GS_EINVAL, "null obstacle array");
  std::vector<double> ob;
  for (int j = 0; j < n_sph; ++j) {
    for (int k = 0; k < 4; ++k)
      if (!std::isfinite(sph[4 * j + k])) return fail(GS_EINVAL, "non-finite sphere");
    if (!(sph[4 * j + 3] > 0)) return fail(GS_EINVAL, "sphere radius must be positive");
    ob.insert(ob.end(), sph + 4 * j, sph + 4 * j + 4);
  }
  for (int j = 0; j < n_pln; ++j) {
    const double* q = pln + 6 * j;
    for (int k = 0; k < 6; ++k)
      if (!std::isfinite(q[k])) return fail(GS_EINVAL, "non-finite plane");
    const double nr = std::sqrt((q[3] * q[3] + q[4] * q[4]) + q[5] * q[5]);
    if (!(nr > 0)) return fail(GS_EINVAL, "plane with zero normal");
    ob.insert(ob.end(), {q[0], q[1], q[2], q[3] / nr, q[4] / nr, q[5] / nr});
  }
  p->ns = n_sph;
  p->np = n_pln;
  p->obst = ob;
  p->slots = 1 + n_sph + n_pln + (p->mo_k > 0 ? 1 : 0);
  return GS_OK;
}

namespace {

// Bounding-volume hierarchy over the obstacle's triangles: median split of
// the centroids along the widest axis, at most 4 triangles per leaf, nodes in
// depth-first order (root first), boxes exact.
int build_mo_tree(const std::vector<double>& tri9, std::vector<int32_t>& order, int lo, int hi,
                  std::vector<MoNode>& nodes, int depth, int& max_depth) {
  max_depth = std::max(max_depth, depth);
  const int id = (int)nodes.size();
  nodes.push_back(MoNode{});
  MoNode nd{};
  for (int k = 0; k < 3; ++k) {
    nd.lo[k] = INFINITY;
    nd.hi[k] = -INFINITY;
  }
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = lo; i < hi; ++i) {
    const double* t = &tri9[9 * (size_t)order[i]];
    for (int k = 0; k < 3; ++k) {
      for (int v = 0; v < 3; ++v) {
        nd.lo[k] = std::min(nd.lo[k], t[3 * v + k]);
        nd.hi[k] = std::max(nd.hi[k], t[3 * v + k]);
      }
      const double cen = (t[k] + t[3 + k] + t[6 + k]) / 3.0;
      clo[k] = std::min(clo[k], cen);
      chi[k] = std::max(chi[k], cen);
    }
  }
  if (hi - lo <= 4) {
    nd.left = nd.right = -1;
    nd.first = lo;
    nd.count = hi - lo;
    nodes[id] = nd;
    return id;
  }
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
  const int mid = (lo + hi) / 2;
  auto cen = [&](int32_t t) { return tri9[9 * (size_t)t + ax] + tri9[9 * (size_t)t + 3 + ax] + tri9[9 * (size_t)t + 6 + ax]; };
  std::nth_element(order.begin() + lo, order.begin() + mid, order.begin() + hi,
                   [&](int32_t a, int32_t b) { return cen(a) < cen(b) || (cen(a) == cen(b) && a < b); });
  nd.left = build_mo_tree(tri9, order, lo, mid, nodes, depth + 1, max_depth);
  nd.right = build_mo_tree(tri9, order, mid, hi, nodes, depth + 1, max_depth);
  nd.first = 0;
  nd.count = 0;
  nodes[id] = nd;
  return id;
}

inline double dot3h(const double* a, const double* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

}  // namespace

gs_status gs_set_mesh_obstacle(gs_problem* p, int32_t n_verts, const double* verts, int32_t n_tris,
                               const int32_t* tris) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (p->bound) return fail(GS_ESTATE, "the mesh obstacle must be set before gs_bind");
  if (n_tris == 0) {
    p->mo_tri.clear();
    p->mo_id.clear();
    p->mo_node.clear();
    p->mo_k = 0;
    p->slots = 1 + p->ns + p->np;
    return GS_OK;
  }
  if (n_verts < 3 || n_tris < 4 || !verts || !tris) return fail(GS_EINVAL, "mesh obstacle: too small or null");
  const size_t m = (size_t)n_verts, k = (size_t)n_tris;
  for (size_t i = 0; i < 3 * m; ++i)
    if (!std::isfinite(verts[i])) return fail(GS_EINVAL, "mesh obstacle: non-finite vertex");
  for (size_t i = 0; i < 3 * k; ++i)
    if (tris[i] < 0 || tris[i] >= n_verts) return fail(GS_EINVAL, "mesh obstacle: vertex index out of range");
  // triangles as [k][3] corners and unit face normals (same operation order
  // as written: n = (b - a) x (c - a), |n| = sqrt((nx^2 + ny^2) + nz^2))
  std::vector<double> tri9(9 * k), fn(3 * k);
  for (size_t t = 0; t < k; ++t) {
    for (int v = 0; v < 3; ++v)
      for (int c = 0; c < 3; ++c) tri9[9 * t + 3 * v + c] = verts[(size_t)c * m + tris[(size_t)v * k + t]];
    const double* a = &tri9[9 * t];
    const double u[3] = {a[3] - a[0], a[4] - a[1], a[5] - a[2]}, w[3] = {a[6] - a[0], a[7] - a[1], a[8] - a[2]};
    const double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    const double ln = std::sqrt(dot3h(n, n));
    if (!(ln > 0)) return fail(GS_EINVAL, "mesh obstacle: degenerate triangle");
    for (int c = 0; c < 3; ++c) fn[3 * t + c] = n[c] / ln;
  }
  // edges (ab, ac, bc of every triangle): each must be shared by exactly two
  // triangles; edge pseudonormal = the sum of their unit normals (ascending
  // triangle order), normalised
  std::map<std::pair<int, int>, int> eid;
  std::vector<int> tedge(3 * k), ecount;
  std::vector<double> en;
  const int lp[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (size_t t = 0; t < k; ++t)
    for (int j = 0; j < 3; ++j) {
      int a = tris[lp[j][0] * k + t], b = tris[lp[j][1] * k + t];
      if (a > b) std::swap(a, b);
      auto it = eid.find({a, b});
      int e;
      if (it == eid.end()) {
        e = (int)ecount.size();
        eid[{a, b}] = e;
        ecount.push_back(0);
        en.insert(en.end(), {0.0, 0.0, 0.0});
      } else {
        e = it->second;
      }
      tedge[3 * t + j] = e;
      ++ecount[e];
    }
  for (int cnt : ecount)
    if (cnt != 2) return fail(GS_EINVAL, "mesh obstacle: not closed (an edge is not shared by two triangles)");
  for (size_t t = 0; t < k; ++t)
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < 3; ++c) en[3 * tedge[3 * t + j] + c] += fn[3 * t + c];
  for (size_t e = 0; e < ecount.size(); ++e) {
    const double l = std::sqrt(dot3h(&en[3 * e], &en[3 * e]));
    for (int c = 0; c < 3; ++c) en[3 * e + c] /= l;
  }
  // vertex pseudonormals: incident unit normals weighted by the angle at the
  // vertex, summed corner slot by corner slot in ascending triangle order
  std::vector<double> vn(3 * m, 0.0);
  for (int i = 0; i < 3; ++i)
    for (size_t t = 0; t < k; ++t) {
      const double* P = &tri9[9 * t];
      const double* o = P + 3 * i;
      const double* q1 = P + 3 * ((i + 1) % 3);
      const double* q2 = P + 3 * ((i + 2) % 3);
      const double u[3] = {q1[0] - o[0], q1[1] - o[1], q1[2] - o[2]}, w[3] = {q2[0] - o[0], q2[1] - o[1], q2[2] - o[2]};
      const double cs = dot3h(u, w) / std::sqrt(dot3h(u, u) * dot3h(w, w));
      const double ang = std::acos(std::min(1.0, std::max(-1.0, cs)));
      const int vv = tris[(size_t)i * k + t];
      for (int c = 0; c < 3; ++c) vn[3 * (size_t)vv + c] += fn[3 * t + c] * ang;
    }
  std::vector<MoNode> nodes;
  std::vector<int32_t> order(k);
  for (size_t t = 0; t < k; ++t) order[t] = (int32_t)t;
  int depth = 0;
  build_mo_tree(tri9, order, 0, (int)k, nodes, 0, depth);
  if (depth > 60) return fail(GS_EINVAL, "mesh obstacle: tree too deep");
  std::vector<double> rec(30 * k);
  for (size_t i = 0; i < k; ++i) {
    const size_t t = (size_t)order[i];
    double* r = &rec[30 * i];
    for (int j = 0; j < 9; ++j) r[j] = tri9[9 * t + j];
    for (int c = 0; c < 3; ++c) r[9 + c] = fn[3 * t + c];
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < 3; ++c) r[12 + 3 * j + c] = en[3 * (size_t)tedge[3 * t + j] + c];
    for (int j = 0; j < 3; ++j) {
      const double* q = &vn[3 * (size_t)tris[(size_t)j * k + t]];
      const double l = std::sqrt(dot3h(q, q));
      for (int c = 0; c < 3; ++c) r[21 + 3 * j + c] = q[c] / l;
    }
  }
  p->mo_tri = std::move(rec);
  p->mo_id = std::move(order);
  p->mo_node = std::move(nodes);
  p->mo_k = n_tris;
  p->slots = 1 + p->ns + p->np + 1;
  return GS_OK;
}

namespace {

// Median-split tree over the tets' rest centroids (4 tets per leaf), then
// relabelled breadth first so that each depth is one contiguous node range.
void build_tet_tree(gs_problem* p) {
  const int T = p->T;
  const size_t n = (size_t)p->n;
  std::vector<double> cen(3 * (size_t)T);
  for (int e = 0; e < T; ++e)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int q = 0; q < 4; ++q) acc += p->X0[k * n + p->tets[(size_t)q * T + e]];
      cen[3 * (size_t)e + k] = acc;
    }
  struct Tmp {
    int left, right, first, count;
  };
  std::vector<Tmp> tmp;
  std::vector<int32_t> order(T);
  std::iota(order.begin(), order.end(), 0);
  std::function<int(int, int)> rec = [&](int lo, int hi) -> int {
    const int id = (int)tmp.size();
    tmp.push_back(Tmp{-1, -1, lo, hi - lo});
    if (hi - lo <= 4) return id;
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = lo; i < hi; ++i)
      for (int k = 0; k < 3; ++k) {
        clo[k] = std::min(clo[k], cen[3 * (size_t)order[i] + k]);
        chi[k] = std::max(chi[k], cen[3 * (size_t)order[i] + k]);
      }
    int ax = 0;
    for (int k = 1; k < 3; ++k)
      if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
    const int mid = (lo + hi) / 2;
    std::nth_element(order.begin() + lo, order.begin() + mid, order.begin() + hi, [&](int32_t a, int32_t b) {
      const double ca = cen[3 * (size_t)a + ax], cb = cen[3 * (size_t)b + ax];
      return ca < cb || (ca == cb && a < b);
    });
    const int l = rec(lo, mid), r = rec(mid, hi);
    tmp[id] = Tmp{l, r, 0, 0};
    return id;
  };
  rec(0, T);
  // breadth-first relabelling
  std::vector<int> bfs{0}, depth{0}, newid(tmp.size(), -1);
  for (size_t h = 0; h < bfs.size(); ++h) {
    const Tmp& t = tmp[bfs[h]];
    if (t.count == 0) {
      bfs.push_back(t.left);
      depth.push_back(depth[h] + 1);
      bfs.push_back(t.right);
      depth.push_back(depth[h] + 1);
    }
  }
  for (size_t h = 0; h < bfs.size(); ++h) newid[bfs[h]] = (int)h;
  p->tree_node.assign(bfs.size(), MoNode{});
  p->tree_level.assign((size_t)depth.back() + 2, 0);
  for (size_t h = 0; h < bfs.size(); ++h) {
    const Tmp& t = tmp[bfs[h]];
    MoNode& nd = p->tree_node[h];
    nd.left = t.count ? -1 : newid[t.left];
    nd.right = t.count ? -1 : newid[t.right];
    nd.first = t.first;
    nd.count = t.count;
    p->tree_level[(size_t)depth[h] + 1] = (int)h + 1;
  }
  p->tree_order = std::move(order);
}

struct TreeScratch {
  size_t node, order, tbox, pairs, count, total;
};

TreeScratch tree_scratch(int64_t nodes, int64_t T, int64_t cap) {
  TreeScratch t{};
  size_t off = 0;
  auto take = [&](size_t b) {
    off = align256(off);
    const size_t o = off;
    off += std::max<size_t>(b, 1);
    return o;
  };
  t.node = take((size_t)nodes * sizeof(MoNode));
  t.order = take((size_t)T * 4);
  t.tbox = take((size_t)T * 48);
  t.pairs = take(2 * (size_t)cap * 4);
  t.count = take(4);
  t.total = align256(off);
  return t;
}

}  // namespace

size_t gs_tree_candidates_scratch(const gs_problem* p, int32_t cap) {
  if (!p || cap < 0) return 0;
  // a median-split tree with at most 4 tets per leaf has fewer than 2T nodes
  return tree_scratch(2 * (int64_t)p->T, p->T, cap).total;
}

gs_status gs_tree_candidates(gs_problem* p, const void* x, int32_t cap, void* scratch, size_t scratch_bytes,
                             int32_t* cand, int32_t* n_cand, double* ms_refit, double* ms_query) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!p->bound) return fail(GS_ESTATE, "not bound");
  if (!x || !scratch || cap < 0 || !n_cand) return fail(GS_EINVAL, "null argument");
  if (p->M != 1) return fail(GS_EINVAL, "the tet tree serves a problem of one mesh");
  if (scratch_bytes < gs_tree_candidates_scratch(p, cap)) return fail(GS_EINVAL, "tree scratch too small");
  if (p->tree_node.empty()) build_tet_tree(p);
  if ((int)p->tree_level.size() - 1 > 60) return fail(GS_EINVAL, "tet tree too deep");
  const TreeScratch ts = tree_scratch((int64_t)p->tree_node.size(), p->T, cap);
  char* b = (char*)scratch;
  hipStream_t s = p->stream;
  HIPCHK(hipMemcpyAsync(b + ts.node, p->tree_node.data(), p->tree_node.size() * sizeof(MoNode),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(b + ts.order, p->tree_order.data(), p->tree_order.size() * 4, hipMemcpyHostToDevice, s));
  const Consts c = make_consts(p);
  hipEvent_t e0, e1, e2;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventCreate(&e2));
  auto run = [&](auto tag) -> hipError_t {
    using R = decltype(tag);
    Dev<R> d = make_dev<R>(p);
    hipError_t e = launch_set_positions<R>(d, c, (const R*)x, s);
    if (e != hipSuccess) return e;
    p->hash_ready = false;
    if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
    if ((e = launch_tree_refit<R>(d, c, (MoNode*)(b + ts.node), (const int32_t*)(b + ts.order),
                                  (double*)(b + ts.tbox), p->tree_level.data(), (int)p->tree_level.size() - 1,
                                  s)) != hipSuccess)
      return e;
    if ((e = hipEventRecord(e1, s)) != hipSuccess) return e;
    if ((e = launch_tree_query<R>(d, c, (const MoNode*)(b + ts.node), (const int32_t*)(b + ts.order),
                                  (const double*)(b + ts.tbox), (int32_t*)(b + ts.pairs), cap,
                                  (int*)(b + ts.count), s)) != hipSuccess)
      return e;
    return hipEventRecord(e2, s);
  };
  hipError_t e = p->prec == 4 ? run(float{}) : run(double{});
  int32_t cnt = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&cnt, b + ts.count, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  float t1 = 0.f, t2 = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t1, e0, e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&t2, e1, e2);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipEventDestroy(e2);
  HIPCHK(e);
  if (ms_refit) *ms_refit = t1;
  if (ms_query) *ms_query = t2;
  *n_cand = cnt;
  if (cnt > cap) return fail(GS_ECAPACITY, "candidate capacity too small");
  std::vector<int32_t> buf(2 * (size_t)cap);
  if (cap > 0) HIPCHK(hipMemcpy(buf.data(), b + ts.pairs, 2 * (size_t)cap * 4, hipMemcpyDeviceToHost));
  std::vector<std::pair<int32_t, int32_t>> pr(cnt);
  for (int i = 0; i < cnt; ++i) pr[i] = {buf[i], buf[cap + i]};
  std::sort(pr.begin(), pr.end());
  if (cand)
    for (int i = 0; i < cnt; ++i) {
      cand[i] = pr[i].first;
      cand[cap + i] = pr[i].second;
    }
  return GS_OK;
}

gs_status gs_info_get(const gs_problem* p, gs_info* info) {
  if (!p || !info) return fail(GS_EINVAL, "null argument");
  info->n_verts = p->n;
  info->n_tets = p->T;
  info->n_surface_faces = p->F;
  info->n_surface_verts = p->n_surf_verts;
  info->n_query_verts = p->S;
  info->nnz = p->nnz;
  info->n_slots = p->slots;
  info->hash_buckets = p->H;
  info->h_ref = p->h_ref;
  info->eps_off = p->eps;
  info->ray_len = p->Lray;
  info->bbox_diag = p->diag;
  info->cell_size = p->cell;
  info->ell_width = p->ell_w;
  info->pcg_grid = p->bound ? p->pcg_grid : 0;
  return GS_OK;
}

gs_status gs_workspace_size(const gs_problem* p, size_t* bytes) {
  if (!p || !bytes) return fail(GS_EINVAL, "null argument");
  *bytes = make_layout(p).total;
  return GS_OK;
}

gs_status gs_bind(gs_problem* p, void* ws, size_t bytes, void* stream) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!ws) return fail(GS_EINVAL, "null workspace");
  if (((uintptr_t)ws & 255) != 0) return fail(GS_EINVAL, "workspace must be 256-byte aligned");
  const Layout L = make_layout(p);
  if (bytes < L.total) return fail(GS_EINVAL, "workspace too small");
  p->lay = L;
  p->ws = (char*)ws;
  p->ws_bytes = bytes;
  p->stream = (hipStream_t)stream;
  p->bound = false;
  p->solved = false;
  p->coarse_G = 0;  // the coarse operator lives in the workspace
  if (!p->hstat) {
    void* h = nullptr;
    if (hipHostMalloc(&h, 2 * sizeof(DevStatus), hipHostMallocDefault) != hipSuccess)
      return fail(GS_EHIP, "hipHostMalloc of the status copies failed");
    p->hstat = (DevStatus*)h;
    for (hipEvent_t& e : p->hev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return fail(GS_EHIP, "hipEventCreate failed");
  }
  const gs_status st = p->prec == 4 ? bind_impl<float>(p) : bind_impl<double>(p);
  if (st == GS_OK) p->bound = true;
  return st;
}

gs_status gs_set_params(gs_problem* p, const gs_params* prm) {
  if (!p) return fail(GS_EINVAL, "null problem");
  gs_status st = check_params(prm);
  if (st != GS_OK) return st;
  if ((st = check_batch_params(prm, p->M)) != GS_OK) return st;
  if (prm->kappa_col != p->prm.kappa_col) {
    for (int s = 0; s < p->S; ++s) p->kq[s] *= prm->kappa_col / p->prm.kappa_col;
    if (p->bound) HIPCHK(hipMemcpyAsync(p->ws + p->lay.kq, p->kq.data(), p->kq.size() * 8, hipMemcpyHostToDevice,
                                        p->stream));
  }
  const double h = p->h_ref;
  p->prm = *prm;
  p->eps = prm->eps_rel * h;
  p->Lray = prm->ray_rel * h;
  if (p->bound) {
    const std::vector<MeshConst> mt = mesh_table(p);
    HIPCHK(upload(p->ws, p->lay.mesh, mt, p->stream));
  }
  if (p->bound) {
    const int maxg = p->prec == 4 ? pcg_max_grid<float>(p->ell_w) : pcg_max_grid<double>(p->ell_w);
    if (maxg < 1) return fail(GS_EHIP, "cannot size the cooperative CG grid");
    p->pcg_maxg = maxg;
    p->pcg_grid = pcg_grid_for(p, maxg);
    const gs_status r = plan_segments(p, maxg);
    if (r != GS_OK) return r;
    HIPCHK(hipStreamSynchronize(p->stream));
  }
  return GS_OK;
}

gs_status gs_solve(gs_problem* p, const void* alpha, void* x, gs_stats* stats) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!p->bound) return fail(GS_ESTATE, "gs_solve before gs_bind");
  if (!x || (p->nch > 0 && !alpha)) return fail(GS_EINVAL, "null device buffer");
  if (p->prec == 4) return solve_impl<float>(p, (const float*)alpha, (float*)x, stats);
  return solve_impl<double>(p, (const double*)alpha, (double*)x, stats);
}

gs_status gs_cg_plan(const gs_problem* p, int32_t M, int32_t* blocks) {
  if (!p || !blocks) return fail(GS_EINVAL, "null argument");
  if (!p->bound) return fail(GS_ESTATE, "gs_cg_plan before gs_bind");
  if (M != p->M) return fail(GS_EINVAL, "M is not the problem's mesh count");
  for (int m = 0; m < M; ++m) blocks[m] = p->seg_k[m];
  return GS_OK;
}

gs_status gs_autotune(gs_problem* p, const void* alpha, void* x, int32_t iters, int32_t* chosen, double* ms_per_iter) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!p->bound) return fail(GS_ESTATE, "gs_autotune before gs_bind");
  if (!x || (p->nch > 0 && !alpha) || iters < 1) return fail(GS_EINVAL, "bad argument");
  hipStream_t s = p->stream;
  const size_t W = (size_t)p->prec, xb = 3 * (size_t)p->n * W;
  const size_t m = (size_t)p->S * p->slots;
  // keep the caller's start positions (in the adjoint iterate's storage, free
  // between calls) and the stored contact set; each trial starts from both
  char* xs = p->ws + p->lay.mu;
  std::vector<uint8_t> act(m);
  std::vector<double> tg(3 * m), nr(3 * m);
  std::vector<int32_t> pr(m);
  HIPCHK(hipMemcpyAsync(xs, x, xb, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(act.data(), p->ws + p->lay.cact, m, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(tg.data(), p->ws + p->lay.ctgt, 3 * m * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(nr.data(), p->ws + p->lay.cnrm, 3 * m * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(pr.data(), p->ws + p->lay.cprim, m * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  auto restore = [&]() -> gs_status {
    HIPCHK(hipMemcpyAsync(x, xs, xb, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(p->ws + p->lay.cact, act.data(), m, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->ws + p->lay.ctgt, tg.data(), 3 * m * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->ws + p->lay.cnrm, nr.data(), 3 * m * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->ws + p->lay.cprim, pr.data(), m * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return GS_OK;
  };
  const int maxg = p->prec == 4 ? pcg_max_grid<float>(p->ell_w) : pcg_max_grid<double>(p->ell_w);
  if (maxg < 1) return fail(GS_EHIP, "cannot size the cooperative CG grid");
  p->pcg_maxg = maxg;
  const gs_params saved = p->prm;
  const bool prof = p->prof.on;
  p->prof.on = false;
  // candidates: the default (about 256 rows per block), every power of two
  // and every 3 x 2^k (the grids between: row ranges and the barrier's cost
  // trade against each other)
  std::vector<int> cand = {std::max(1, std::min({cdiv(p->n, kPcgRowsPerBlock), maxg, kMaxPcgGrid, p->nparts / 2}))};
  const int glim = std::min({maxg, kMaxPcgGrid, p->nparts / 2});
  for (int g = 1; g <= glim; g *= 2) {
    if (g != cand[0]) cand.push_back(g);
    const int h = 3 * g;
    if (g >= 1 && h <= glim && h < 4 * g && h != cand[0] && (h & (h - 1)) != 0) cand.push_back(h);
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double best_ms = INFINITY;
  int best = cand[0];
  gs_status st = GS_OK;
  for (int g : cand) {
    p->prm.fixed_iters = iters;
    p->prm.pcg_blocks = g;
    p->pcg_grid = g;
    if ((st = plan_segments(p, maxg)) != GS_OK) break;
    for (int rep = 0; rep < 2 && st == GS_OK; ++rep) {  // the first run warms up
      if ((st = restore()) != GS_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) st = fail(GS_EHIP, "event record");
      gs_stats sts{};
      const gs_status r = p->prec == 4 ? solve_impl<float>(p, (const float*)alpha, (float*)x, &sts)
                                       : solve_impl<double>(p, (const double*)alpha, (double*)x, &sts);
      if (r < 0) st = r;
      if (st == GS_OK && hipEventRecord(e1, s) != hipSuccess) st = fail(GS_EHIP, "event record");
      if (st == GS_OK && hipEventSynchronize(e1) != hipSuccess) st = fail(GS_EHIP, "event sync");
      float ms = 0.f;
      if (st == GS_OK && rep == 1 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best_ms) {
        best_ms = ms;
        best = g;
      }
    }
    if (st != GS_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->prm = saved;
  p->prof.on = prof;
  if (st == GS_OK) st = restore();
  p->solved = false;
  if (st != GS_OK) {
    p->pcg_grid = pcg_grid_for(p, maxg);
    (void)plan_segments(p, maxg);
    return st;
  }
  p->prm.pcg_blocks = best;
  p->pcg_grid = pcg_grid_for(p, maxg);
  if ((st = plan_segments(p, maxg)) != GS_OK) return st;
  if (chosen) *chosen = per_mesh_cg(p) ? best : p->pcg_grid;
  if (ms_per_iter) *ms_per_iter = best_ms / iters;
  return GS_OK;
}

size_t gs_unrolled_scratch_size(const gs_problem* p, int32_t K) {
  if (!p || K < 1) return 0;
  return unrolled_records(K) * record_layout(p).bytes;
}

gs_status gs_adjoint_unrolled(gs_problem* p, const void* alpha, const void* x0, int32_t K, const void* dLdx,
                              void* dLdalpha, void* dLdx0, void* xK, void* scratch, size_t scratch_bytes,
                              gs_stats* stats) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!p->bound) return fail(GS_ESTATE, "gs_adjoint_unrolled before gs_bind");
  if (K < 1 || !x0 || !dLdx || !scratch || (p->nch > 0 && (!alpha || !dLdalpha)))
    return fail(GS_EINVAL, "bad argument");
  if (p->mo_k > 0 && p->prm.obstacle_collision)
    return fail(GS_EINVAL, "gradients through a triangle-mesh obstacle are not supported");
  if (((uintptr_t)scratch & 255) != 0) return fail(GS_EINVAL, "scratch must be 256-byte aligned");
  if (scratch_bytes < gs_unrolled_scratch_size(p, K)) return fail(GS_EINVAL, "scratch too small");
  if (p->prec == 4)
    return unrolled_impl<float>(p, (const float*)alpha, (const float*)x0, K, (const float*)dLdx, (float*)dLdalpha,
                                (float*)dLdx0, (float*)xK, (char*)scratch, stats);
  return unrolled_impl<double>(p, (const double*)alpha, (const double*)x0, K, (const double*)dLdx,
                               (double*)dLdalpha, (double*)dLdx0, (double*)xK, (char*)scratch, stats);
}

gs_status gs_adjoint(gs_problem* p, const void* dLdx, void* dLdalpha, void* mu, gs_stats* stats) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!p->bound) return fail(GS_ESTATE, "gs_adjoint before gs_bind");
  if (!p->solved) return fail(GS_ESTATE, "gs_adjoint needs a gs_solve first");
  if (!dLdx || (p->nch > 0 && !dLdalpha)) return fail(GS_EINVAL, "null device buffer");
  if (p->mo_k > 0 && p->prm.obstacle_collision)
    return fail(GS_EINVAL, "gradients through a triangle-mesh obstacle are not supported");
  if (p->prec == 4) return adjoint_impl<float>(p, (const float*)dLdx, (float*)dLdalpha, (float*)mu, stats);
  return adjoint_impl<double>(p, (const double*)dLdx, (double*)dLdalpha, (double*)mu, stats);
}

gs_status gs_reset_contacts(gs_problem* p) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!p->bound) return fail(GS_ESTATE, "not bound");
  HIPCHK(hipMemsetAsync(p->ws + p->lay.cact, 0, (size_t)p->S * p->slots, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return GS_OK;
}

gs_status gs_contacts(gs_problem* p, int32_t cap, int32_t* v, int32_t* type, int32_t* prim, double* target,
                      double* normal, int32_t* fresh, int32_t* count) {
  if (!p || !count) return fail(GS_EINVAL, "null argument");
  if (!p->bound) return fail(GS_ESTATE, "not bound");
  const size_t m = (size_t)p->S * p->slots;
  std::vector<uint8_t> act(m);
  std::vector<double> tg(3 * m), nr(3 * m);
  std::vector<int32_t> pr(m);
  HIPCHK(hipMemcpyAsync(act.data(), p->ws + p->lay.cact, m, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipMemcpyAsync(tg.data(), p->ws + p->lay.ctgt, 3 * m * 8, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipMemcpyAsync(nr.data(), p->ws + p->lay.cnrm, 3 * m * 8, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipMemcpyAsync(pr.data(), p->ws + p->lay.cprim, m * 4, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  int k = 0;
  for (size_t i = 0; i < m; ++i) k += act[i] ? 1 : 0;
  *count = k;
  if (k > cap) return fail(GS_ECAPACITY, "contact capacity too small");
  int o = 0;
  for (int s = 0; s < p->S; ++s)
    for (int sl = 0; sl < p->slots; ++sl) {
      const size_t i = (size_t)s * p->slots + sl;
      if (!act[i]) continue;
      if (v) v[o] = p->qverts[s];
      if (type)
        type[o] = sl == 0 ? GS_CONTACT_SELF
                          : (sl <= p->ns ? GS_CONTACT_SPHERE : (sl <= p->ns + p->np ? GS_CONTACT_PLANE : GS_CONTACT_MESH));
      if (prim) prim[o] = pr[i];
      if (fresh) fresh[o] = act[i] == 2 ? 1 : 0;
      for (int c = 0; c < 3; ++c) {
        if (target) target[3 * o + c] = tg[3 * i + c];
        if (normal) normal[3 * o + c] = nr[3 * i + c];
      }
      ++o;
    }
  return GS_OK;
}

gs_status gs_set_contacts(gs_problem* p, int32_t count, const int32_t* v, const int32_t* type, const int32_t* prim,
                          const double* target, const double* normal, const int32_t* fresh) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!p->bound) return fail(GS_ESTATE, "not bound");
  if (count < 0 || (count > 0 && (!v || !type || !prim || !target || !normal))) return fail(GS_EINVAL, "bad arrays");
  const size_t m = (size_t)p->S * p->slots;
  std::vector<uint8_t> act(m, 0);
  std::vector<double> tg(3 * m, 0.0), nr(3 * m, 0.0);
  std::vector<int32_t> pr(m, -1);
  for (int i = 0; i < count; ++i) {
    if (v[i] < 0 || v[i] >= p->n || p->vq[v[i]] < 0) return fail(GS_EINVAL, "contact vertex is not a query vertex");
    int sl;
    if (type[i] == GS_CONTACT_SELF) {
      if (prim[i] < 0 || prim[i] >= p->F) return fail(GS_EINVAL, "self contact face out of range");
      sl = 0;
    } else if (type[i] == GS_CONTACT_SPHERE) {
      if (prim[i] < 0 || prim[i] >= p->ns) return fail(GS_EINVAL, "sphere index out of range");
      sl = 1 + prim[i];
    } else if (type[i] == GS_CONTACT_PLANE) {
      if (prim[i] < 0 || prim[i] >= p->np) return fail(GS_EINVAL, "plane index out of range");
      sl = 1 + p->ns + prim[i];
    } else if (type[i] == GS_CONTACT_MESH && p->mo_k > 0) {
      if (prim[i] < 0 || prim[i] >= p->mo_k) return fail(GS_EINVAL, "mesh obstacle triangle out of range");
      sl = 1 + p->ns + p->np;
    } else {
      return fail(GS_EINVAL, "bad contact type");
    }
    const size_t j = (size_t)p->vq[v[i]] * p->slots + sl;
    if (act[j]) return fail(GS_EINVAL, "duplicate contact");
    const bool fr = fresh && fresh[i];
    if (fr && sl != 0) return fail(GS_EINVAL, "only self contacts can be fresh");
    act[j] = fr ? 2 : 1;
    pr[j] = prim[i];
    for (int c = 0; c < 3; ++c) {
      tg[3 * j + c] = target[3 * i + c];
      nr[3 * j + c] = normal[3 * i + c];
    }
  }
  HIPCHK(hipMemcpyAsync(p->ws + p->lay.cact, act.data(), m, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(p->ws + p->lay.ctgt, tg.data(), 3 * m * 8, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(p->ws + p->lay.cnrm, nr.data(), 3 * m * 8, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(p->ws + p->lay.cprim, pr.data(), m * 4, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return GS_OK;
}

gs_status gs_local_step_debug(gs_problem* p, const void* x, const void* alpha, void* targets) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!p->bound) return fail(GS_ESTATE, "not bound");
  if (!x || !targets || (p->nch > 0 && !alpha)) return fail(GS_EINVAL, "null device buffer");
  const Consts c = make_consts(p);
  if (p->prec == 4) {
    HIPCHK(launch_local_debug<float>(make_dev<float>(p), c, (const float*)alpha, (const float*)x, (float*)targets,
                                     p->stream));
  } else {
    HIPCHK(launch_local_debug<double>(make_dev<double>(p), c, (const double*)alpha, (const double*)x,
                                      (double*)targets, p->stream));
  }
  return GS_OK;
}

gs_status gs_remesh_flags(gs_problem* p, const void* x, const void* x_ref, double alpha_max, double d_max,
                          uint8_t* flags, int32_t* n_flagged) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!p->bound) return fail(GS_ESTATE, "gs_remesh_flags before gs_bind");
  if (!x || !flags) return fail(GS_EINVAL, "null device buffer");
  if (!(alpha_max > 0) || !std::isfinite(alpha_max) || !(d_max > 0) || !std::isfinite(d_max))
    return fail(GS_EINVAL, "alpha_max and d_max must be finite and > 0");
  const Consts c = make_consts(p);
  int* cnt = (int*)(p->ws + p->lay.rcount);
  hipError_t e;
  if (p->prec == 4)
    e = timed(p, K_REMESH, [&] {
      return launch_remesh_flags<float>(make_dev<float>(p), c, (const float*)x, (const float*)x_ref, alpha_max, d_max,
                                        flags, cnt, p->stream);
    });
  else
    e = timed(p, K_REMESH, [&] {
      return launch_remesh_flags<double>(make_dev<double>(p), c, (const double*)x, (const double*)x_ref, alpha_max,
                                         d_max, flags, cnt, p->stream);
    });
  HIPCHK(e);
  int32_t h = 0;
  HIPCHK(hipMemcpyAsync(&h, cnt, 4, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  if (n_flagged) *n_flagged = h;
  return GS_OK;
}

gs_status gs_solve_progressive(gs_problem* p, const void* alpha, void* x, double alpha_max, double d_max,
                               int32_t stop_on_flag, uint8_t* flags, int32_t cap, gs_stage* stages,
                               int32_t* n_stages) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!p->bound) return fail(GS_ESTATE, "gs_solve_progressive before gs_bind");
  if (!x || !flags || (p->nch > 0 && !alpha) || (cap > 0 && !stages)) return fail(GS_EINVAL, "null buffer");
  if (!(alpha_max > 0) || !std::isfinite(alpha_max) || !(d_max > 0) || !std::isfinite(d_max))
    return fail(GS_EINVAL, "alpha_max and d_max must be finite and > 0");
  const size_t W = (size_t)p->prec, nch = (size_t)p->nch;
  std::vector<double> a(nch);
  if (nch) {
    std::vector<char> raw(nch * W);
    HIPCHK(hipMemcpyAsync(raw.data(), alpha, nch * W, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    for (size_t i = 0; i < nch; ++i)
      a[i] = W == 4 ? (double)((const float*)raw.data())[i] : ((const double*)raw.data())[i];
  }
  // stage k actuates min(alpha, (k+1) alpha_max) per chamber; the last stage
  // is the first whose actuation reaches alpha everywhere
  for (double v : a)
    if (!std::isfinite(v)) return fail(GS_EINVAL, "non-finite alpha");
  int K = 0;
  for (bool reached = false; !reached;) {
    if (++K > (1 << 20)) return fail(GS_EINVAL, "alpha / alpha_max too large");
    reached = true;
    for (double v : a) reached &= std::min(v, K * alpha_max) >= v;
  }
  if (K > cap) return fail(GS_EINVAL, "stages array shorter than the number of stages");
  char* ak = p->ws + p->lay.alpha_stage;
  std::vector<char> host(nch * W);
  bool all_converged = true;
  int done = 0;
  for (int k = 0; k < K; ++k) {
    double top = 0.0;
    for (size_t i = 0; i < nch; ++i) {
      const double v = std::min(a[i], (k + 1) * alpha_max);
      top = std::max(top, v);
      if (W == 4)
        ((float*)host.data())[i] = (float)v;
      else
        ((double*)host.data())[i] = v;
    }
    if (nch) HIPCHK(hipMemcpyAsync(ak, host.data(), nch * W, hipMemcpyHostToDevice, p->stream));
    gs_stage& st = stages[k];
    std::memset(&st, 0, sizeof(st));
    const gs_status r = gs_solve(p, nch ? ak : nullptr, x, &st.solve);
    if (r != GS_OK && r != GS_NOT_CONVERGED) return r;
    all_converged &= (r == GS_OK);
    st.status = r;
    st.alpha_top = top;
    const gs_status rf = gs_remesh_flags(p, x, nullptr, alpha_max, d_max, flags, &st.n_flagged);
    if (rf != GS_OK) return rf;
    done = k + 1;
    if (n_stages) *n_stages = done;
    if (stop_on_flag && st.n_flagged > 0) break;
  }
  if (n_stages) *n_stages = done;
  return all_converged ? GS_OK : GS_NOT_CONVERGED;
}

gs_status gs_tets(const gs_problem* p, int32_t* tets) {
  if (!p || !tets) return fail(GS_EINVAL, "null argument");
  std::memcpy(tets, p->tets.data(), p->tets.size() * 4);
  return GS_OK;
}

gs_status gs_faces(const gs_problem* p, int32_t* faces) {
  if (!p || !faces) return fail(GS_EINVAL, "null argument");
  std::memcpy(faces, p->faces.data(), p->faces.size() * 4);
  return GS_OK;
}

size_t gs_collide_debug_scratch(int32_t cap) { return 16 * (size_t)std::max(cap, 0) + 256; }

gs_status gs_collide_debug(gs_problem* p, const void* x, int32_t cap, void* scratch, size_t scratch_bytes,
                           int32_t* cand_tet, int32_t* n_cand_tet, int32_t* cand_tri, int32_t* n_cand_tri,
                           int32_t* contacts, double* target, int32_t* n_contacts) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (!p->bound) return fail(GS_ESTATE, "not bound");
  if (!x || !scratch || cap < 0 || !n_cand_tet || !n_cand_tri || !n_contacts) return fail(GS_EINVAL, "null argument");
  if (scratch_bytes < gs_collide_debug_scratch(cap)) return fail(GS_EINVAL, "debug scratch too small");
  hipStream_t s = p->stream;
  const size_t m = (size_t)p->S * p->slots;
  // keep the stored active set: save it, run one check, restore it
  std::vector<uint8_t> act(m);
  std::vector<double> tg(3 * m), nr(3 * m);
  std::vector<int32_t> pr(m);
  HIPCHK(hipMemcpyAsync(act.data(), p->ws + p->lay.cact, m, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(tg.data(), p->ws + p->lay.ctgt, 3 * m * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(nr.data(), p->ws + p->lay.cnrm, 3 * m * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(pr.data(), p->ws + p->lay.cprim, m * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const Consts c = make_consts(p);
  DevStatus h{};
  gs_status st = GS_OK;
  auto run = [&](auto tag) -> gs_status {
    using R = decltype(tag);
    Dev<R> d = make_dev<R>(p);
    d.dbg_cap = cap;
    d.dbg_tet = (int32_t*)scratch;
    d.dbg_tri = (int32_t*)scratch + 2 * (size_t)cap;
    HIPCHK(launch_set_positions<R>(d, c, (const R*)x, s));
    p->hash_ready = false;
    if (c.self_col)
      for (int stg = 0; stg < N_COLLIDE_STAGES; ++stg) HIPCHK(launch_collide_stage<R>(d, c, stg, true, s));
    if (c.mo) HIPCHK(launch_mesh_obstacle<R>(d, c, s));
    if (c.self_col || c.obst_col || c.mo) HIPCHK(launch_contacts<R>(d, c, s));
    HIPCHK(hipMemcpyAsync(&h, d.st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return GS_OK;
  };
  st = p->prec == 4 ? run(float{}) : run(double{});
  if (st != GS_OK) return st;
  *n_cand_tet = h.cand_tet;
  *n_cand_tri = h.cand_tri;
  auto sorted_pairs = [&](const int32_t* dev, int cnt, int32_t* out, int32_t* nout) -> gs_status {
    const int k = std::min(cnt, cap);
    std::vector<int32_t> buf(2 * (size_t)cap);
    if (cap > 0) HIPCHK(hipMemcpy(buf.data(), dev, 2 * (size_t)cap * 4, hipMemcpyDeviceToHost));
    std::vector<std::pair<int32_t, int32_t>> pr2(k);
    for (int i = 0; i < k; ++i) pr2[i] = {buf[i], buf[cap + i]};
    std::sort(pr2.begin(), pr2.end());
    pr2.erase(std::unique(pr2.begin(), pr2.end()), pr2.end());
    *nout = (int32_t)pr2.size();
    if (out)
      for (size_t i = 0; i < pr2.size(); ++i) {
        out[i] = pr2[i].first;
        out[cap + i] = pr2[i].second;
      }
    return GS_OK;
  };
  const bool over = h.cand_tet > cap || h.cand_tri > cap;
  if (!over) {
    if ((st = sorted_pairs((const int32_t*)scratch, h.cand_tet, cand_tet, n_cand_tet)) != GS_OK) return st;
    if ((st = sorted_pairs((const int32_t*)scratch + 2 * (size_t)cap, h.cand_tri, cand_tri, n_cand_tri)) != GS_OK)
      return st;
  }
  // resulting active set, then restore the stored one
  std::vector<int32_t> cv(std::max<size_t>(m, 1)), ct(std::max<size_t>(m, 1)), cp(std::max<size_t>(m, 1));
  std::vector<double> ctg(3 * std::max<size_t>(m, 1)), cnr(3 * std::max<size_t>(m, 1));
  int32_t cnt = 0;
  st = gs_contacts(p, (int32_t)m, cv.data(), ct.data(), cp.data(), ctg.data(), cnr.data(), nullptr, &cnt);
  HIPCHK(hipMemcpyAsync(p->ws + p->lay.cact, act.data(), m, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->ws + p->lay.ctgt, tg.data(), 3 * m * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->ws + p->lay.cnrm, nr.data(), 3 * m * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->ws + p->lay.cprim, pr.data(), m * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  if (st != GS_OK) return st;
  *n_contacts = cnt;
  if (cnt <= cap && contacts)
    for (int i = 0; i < cnt; ++i) {
      contacts[i] = cv[i];
      contacts[cap + i] = ct[i];
      contacts[2 * (size_t)cap + i] = cp[i];
      if (target)
        for (int k = 0; k < 3; ++k) target[k * (size_t)cap + i] = ctg[3 * i + k];
    }
  if (over || cnt > cap) return fail(GS_ECAPACITY, "candidate or contact capacity too small");
  return GS_OK;
}

gs_status gs_collide_debug_static(gs_problem* p, const void* x, int32_t cap, int32_t* cand_tet, int32_t* n_cand_tet,
                                  int32_t* cand_tri, int32_t* n_cand_tri, int32_t* contacts, double* target,
                                  int32_t* n_contacts) {
  if (!p) return fail(GS_EINVAL, "null problem");
  if (cap < 0 || cap > kStaticCandCap)
    return fail(GS_EINVAL, "cap exceeds the static candidate buffer (" + std::to_string(kStaticCandCap) + " pairs)");
  if (!p->bound) return fail(GS_ESTATE, "not bound");
  void* scratch = nullptr;
  HIPCHK(static_candidate_scratch(&scratch));
  // the staging layout is [2][cap] tet pairs then [2][cap] triangle pairs:
  // the whole array serves any cap up to kStaticCandCap
  return gs_collide_debug(p, x, cap, scratch, gs_collide_debug_scratch(kStaticCandCap), cand_tet, n_cand_tet, cand_tri,
                          n_cand_tri, contacts, target, n_contacts);
}

gs_status gs_trace(gs_problem* p, int32_t cap, double* rows, int32_t* count) {
  if (!p || !count || (cap > 0 && !rows)) return fail(GS_EINVAL, "null argument");
  if (!p->bound) return fail(GS_ESTATE, "not bound");
  const int k = std::min({p->last_iters, p->trace_len, std::max(cap, 0)});
  *count = k;
  if (k > 0) {
    HIPCHK(hipMemcpyAsync(rows, p->ws + p->lay.trace, (size_t)k * 6 * 8, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
  }
  return GS_OK;
}

gs_status gs_profile(gs_problem* p, int32_t enable) {
  if (!p) return fail(GS_EINVAL, "null problem");
  p->prof.reset();
  p->prof.on = enable != 0;
  return GS_OK;
}

gs_status gs_profile_read(const gs_problem* p, double* ms, int64_t* launches) {
  if (!p || !ms || !launches) return fail(GS_EINVAL, "null argument");
  for (int k = 0; k < kNKernels; ++k) {
    ms[k] = p->prof.ms[k];
    launches[k] = p->prof.cnt[k];
  }
  return GS_OK;
}

const char* gs_kernel_name(int32_t k) { return (k >= 0 && k < kNKernels) ? kKernelNames[k] : ""; }

void gs_destroy(gs_problem* p) { delete p; }

}  // extern "C"
