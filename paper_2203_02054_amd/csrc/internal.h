// Internal declarations shared by the host layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geosim.h"

namespace gs {

constexpr int kBlock = 256;          // threads per block of the streaming kernels
constexpr int kCellCap = 64;         // hash cells a tet box may span before the brute-force path
constexpr int kHashCap = 8;          // entries stored in a hash bucket before the overflow list
constexpr int kMaxSlots = 1 + 8 + 8 + 1; // self + spheres + planes + the triangle-mesh obstacle
constexpr int kPcgThreads = 512;     // threads per block of the persistent CG kernel
constexpr int kPcgRowsPerBlock = 256; // default rows per CG block (grid = n / 256, capped)
// Tet count from which the tet query runs its one-lane-per-tet,
// lower-register variant (the GPU then holds enough waves that occupancy
// beats prefetching and lane sharing) and is not fused with the local step.
constexpr int kTetQueryWide = 1 << 18;
constexpr int kMaxPcgGrid = 1024;     // workgroups of the persistent CG kernel at most
constexpr int kBarGroups = 8;          // groups of the two-level grid barrier (one per XCD)
constexpr int kBarWords = 64 * (kBarGroups + 1);  // its group counters a cache line apart, then the top counter
constexpr int kAaMaxMem = 16;         // Anderson memory at most (forward and adjoint)
constexpr int kFaaRows = 1024;        // rows per block of the acceleration's dot-product kernel
constexpr int kStaticCandCap = 1 << 17;  // candidate pairs per list of the allocation-free collision check
constexpr int kMaxDevices = 64;
constexpr int kCoarseNb = 8;          // coarse unknowns a CG workgroup's rows reach (its own first)
constexpr int kCoarseMaxG = 256;      // CG workgroups at most with the coarse correction

// Completion codes kept on the device (DevStatus::done).
// STALLED: a grid barrier of the CG kernel gave up waiting (see grid_barrier).
enum { RUNNING = 0, CONVERGED = 1, MAXITER = 2, BREAKDOWN = 3, FIXED_DONE = 4, STALLED = 5 };

struct DevStatus {
  int iters;            // outer iterations completed
  int done;             // RUNNING / CONVERGED / ...
  int changed;          // active set changed in the current iteration
  int pcg_total;        // inner CG iterations summed
  int ray_miss;         // current iteration
  int ray_miss_last;    // last completed iteration
  int n_pen;            // penetrating query vertices (current iteration)
  int ticket;           // last-block ticket of the finish kernel
  int n_contacts;       // active springs (current iteration)
  int n_contacts_last;
  int cand_tet, cand_tri;  // debug candidate counters
  int n_over;           // hash entries in the overflow list (current iteration)
  int pcg_last;         // inner iterations of the last outer iteration
  int changed_last;
  int n_active;         // meshes still iterating
  double residual;      // r_k of the last completed iteration
  double energy;        // Eq. 9 at x_k with the iteration's targets
  unsigned bar_count;    // grid-barrier arrivals of the running CG launch (0 between launches)
  int aa_pending;        // accelerated iteration: an iteration's position update is due
  int aa_ticket;         // last-block ticket of the position-update kernel
  unsigned mb_last;      // one-workgroup-per-mesh CG: the longest mesh's iterations, bit 31 a breakdown
};

// Anderson acceleration of the local/global iteration: per-mesh state.
// `act` is the decision the CG kernel's last block takes for the iteration
// just finished, read by the acceleration kernels that follow it.
enum { AA_NONE = 0, AA_ACCEPT = 1, AA_REJECT = 2 };
struct AaMesh {
  int k;         // difference columns held (<= memory); columns 0..k-1 are valid
  int head;      // column the next difference goes to
  int has_prev;  // the last accepted point and its residual are stored
  int cand;      // the current point is an accelerated one (not yet tested)
  int act;       // AA_NONE (mesh done or frozen) / AA_ACCEPT / AA_REJECT
  int rejected;  // accelerated points rejected in this solve
  int ok;        // the last least-squares solve succeeded
  int pad;
  double r_acc;  // residual at the last accepted point (residual guard)
  double e_acc;  // energy at the last accepted point (energy guard)
};

// A block of the acceleration's dot-product kernel: rows [v0, v1) of mesh m.
struct AaBlock {
  int m, v0, v1, pad;
};

// A node of the triangle-mesh obstacle's bounding-volume hierarchy: a leaf
// (count > 0) holds triangles [first, first + count) of the leaf-ordered
// records; an inner node (count == 0) its two children.
struct MoNode {
  double lo[3], hi[3];
  int left, right, first, count;
};

// Per-mesh constants of a problem made of one or several meshes.
struct MeshConst {
  double eps;       // offset of the collided boundary (eps_rel * h_ref)
  double Lray;      // length of the inverse-normal search (ray_rel * h_ref)
  double inv_cell;  // 1 / hash cell size
  double inv_diag;  // 1 / bounding-box diagonal (residual scale)
  double inv_mean_vol;  // 1 / mean rest tet volume (omega_e = Vol(e) / mean Vol)
  int fbeg, fend;   // boundary faces of the mesh
  int sbeg, send;   // query vertices of the mesh
  int vbeg, vend;   // vertices of the mesh
};

// Scalars of one problem (passed by value to kernels).
struct Consts {
  int n, T, S, F, nch, slots, H, ns, np;
  int M;                // meshes
  int mask_done;        // freeze meshes once they converge (not with fixed_iters)
  int self_col, obst_col, hyper;
  int mo;               // the triangle-mesh obstacle is on (its slot is the last one)
  int coarse;           // the CG preconditioner has the coarse correction (built for this grid)
  int max_iter, fixed_iters, pcg_max;
  int nparts;           // partial-sum slots per reduction array
  int ell_w;            // off-diagonal entries per row of the ELL matrix (16, 32 or 64)
  int trace_len;        // rows of the per-iteration trace
  int aa_m;             // adjoint: Anderson memory (0: plain fixed-point iteration)
  int adj_jt;           // adjoint gather writes (db/dx)^T mu alone to `lam` (unrolled reverse sweep)
  int a_parts;          // energy partials the local step writes per iteration (part_a)
  int cg_soa;           // CG state layout for the current grid: 1 = [3][n] (paired variant), 0 = [n][3]
  unsigned long long bar_timeout;  // grid-barrier wait limit in wall-clock ticks
  int faa_m;            // Anderson memory of the local/global iteration (0: plain)
  int faa_guard;        // GS_AA_GUARD_*
  int faa_nblk;         // blocks of the acceleration's dot-product kernel
  int per_mesh;         // a batch's CG runs per mesh (its own workgroups, scalars and stopping test)
  int cg_wb;            // CG state stored write-back (1) or write-through (0)
  int bar2;             // the whole-grid CG kernel uses the two-level grid barrier
  double c1, c2, kappa, tol, pcg_eta;
  double pcg_eta_min;   // > 0: forward solves stop at clamp(previous r_k, pcg_eta_min, pcg_eta)
  double faa_slack;     // relative slack of the guard test
};

// Device pointers, all inside the caller's workspace except the in/out buffers.
template <typename R>
struct Dev {
  // static
  const double* X0;        // [3][n]
  const int32_t* tets;     // [4][T]
  const int32_t* tag;      // [T] mode | (chamber << 3)
  const int32_t* inc_start;  // [n+1]
  const int32_t* inc_pos;  // [4][T]
  const int32_t* ell_col;  // [ell_w][n] off-diagonal columns of A_el (free rows/cols; padding: own row)
  const R* ell_val;        // [ell_w][n] (padding: 0)
  R* ell_scaled;           // [ell_w][n] ell_val / dg[col], rebuilt by each CG solve
  const R* adiag;          // [n] diagonal of A_el (1 on fixed rows)
  const uint8_t* freem;    // [n]
  const int32_t* faces;    // [3][F]
  const int32_t* qverts;   // [S]
  const int32_t* vq;       // [n] query index or -1
  const int32_t* qf_start; // [S+1]
  const int32_t* qf_list;  // incident boundary faces of each query vertex, ascending
  const double* kq;        // [S] spring stiffness
  const double* obst;      // spheres [ns][4] then planes [np][6]
  const MeshConst* mesh;   // [M]
  const int32_t* vmesh;    // [n] mesh of each vertex
  const int32_t* tmesh;    // [T] mesh of each tet
  // iteration state
  R* u;                    // [3][n] displacement from X0
  double* xc;              // [3][n] X0 + u in double (collision positions)
  R* res4;                 // [4T][4] element residual columns in incidence order
  R* cg;                   // [2][3n][4] CG state, two buffers of r, w = A M^-1 r, s = A p: [3][n] or [n][3] (cg_soa)
                           //   (each as x, y, z, pad); buffer 0 holds the right-hand side on entry
  R* dl;                   // [n][4] correction (kept across iterations: the warm start)
  R* dlp;                  // [n][4] correction of the previous outer iteration
  R* dlpp;                 // [n][4] correction two outer iterations back
  R* p;                    // [n][4]
  R* dg;                   // [n] Jacobi diagonal
  R* dsp;                  // [n] spring diagonal
  int32_t* pen;            // [S] penetration flag of each query vertex (this iteration)
  int32_t* hcount;         // [H] entries inserted per bucket (may exceed kHashCap)
  double* hslot;           // [H][kHashCap][4] bucket entries (x, y, z, and as bits: query index | vertex << 32)
  double* hover;           // [S][4] entries of full buckets (scanned by every tet)
  int32_t* penlist;        // [S] penetrating query vertices (unordered)
  int32_t* fhit;           // [S] fresh self hit face or -1
  double* fc;              // [S][3] fresh self target
  double* fn;              // [S][3] fresh self normal
  uint8_t* cact;           // [S][slots] 0 inactive, 1 active, 2 self contact given a new target this iteration
  double* ctgt;            // [S][slots][3]
  double* cnrm;            // [S][slots][3]
  int32_t* cprim;          // [S][slots]
  double* part_a;          // [nparts] reductions
  double* part_b;
  double* part_c;
  double* part_d;
  double* part_e;
  double* part_f;
  unsigned long long* mres;  // [M] max |d| per mesh (double bits; non-negative, so integer max works)
  int32_t* mchanged;       // [M] active set of the mesh changed this iteration
  int32_t* mdone;          // [M] iteration at which the mesh converged (0: still running)
  DevStatus* st;
  double* trace;           // [trace_len][6]
  // implicit adjoint (gs_adjoint); the adjoint iteration runs with its own
  // status block and per-mesh done flags in place of st / mdone
  R* mu;                   // [3][n] adjoint iterate
  const R* gL;             // [3][n] dL/dx (caller's buffer)
  double* acc3;            // [3][n] adjoint of the new self-contact targets, scattered as 64-bit fixed-point
                           //   integers (cleared by the gather)
  unsigned long long* acc_max;  // [1] largest scattered magnitude of the iteration (double bits)
  double* ga;              // [T] per-tet contribution to dL/dalpha
  const int32_t* ch_start; // [nch+1] chamber -> tets
  const int32_t* ch_tets;  // chamber tets grouped by chamber, ascending
  unsigned long long* mmax;  // [M] max |mu| per mesh (double bits)
  double* mgam;              // [M][2] warm-start weights per mesh of a batch
  R* alpha_last;           // [nch] volume ratios of the last solve
  // Anderson acceleration of the adjoint iteration (memory m = Consts::aa_m)
  R* aa_dx;                // [m][3][n] differences of successive iterates
  R* aa_df;                // [m][3][n] differences of successive residuals (corrections)
  R* aa_xp;                // [3][n] previous iterate
  R* aa_fp;                // [3][n] previous residual
  double* aa_h;            // [m][m] Gram matrix of aa_df
  double* aa_gamma;        // [m] least-squares coefficients
  double* aa_part;         // [2m][nparts] block partials of the dot products
  int32_t* aa_k;           // [1] iterations taken by the accelerated loop
  // Anderson acceleration of the local/global iteration (memory Consts::faa_m;
  // shares aa_dx / aa_df / aa_xp / aa_fp with the adjoint's)
  AaMesh* faa;             // [M]
  double* faa_h;           // [M][kAaMaxMem][kAaMaxMem] Gram matrices of the residual differences
  double* faa_gam;         // [M][kAaMaxMem] least-squares coefficients
  const AaBlock* faa_blk;  // [faa_nblk] row ranges of the dot-product kernel, grouped by mesh
  const int32_t* faa_mblk; // [M+1] first block of each mesh
  uint8_t* cact_s;         // the active set at the last accepted point (restored on a rejection)
  double* ctgt_s;
  double* cnrm_s;
  int32_t* cprim_s;
  // unrolled reverse sweep
  R* lam;                  // [3][n] adjoint of the positions
  double* ga_acc;          // [nch] dL/dalpha accumulated over the reverse steps
  // coarse correction of the CG preconditioner (one unknown per workgroup's
  // row range): the inverse of R0 A_el R0^T [G][G], the coarse unknowns each
  // workgroup's rows reach [G][kCoarseNb] (own first, -1 padded), and per
  // row its couplings (x: off-diagonal sum over its own range; y, z: sums
  // over the other ranges cz_ri names, low and high 16 bits)
  const double* cz_inv;
  const int32_t* cz_nb;
  const R* cz_rho;         // [n][4]
  const int32_t* cz_ri;
  // triangle-mesh obstacle (static tree; per-query-vertex results of its kernel)
  const double* mo_tri;    // [k][30] leaf-ordered triangles: a, b, c, face, edge (ab, ac, bc) and vertex
                           //   (a, b, c) pseudonormals
  const int32_t* mo_id;    // [k] triangle id of each record
  const MoNode* mo_node;   // tree nodes, root first
  uint8_t* mo_flag;        // [S] 0 not tested, 1 tested and outside, 2 inside
  double* mo_tgt;          // [S][3] target c + eps u
  double* mo_nrm;          // [S][3] outward direction u
  int32_t* mo_prim;        // [S] triangle of the closest point
  // debug candidate buffers (null outside gs_collide_debug)
  int32_t* dbg_tet;        // [2][cap]
  int32_t* dbg_tri;        // [2][cap]
  int dbg_cap;
  // per-mesh CG (a batch): each workgroup's {mesh, index within the mesh,
  // the mesh's workgroups, the mesh's first workgroup}; barrier counters
  const int4* seg;         // [grid]
  unsigned* mbar;          // [M] arrivals at the mesh's barrier in the running launch (0 between launches)
  unsigned* bar2;          // [9 * 64] two-level grid barrier: group counters (64 words apart), top counter
};

// ---------------------------------------------------------------------------
// launchers (one per kernel family); all enqueue on `s` and return hipError_t
template <typename R> hipError_t launch_init(const Dev<R>& d, const Consts& c, const R* xin, hipStream_t s);
template <typename R>
hipError_t launch_hash_clear(const Dev<R>& d, const Consts& c, hipStream_t s);
template <typename R> hipError_t launch_output(const Dev<R>& d, const Consts& c, R* xout, hipStream_t s);
// collision stages, in launch order
enum { STAGE_HASH_INSERT = 0, STAGE_TET_QUERY, STAGE_RAY, N_COLLIDE_STAGES };
template <typename R>
hipError_t launch_collide_stage(const Dev<R>& d, const Consts& c, int stage, bool debug, hipStream_t s);
template <typename R> hipError_t launch_contacts(const Dev<R>& d, const Consts& c, hipStream_t s);
template <typename R> hipError_t launch_local(const Dev<R>& d, const Consts& c, const R* alpha, hipStream_t s);
template <typename R> hipError_t launch_query_local(const Dev<R>& d, const Consts& c, const R* alpha, hipStream_t s);
template <typename R> hipError_t launch_local_debug(const Dev<R>& d, const Consts& c, const R* alpha, const R* x,
                                                    R* targets, hipStream_t s);
template <typename R>
hipError_t launch_pcg(const Dev<R>& d, const Consts& c, int grid, hipStream_t s, bool adjoint, bool cooperative,
                      hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// implicit adjoint
template <typename R> hipError_t launch_adj_init(const Dev<R>& d, const Consts& c, hipStream_t s);
template <typename R> hipError_t launch_adj_springs(const Dev<R>& d, const Consts& c, hipStream_t s);
template <typename R>
hipError_t launch_adj_local(const Dev<R>& d, const Consts& c, bool alpha_grad, hipStream_t s);
template <typename R> hipError_t launch_adj_gather(const Dev<R>& d, const Consts& c, hipStream_t s);
template <typename R> hipError_t launch_adj_chamber_sum(const Dev<R>& d, const Consts& c, R* out, hipStream_t s);
template <typename R> hipError_t launch_adj_anderson(const Dev<R>& d, const Consts& c, hipStream_t s);
// Anderson step of the local/global iteration, after the CG kernel
template <typename R> hipError_t launch_fwd_anderson(const Dev<R>& d, const Consts& c, hipStream_t s);
template <typename R> hipError_t launch_mesh_obstacle(const Dev<R>& d, const Consts& c, hipStream_t s);
template <typename R>
hipError_t launch_tree_refit(const Dev<R>& d, const Consts& c, MoNode* nodes, const int32_t* order, double* tbox,
                             const int* level_start, int levels, hipStream_t s);
template <typename R>
hipError_t launch_tree_query(const Dev<R>& d, const Consts& c, const MoNode* nodes, const int32_t* order,
                             const double* tbox, int32_t* pairs, int cap, int* count, hipStream_t s);
template <typename R>
hipError_t launch_remesh_flags(const Dev<R>& d, const Consts& c, const R* x, const R* xref, double amax, double dmax,
                               uint8_t* flags, int* count, hipStream_t s);
// unrolled adjoint helpers
enum { ADJ_RESIDUAL = 0, ADJ_ALPHA = 1, ADJ_JT = 2 };
template <typename R> hipError_t launch_adj_local_mode(const Dev<R>& d, const Consts& c, int mode, hipStream_t s);
template <typename R> hipError_t launch_unr_restore(const Dev<R>& d, const Consts& c, DevStatus* run, hipStream_t s);
template <typename R> hipError_t launch_unr_rhs(const Dev<R>& d, const Consts& c, hipStream_t s);
template <typename R>
hipError_t launch_unr_accumulate(const Dev<R>& d, const Consts& c, hipStream_t s);
template <typename R>
hipError_t launch_unr_finish(const Dev<R>& d, const Consts& c, R* dalpha, R* dx0, hipStream_t s);
template <typename R> hipError_t launch_set_positions(const Dev<R>& d, const Consts& c, const R* x, hipStream_t s);
template <typename R> int pcg_max_grid(int ell_w);
// this device's copy of the allocation-free collision check's staging array
hipError_t static_candidate_scratch(void** ptr);

__host__ __device__ inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// Rows per block of the CG kernel for n rows on a grid of G blocks (a
// multiple of 64; the kernel derives the same value).
__host__ __device__ inline int pcg_chunk(int n, int G) { return (cdiv(n, G) + 63) & ~63; }

// Whether a CG launch on G blocks runs the paired-lane variant (FP32, ELL
// width 16, at most one lane pair per row).  That variant keeps the CG state
// as three arrays of rows, the others as rows of three vectors (Consts::cg_soa).
__host__ __device__ inline bool pcg_paired(int real_bytes, int ell_w, int n, int G) {
  return real_bytes == 4 && ell_w <= 16 && 2 * pcg_chunk(n, G) <= kPcgThreads;
}

}  // namespace gs
