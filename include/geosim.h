/*
 * geosim.h - C ABI of the MI355X (gfx950) library for collision-aware,
 * geometry-based soft-robot simulation on tetrahedral meshes.
 *
 * The method (Fang, Tian, Weightman, Wang, "Collision-Aware Fast Simulation
 * for Soft Robots by Optimization-Based Geometric Computing") finds the
 * deformed shape of an actuated soft robot by minimising the augmented
 * geometric objective of Eq. (9) with a local/global iteration
 * (Section III-B, inner loop of Algorithm 1):
 *
 *   local step   every tet is projected onto its target shape: chamber
 *                elements onto their volume-scaled rest shape (Section
 *                III-A.1, Eq. 2), body elements onto the Mooney-Rivlin blend
 *                of Eq. (6) rescaled to the rest volume by Eq. (7); the
 *                rotation is the SVD (Kabsch) fit below Eq. (1);
 *   collision    surface vertices inside other tets (Eq. 3) or inside
 *                obstacles (Eq. 4) get virtual springs (Eq. 5) towards
 *                targets on the offset boundary (Section II-C), kept or
 *                released by Eq. (8);
 *   global step  with targets fixed, Eq. (9) is a linear least-squares
 *                problem in the vertex positions, solved here by a
 *                Jacobi-preconditioned conjugate gradient on the sparse
 *                matrix in ELL form (16, 32 or 64 entries per row).
 *
 * Conventions
 * -----------
 * - All arrays are structure-of-arrays: positions [3][n] (x row, y row,
 *   z row), tets [4][T].  Indices are int32, zero-based.
 * - "dev_" pointers are device (HIP) memory owned by the caller; all other
 *   pointers are host memory.  The library never allocates or frees device
 *   memory: the caller provides one workspace (gs_workspace_size bytes) at
 *   gs_bind, plus the in/out buffers of each call.
 * - Every device call is enqueued on the stream given to gs_bind (a
 *   hipStream_t passed as void*).  Calls that return host data (statistics,
 *   contacts, candidate lists) synchronise that stream.
 * - Status codes: 0 ok, > 0 warning, < 0 error.  A negative code leaves the
 *   handle usable except after GS_EHIP.  gs_last_error() gives a message for
 *   the last failing call on the calling thread.  No C++ exception crosses
 *   this interface.
 * - Floating-point width of the solve is chosen per problem
 *   (gs_mesh_desc.precision = 4 or 8): dev_x, dev_alpha and the debug
 *   outputs use that width; geometric predicates are always evaluated in
 *   double precision.
 */
#ifndef GEOSIM_H
#define GEOSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GEOSIM_VERSION 211

typedef int32_t gs_status;

enum {
  GS_OK = 0,
  GS_NOT_CONVERGED = 1, /* max_iter reached; the last iterate is written      */
  GS_EINVAL = -1,       /* bad size, index, null pointer or non-finite input  */
  GS_EDEGENERATE = -2,  /* rest tet with |Vol| <= 1e-12 h_ref^3               */
  GS_EBREAKDOWN = -3,   /* NaN/Inf in the iteration or CG curvature p'Ap <= 0 */
  GS_ECAPACITY = -4,    /* caller buffer too small; the needed count is given */
  GS_ESTATE = -5,       /* call out of order (e.g. solve before bind)         */
  GS_EHIP = -6          /* HIP runtime error; see gs_last_error()             */
};

/* Element classes (Section II-A): body elements (M_b) and chamber elements
 * (M_c).  A chamber element of class GS_CH_ISO targets alpha^(1/3) times its
 * rest shape (Section III-A.1); GS_CH_AX_{X,Y,Z} stretch the rest shape by
 * alpha along one rest-frame axis (length actuation, footnote of Section
 * II-A).  Both reach volume ratio alpha (Eq. 2). */
enum { GS_BODY = 0, GS_CH_ISO = 1, GS_CH_AX_X = 2, GS_CH_AX_Y = 3, GS_CH_AX_Z = 4 };

/* Contact types of the virtual springs (Section II-C). */
enum { GS_CONTACT_SELF = 0, GS_CONTACT_SPHERE = 1, GS_CONTACT_PLANE = 2, GS_CONTACT_MESH = 3 };

/* Tet mesh M = M_c + M_b (Section II-A).  Host pointers, copied by gs_create. */
typedef struct {
  int32_t n_verts, n_tets, n_chambers;
  int32_t precision;          /* 4 (float) or 8 (double)                          */
  const double* rest_xyz;     /* [3][n_verts] rest positions X0 (mm)              */
  const int32_t* tets;        /* [4][n_tets] vertex ids, any orientation          */
  const uint8_t* tet_mode;    /* [n_tets] GS_BODY / GS_CH_*                       */
  const int16_t* tet_chamber; /* [n_tets] chamber id in [0, n_chambers), -1 body  */
  const uint8_t* fixed;       /* [n_verts] 1 = held at its rest position          */
} gs_mesh_desc;

typedef struct {
  double c1, c2;          /* Mooney-Rivlin constants of the body (Section IV)     */
  int32_t hyperelastic;   /* 0: R_w == 1 (as-rigid-as-possible body targets)      */
  double kappa_col;       /* spring stiffness k_v = kappa_col * A_el[v,v]         */
  double eps_rel;         /* offset eps of the collided boundary, x h_ref (0.05)  */
  double ray_rel;         /* length of the inverse-normal search, x h_ref (4)     */
  int32_t self_collision, obstacle_collision;
  double tol;             /* outer residual max_v|dx_v| / bbox diagonal (1e-6)    */
  int32_t max_iter;       /* outer iteration cap                                  */
  int32_t fixed_iters;    /* > 0: run exactly this many outer iterations          */
  double pcg_eta;         /* inner CG stop: sqrt(r'z) <= pcg_eta sqrt(b'D^-1 b),
                             b = right-hand side, CG warm-started at the previous
                             correction                                           */
  int32_t pcg_max;        /* inner CG iteration cap per outer iteration           */
  int32_t check_every;    /* outer iterations between host convergence polls     */
  int32_t pcg_blocks;     /* workgroups of the persistent CG kernel (0: auto)     */
  int32_t trace_len;      /* iterations recorded by gs_trace (workspace grows)    */
  double adj_tol;         /* adjoint stop: max|d mu| <= adj_tol max|mu| per mesh  */
  int32_t adj_max_iter;   /* adjoint iteration cap                                */
  int32_t adj_aa_m;       /* Anderson memory of the adjoint iteration, 0..16 (0:
                             plain fixed-point iteration); the workspace holds
                             the value given at gs_create                         */
  int32_t aa_m;           /* Anderson memory of the local/global iteration, 0..16
                             (0: the plain iteration; end of Section III-B); the
                             workspace holds max(aa_m, adj_aa_m) given at
                             gs_create, a later larger value is clamped to it     */
  int32_t aa_guard;       /* tests an accelerated point must pass (GS_AA_GUARD_*) */
  double aa_slack;        /* relative slack of that test                          */
  double barrier_timeout_ms; /* bound on one wait of the CG kernel's grid barrier;
                             a workgroup that waits longer gives up and the call
                             returns GS_EHIP (0: give up at the first wait)      */
  double pcg_eta_min;     /* 0: the inner CG stops at pcg_eta; else iteration k's
                             solve stops at min(pcg_eta, max(r_{k-1}, pcg_eta_min))
                             (loose far from the fixed point, tighter near it;
                             the accelerated iteration needs accurate steps
                             where the map contracts slowly); r is the
                             adjoint's residual in gs_adjoint; the unrolled
                             sweep's solves always stop at pcg_eta               */
  int32_t pcg_coarse;     /* 1: the global step's CG adds a coarse correction to
                             its Jacobi preconditioner (one unknown per CG
                             workgroup's row range, its matrix from A_el; one
                             mesh, rows-of-three-vectors kernel variant, at
                             most 256 workgroups); 0 (default): Jacobi alone */
  int32_t pcg_per_mesh;   /* a batch (M > 1) only.  1 or 2: the global step's
                             CG runs on each mesh's own workgroups (the plan
                             gs_cg_plan reports), each mesh with its own
                             scalars, stopping test and iteration count (a
                             mesh's iterations and positions are those of
                             solving it alone with as many CG workgroups);
                             1 shares the budget pcg_blocks by rows, 2 plans
                             by longest processing time (see gs_cg_plan).
                             0 (default): one CG over the whole batch's rows
                             with per-mesh warm starts and a shared stopping
                             test.  Ignored for one mesh.                   */
  int32_t graph;          /* 1: gs_solve runs each chunk of check_every outer
                             iterations after the first as one HIP graph
                             launch (the chunk's kernels, captured once and
                             kept while the problem, its binding and its
                             parameters stay the same), when every kernel of
                             the iteration takes an ordinary launch and
                             profiling is off.  Results are the same as with
                             0 (default): each kernel launched on its own.  */
  int32_t pcg_store;      /* how the CG kernel stores the state other
                             workgroups read after a barrier: 1 written
                             through to memory (the barrier's release then
                             has little to write back: best while the state
                             is cache-resident and the iteration waits on
                             the barrier), 2 through L2 (a row record's
                             vectors merge into whole lines: fewer HBM writes
                             when the iteration is bound by memory traffic),
                             0 (default): 2 above 700,000 rows, else 1.
                             Results are the same either way.              */
} gs_params;

/* Safeguards of the accelerated iteration.  Every iteration evaluates the
 * plain map at the current point x_k: collision, local step and global step
 * give G(x_k), the active set A_k, the residual r_k = max_v |G(x_k)_v -
 * x_k,v| / diag and the energy E_k of Eq. (9).  An accelerated point that
 * fails the test is rejected: the next point is the plain step from the last
 * accepted point, taken with that point's active set (so a rejection leaves
 * exactly the plain iteration's state behind), and the Anderson history is
 * cleared.  aa_guard is one of
 *   RESIDUAL  reject when r_k > (1 + aa_slack) r_acc (r_acc: residual at the
 *             last accepted point);
 *   ENERGY    reject when E_k > E_acc + aa_slack |E_acc| (one mesh only; Eq. 9
 *             decreases along plain steps only with as-rigid-as-possible
 *             body targets, hyperelastic = 0);
 *   NONE      no value test;
 * optionally or-ed with
 *   SET       also reject when A_k differs from the last accepted point's
 *             set (an accelerated step may not create or release contacts:
 *             the active set evolves along plain steps only).
 * An accepted point whose set changed clears the history (the map changed). */
enum { GS_AA_GUARD_NONE = 0, GS_AA_GUARD_RESIDUAL = 1, GS_AA_GUARD_ENERGY = 2, GS_AA_GUARD_SET = 4 };

typedef struct {
  int32_t iters;           /* outer iterations run                                */
  int32_t pcg_iters_total; /* inner CG iterations summed over the solve           */
  int32_t n_contacts;      /* active springs after the last iteration             */
  int32_t ray_miss;        /* penetrating vertices whose ray found no boundary    */
  double residual;         /* r_k of the last iteration                           */
  double energy;           /* Eq. (9) at x_k with the last targets                */
  int32_t aa_rejected;     /* accelerated points rejected by the safeguard        */
  int32_t pad;
} gs_stats;

/* Sizes derived by gs_create (set-up step). */
typedef struct {
  int32_t n_verts, n_tets, n_surface_faces, n_surface_verts, n_query_verts, nnz;
  int32_t n_slots;         /* contact slots per query vertex: 1 + spheres + planes */
  int32_t hash_buckets;
  double h_ref, eps_off, ray_len, bbox_diag, cell_size;
  int32_t ell_width;       /* off-diagonal slots per row of the stored matrix      */
  int32_t pcg_grid;        /* workgroups of the CG kernel (0 before gs_bind)       */
} gs_info;

typedef struct gs_problem gs_problem;

int32_t gs_version(void);
const char* gs_last_error(void);

/* Defaults: Ecoflex 00-30 (c1 = 0.0418, c2 = 0.0106 MPa), hyperelastic on,
 * kappa_col 1, eps_rel 0.05, ray_rel 4, no collision, tol 1e-6,
 * max_iter 20000, fixed_iters 0, pcg_eta 1e-3, pcg_max 200, check_every 16,
 * pcg_blocks 0, trace_len 0, adj_tol 1e-6, adj_max_iter 20000, adj_aa_m 16,
 * aa_m 8, aa_guard GS_AA_GUARD_RESIDUAL | GS_AA_GUARD_SET, aa_slack 0.5,
 * barrier_timeout_ms 2000, pcg_eta_min 0. */
void gs_default_params(gs_params* params);

/* Host set-up for one mesh (done once per mesh; not per iteration): orient
 * tets to positive rest volume (swapping slots 2 and 3 of negative ones),
 * rest shapes and weights omega_e = Vol(e)/mean Vol (Eq. 9), boundary faces
 * (faces of exactly one tet, outward), query vertices (non-fixed boundary
 * vertices), A_el = sum_e omega_e S_e^T N S_e with N = I - 11^T/4 (below
 * Eq. 1) with fixed rows/columns removed (kept in ELL form), h_ref (mean rest edge
 * length), eps = eps_rel h_ref, L_ray = ray_rel h_ref and the spatial-hash
 * geometry.  Errors: GS_EINVAL, GS_EDEGENERATE.  *out is owned by the caller
 * and released with gs_destroy. */
gs_status gs_create(const gs_mesh_desc* mesh, const gs_params* params, gs_problem** out);

/* Batch of meshes solved together (one problem): the arrays of all calls are
 * the meshes' arrays concatenated in order (positions [3][sum n], alpha
 * [sum n_chambers]); chamber ids, vertex ids and boundary-face ids are offset
 * per mesh; there are no contacts between meshes.  Each mesh keeps its own
 * h_ref, eps, L_ray, weights and residual scale (its bounding-box diagonal);
 * in a convergence solve a mesh whose r_k <= tol with an unchanged active set
 * is frozen (its correction is zero from then on) and the solve ends when
 * every mesh is frozen.  All meshes share one precision.  Errors as
 * gs_create, prefixed with the mesh number. */
gs_status gs_create_batch(int32_t n_mesh, const gs_mesh_desc* meshes, const gs_params* params,
                          gs_problem** out);

/* Offsets of mesh m's vertices, tets and chambers in the concatenated arrays:
 * entries m and m + 1 of each array (cap >= n_mesh + 1).  A single mesh is a
 * batch of one. */
gs_status gs_batch_layout(const gs_problem* p, int32_t cap, int32_t* vert_offset,
                          int32_t* tet_offset, int32_t* chamber_offset, int32_t* n_mesh);

/* Iteration at which each mesh of the last convergence solve converged (0:
 * did not converge), cap >= n_mesh. */
gs_status gs_mesh_iters(gs_problem* p, int32_t cap, int32_t* iters);

/* Analytic obstacles O_obs (Eq. 4): n_sph spheres (cx, cy, cz, r) and n_pln
 * half-spaces (px, py, pz, nx, ny, nz) whose inside is n.(x - p) < 0 (the
 * normal is normalised here).  Must be called before gs_bind.  GS_EINVAL for
 * r <= 0, a zero normal or non-finite values. */
gs_status gs_set_obstacles(gs_problem* p, int32_t n_sph, const double* sph, int32_t n_pln,
                           const double* pln);

/* A closed, outward-oriented triangle-mesh obstacle (Section II-B, the
 * obstacle term of Eq. 4; Section II-C): verts [3][n_verts] (host, FP64),
 * tris [3][n_tris] (host, vertex ids; every edge shared by exactly two
 * triangles).  Copied; must be called before gs_bind; n_tris = 0 removes it.
 * With obstacle_collision on, every query vertex inside the obstacle's box
 * or holding a contact with it is tested against its closest point c on the
 * mesh (smallest squared distance, ties to the lowest triangle id; found by
 * a tree built here over the triangles): it is inside when (x - c) . psi < 0,
 * psi the angle-weighted pseudonormal of the face, edge or vertex c lies on;
 * the spring target is c + eps_off u and the contact normal u, u the outward
 * unit direction ((x - c)/|x - c| outside, (c - x)/|x - c| inside, psi on
 * the surface), recomputed at every check; the release rule is Eq. 8's.
 * Contacts with it are listed with type GS_CONTACT_MESH and the triangle id
 * as prim, in the last slot.  Gradients (gs_adjoint, gs_adjoint_unrolled)
 * refuse a problem whose mesh obstacle is on.  GS_EINVAL for non-finite
 * vertices, bad indices, a degenerate triangle or an open mesh. */
gs_status gs_set_mesh_obstacle(gs_problem* p, int32_t n_verts, const double* verts, int32_t n_tris,
                               const int32_t* tris);

gs_status gs_info_get(const gs_problem* p, gs_info* info);

/* Bytes of device workspace gs_bind needs (256-byte aligned start). */
gs_status gs_workspace_size(const gs_problem* p, size_t* bytes);

/* Attach a workspace and a stream, and upload the static data.  The
 * workspace must stay valid until gs_destroy or the next gs_bind.
 * Errors: GS_EINVAL (null/small/misaligned workspace), GS_EHIP. */
gs_status gs_bind(gs_problem* p, void* dev_workspace, size_t bytes, void* hip_stream);

/* Replace the solver constants (c1, c2, tolerances, collision switches,
 * iteration limits).  Obstacles and mesh stay.  GS_EINVAL on bad values. */
gs_status gs_set_params(gs_problem* p, const gs_params* params);

/* Solve (Section III-B, inner loop of Algorithm 1): iterate from dev_x (warm
 * start; fixed vertices are reset to X0) and the stored active contact set
 * (empty after gs_bind, or the set left by the previous solve /
 * gs_set_contacts), for the per-chamber volume ratios dev_alpha[n_chambers],
 * until r_k <= tol with the active set unchanged, or exactly fixed_iters
 * iterations.  Each iteration evaluates the plain local/global map G at the
 * current point x_k (collision check and response, local step, global step),
 * r_k = max_v |G(x_k)_v - x_k,v| / bbox diagonal.  With aa_m = 0 the next
 * point is G(x_k); with aa_m > 0 it is the Anderson point (Walker & Ni 2011)
 * built from the last aa_m accepted points and residuals, or, when the
 * guard (aa_guard) rejects x_k, the plain step from the last accepted point;
 * the history is cleared whenever the active set changes.  Either way the
 * result is G(x_k) of the last iteration, and the stopping rule is the plain
 * iteration's.  In a batch each mesh has its own history and decisions.
 * dev_x [3][n] receives the result.  Returns GS_OK, GS_NOT_CONVERGED (last
 * iterate written), GS_EBREAKDOWN, GS_ESTATE (not bound), GS_EINVAL (null
 * pointers), GS_EHIP (also when a grid barrier gave up, see
 * barrier_timeout_ms).  stats may be NULL. */
gs_status gs_solve(gs_problem* p, const void* dev_alpha, void* dev_x, gs_stats* stats);

/* Forget the stored active contact set (the next solve starts from none). */
gs_status gs_reset_contacts(gs_problem* p);

/* Copy out the stored active set sorted by (vertex, type, prim): prim is the
 * hit boundary-face id for self contacts and the obstacle index otherwise;
 * target/normal are [cap][3] (x,y,z per row); fresh[i] is 1 for a self
 * contact whose target was recomputed from the current positions in the
 * last collision check (its vertex penetrates and its ray hit prim), 0 for
 * one kept with its stored target (Eq. 8) and for obstacle contacts.  Any
 * output pointer may be NULL.  *count receives the number of contacts;
 * GS_ECAPACITY if it exceeds cap (nothing else written). */
gs_status gs_contacts(gs_problem* p, int32_t cap, int32_t* v, int32_t* type, int32_t* prim,
                      double* target, double* normal, int32_t* fresh, int32_t* count);

/* Import an active set (for resuming a solve, or to fix the state an adjoint
 * linearises).  Rows as gs_contacts gives them (fresh may be NULL: all 0); at
 * most one contact per (vertex, type, prim) slot.  GS_EINVAL for a vertex
 * that is not a query vertex, an out-of-range prim, or fresh set on an
 * obstacle contact. */
gs_status gs_set_contacts(gs_problem* p, int32_t count, const int32_t* v, const int32_t* type,
                          const int32_t* prim, const double* target, const double* normal,
                          const int32_t* fresh);

/* Unrolled adjoint over a fixed iteration budget (the differentiable form of
 * a K-iteration solve; not in the paper).  Runs K local/global iterations
 * from dev_x0 [3][n] with the stored contact set as the previous one (as
 * gs_solve with fixed_iters = K), then the reverse sweep: with the contact
 * set A_k each iteration found held as recorded (new self-contact targets
 * follow x_k, kept ones are constants, obstacle targets follow x_k),
 * x_{k+1} = M_k^-1 b_k(x_k, alpha) is differentiated exactly:
 *   lambda_K = g;  for k = K-1..0:  nu = M_k^-1 lambda_{k+1},
 *   dL/dalpha += (db_k/dalpha)^T nu,  lambda_k = (db_k/dx_k)^T nu.
 * Each M_k^-1 is the solve's CG (pcg_eta / pcg_max apply; a small pcg_eta
 * keeps the forward path close to exact global steps).  States are
 * checkpointed every ceil(sqrt(K)) iterations in dev_scratch (caller-owned,
 * 256-byte aligned, gs_unrolled_scratch_size(p, K) bytes) and each segment
 * is recomputed once.  Outputs (device, problem width): dev_dLdalpha
 * [n_chambers]; dev_dLdx0 [3][n] = lambda_0 (may be NULL); dev_xK [3][n]
 * the positions after K iterations (may be NULL).  The stored contact set
 * afterwards is the one the K-th iteration found, as after gs_solve.
 * stats (may be NULL): iters = K, pcg_iters_total = forward + reverse CG
 * iterations, residual / energy of the last forward iteration.  Errors:
 * GS_EINVAL (bad sizes, null or small scratch), GS_ESTATE, GS_EBREAKDOWN,
 * GS_EHIP.  The implicit adjoint state of an earlier gs_solve is discarded. */
size_t gs_unrolled_scratch_size(const gs_problem* p, int32_t K);
gs_status gs_adjoint_unrolled(gs_problem* p, const void* dev_alpha, const void* dev_x0, int32_t K,
                              const void* dev_dLdx, void* dev_dLdalpha, void* dev_dLdx0, void* dev_xK,
                              void* dev_scratch, size_t scratch_bytes, gs_stats* stats);

/* Choose the CG kernel's grid for this problem: times `iters` fixed
 * iterations from dev_x (with the stored contact set) for the default grid
 * (about 256 rows per block) and every grid of 2^k or 3 x 2^k workgroups
 * that can be resident, keeps the fastest in params.pcg_blocks, and restores dev_x and
 * the stored contact set.  *chosen (may be NULL) receives the grid,
 * *ms_per_iter (may be NULL) its time per outer iteration.  With
 * pcg_per_mesh on a batch the candidates are budgets the per-mesh plan
 * shares out (gs_cg_plan), and *chosen is the budget kept.  Errors as
 * gs_solve; the last solve's adjoint state is discarded (gs_adjoint then
 * needs a new gs_solve). */
gs_status gs_autotune(gs_problem* p, const void* dev_alpha, void* dev_x, int32_t iters, int32_t* chosen,
                      double* ms_per_iter);

/* The per-mesh CG plan of a bound batch (params.pcg_per_mesh = 1 or 2,
 * M > 1): blocks[m] (host array of M int32, caller-owned) receives the
 * number of CG workgroups mesh m gets.  A mesh's global step (Eq. 8's linear
 * system, one per mesh) is then solved as a solve of that mesh alone with
 * pcg_blocks = blocks[m] would solve it.  With 1 the plan gives each mesh one
 * workgroup plus its share, by rows, of the budget (pcg_blocks, else the
 * workgroups that can be resident at once) beyond one per mesh; all of them
 * fit on the device at once.  With 2 (longest processing time) every
 * workgroup gets about (all rows) / budget rows, so a large mesh is split and
 * a small one keeps one workgroup; the grid may exceed what can be resident,
 * the split meshes come first in block order within half the resident
 * capacity, and the single-workgroup meshes follow largest first, the
 * smallest queueing for the workgroups that finish first.  Either way at
 * most one workgroup per 512 rows.  Without the per-mesh CG every entry is
 * 1.  GS_EINVAL for a null argument or M other than the problem's mesh
 * count; GS_ESTATE before gs_bind. */
gs_status gs_cg_plan(const gs_problem* p, int32_t M, int32_t* blocks);

/* Implicit adjoint of the last gs_solve (not in the paper: the gradient of
 * its fixed point).  At the positions x the solve returned, with the stored
 * active set held fixed and the volume ratios alpha of that solve, the free
 * coordinates satisfy M_FF x_F = b_F(x, alpha) - M_FC x_C (M = A_el +
 * springs, b = element targets of Section III-A plus spring targets of
 * Section II-C); for dev_dLdx [3][n] = dL/dx this computes
 *   dev_dLdalpha[n_chambers] = (db_F/dalpha)^T mu,  (M_FF - db_F/dx_F)^T mu = g_F
 * by the iteration mu <- M^-1 (g + (db/dx)^T mu) in correction form (same CG
 * as the solve, pcg_eta / pcg_max apply), with Anderson acceleration of
 * memory adj_aa_m (Walker & Ni 2011) when it is > 0, until
 * max|d mu| <= adj_tol max|mu| (d the correction of the last iteration; per
 * mesh, and on every mesh at once when accelerated) or adj_max_iter
 * iterations.  Self contacts flagged fresh
 * (gs_contacts) follow x through the ray target; kept self contacts are
 * constant; obstacle targets follow x in closed form.  dev_mu [3][n] (may be
 * NULL) receives mu (zero on fixed vertices).  Both outputs use the
 * problem's width.  stats (may be NULL): iters = adjoint iterations,
 * pcg_iters_total, residual = the largest max|d mu| / max|mu|.  Returns
 * GS_OK, GS_NOT_CONVERGED (gradient of the last iterate written),
 * GS_ESTATE (no solve since gs_bind), GS_EINVAL, GS_EBREAKDOWN, GS_EHIP. */
gs_status gs_adjoint(gs_problem* p, const void* dev_dLdx, void* dev_dLdalpha, void* dev_mu, gs_stats* stats);

/* Local step alone (Section III-A) at positions dev_x [3][n]: writes the
 * centred target shapes to dev_targets [3][4][T] (row c, tet slot j, tet e
 * at ((c*4 + j) * T + e)); slots follow the oriented tets (gs_tets). */
gs_status gs_local_step_debug(gs_problem* p, const void* dev_x, const void* dev_alpha,
                              void* dev_targets);

/* Oriented tets [4][T] as used internally (host copy). */
gs_status gs_tets(const gs_problem* p, int32_t* tets);
/* Outward boundary faces [3][F] in their id order (host copy). */
gs_status gs_faces(const gs_problem* p, int32_t* faces);

/* Device scratch bytes gs_collide_debug needs for a candidate capacity cap. */
size_t gs_collide_debug_scratch(int32_t cap);

/* One collision check (Section II-B/II-C) at positions dev_x [3][n] given the
 * stored active set as A_{k-1}; the stored set is not modified.  dev_scratch
 * (gs_collide_debug_scratch(cap) bytes, caller-owned device memory) stages
 * the candidate lists.  Outputs (host, each sorted ascending and free of
 * duplicates; row r of a [m][cap] array is at r * cap):
 *   cand_tet [2][cap]   (v, e) with v a query vertex not in e and x_v inside
 *                       the min/max box of e (inclusive)
 *   cand_tri [2][cap]   (v, f) for penetrating v: f a boundary face not
 *                       containing v whose box meets the box of the segment
 *                       [x_v, x_v - L_ray n_v]
 *   contacts [3][cap]   (v, type, prim) of the resulting active set, with
 *                       target [3][cap]
 * and the counts.  GS_ECAPACITY if any count exceeds cap (counts still set). */
gs_status gs_collide_debug(gs_problem* p, const void* dev_x, int32_t cap, void* dev_scratch,
                           size_t scratch_bytes, int32_t* cand_tet, int32_t* n_cand_tet,
                           int32_t* cand_tri, int32_t* n_cand_tri, int32_t* contacts,
                           double* target, int32_t* n_contacts);

/* gs_collide_debug for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * allocation): the candidate lists are staged in a static device array of
 * the library (GS_STATIC_CAND_CAP pairs per list, 2 MiB per device, held by
 * each device the library runs on until the process ends) instead of a
 * caller scratch; nothing is allocated.  Arguments and outputs as
 * gs_collide_debug; GS_EINVAL when cap > GS_STATIC_CAND_CAP, GS_ESTATE when
 * not bound.  Calls on one device share the array: calls that overlap on one
 * device race. */
#define GS_STATIC_CAND_CAP 131072
gs_status gs_collide_debug_static(gs_problem* p, const void* dev_x, int32_t cap, int32_t* cand_tet,
                                  int32_t* n_cand_tet, int32_t* cand_tri, int32_t* n_cand_tri,
                                  int32_t* contacts, double* target, int32_t* n_contacts);

/* Self-collision broadphase by a refit-only AABB tree over the tets
 * (Section II-B: the tree keeps its structure through the deformation and
 * only its boxes follow the positions).  The topology is built once, on the
 * first call, by median splits of the rest centroids (at most 4 tets per
 * leaf); every call refits the boxes to dev_x ([3][n], exact min/max of the
 * FP64 positions, bottom-up one depth per launch) and walks it for every
 * query vertex, returning C_tet = {(v, e): v not a vertex of e, lo_e <= x_v
 * <= hi_e}, the same set as the spatial hash the solver uses (see
 * gs_collide_debug).  cand [2][cap] (host) receives the pairs sorted by
 * (v, e), *n_cand their number (GS_ECAPACITY when above cap, pairs not
 * written); ms_refit / ms_query (may be NULL) the two phases' device times.
 * dev_scratch holds gs_tree_candidates_scratch(p, cap) bytes (caller-owned).
 * Problems of one mesh only.  Synchronises the bound stream. */
size_t gs_tree_candidates_scratch(const gs_problem* p, int32_t cap);
gs_status gs_tree_candidates(gs_problem* p, const void* dev_x, int32_t cap, void* dev_scratch, size_t scratch_bytes,
                             int32_t* cand, int32_t* n_cand, double* ms_refit, double* ms_query);

/* Per-iteration trace of the last solve: rows of GS_TRACE_COLS doubles
 * (r_k, E_k, active springs, set changed, inner CG iterations, ray misses)
 * for the first min(iters, trace_len) iterations; trace_len is fixed at
 * gs_create.  *count receives the number of rows written (<= cap). */
#define GS_TRACE_COLS 6
gs_status gs_trace(gs_problem* p, int32_t cap, double* rows, int32_t* count);

/* Remesh checks (Section III-B; the check that follows each stage of
 * Algorithm 1's outer loop).  For every chamber element (M_c) at positions
 * dev_x ([3][n], the precision of the problem) against the reference
 * positions dev_x_ref (same layout; NULL: the rest shape X0, i.e. the mesh
 * as last meshed), with D the three edges from the element's first vertex
 * and F = D_x D_ref^-1:
 *   GS_REMESH_VOLUME      det(D_x) / det(D_ref) > alpha_max (volume gain);
 *   GS_REMESH_DISTORTION  norm(Sigma) > d_max, Sigma the singular values of
 *                         the affine map taking the deformed element back to
 *                         the reference (F^-1), norm the 2-norm, so
 *                         norm(Sigma) = 1 / sigma_min(F) (infinite for a
 *                         flattened element).
 * Both decisions are taken in FP64.  dev_flags (device, one byte per tet in
 * the order of gs_tets, caller-owned) receives the or-ed bits, 0 for body
 * elements; *n_flagged (host, may be NULL) the number of elements with a bit
 * set.  The paper uses alpha_max = d_max = 4.  Synchronises the bound stream.
 * GS_EINVAL for null buffers or thresholds that are not finite and > 0,
 * GS_ESTATE before gs_bind, GS_EHIP. */
enum { GS_REMESH_VOLUME = 1, GS_REMESH_DISTORTION = 2 };
gs_status gs_remesh_flags(gs_problem* p, const void* dev_x, const void* dev_x_ref, double alpha_max, double d_max,
                          uint8_t* dev_flags, int32_t* n_flagged);

/* One stage of gs_solve_progressive. */
typedef struct {
  gs_stats solve;          /* the stage's solve                                  */
  int32_t status;          /* its status: GS_OK or GS_NOT_CONVERGED              */
  int32_t n_flagged;       /* elements flagged by the remesh checks after it     */
  double alpha_top;        /* the stage's largest per-chamber actuation          */
} gs_stage;

/* Progressive actuation (Algorithm 1's outer loop, without the remesher):
 * stage k = 0, 1, ... solves (gs_solve, warm-started from the previous
 * stage's positions in dev_x and its active contact set) with the
 * per-chamber actuation alpha_k = min(alpha, (k+1) alpha_max), rounded to
 * the problem's precision, then runs gs_remesh_flags against the rest shape
 * into dev_flags.  The last stage is the first whose actuation reaches
 * dev_alpha in every chamber (one stage when alpha <= alpha_max).  With
 * stop_on_flag != 0 the loop ends after the first stage that flags an
 * element: remeshing is the caller's (a new problem on the new mesh, from the
 * returned positions).  stages[cap] (host) receives one record per stage run
 * and *n_stages their number.  Returns GS_OK when every stage converged,
 * GS_NOT_CONVERGED when one did not (later stages still run), GS_EINVAL for
 * null buffers, non-finite alpha, thresholds that are not finite and > 0 or
 * cap below the number of stages, and any error of gs_solve. */
gs_status gs_solve_progressive(gs_problem* p, const void* dev_alpha, void* dev_x, double alpha_max, double d_max,
                               int32_t stop_on_flag, uint8_t* dev_flags, int32_t cap, gs_stage* stages,
                               int32_t* n_stages);

/* Kernel timing.  gs_profile(p, 1) resets the totals and brackets every
 * kernel that gs_solve launches with a pair of HIP events on the bound
 * stream (gs_adjoint likewise: its kernels are named "adj_*");
 * gs_profile_read returns, per kernel id k < GS_N_KERNELS, the summed
 * duration in milliseconds and the number of launches; gs_kernel_name(k)
 * names the kernel ("pcg", "local", ...); the CG kernel also applies the
 * correction and takes the convergence decision.  Fused launches are counted
 * under one name: "pcg" also updates the contact set and gathers the
 * right-hand side ("contacts" and "gather" count no launches in a solve);
 * with self-collision on a mesh below 2^18 tets, "tet_query" includes the
 * local step ("local" then counts none); "hash_insert" runs only on a solve's
 * first iteration (the CG kernel refills the hash, or, with aa_m > 0, the
 * accelerated iteration's position update); "anderson" is that update with
 * its dot products and least-squares solve (three launches counted as one);
 * "remesh_flags" is gs_remesh_flags (two launches: the count is cleared
 * first); "mesh_obstacle" the closest-point search of the triangle-mesh
 * obstacle.  gs_profile(p, 0) stops. */
#define GS_N_KERNELS 14
gs_status gs_profile(gs_problem* p, int32_t enable);
gs_status gs_profile_read(const gs_problem* p, double* ms, int64_t* launches);
const char* gs_kernel_name(int32_t k);

void gs_destroy(gs_problem* p);

#ifdef __cplusplus
}
#endif

#endif /* GEOSIM_H */
