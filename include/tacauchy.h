/*
 * tacauchy.h - C ABI of the MI355X tactile-FEM hot path.
 *
 * One implicit time step of a tetrahedral Stable Neo-Hookean gel pad pressed
 * by rigid indenters, followed by Cauchy stress and surface traction
 * extraction (TaCauchy, Sec. III-B/C, Alg. 1 and Alg. 2):
 *
 *   physics   minimise the incremental potential
 *               E(x) = 1/2 |x - xhat|_M^2 + dt^2 [ sum_e V_e Psi(F_e) + E_b(x) ]
 *             (Psi: energy density whose derivative is the first Piola stress
 *             of Eq. 2; E_b: IPC log barrier with threshold d_hat, Sec. III-B)
 *             by Newton with a matrix-free-assembled, block-Jacobi
 *             preconditioned CG solve and backtracking line search;
 *   stress    per tet sigma = J^-1 P F^T = (mu/J) F F^T + lambda (J - alpha) I
 *             (Eq. 3 and Eq. 4);
 *   traction  per surface triangle t = sigma n, p_n = t . n, t_tau = t - p_n n
 *             (Alg. 1, Eq. 6-9);
 *   contact   per contact vertex f = -dE_b/dx, normal/tangential split,
 *             pressure |f| / A (Alg. 2).
 *
 * Conventions
 *   - Every call returns tc_status: TC_OK (0) or a negative error code.
 *     tc_last_error() returns a message for the calling thread's last error.
 *   - No call throws; no torch or HIP type appears in a signature.  Device
 *     pointers are plain void* into memory of the context's device.
 *   - Units: metres, seconds, kilograms, pascals, newtons.
 *   - Arrays are row-major; [N][3] means N consecutive xyz triples.
 *   - Every input array is copied; the caller keeps ownership of its memory.
 *   - Entry points marked "host only" touch no GPU and may run on a machine
 *     without one.  All others need a context on an MI355X (gfx950).
 *   - Calls on one context are not thread-safe with respect to each other,
 *     except tc_server_submit / tc_server_poll, which may be called from any
 *     thread while the server's own thread drives the device.
 */
#ifndef TACAUCHY_H
#define TACAUCHY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef int32_t tc_status;
#define TC_OK               0
#define TC_E_INVALID_ARG   -1  /* null pointer, bad size, value out of range */
#define TC_E_BAD_MESH      -2  /* index out of range, non-positive tet volume */
#define TC_E_NO_MEMORY     -3  /* HBM budget exceeded or allocation failed */
#define TC_E_HIP           -4  /* HIP runtime error (message has details) */
#define TC_E_INFEASIBLE    -5  /* indenter pose leaves no feasible start */
#define TC_E_NOT_CONVERGED -6  /* Newton hit max_newton iterations */
#define TC_E_LINESEARCH    -7  /* no energy decrease within max_halvings */
#define TC_E_NO_DEVICE     -8  /* no usable gfx950 device */
#define TC_E_BUSY          -9  /* pad has a request in flight on a server */

/* ------------------------------------------------------------- constants */
#define TC_PREC_FP64  0   /* every kernel in float64 */
#define TC_PREC_MIXED 1   /* element/assembly/SpMV in float32; positions,
                             residual, dot products, line-search energy and
                             barrier in float64 */

#define TC_PRECOND_BLOCK_JACOBI  0  /* inverse of each vertex's 3x3 diagonal block */
#define TC_PRECOND_JACOBI        1  /* inverse of the scalar diagonal */

/* Indenter shapes (local frame; the solid is where phi < 0):
 *   SPHERE   prm[0] = radius                               phi = |y| - r
 *   CYLINDER prm[0] = radius, prm[1] = half height, axis z
 *   BOX      prm[0..2] = half extents
 *   TORUS    prm[0] = ring radius, prm[1] = tube radius, axis z
 *   TEXTURE  prm[0] = amplitude A, prm[1] = period L: plate occupying
 *            y_z >= A sin(2 pi y_x / L) sin(2 pi y_y / L); phi is the
 *            1-Lipschitz bound (eta - y_z) / sqrt(1 + (2 pi A / L)^2).
 *   MESH     a closed rigid triangle mesh registered with
 *            tc_rigid_mesh_create; tc_indenter.reserved = its id, prm
 *            unused (finite).  phi is the signed distance to its surface. */
#define TC_SPHERE   0
#define TC_CYLINDER 1
#define TC_BOX      2
#define TC_TORUS    3
#define TC_TEXTURE  4
#define TC_MESH     5
#define TC_MAX_MESHES 64     /* rigid meshes per context */

#define TC_MAX_INDENTERS 5   /* per pad and step */
#define TC_MAX_MATERIALS 8   /* per pad */

/* Output / state fields for tc_pad_read (and tc_pad_write where noted).
 * dtype "real" is float64 in TC_PREC_FP64 and float32 in TC_PREC_MIXED;
 * tc_field_info reports it. */
#define TC_F_POSITIONS        0  /* f64 [V][3] committed positions (writable) */
#define TC_F_VELOCITIES       1  /* f64 [V][3] committed velocities (writable) */
#define TC_F_REST             2  /* f64 [V][3] rest positions */
#define TC_F_SIGMA            3  /* real [T][6] Cauchy stress (xx,yy,zz,yz,xz,xy) */
#define TC_F_TRACTION         4  /* real [S][3] t = sigma n per surface triangle */
#define TC_F_PRESSURE         5  /* real [S] p_n = t . n (> 0 tension) */
#define TC_F_TANGENTIAL       6  /* real [S][3] t_tau = t - p_n n */
#define TC_F_TRI_AREA         7  /* real [S] current triangle area */
#define TC_F_TRI_NORMAL       8  /* real [S][3] current unit normal */
#define TC_F_CONTACT_FORCE    9  /* f64 [C][3] f_k = -dE_b/dx_k */
#define TC_F_CONTACT_NORMAL  10  /* f64 [C][3] area-weighted vertex normal */
#define TC_F_CONTACT_AREA    11  /* f64 [C] 1/3 of incident contact-face area
                                     (side-face vertices: of incident surface area) */
#define TC_F_CONTACT_FN      12  /* f64 [C][3] (f . n) n */
#define TC_F_CONTACT_FT      13  /* f64 [C][3] f - f_n */
#define TC_F_CONTACT_PRESSURE 14 /* f64 [C] |f| / A */
#define TC_F_REACTION        15  /* f64 [3] force on the indenters = -sum f_k */
#define TC_F_TRACTION_SUM    16  /* f64 [3] sum over contact-face tris of t A */
#define TC_F_SURFACE_TRIS    17  /* i32 [S][3] outward-wound surface triangles */
#define TC_F_SURFACE_PARENT  18  /* i32 [S] owning tet of each triangle */
#define TC_F_SURFACE_IS_TOP  19  /* u8  [S] 1 = contact face */
#define TC_F_CANDIDATES      20  /* i32 [C] contact vertex ids, ascending */
#define TC_F_CAND_REST_AREA  21  /* f64 [C] barrier weight A_k (rest) */
#define TC_F_MASS            22  /* f64 [V] lumped mass */
#define TC_F_FIXED           23  /* u8  [V] xyz bitmask of fixed components */
#define TC_F_TETS            24  /* i32 [T][4] */
#define TC_F_COUNT           25

#define TC_DT_F64 0
#define TC_DT_F32 1
#define TC_DT_I32 2
#define TC_DT_U8  3

/* ---------------------------------------------------------------- types */
typedef struct tc_context tc_context;
typedef struct tc_pad tc_pad;
typedef struct tc_server tc_server;

/* Tet mesh (Alg. 1 / Alg. 2 input (V, T)). */
typedef struct {
  int32_t n_verts;
  int32_t n_tets;
  const double* rest_xyz;      /* [n_verts][3] host */
  const int32_t* tets;         /* [n_tets][4] host, det(Dm) > 0 */
  const uint8_t* fixed;        /* [n_verts] bit c set = component c fixed;
                                  NULL = the base (minimum along the thinnest
                                  bounding-box axis) fully fixed */
  const int32_t* tet_material; /* [n_tets] index into the material table, or
                                  NULL = material 0 everywhere */
} tc_mesh;

/* Eq. 1 inputs: Young's modulus [Pa] > 0, Poisson ratio in (-1, 0.5),
 * density [kg/m^3] > 0. */
typedef struct {
  double E;
  double nu;
  double density;
} tc_material;

typedef struct {
  double dt;            /* time step [s] > 0 */
  double dhat;          /* barrier threshold d_hat [m] > 0 */
  double kappa;         /* barrier stiffness [Pa] > 0 */
  double newton_tol;    /* converged when |p|_inf <= tol * bbox diagonal */
  double cg_rel_tol;    /* CG stops at sqrt(r.z / r0.z0) <= this */
  int32_t max_newton;   /* Newton cap (1024 in Sec. III-B) */
  int32_t max_cg;       /* CG cap per Newton iteration */
  int32_t quasi_static; /* 1 = drop the inertia term */
  int32_t precision;    /* TC_PREC_* (fixed at pad creation) */
  double gravity[3];    /* [m/s^2], enters xhat = x + dt v + dt^2 g */
  int32_t literal_alpha;/* 1 = rest shift alpha = 1 exactly as Eq. 2 prints */
  int32_t precond;      /* TC_PRECOND_* */
  int32_t max_halvings; /* line-search halvings before TC_E_LINESEARCH */
  int32_t cg_forcing;   /* 0: CG to cg_rel_tol every Newton iteration;
                           1: adaptive forcing within [cg_rel_tol,
                           cg_eta_max]: Eisenstat-Walker eta_k = 0.9 (|g_k| /
                           |g_k-1|)^2 (preconditioned norms, safeguarded)
                           while the gradient falls by 2x or more per
                           iteration, eta_k = eta_k-1 / 4 otherwise;
                           2: Eisenstat-Walker choice 2 throughout (slow
                           Newton progress keeps the solve loose) */
  int32_t hess_proj;    /* Hessian filters.  Bits 0-1, element eigenvalues:
                           0 clamp negatives to 0, 1 absolute value, 2 clamp
                           until a full Newton step is accepted, then the
                           unfiltered Hessian (CG stops at negative
                           curvature; a breakdown reverts to clamping for the
                           rest of the step).  Bits 2-3, barrier 3x3: 0 clamp,
                           1 unfiltered, 2 normal term only, 3 clamp until a
                           full Newton step is accepted, then unfiltered.  In
                           every mode a CG breakdown (negative curvature)
                           never counts as convergence: its iterate is used
                           as a descent direction, the element Hessians are
                           clamped for the rest of the step, and so are the
                           barrier Hessians once a breakdown leaves a zero
                           iterate or happens a second time. */
  int32_t init_guess;   /* Newton start: 0 = x_t, 1 = x_t + dt v_t (free
                           components); either is then made feasible */
  double cg_conv_tol;   /* CG tolerance of the direction on which Newton
                           convergence is accepted (0 = cg_rel_tol) */
  double cg_eta_max;    /* largest forcing term (first Newton iteration) */
  int32_t ls_expand;    /* after a full Newton step passes the line search,
                           up to this many doublings of the step while the
                           energy keeps falling (within the collision-free
                           bound); 0 = off.  Same minimiser, fewer
                           iterations where the filtered Hessian is stiffer
                           than the energy along the direction.  In the
                           other case (a full step that passes with much
                           less decrease than the model predicts, the
                           energy curving up at least 1.4 times as fast
                           along the direction) the minimum of the
                           quadratic through E(0), g.d and E(1) is tried
                           instead, whatever ls_expand. */
  int32_t mesh_contact; /* rigid meshes (TC_MESH): 0 = barrier of the
                           distance to the whole surface, b(phi / d_hat);
                           1 = barrier summed over the mesh's triangles
                           nearer than d_hat, sum_t b(d_t / d_hat) (IPC's
                           point-triangle pairs, Sec. III-B).  The distance
                           to a whole non-convex mesh has a kink on the
                           bisector plane of every concave edge, where
                           Newton can stall; each d_t is C1 off its
                           triangle.  A point near an edge or a vertex
                           counts once per triangle in reach.  The step
                           bound and the feasible start use phi in both
                           modes.  With friction, mode 1 lags lambda n =
                           -kappa A sum_t b'(d_t / d_hat) grad d_t (lambda
                           its length, n its direction).  2 = mode 1
                           plus the pairs whose pad side is a surface
                           triangle or edge (IPC's other primitives, Sec.
                           III-B): every mesh vertex y against every pad
                           surface triangle t, kappa a_y d_hat b(d / d_hat)
                           with a_y a third of the area of y's mesh
                           triangles; every mesh edge e against every pad
                           surface edge f, kappa (|e| |f|_0 / 4) d_hat m(c)
                           b(d / d_hat) with IPC's mollifier m(c) = (2 -
                           c/c0) c/c0 below c0 = 1e-3 |e|^2 |f|_0^2 (1
                           above), c = |e x f|^2 (|f|_0 the rest length);
                           d the distance between the closed features.
                           Their Hessians are Gauss-Newton (PSD); their
                           step bound is alpha <= 0.9 d / max |p| over the
                           pad feature's vertices; the feasible start also
                           pushes a pad triangle or edge that a mesh vertex
                           or edge came through (within the mesh's travel
                           since the previous pose plus d_hat) back along
                           its outward normal, and fails with
                           TC_E_INFEASIBLE if one stays through.  A mesh
                           corner or edge pressed between pad vertices is
                           then seen.  Friction takes the pad-vertex pairs
                           only.  Analytic shapes ignore it. */
  double friction;      /* friction ratio mu >= 0 of the lagged smoothed
                           Coulomb friction against the indenters (Sec.
                           III-B: 0.5); 0 = frictionless.  Per contact
                           vertex k and indenter m, at the step start (x_t
                           and the previous poses): normal force lambda =
                           -kappa A_k b'(d/d_hat), normal n = grad(phi);
                           the indenter point at x_t moves by w = R R_prev^T
                           (x_t - c_prev) + c - x_t.  The step potential gains
                           dt^2 mu sum lambda f0(|u|), u = (I - n n^T)((x -
                           x_t) - w), f0 the C1 cubic/linear mollifier with
                           threshold eps_v dt.  Previous poses: those of the
                           pad's last completed step when it had as many
                           indenters, else the step's own (w = 0). */
  double eps_v;         /* friction velocity threshold [m/s] > 0 (Sec.
                           III-B: 0.01) */
  int32_t cg_warm;      /* 1: from the second Newton iteration of a step on,
                           CG starts from the best multiple of the previous
                           Newton direction, gamma d_prev with gamma =
                           -g.d_prev / d_prev.H d_prev (one extra product,
                           skipped when d_prev.H d_prev <= 0), instead of
                           0; its stopping test stays relative to the cold
                           start's r0.z0.  Where Newton converges linearly
                           along a slowly turning direction, that start
                           already meets the CG tolerance.  0 = cold start. */
  int32_t reserved0;    /* 0 */
} tc_params;

/* Rigid indenter pose at the end of the step: world x = R y + c. */
typedef struct {
  int32_t shape;        /* TC_SPHERE ... TC_MESH */
  int32_t reserved;     /* TC_MESH: mesh id; otherwise 0 */
  double R[9];          /* row-major rotation, orthonormal to 1e-9, det +1 */
  double c[3];          /* centre [m] */
  double prm[4];        /* shape parameters [m], see TC_SPHERE ... */
} tc_indenter;

typedef struct {
  int32_t status;          /* TC_OK or the step's error */
  int32_t newton_iters;
  int32_t cg_iters;        /* summed over Newton iterations */
  int32_t ls_halvings;     /* summed over Newton iterations */
  double final_step_inf;   /* |p|_inf of the last Newton direction [m] */
  double energy;           /* E at the accepted state [J] */
  double reaction[3];      /* force on the indenters [N] */
  double ms;               /* wall time of the call [ms] */
} tc_step_stats;

typedef struct {
  int32_t n_verts, n_tets, n_surface_tris, n_top_tris, n_candidates;
  int32_t ell_width;       /* stored blocks per matrix row */
  int32_t precision;
  int32_t n_materials;
  uint64_t resident_bytes; /* HBM held while the pad exists */
  uint64_t scratch_bytes;  /* HBM needed while a step runs */
  double bbox_diag;        /* [m] */
} tc_pad_info;

/* ---------------------------------------------------- host-only helpers */
const char* tc_version(void);                 /* host only */
const char* tc_status_string(tc_status s);    /* host only */
const char* tc_last_error(void);              /* host only, thread-local */

/* Defaults: dt 1/60, d_hat 1e-4, kappa 1e3, newton_tol 1e-6, cg_rel_tol 1e-4,
 * max_newton 1024, max_cg 4000, dynamic, MIXED, block Jacobi, 40 halvings,
 * Eisenstat-Walker CG forcing. */
tc_status tc_params_default(tc_params* out);  /* host only */

/* Argument checks used by every entry point (host only):
 * mesh: counts > 0, pointers non-null, indices in range, distinct vertices
 *       per tet, det(Dm) > 0 (TC_E_BAD_MESH), fixed bits <= 7, material ids
 *       in [0, n_materials);
 * material: E > 0, -1 < nu < 0.5, density > 0 (all finite);
 * params: dt, dhat, kappa, tolerances > 0 and finite, caps >= 1, known enums;
 * indenters: 0 <= n <= TC_MAX_INDENTERS, known shape, positive parameters,
 *       R orthonormal with det +1 to 1e-9, finite centre. */
tc_status tc_validate_mesh(const tc_mesh* mesh, int32_t n_materials);
tc_status tc_validate_materials(int32_t n, const tc_material* m);
tc_status tc_validate_params(const tc_params* p);
tc_status tc_validate_indenters(int32_t n, const tc_indenter* ind);

/* Alg. 1 (surface extraction) on the host: surface triangles (faces owned by exactly
 * one tet, outward winding, ascending (tet, local face) order), their parent
 * tets, the contact-face label (rest outward normal >= 0.5 along the thinnest
 * bounding-box axis, on the side away from the base) and the contact vertices
 * (every surface vertex with a free component, side faces included,
 * ascending; Sec. III-B puts the IPC barrier on the whole pad surface).
 * Two-call pattern: with tris == NULL only the counts are written.  Capacity
 * arguments are element counts of the caller's arrays (host only). */
tc_status tc_mesh_surface(const tc_mesh* mesh,
                          int32_t* n_tris, int32_t* n_candidates,
                          int32_t* tris, int32_t* parent, uint8_t* is_top,
                          int32_t* candidates,
                          int32_t tris_capacity, int32_t cand_capacity);

/* ---------------------------------------------------------------- context */
/* device: HIP ordinal; hip_stream: a hipStream_t of that device (e.g. torch's
 * current stream) or NULL for a stream the context creates; hbm_budget: bytes
 * the context may hold in total (resident pads + step scratch), 0 = no limit
 * beyond the device. */
tc_status tc_context_create(int32_t device, void* hip_stream, uint64_t hbm_budget,
                            tc_context** out);
/* Destroys the context.  Its pads and servers hold pointers into it, so they
 * must be destroyed first: while any remains the call returns TC_E_BUSY and
 * changes nothing. */
tc_status tc_context_destroy(tc_context* ctx);
/* Bytes currently held (resident + scratch pool) and the budget. */
tc_status tc_context_memory(const tc_context* ctx, uint64_t* used, uint64_t* budget);

/* Per-kernel timing on the context stream (for roofline reporting).
 * enable = 0 off; k >= 1: every launch of the Newton-level kernels is timed
 * with a pair of events recorded by its dispatch, and every k-th launch of
 * the CG kernels (tens of thousands of launches per run) times itself from
 * its blocks' GPU wall clock (k = 1 times every launch; a larger k keeps the
 * sampling's own cost out of the run).  tc_context_timing fills, for up to
 * cap kernels, the average duration of the timed launches, the number of
 * launches made while timing was on, and the algorithmic bytes per launch
 * (model of each kernel's compulsory HBM traffic, averaged over all those
 * launches). */
#define TC_TIMER_NAME_LEN 32
tc_status tc_context_set_timing(tc_context* ctx, int32_t enable);
tc_status tc_context_timing(tc_context* ctx, int32_t cap, int32_t* n,
                            char (*names)[TC_TIMER_NAME_LEN], double* avg_ms,
                            int64_t* launches, double* bytes_per_launch);
tc_status tc_context_reset_timing(tc_context* ctx);

/* Launch-shape autotuner.  First it times the element and CG kernels on
 * the given pads for each candidate block size (vertex rows and SpMV 128 to
 * 1024, element 64 to 256) and keeps the fastest per kernel; then, by the
 * wall time of whole probe steps, the number of streams a batch is split
 * over (1 to 4, at least 2 pads each) and the CG iterations between host
 * checks (8, 16, 32), a candidate winning only by more than 2 %.  Every
 * probe starts from the same saved state and leaves the committed pad state
 * unmodified.  chosen (may be NULL) receives 5 values: vertex-row block,
 * element block, SpMV block, CG iterations per host check, streams. */
tc_status tc_autotune(tc_context* ctx, int32_t n, tc_pad* const* pads,
                      const int32_t* n_ind, const tc_indenter* ind, int32_t* chosen);
/* Force a launch shape: block sizes of the vertex-row kernels (64..1024),
 * the element kernels (64..256) and the SpMV (64..1024), all multiples of 64;
 * CG iterations between host checks of convergence (even, >= 2; default 12);
 * use_graphs 1 replays those iterations of a whole batch as one captured HIP
 * graph, 0 (default) launches them directly, -1 leaves it unchanged.
 * 0 leaves a value unchanged. */
tc_status tc_set_launch(tc_context* ctx, int32_t cg_block, int32_t elem_block, int32_t spmv_block,
                        int32_t cg_per_replay, int32_t use_graphs);

/* Streams a batch step is split over (default 1).  With n > 1, tc_step_batch
 * divides its pads into n groups: the pads with the most Newton iterations
 * in their last step (up to a quarter of the batch's tets) form the first,
 * the others are split into groups of about equal cost (tets x Newton
 * iterations).  Each group is stepped on a stream of its own, driven by a
 * host thread of its own, so the slow pads' long chains of small launches
 * and every group's host round trips overlap with the other groups' large
 * launches.  Every pad's result is bitwise the same for any n
 * (pads never share arithmetic).  Streams keep the default priority.  The
 * setting takes effect from the next batch; extraction-only calls and
 * single pads use the context stream. */
#define TC_MAX_STREAMS 4
tc_status tc_set_streams(tc_context* ctx, int32_t n_streams);

/* How a batch step orders its pads' Newton iterations (Sec. III-B: each pad
 * runs its own Newton solve of the incremental potential, with CG for the
 * linear systems and a backtracking line search).
 *   staged = 1 (default): every pad moves through the stages of its Newton
 *     iterations (Hessians and assembly, CG, direction and step bound, line
 *     search, update) at its own pace.  The step runs in rounds: pads whose
 *     CG has ended are taken through direction, step bound, line_search_evals
 *     trial energies and, when the search ends, the update and the next
 *     iteration's assembly, while every pad in CG runs a chunk of CG
 *     iterations (cg_per_replay of tc_set_launch); one host readback per
 *     round.  Pads that converge in few iterations no longer wait for the
 *     slowest pad at every iteration, and the launches of the slowest pads'
 *     iterations carry the other pads' work.
 *   staged = 0: lockstep; one Newton iteration of every running pad at a
 *     time, each stage waiting for its slowest pad.
 * line_search_evals: 1..8 (0 keeps the current value; default 3).  Every
 * pad's result is bitwise the same under both schedules: each runs the same
 * kernels on its own data in the same order.  Takes effect from the next
 * batch.  The serving loop follows the same setting: one Newton iteration
 * (lockstep) or one round (staged) of its running pads per tick; a staged
 * round also initialises the requests admitted since the last tick and
 * extracts the ones that had ended, so its readback is the tick's only host
 * round trip. */
tc_status tc_set_schedule(tc_context* ctx, int32_t staged, int32_t line_search_evals);

/* ------------------------------------------------------------------- pads */
/* Copies the mesh and materials into HBM and runs the setup kernels: Eq. 1
 * Lame parameters, Dm^-1 and V_e, lumped mass, rest contact areas; builds the
 * surface (Alg. 1 (surface extraction)) and the sparsity of the assembled Hessian on
 * the host.  State starts at rest (x = X, v = 0). */
tc_status tc_pad_create(tc_context* ctx, const tc_mesh* mesh,
                        int32_t n_materials, const tc_material* materials,
                        const tc_params* params, tc_pad** out);
tc_status tc_pad_destroy(tc_pad* pad);
tc_status tc_pad_get_info(const tc_pad* pad, tc_pad_info* out);
/* ------------------------------------------------------- mesh refinement */
/* Contact sizing field of Sec. III-A: the thickness axis (thinnest bounding-
 * box axis unless given) and the contact face at its maximum (side +1) or
 * minimum (-1); points within band x thickness of that face form the contact
 * band, where a radial profile over the two planar axes applies with the
 * radius normalised by the planar half-extents,
 *   rho = |((p_u - c_u) / h_u, (p_v - c_v) / h_v)|   (u < v the planar axes):
 * h = l_contact for rho <= inner, l_global for rho >= inner + transition,
 * cosine blend l_g + (l_c - l_g) (1 + cos(pi (rho - inner) / transition)) / 2
 * between; h = l_global outside the band.  Defaults (tc_sizing_default):
 * band 0.15, inner 0.4, transition 0.2, l_contact 0.8 mm, l_global 3.2 mm,
 * centre NaN = bounding-box centre, max_tets 2^24. */
typedef struct {
  int32_t axis;         /* 0..2, or -1 = thinnest bounding-box axis */
  int32_t side;         /* +1 or -1 */
  double band, inner, transition;
  double l_contact, l_global;   /* [m] > 0 */
  double centre[2];     /* (c_u, c_v) [m]; NaN = bounding-box centre */
  int64_t max_tets;     /* refinement stops with TC_E_INVALID_ARG beyond this */
} tc_sizing;

tc_status tc_sizing_default(tc_sizing* out);   /* host only */

/* Host only: conforming adaptive refinement of a valid tet mesh by
 * terminal-edge bisection under the field above (the paper imposes the
 * field inside WildMeshing's tetrahedralisation; here it drives bisection of
 * a given mesh).  h is read as a cell size: edge ab is too long when
 * |x_a - x_b|^2 > 3 h(m)^2, m its midpoint.  Edges are ordered by (squared
 * length, smaller vertex id, larger vertex id); tets are visited first-in
 * first-out from 0 .. T-1; while the visited tet has a too-long edge, its
 * longest edge is replaced by the largest longest-edge of the tets around it
 * until that is the edge itself (terminal edge), which is bisected: vertex
 * m = 0.5 (x_a + x_b) is appended and each tet around ab (a < b), in
 * ascending index, keeps its index with b replaced by m while a new tet
 * with a replaced by m (same material) is appended; both are queued.  The
 * result is conforming, positively oriented and reproducible bit for bit.
 * Input vertices keep their indices.  Outputs (host): xyz_out [cap_verts][3],
 * tets_out [cap_tets][4], mat_out [cap_tets] (may be NULL); n_verts_out and
 * n_tets_out receive the sizes, also when the capacities are too small
 * (then TC_E_INVALID_ARG and nothing is written). */
tc_status tc_refine_mesh(const tc_mesh* in, const tc_sizing* sizing, int32_t cap_verts, int32_t cap_tets,
                         double* xyz_out, int32_t* tets_out, int32_t* mat_out, int32_t* n_verts_out,
                         int32_t* n_tets_out);

/* ------------------------------------------------------- rigid meshes */
/* Register a rigid triangle mesh as an indenter shape (the rigid objects of
 * Sec. III-B and the grasped test objects of Sec. IV-D).  verts: host
 * [n_verts][3] float64 in the indenter's local frame [m]; tris: host
 * [n_tris][3] int32.  The surface must be closed and consistently oriented
 * with outward normals: every edge shared by exactly two triangles in
 * opposite directions, no zero-area triangle, positive enclosed volume,
 * n_tris <= 2^24 (TC_E_INVALID_ARG otherwise).  The library copies the mesh
 * to the device with its bounding-volume hierarchy and pseudonormals
 * (context memory, counted in the budget); *id receives the handle for
 * tc_indenter.reserved.  Against it phi is the signed distance to the
 * surface: nearest point over the triangles, sign from the angle-weighted
 * pseudonormal of the nearest feature; contact acts on pad vertices (as
 * for the analytic shapes; tc_params.mesh_contact selects the distance or
 * the point-triangle pair barrier).  The collision-free step bound is
 * conservative advancement along each vertex's segment; a mesh that is one
 * connected surface without concave edges (checked here) bounds a convex
 * body, and takes the convex shapes' tangent-line bound instead. */
tc_status tc_rigid_mesh_create(tc_context* ctx, int32_t n_verts, const double* verts, int32_t n_tris,
                               const int32_t* tris, int32_t* id);
/* Host only: the checks of tc_rigid_mesh_create without a context. */
tc_status tc_validate_rigid_mesh(int32_t n_verts, const double* verts, int32_t n_tris, const int32_t* tris);
/* Release a mesh.  TC_E_BUSY while any pad of the context has a request on a
 * server (it may name the mesh); TC_E_INVALID_ARG for an unknown id. */
tc_status tc_rigid_mesh_destroy(tc_context* ctx, int32_t id);

/* Replace solver parameters (precision cannot change; TC_E_INVALID_ARG).
 * TC_E_BUSY while the pad has a request in flight on a server. */
tc_status tc_pad_set_params(tc_pad* pad, const tc_params* params);
/* Back to rest: x = X, v = 0, no previous indenter poses. */
tc_status tc_pad_reset(tc_pad* pad);
/* Release the pad's step scratch back to the context pool (it is taken again
 * by the next step). */
tc_status tc_pad_release_scratch(tc_pad* pad);

/* ------------------------------------------------------------------- step */
/* Alg. 2 one iteration: physics, stress, traction, contact for one pad under
 * n_ind end-of-step indenter poses.  Synchronous on the context stream and
 * transactional: on error the committed state (x, v) is unchanged. */
tc_status tc_step(tc_pad* pad, int32_t n_ind, const tc_indenter* ind,
                  tc_step_stats* stats);

/* The same for n pads fused into one set of launches (uneven pads share every
 * kernel launch).  n_ind[i] poses for pad i are consecutive in ind.  stats[i]
 * receives pad i's outcome; the return value is TC_OK when every pad
 * succeeded, else the first failing pad's status.  Each pad is transactional
 * on its own.  A pad may appear only once. */
tc_status tc_step_batch(tc_context* ctx, int32_t n, tc_pad* const* pads,
                        const int32_t* n_ind, const tc_indenter* ind,
                        tc_step_stats* stats);

/* Extraction only (Alg. 2 stress/traction/contact) on the committed positions
 * under the given poses: fills SIGMA ... TRACTION_SUM.  Its contact forces are
 * the barrier's only: friction forces depend on the start state of the step
 * that produced the positions and come with tc_step's extraction. */
tc_status tc_extract(tc_pad* pad, int32_t n_ind, const tc_indenter* ind);

/* tc_extract for callers that cannot allocate device memory: code under HIP
 * stream capture, tight serving loops, harnesses that forbid allocation.  It
 * allocates nothing (no hipMalloc, hipFree or allocating library call): its
 * launch descriptor, state, poses, tile lists and partial sums live in one
 * fixed device array of TC_NOALLOC_SCRATCH_BYTES per device, held from the
 * first context on that device until the process ends.  The outputs are the
 * pad's own fields, as with tc_extract, and equal tc_extract's bitwise (same
 * kernels, same inputs).  reaction (host, [3], may be NULL) receives
 * -sum_k f_k.  A pad whose tables need more than the array returns
 * TC_E_INVALID_ARG (the array holds pads up to tens of millions of tets at
 * the default launch shape), and so does a pad with vertex-face / edge-edge
 * pairs on (mesh_contact 2 with a TC_MESH indenter), whose pair records
 * live in its step scratch.  Every call on a device shares that device's
 * array: calls through one context are serialised, but calls that overlap on
 * one device through different contexts race. */
#define TC_NOALLOC_SCRATCH_BYTES (4u << 20)
tc_status tc_extract_noalloc(tc_pad* pad, int32_t n_ind, const tc_indenter* ind, double* reaction);

/* Inspection: one Newton direction at the committed positions (taken as the
 * current iterate as they are: no feasible-start projection) under the given
 * poses.  Assembles the element and barrier Hessians and gradient and runs
 * CG to cg_conv_tol (else cg_rel_tol).  dir and grad (host, [V][3] float64,
 * grad may be NULL) receive p and dE/dx (inertia + dt^2 (elastic + barrier),
 * fixed components zeroed).  The pad state is not modified. */
tc_status tc_pad_newton_direction(tc_pad* pad, int32_t n_ind, const tc_indenter* ind, double* dir,
                                  double* grad);

/* ------------------------------------------------------------------ fields */
tc_status tc_field_info(const tc_pad* pad, int32_t field, int32_t* dtype,
                        int64_t* count, int32_t* components);
/* Copy a field into dst (bytes must be >= its size, else TC_E_INVALID_ARG).
 * dst_is_device: 1 = dst is device memory on the context's device. */
tc_status tc_pad_read(const tc_pad* pad, int32_t field, void* dst, size_t bytes,
                      int32_t dst_is_device);
/* Overwrite POSITIONS or VELOCITIES (bytes must equal the field size). */
tc_status tc_pad_write(tc_pad* pad, int32_t field, const void* src, size_t bytes,
                       int32_t src_is_device);

/* ------------------------------------------------------ checkpoint/resume */
/* Serialise x, v, the step counter and the previous indenter poses.  With buf == NULL *bytes receives the
 * size needed; otherwise *bytes is the capacity on input and the size written
 * on output.  load restores a buffer written for a pad with the same mesh. */
tc_status tc_pad_save_state(const tc_pad* pad, void* buf, size_t* bytes);
tc_status tc_pad_load_state(tc_pad* pad, const void* buf, size_t bytes);

/* --------------------------------------------------------------- serving */
typedef struct {
  uint64_t ticket;
  int32_t status;          /* step status */
  int32_t pad_index;       /* caller tag given at submit */
  double t_arrive_ms;      /* submit time, ms on the server clock */
  double t_admit_ms;       /* admission into the running batch */
  double t_done_ms;        /* result committed and readable */
  tc_step_stats stats;
} tc_result;

typedef struct {
  int64_t submitted, admitted, completed, rejected;
  int32_t queued, running;
  int32_t max_running_seen;
  int64_t ticks;           /* batched ticks executed (Newton iterations in
                              lockstep, rounds in the staged schedule) */
  uint64_t scratch_in_use; /* bytes of step scratch held by running requests */
  int64_t evictions;       /* step scratch released to make room (context total) */
} tc_server_stats;

/* Continuous-batching request loop on its own host thread.  Pads stay
 * resident; a request (pad, poses) is admitted when a slot is free and its
 * step scratch fits the context budget, joins the running batch at the next
 * tick (see tc_set_schedule) and leaves it when its step completes.  When the
 * budget is short, the step scratch of pads with no step on the device is
 * released (their committed state stays resident); a request that cannot fit
 * even then, with nothing running, completes with TC_E_NO_MEMORY.
 * max_slots: requests on the device at once (>= 1). */
tc_status tc_server_create(tc_context* ctx, int32_t max_slots, tc_server** out);
/* Queue one step request.  The pad must belong to the server's context;
 * requests for the same pad run in submission order.  tag is echoed in the
 * result's pad_index. */
tc_status tc_server_submit(tc_server* srv, tc_pad* pad, int32_t tag, int32_t n_ind,
                           const tc_indenter* ind, uint64_t* ticket);
/* Collect up to cap finished results; waits up to wait_us microseconds for
 * the first one (0 = do not wait). */
tc_status tc_server_poll(tc_server* srv, tc_result* out, int32_t cap, int32_t* n,
                         int32_t wait_us);
tc_status tc_server_get_stats(tc_server* srv, tc_server_stats* out);
/* Stops the thread after finishing running requests; queued ones are
 * dropped with status TC_E_BUSY. */
tc_status tc_server_destroy(tc_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* TACAUCHY_H */
