// Device-visible data of the tactile FEM step: per-pad descriptors, per-step
// state and tile tables shared by the kernels (kernels.hip) and the runtime
// that launches them (runtime.hip).
#pragma once

#include <cstdint>

namespace tc {

constexpr int MAX_IND = 5;
constexpr int MAX_MAT = 8;
// Per-tet record the element kernel accumulates in registers: the 78
// independent entries of the symmetric 12x12 element Hessian in 10 blocks
// (a <= b), then the 12 gradient entries, padded to 96 values.
constexpr int KE_STRIDE = 96;
constexpr int KE_GRAD = 78;
// Values per block of the element block streams.  The element kernel
// scatters each tet's 4 diagonal blocks into the diagonal stream (grouped by
// vertex row, tets ascending) and its 6 edge blocks into the edge stream
// (grouped by unique edge i < j, tets ascending), so assembly reads every row
// and every edge contiguously.  Diagonal block: xx, xy, xz, yy, yz, zz and the
// gradient of the vertex; edge block: the 3x3 block (row i, column j),
// row-major.
constexpr int KC = 9;
// rows handled by each lane group of the vectorised SpMV per tile
constexpr int SPMV_ROWS_PER_GROUP = 4;

// offset of block (a, b), a <= b, inside the record; diagonal blocks hold
// (xx, xy, xz, yy, yz, zz), off-diagonal blocks row-major 3x3
__host__ __device__ constexpr int ke_block_offset(int a, int b) {
  return a == 0 ? (b == 0 ? 0 : 6 + 9 * (b - 1))
       : a == 1 ? (b == 1 ? 33 : 39 + 9 * (b - 2))
       : a == 2 ? (b == 2 ? 57 : 63)
       : 72;
}

struct DevIndenter {
  int32_t shape;
  int32_t reserved;
  double R[9];
  double c[3];
  double prm[4];
};

// Rigid triangle meshes registered with a context (TC_MESH indenters).
constexpr int MAX_MESHES = 64;
// stack of the closest-triangle traversal; the host builds trees of depth
// below this (median splits, at most 2^24 triangles)
constexpr int BVH_STACK = 64;

// Bounding-volume hierarchy node, depth-first order (an inner node's left
// child follows it).  count > 0: leaf over triangles [first, first + count);
// count == 0: inner node whose right child is node `first`.
struct BvhNode {
  double lo[3], hi[3];
  int32_t first;
  int32_t count;
};

// One registered mesh (local frame), triangles in leaf order.  n_tri == 0:
// free slot.
struct DevMesh {
  int32_t n_tri, n_node;
  int32_t convex;          // 1: one component, no concave edge (the distance outside is convex)
  int32_t n_vert;
  const double* tv;        // [n_tri][9] corners a, b, c (counter-clockwise from outside)
  const double* tn;        // [n_tri][3] unit outward face normal
  const int32_t* tid;      // [n_tri][6] vertex ids of a, b, c; edge ids of ab, bc, ca
  const double* en;        // [n_edge][3] edge pseudonormal (sum of the two face normals)
  const double* vn;        // [n_vert][3] vertex pseudonormal (angle-weighted normal sum)
  const BvhNode* nodes;
  // vertex-face and edge-edge pairs (mesh_contact 2)
  const double* mv;        // [n_vert][3] vertex positions
  const double* va;        // [n_vert] a third of the area of the vertex's triangles
  const int32_t* me;       // [n_edge][2] edge end vertex ids
  const double* mel;       // [n_edge] edge length
  const uint8_t* own;      // [n_tri] bit k: this triangle owns vertex tid[k], bit 3 + k: edge
                           // tid[3 + k] (each vertex and edge owned by its first triangle in
                           // leaf order, so a traversal meets it once)
};

// Indenter poses of one pad for the current step (uploaded at step start)
// and the poses the friction lag is taken under (the previous step's, or
// the current ones when there is none).
struct EnvPose {
  int32_t n_ind;
  int32_t pairs;             // vertex-face / edge-edge pairs on (mesh_contact 2 and a mesh indenter)
  DevIndenter ind[MAX_IND];
  DevIndenter prev[MAX_IND];
  double travel[MAX_IND];    // largest move of a mesh vertex from the previous pose (mesh indenters)
};

// Pair record of one pad surface primitive (triangle j < S, surface edge
// S + f), float64: gradient of its vertices' pair terms [3][3] (edges use
// the first two), then the symmetric 3x3 Gauss-Newton blocks (6 values
// each: 00 01 02 11 12 22) of vertex pairs (0,0) (1,1) (2,2) (0,1) (1,2)
// (2,0).  During the feasible start the first four values hold the push
// of the primitive's vertices and the number of pushes.
constexpr int PREC = 48;

// Lagged friction record of one (indenter, contact vertex) pair, float64:
// normal force lambda (0 = no friction), normal n, indenter point motion w.
constexpr int FRIC_STRIDE = 8;
constexpr int FRIC_LAM = 0, FRIC_N = 1, FRIC_W = 4;

// Life cycle of a pad's step inside a batch.
enum Phase : int32_t {
  PH_INIT = 0,    // predict + feasible start + E(x0) pending
  PH_RUN = 1,     // Newton iterations
  PH_FINISH = 2,  // Newton ended (or extraction only): extraction/commit pending
  PH_DONE = 3,    // results readable, slot free
  PH_IDLE = 4     // slot not in use
};

// Stage of a running pad inside its Newton iteration.  Every kernel of an
// iteration acts only on pads at its own stage, so one launch may carry
// pads at different stages (pads of a batch need not iterate in step).
enum Stage : int32_t {
  ST_START = 0,   // next: reset of the iteration's counters
  ST_ASM = 1,     // element and barrier Hessians, assembly
  ST_CG = 2,      // CG running; with cg_done the direction is ready
  ST_LS = 3,      // line search
  ST_UPD = 4      // step accepted (or converged): update pending
};

// Mutable per-pad state of one step, in device memory (one slot of a pool).
// The runtime initialises it at step start; kernels own it afterwards.
struct EnvState {
  int32_t phase;
  int32_t stage;           // Stage, while phase == PH_RUN
  int32_t extracting;      // the extraction kernels were launched for this pad (set by k_sigma)
  int32_t mode;            // 0 = full step, 1 = extraction only
  int32_t status;          // TC_OK or TC_E_*
  int32_t infeasible;
  int32_t newton_done;
  int32_t newton_iters;
  int32_t cg_total;
  int32_t ls_total;
  double final_step_inf;
  double reaction[3];
  // per Newton iteration
  int32_t dir_conv;
  int32_t apply;
  int32_t ls_done;
  int32_t ls_halv;
  double ls_alpha;
  int32_t ls_expanding;    // the line search is doubling an accepted full step
  int32_t ls_expand_n;     // doublings taken
  int32_t ls_contracting;  // trying the shorter step of the quadratic fit after a full step
  double ls_best_alpha;    // best accepted step and its energy while doubling
  double ls_best_E;
  double alpha_max;
  double gTd;
  double E_cur;
  double E_next;
  // CG (ping-pong slots indexed by iteration parity)
  double rzp[2];
  double rz0;
  int32_t it[2];
  int32_t cg_done;
  int32_t warm;            // this iteration's CG starts from gamma d_prev (iteration -1)
  int32_t cg_iters;
  int32_t breakdown;
  int32_t force_tight;     // next CG must reach the floor tolerance
  int32_t true_hess;       // element Hessians unfiltered in this iteration
  int32_t no_true_hess;    // a breakdown happened: filtered for the rest of the step
  int32_t filt_all;        // the same for the barrier Hessians (any unfiltered mode)
  int32_t n_breakdown;     // CG breakdowns in this step
  double cg_tol2;
  double rz0_prev;         // r0.z0 of the previous Newton iteration (< 0: none)
  double eta_prev;
};

// Immutable-per-batch description of one pad: pointers into its resident
// arrays, step scratch and outputs, sizes, material table and parameters.
struct EnvDesc {
  int32_t V, T, C, S, W;
  int32_t V_E;               // unique edges (off-diagonal block pairs)
  int32_t Se;                // surface edges
  int32_t n_vt, n_tt, n_ct, n_st, n_at, n_te, n_spt;   // tiles per kernel class
  int32_t n_pt;              // pair tiles over S + Se surface primitives (mesh_contact 2, else 0)
  // resident inputs
  const double* X;
  double* x;
  double* v;
  const int32_t* tets;       // [T][4]
  const void* Dminv;         // real [T][9]
  const void* vol;           // real [T]
  const int8_t* mat;         // [T] material index or null
  const double* mass;        // [V]
  const uint8_t* fixed;      // [V]
  const int32_t* cand;       // [C]
  const int32_t* cand_of_vert;  // [V], -1 if not a candidate
  const double* cand_area;   // [C] rest barrier weight
  const int32_t* tris;       // [S][3]
  const int32_t* parent;     // [S]
  const uint8_t* is_top;     // [S]
  const int32_t* ctri_ptr;   // [C+1] triangles of each candidate: incident contact-face tris, or
                             // all incident surface tris for a side-face vertex
  const int32_t* ctri_idx;
  const int32_t* col;        // [V][W] block column of each stored block, -1 = empty
  const int32_t* cptr;       // [V*W+1] contribution ranges per (row, slot)
  const uint32_t* clist;     // (tet << 4) | (a << 2) | b
  const int32_t* dptr;       // [V+1] diagonal-stream range of each row
  const int32_t* eptr;       // [V_E+1] edge-stream range of each edge
  const int32_t* eitem;      // [V_E][2] blocks (i, slot of j), (j, slot of i)
  const int32_t* cpos;       // [T][10] stream positions: 4 diagonal, 6 edge blocks
  const int32_t* sedge;      // [Se][2] surface edges (i < j), ascending
  const double* sedge_len0;  // [Se] rest length
  const int32_t* sedge_adj;  // [Se][2] its surface triangles: tri << 3 | pair block (3 ab, 4 bc, 5 ca)
  const int32_t* edge_sedge; // [V_E] surface edge of each unique edge, -1 if interior
  const int32_t* vp_ptr;     // [C+1] surface primitives of each contact vertex
  const int32_t* vp_idx;     //   primitive << 2 | its local vertex (triangles j, edges S + f)
  // outputs
  void* sigma;               // real [T][6]
  void* traction;            // real [S][3]
  void* pressure;            // real [S]
  void* tangential;          // real [S][3]
  void* tri_area;            // real [S]
  void* tri_normal;          // real [S][3]
  double* tri_cross;         // [S][3] e1 x e2 (current)
  double* c_force;           // [C][3]
  double* c_normal;
  double* c_area;
  double* c_fn;
  double* c_ft;
  double* c_press;
  double* reaction;          // [3]
  double* traction_sum;      // [3]
  // step scratch
  void* Ke;                  // real [4 T][KC] diagonal stream, then [6 T][KC] edge stream
  void* A;                   // real [V][W][9] row-major 3x3 blocks
  double* xn;                // Newton iterate [V][3]
  double* xhat;
  double* g;                 // gradient [V][3]
  void* d;                   // real [V][3] Newton direction (CG solution)
  double* r;                 // CG residual
  void* z;                   // real
  void* p0;                  // real, ping-pong search directions
  void* p1;
  void* q;                   // real, A p
  void* Pinv;                // real [V][6] symmetric preconditioner blocks
  double* gb;                // [C][3] barrier gradient
  double* Hb;                // [C][6] projected barrier Hessian
  double* fric;              // [MAX_IND][C][FRIC_STRIDE] lagged friction (friction on)
  double* part_rz;           // [n_vt]
  double* part_pq;           // [n_spt]
  double* part_g2;           // [n_vt]
  double* part_e;            // [n_te + n_vt + n_ct + n_pt]
  double* part_dir;          // [2 n_vt]
  double* part_filt;         // [n_ct + n_pt]
  double* part_c3;           // [3 n_ct]
  double* part_s3;           // [3 n_st]
  double* prec;              // [S + Se][PREC] pair records (mesh_contact 2)
  int32_t* pflag;            // [S + Se] 1 where the record holds pairs
  EnvState* st;
  const EnvPose* pose;
  const DevMesh* meshes;     // [MAX_MESHES] the context's rigid meshes
  // material table (Eq. 1) and parameters
  // cshift = lam (alpha - 1): mu for the rest-stable shift, 0 for alpha = 1
  double mu[MAX_MAT], lam[MAX_MAT], alpha[MAX_MAT], rho[MAX_MAT], cshift[MAX_MAT];
  double h, dhat, kappa, tol_abs, noise, cg_rel_tol, cg_conv_tol, cg_eta_max;
  double gravity[3];
  int32_t quasi_static, max_cg, max_newton, max_halvings, precond, cg_forcing, hess_proj, init_guess;
  int32_t ls_expand;
  int32_t cg_warm;           // CG starts from the best multiple of the previous direction
  int32_t mesh_pairs;        // rigid meshes: 0 distance; 1 barrier summed over triangles within
                             // d_hat; 2 that plus vertex-face and edge-edge pairs
  double fr_mu, fr_eps;      // friction ratio (0 = off) and slip threshold eps_v h [m]
};

// One block of a launch: pad `env`, tile index `tile` within that pad's
// work of the kernel's class.
struct Tile {
  int32_t env;
  int32_t tile;
};

}  // namespace tc
