// Host-side mesh topology of a pad: validation, surface extraction
// (Alg. 1 (surface extraction)), contact-face labels and contact vertices, and the
// sparsity of the assembled Hessian with its per-block gather lists.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tacauchy.h"

namespace tc {

struct Topology {
  int V = 0, T = 0;
  int axis = 2;                   // thickness axis (thinnest bounding-box extent)
  double bbox_diag = 0.0;
  std::vector<int32_t> tris;      // [S][3] outward winding
  std::vector<int32_t> parent;    // [S]
  std::vector<uint8_t> is_top;    // [S]
  std::vector<uint8_t> fixed;     // [V]
  std::vector<int32_t> cand;      // [C] ascending
  std::vector<int32_t> cand_of_vert;  // [V]
  std::vector<int32_t> ctri_ptr;  // [C+1] triangles of each contact vertex (contact face first)
  std::vector<int32_t> ctri_idx;
  // assembled Hessian: W stored 3x3 blocks per vertex row, slot 0 = diagonal,
  // then neighbours ascending; col[i * W + s] = -1 past the row's end
  int W = 0;
  int64_t nnz_blocks = 0;
  std::vector<int32_t> col;       // [W*V]
  std::vector<int32_t> cptr;      // [V*W+1] gather range of each (row, slot)
  std::vector<uint32_t> clist;    // (tet << 4) | (a << 2) | b, ascending tet
  // element block streams of assembly: diagonal blocks by row (ascending
  // tet), off-diagonal blocks by unique edge i < j (ascending tet)
  std::vector<int32_t> dptr;      // [V+1] diagonal-stream range of each row
  std::vector<int32_t> eptr;      // [NE+1] off-diagonal-stream range of each edge
  std::vector<int32_t> eitem;     // [NE][2] blocks (i, slot of j) and (j, slot of i)
  std::vector<int32_t> cpos;      // [T][10] stream positions: diagonal a = 0..3,
                                  // then pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
};

// Checks of tacauchy.h (tc_validate_mesh); err receives the message.
tc_status validate_mesh(const tc_mesh* m, int n_materials, std::string& err);
tc_status validate_materials(int n, const tc_material* m, std::string& err);
tc_status validate_params(const tc_params* p, std::string& err);
tc_status validate_indenters(int n, const tc_indenter* ind, std::string& err);

// Surface, labels, fixed mask, contact vertices (needs a validated mesh).
void build_surface(const tc_mesh* m, Topology& t);
// Block sparsity and assembly gather lists.
void build_sparsity(const tc_mesh* m, Topology& t);

}  // namespace tc
