// Host-side topology of a pad (see topology.h).
#include "topology.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>

namespace tc {

namespace {

// Outward faces of a positively oriented tet (v0, v1, v2, v3):
// (b - a) x (c - a) points away from the vertex not on the face.
constexpr int kFaces[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};

bool finite(double v) { return std::isfinite(v); }

std::string fmt(const char* f, long long a = 0, long long b = 0) {
  char buf[256];
  std::snprintf(buf, sizeof buf, f, a, b);
  return buf;
}

}  // namespace

tc_status validate_mesh(const tc_mesh* m, int n_materials, std::string& err) {
  if (!m) { err = "mesh is null"; return TC_E_INVALID_ARG; }
  if (m->n_verts < 4 || m->n_tets < 1) { err = "mesh needs >= 4 vertices and >= 1 tet"; return TC_E_INVALID_ARG; }
  if (!m->rest_xyz || !m->tets) { err = "mesh arrays are null"; return TC_E_INVALID_ARG; }
  if ((int64_t)m->n_tets >= (int64_t(1) << 27)) { err = "too many tets (limit 2^27)"; return TC_E_INVALID_ARG; }
  const int V = m->n_verts;
  for (int64_t i = 0; i < 3LL * V; ++i)
    if (!finite(m->rest_xyz[i])) { err = fmt("rest position %lld is not finite", i / 3); return TC_E_INVALID_ARG; }
  for (int e = 0; e < m->n_tets; ++e) {
    const int32_t* t = m->tets + 4 * (int64_t)e;
    for (int a = 0; a < 4; ++a)
      if (t[a] < 0 || t[a] >= V) { err = fmt("tet %lld references vertex %lld out of range", e, t[a]); return TC_E_BAD_MESH; }
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        if (t[a] == t[b]) { err = fmt("tet %lld repeats a vertex", e); return TC_E_BAD_MESH; }
    const double* X = m->rest_xyz;
    double D[3][3];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) D[i][k] = X[3 * t[k + 1] + i] - X[3 * t[0] + i];
    const double det = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) -
                       D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
                       D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
    if (!(det > 0.0)) { err = fmt("tet %lld has non-positive rest volume", e); return TC_E_BAD_MESH; }
  }
  if (m->fixed)
    for (int i = 0; i < V; ++i)
      if (m->fixed[i] > 7) { err = fmt("fixed mask of vertex %lld > 7", i); return TC_E_INVALID_ARG; }
  if (m->tet_material)
    for (int e = 0; e < m->n_tets; ++e)
      if (m->tet_material[e] < 0 || m->tet_material[e] >= n_materials) {
        err = fmt("tet %lld material id out of range", e);
        return TC_E_INVALID_ARG;
      }
  return TC_OK;
}

tc_status validate_materials(int n, const tc_material* m, std::string& err) {
  if (n < 1 || n > 8 || !m) { err = "need 1..8 materials"; return TC_E_INVALID_ARG; }
  for (int k = 0; k < n; ++k) {
    const tc_material& q = m[k];
    if (!finite(q.E) || !(q.E > 0)) { err = fmt("material %lld: E must be > 0", k); return TC_E_INVALID_ARG; }
    if (!finite(q.nu) || !(q.nu > -1.0 && q.nu < 0.5)) { err = fmt("material %lld: nu must be in (-1, 0.5)", k); return TC_E_INVALID_ARG; }
    if (!finite(q.density) || !(q.density > 0)) { err = fmt("material %lld: density must be > 0", k); return TC_E_INVALID_ARG; }
  }
  return TC_OK;
}

tc_status validate_params(const tc_params* p, std::string& err) {
  if (!p) { err = "params is null"; return TC_E_INVALID_ARG; }
  const double pos[] = {p->dt, p->dhat, p->kappa, p->newton_tol, p->cg_rel_tol};
  const char* names[] = {"dt", "dhat", "kappa", "newton_tol", "cg_rel_tol"};
  for (int k = 0; k < 5; ++k)
    if (!finite(pos[k]) || !(pos[k] > 0)) { err = std::string(names[k]) + " must be finite and > 0"; return TC_E_INVALID_ARG; }
  if (p->max_newton < 1 || p->max_cg < 1 || p->max_halvings < 0) { err = "iteration caps must be >= 1"; return TC_E_INVALID_ARG; }
  if (p->precision != TC_PREC_FP64 && p->precision != TC_PREC_MIXED) { err = "unknown precision"; return TC_E_INVALID_ARG; }
  if (p->precond != TC_PRECOND_BLOCK_JACOBI && p->precond != TC_PRECOND_JACOBI) { err = "unknown preconditioner"; return TC_E_INVALID_ARG; }
  if (p->cg_forcing < 0 || p->cg_forcing > 2) { err = "cg_forcing must be 0, 1 or 2"; return TC_E_INVALID_ARG; }
  if (p->literal_alpha != 0 && p->literal_alpha != 1) { err = "literal_alpha must be 0 or 1"; return TC_E_INVALID_ARG; }
  if (p->quasi_static != 0 && p->quasi_static != 1) { err = "quasi_static must be 0 or 1"; return TC_E_INVALID_ARG; }
  if (!finite(p->cg_conv_tol) || p->cg_conv_tol < 0) { err = "cg_conv_tol must be >= 0"; return TC_E_INVALID_ARG; }
  if (!finite(p->cg_eta_max) || !(p->cg_eta_max > 0 && p->cg_eta_max < 1)) { err = "cg_eta_max must be in (0, 1)"; return TC_E_INVALID_ARG; }
  if (p->ls_expand < 0 || p->ls_expand > 16) { err = "ls_expand must be in 0..16"; return TC_E_INVALID_ARG; }
  if (p->hess_proj < 0 || p->hess_proj > 15 || (p->hess_proj & 3) == 3) { err = "hess_proj: element mode 0..2 in bits 0-1, barrier mode 0..3 in bits 2-3"; return TC_E_INVALID_ARG; }
  if (p->init_guess != 0 && p->init_guess != 1) { err = "init_guess must be 0 or 1"; return TC_E_INVALID_ARG; }
  if (!finite(p->friction) || p->friction < 0) { err = "friction must be finite and >= 0"; return TC_E_INVALID_ARG; }
  if (p->friction > 0 && (!finite(p->eps_v) || !(p->eps_v > 0))) { err = "eps_v must be finite and > 0 with friction on"; return TC_E_INVALID_ARG; }
  if (p->mesh_contact < 0 || p->mesh_contact > 2) { err = "mesh_contact must be 0, 1 or 2"; return TC_E_INVALID_ARG; }
  if (p->cg_warm < 0 || p->cg_warm > 1) { err = "cg_warm must be 0 or 1"; return TC_E_INVALID_ARG; }
  for (int c = 0; c < 3; ++c)
    if (!finite(p->gravity[c])) { err = "gravity must be finite"; return TC_E_INVALID_ARG; }
  return TC_OK;
}

tc_status validate_indenters(int n, const tc_indenter* ind, std::string& err) {
  if (n < 0 || n > TC_MAX_INDENTERS) { err = "0..5 indenters per pad"; return TC_E_INVALID_ARG; }
  if (n > 0 && !ind) { err = "indenter array is null"; return TC_E_INVALID_ARG; }
  for (int k = 0; k < n; ++k) {
    const tc_indenter& q = ind[k];
    if (q.shape < TC_SPHERE || q.shape > TC_MESH) { err = fmt("indenter %lld: unknown shape", k); return TC_E_INVALID_ARG; }
    if (q.shape == TC_MESH) {
      if (q.reserved < 0 || q.reserved >= TC_MAX_MESHES) { err = fmt("indenter %lld: mesh id out of range", k); return TC_E_INVALID_ARG; }
      for (int j = 0; j < 4; ++j)
        if (!finite(q.prm[j])) { err = fmt("indenter %lld: parameter %lld not finite", k, j); return TC_E_INVALID_ARG; }
    } else {
      const int need = q.shape == TC_SPHERE ? 1 : q.shape == TC_BOX ? 3 : 2;
      for (int j = 0; j < need; ++j)
        if (!finite(q.prm[j]) || !(q.prm[j] > 0)) { err = fmt("indenter %lld: parameter %lld must be > 0", k, j); return TC_E_INVALID_ARG; }
    }
    for (int j = 0; j < 3; ++j)
      if (!finite(q.c[j])) { err = fmt("indenter %lld: centre not finite", k); return TC_E_INVALID_ARG; }
    // R^T R = I and det R = +1
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0;
        for (int r = 0; r < 3; ++r) s += q.R[3 * r + a] * q.R[3 * r + b];
        if (!finite(s) || std::fabs(s - (a == b ? 1.0 : 0.0)) > 1e-9) { err = fmt("indenter %lld: R is not orthonormal", k); return TC_E_INVALID_ARG; }
      }
    const double* R = q.R;
    const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                       R[2] * (R[3] * R[7] - R[4] * R[6]);
    if (std::fabs(det - 1.0) > 1e-9) { err = fmt("indenter %lld: det R != 1", k); return TC_E_INVALID_ARG; }
  }
  return TC_OK;
}

void build_surface(const tc_mesh* m, Topology& t) {
  const int V = m->n_verts, T = m->n_tets;
  const double* X = m->rest_xyz;
  t.V = V;
  t.T = T;
  // faces keyed by their sorted vertex triple; a face is on the surface iff
  // its key occurs once
  const int64_t NF = 4LL * T;
  std::vector<std::array<int32_t, 3>> key(NF);
  for (int e = 0; e < T; ++e)
    for (int f = 0; f < 4; ++f) {
      std::array<int32_t, 3> k = {m->tets[4LL * e + kFaces[f][0]], m->tets[4LL * e + kFaces[f][1]],
                                  m->tets[4LL * e + kFaces[f][2]]};
      std::sort(k.begin(), k.end());
      key[4LL * e + f] = k;
    }
  std::vector<int64_t> order(NF);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return key[a] != key[b] ? key[a] < key[b] : a < b;
  });
  std::vector<uint8_t> once(NF, 0);
  for (int64_t s = 0; s < NF;) {
    int64_t r = s + 1;
    while (r < NF && key[order[r]] == key[order[s]]) ++r;
    if (r - s == 1) once[order[s]] = 1;
    s = r;
  }
  t.tris.clear();
  t.parent.clear();
  for (int64_t idx = 0; idx < NF; ++idx)
    if (once[idx]) {
      const int e = (int)(idx / 4), f = (int)(idx % 4);
      for (int c = 0; c < 3; ++c) t.tris.push_back(m->tets[4LL * e + kFaces[f][c]]);
      t.parent.push_back(e);
    }
  const int S = (int)t.parent.size();
  // thickness axis = thinnest bounding-box extent (first on ties)
  double lo[3], hi[3];
  for (int c = 0; c < 3; ++c) { lo[c] = X[c]; hi[c] = X[c]; }
  for (int i = 0; i < V; ++i)
    for (int c = 0; c < 3; ++c) { lo[c] = std::min(lo[c], X[3 * i + c]); hi[c] = std::max(hi[c], X[3 * i + c]); }
  double ext[3];
  for (int c = 0; c < 3; ++c) ext[c] = hi[c] - lo[c];
  int a = 0;
  if (ext[1] < ext[a]) a = 1;
  if (ext[2] < ext[a]) a = 2;
  t.axis = a;
  t.bbox_diag = std::sqrt(ext[0] * ext[0] + ext[1] * ext[1] + ext[2] * ext[2]);
  // contact face: rest outward normal component >= 0.5 along the axis
  t.is_top.assign(S, 0);
  for (int j = 0; j < S; ++j) {
    const double* v0 = X + 3 * t.tris[3 * j];
    const double* v1 = X + 3 * t.tris[3 * j + 1];
    const double* v2 = X + 3 * t.tris[3 * j + 2];
    const double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
    const double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
    const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                         e1[0] * e2[1] - e1[1] * e2[0]};
    const double L = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    t.is_top[j] = (c[a] / L >= 0.5) ? 1 : 0;
  }
  // fixed: given mask, or the base (minimum along the axis) fully fixed
  t.fixed.assign(V, 0);
  if (m->fixed) {
    std::copy(m->fixed, m->fixed + V, t.fixed.begin());
  } else {
    for (int i = 0; i < V; ++i)
      if (X[3 * i + a] <= lo[a] + 1e-9 * ext[a]) t.fixed[i] = 7;
  }
  // contact vertices (barrier candidates): every surface vertex with a free
  // component, side faces included, so that an indenter reaching past the
  // contact face still meets a barrier
  std::vector<uint8_t> on(V, 0);
  for (int j = 0; j < S; ++j)
    for (int c = 0; c < 3; ++c) on[t.tris[3 * j + c]] = 1;
  t.cand.clear();
  t.cand_of_vert.assign(V, -1);
  for (int i = 0; i < V; ++i)
    if (on[i] && t.fixed[i] != 7) {
      t.cand_of_vert[i] = (int)t.cand.size();
      t.cand.push_back(i);
    }
  const int C = (int)t.cand.size();
  // triangles whose share each contact vertex takes (rest barrier weight,
  // Alg. 2 normal and area): its incident contact-face triangles when it
  // lies on the contact face, else all its incident surface triangles
  std::vector<uint8_t> on_top(V, 0);
  for (int j = 0; j < S; ++j)
    if (t.is_top[j])
      for (int c = 0; c < 3; ++c) on_top[t.tris[3 * j + c]] = 1;
  auto takes = [&](int j, int vtx) { return t.is_top[j] || !on_top[vtx]; };
  t.ctri_ptr.assign(C + 1, 0);
  for (int j = 0; j < S; ++j)
    for (int c = 0; c < 3; ++c) {
      const int v = t.tris[3 * j + c];
      const int k = t.cand_of_vert[v];
      if (k >= 0 && takes(j, v)) t.ctri_ptr[k + 1]++;
    }
  for (int k = 0; k < C; ++k) t.ctri_ptr[k + 1] += t.ctri_ptr[k];
  t.ctri_idx.assign(t.ctri_ptr[C], 0);
  std::vector<int32_t> fill(t.ctri_ptr.begin(), t.ctri_ptr.end() - 1);
  for (int j = 0; j < S; ++j)
    for (int c = 0; c < 3; ++c) {
      const int v = t.tris[3 * j + c];
      const int k = t.cand_of_vert[v];
      if (k >= 0 && takes(j, v)) t.ctri_idx[fill[k]++] = j;
    }
}

void build_sparsity(const tc_mesh* m, Topology& t) {
  const int V = m->n_verts, T = m->n_tets;
  std::vector<std::vector<int32_t>> nb(V);
  for (int i = 0; i < V; ++i) nb[i].push_back(i);
  for (int e = 0; e < T; ++e) {
    const int32_t* tv = m->tets + 4LL * e;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        auto& L = nb[tv[a]];
        if (std::find(L.begin(), L.end(), tv[b]) == L.end()) L.push_back(tv[b]);
      }
  }
  int W = 0;
  t.nnz_blocks = 0;
  for (int i = 0; i < V; ++i) {
    std::sort(nb[i].begin() + 1, nb[i].end());
    W = std::max(W, (int)nb[i].size());
    t.nnz_blocks += (int64_t)nb[i].size();
  }
  t.W = W;
  t.col.assign((size_t)W * V, -1);
  for (int i = 0; i < V; ++i)
    for (size_t s = 0; s < nb[i].size(); ++s) t.col[(size_t)i * W + s] = nb[i][s];
  auto slot_of = [&](int row, int c) {
    const auto& L = nb[row];
    return (int)(std::find(L.begin(), L.end(), c) - L.begin());
  };
  const int64_t NI = (int64_t)W * V;
  std::vector<int32_t> cnt(NI + 1, 0);
  std::vector<int32_t> item(16LL * T);
  for (int e = 0; e < T; ++e) {
    const int32_t* tv = m->tets + 4LL * e;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const int64_t it = (int64_t)tv[a] * W + slot_of(tv[a], tv[b]);
        item[16LL * e + 4 * a + b] = (int32_t)it;
        cnt[it + 1]++;
      }
  }
  for (int64_t k = 0; k < NI; ++k) cnt[k + 1] += cnt[k];
  t.cptr = cnt;
  t.clist.assign(16LL * T, 0);
  std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
  for (int e = 0; e < T; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const int64_t it = item[16LL * e + 4 * a + b];
        t.clist[pos[it]++] = ((uint32_t)e << 4) | ((uint32_t)a << 2) | (uint32_t)b;
      }
  // streams: diagonal blocks grouped by row, off-diagonal blocks grouped by
  // unique edge (i < j, in row-major (i, slot) order), tets ascending in each
  t.dptr.assign(V + 1, 0);
  for (int i = 0; i < V; ++i) t.dptr[i + 1] = t.dptr[i] + (cnt[(int64_t)i * W + 1] - cnt[(int64_t)i * W]);
  std::vector<int64_t> edge_of(NI, -1);
  t.eitem.clear();
  for (int i = 0; i < V; ++i)
    for (size_t sl = 1; sl < nb[i].size(); ++sl) {
      const int j = nb[i][sl];
      if (j < i) continue;
      edge_of[(int64_t)i * W + sl] = (int64_t)(t.eitem.size() / 2);
      t.eitem.push_back((int32_t)((int64_t)i * W + sl));
      t.eitem.push_back((int32_t)((int64_t)j * W + slot_of(j, i)));
    }
  const int64_t NE = (int64_t)t.eitem.size() / 2;
  t.eptr.assign(NE + 1, 0);
  for (int64_t k = 0; k < NE; ++k) {
    const int64_t it = t.eitem[2 * k];
    t.eptr[k + 1] = t.eptr[k] + (cnt[it + 1] - cnt[it]);
  }
  t.cpos.assign(10LL * T, 0);
  std::vector<int32_t> dfill(t.dptr.begin(), t.dptr.end() - 1);
  std::vector<int32_t> efill(t.eptr.begin(), t.eptr.end() - 1);
  static const int kPair[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  for (int e = 0; e < T; ++e) {
    const int32_t* tv = m->tets + 4LL * e;
    for (int a = 0; a < 4; ++a) t.cpos[10LL * e + a] = dfill[tv[a]]++;
    for (int k = 0; k < 6; ++k) {
      const int i = std::min(tv[kPair[k][0]], tv[kPair[k][1]]), j = std::max(tv[kPair[k][0]], tv[kPair[k][1]]);
      const int64_t ek = edge_of[(int64_t)i * W + slot_of(i, j)];
      t.cpos[10LL * e + 4 + k] = efill[ek]++;
    }
  }
}

}  // namespace tc
