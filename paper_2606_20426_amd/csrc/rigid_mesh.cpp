// Rigid triangle meshes as indenter shapes (TC_MESH): validation,
// pseudonormals and a bounding-volume hierarchy built on the host, one
// device allocation per mesh, registered in the context's device table that
// the kernels index by tc_indenter.reserved.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <utility>
#include <vector>

#include "runtime.h"

namespace tc {

namespace {

constexpr int kLeaf = 4;   // triangles per leaf

using Vec3 = std::array<double, 3>;

Vec3 sub(const Vec3& a, const Vec3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
Vec3 cross(const Vec3& a, const Vec3& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
double dot(const Vec3& a, const Vec3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
double norm(const Vec3& a) { return std::sqrt(dot(a, a)); }

struct Tree {
  std::vector<BvhNode> nodes;
  std::vector<int> order;   // triangle of each leaf slot
};

// Median split on the longest axis of the centroids' box (ties broken by
// triangle index, so the tree is deterministic); depth-first node order.
int build(Tree& t, int lo, int hi, const std::vector<Vec3>& cen, const std::vector<std::array<double, 6>>& box) {
  const int me = (int)t.nodes.size();
  t.nodes.push_back(BvhNode{});
  BvhNode nd{};
  for (int i = 0; i < 3; ++i) { nd.lo[i] = INFINITY; nd.hi[i] = -INFINITY; }
  Vec3 clo{INFINITY, INFINITY, INFINITY}, chi{-INFINITY, -INFINITY, -INFINITY};
  for (int k = lo; k < hi; ++k) {
    const int f = t.order[k];
    for (int i = 0; i < 3; ++i) {
      nd.lo[i] = std::min(nd.lo[i], box[f][i]);
      nd.hi[i] = std::max(nd.hi[i], box[f][3 + i]);
      clo[i] = std::min(clo[i], cen[f][i]);
      chi[i] = std::max(chi[i], cen[f][i]);
    }
  }
  if (hi - lo <= kLeaf) {
    nd.first = lo;
    nd.count = hi - lo;
    t.nodes[me] = nd;
    return me;
  }
  int ax = 0;
  for (int i = 1; i < 3; ++i)
    if (chi[i] - clo[i] > chi[ax] - clo[ax]) ax = i;
  const int mid = (lo + hi) / 2;
  std::nth_element(t.order.begin() + lo, t.order.begin() + mid, t.order.begin() + hi, [&](int a, int b) {
    return cen[a][ax] < cen[b][ax] || (cen[a][ax] == cen[b][ax] && a < b);
  });
  build(t, lo, mid, cen, box);
  const int right = build(t, mid, hi, cen, box);
  nd.first = right;
  nd.count = 0;
  t.nodes[me] = nd;
  return me;
}

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

tc_status check_meshes(const tc_context* ctx, int n_ind, const tc_indenter* ind) {
  std::lock_guard<std::mutex> lk(ctx->mesh_mu);
  for (int k = 0; k < n_ind; ++k)
    if (ind[k].shape == TC_MESH) {
      const int id = ind[k].reserved;
      if (id < 0 || id >= (int)ctx->mesh_slots.size() || !ctx->mesh_slots[id].live)
        return set_error(TC_E_INVALID_ARG, "indenter " + std::to_string(k) + ": mesh id " + std::to_string(id) +
                                               " is not registered");
    }
  return TC_OK;
}

void free_meshes(tc_context* ctx) {
  std::lock_guard<std::mutex> lk(ctx->mesh_mu);
  for (auto& m : ctx->mesh_slots)
    if (m.live) {
      ctx->dev_free(m.mem, m.bytes);
      m = tc_context::MeshSlot{};
    }
}

}  // namespace tc

using namespace tc;

namespace {

// Host tables of a mesh: hierarchy nodes, triangles in leaf order with their
// normals and feature ids, edge and vertex pseudonormals.
struct Tables {
  Tree tree;
  std::vector<double> tv, tn, enf, vnf;
  std::vector<int32_t> tid_l;
  // vertex-face and edge-edge pairs: vertex positions and areas (a third of
  // the incident triangle areas), edge ends and lengths, and per leaf slot
  // the vertices and edges that slot owns (first slot in leaf order that
  // has them)
  std::vector<double> mv, va, mel;
  std::vector<int32_t> me;
  std::vector<uint8_t> own;
  bool convex = false;
};

// A closed, consistently oriented surface bounds a convex body when it is
// connected and no edge is concave (the far corner of each neighbouring
// triangle lies on or below a triangle's plane); the distance to it is then
// a convex function outside.
bool surface_is_convex(const std::vector<Vec3>& V, const int32_t* tris, int n_tris, const std::vector<Vec3>& fn) {
  std::map<std::pair<int, int>, int> dir_tri;
  for (int f = 0; f < n_tris; ++f)
    for (int k = 0; k < 3; ++k) dir_tri[{tris[3 * f + k], tris[3 * f + (k + 1) % 3]}] = f;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (const Vec3& v : V)
    for (int i = 0; i < 3; ++i) { lo[i] = std::min(lo[i], v[i]); hi[i] = std::max(hi[i], v[i]); }
  const double tol = 1e-9 * std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                      (hi[2] - lo[2]) * (hi[2] - lo[2]));
  std::vector<int> parent(n_tris);
  std::iota(parent.begin(), parent.end(), 0);
  auto root = [&](int x) {
    while (parent[x] != x) x = parent[x] = parent[parent[x]];
    return x;
  };
  bool convex = true;
  for (const auto& de : dir_tri) {
    const int f1 = de.second, f2 = dir_tri.at({de.first.second, de.first.first});
    parent[root(f1)] = root(f2);
    int far = -1;
    for (int k = 0; k < 3; ++k) {
      const int v = tris[3 * f2 + k];
      if (v != de.first.first && v != de.first.second) far = v;
    }
    if (dot(fn[f1], sub(V[far], V[de.first.first])) > tol) convex = false;
  }
  for (int f = 0; f < n_tris; ++f)
    if (root(f) != root(0)) convex = false;
  return convex;
}

tc_status mesh_tables(int32_t n_verts, const double* verts, int32_t n_tris, const int32_t* tris, Tables& out) {
  if (!verts || !tris) return set_error(TC_E_INVALID_ARG, "null argument");
  if (n_verts < 4 || n_tris < 4 || n_tris > (1 << 24))
    return set_error(TC_E_INVALID_ARG, "a closed mesh needs >= 4 vertices and 4..2^24 triangles");
  {
    std::vector<Vec3> V(n_verts);
    for (int i = 0; i < n_verts; ++i) {
      for (int c = 0; c < 3; ++c) {
        V[i][c] = verts[3 * i + c];
        if (!std::isfinite(V[i][c])) return set_error(TC_E_INVALID_ARG, "vertex coordinates must be finite");
      }
    }
    // closed and consistently oriented: each directed edge once, its
    // reverse once
    std::map<std::pair<int, int>, int> directed;
    std::vector<Vec3> fn(n_tris), cen(n_tris);
    std::vector<std::array<double, 6>> box(n_tris);
    double vol6 = 0.0;
    for (int f = 0; f < n_tris; ++f) {
      const int a = tris[3 * f], b = tris[3 * f + 1], c = tris[3 * f + 2];
      if (a < 0 || b < 0 || c < 0 || a >= n_verts || b >= n_verts || c >= n_verts || a == b || b == c || a == c)
        return set_error(TC_E_INVALID_ARG, "triangle " + std::to_string(f) + ": bad vertex index");
      const int t[3] = {a, b, c};
      for (int k = 0; k < 3; ++k)
        if (++directed[{t[k], t[(k + 1) % 3]}] > 1)
          return set_error(TC_E_INVALID_ARG, "mesh is not consistently oriented (directed edge used twice)");
      const Vec3 cr = cross(sub(V[b], V[a]), sub(V[c], V[a]));
      const double L = norm(cr);
      const double e2 = std::max({dot(sub(V[b], V[a]), sub(V[b], V[a])), dot(sub(V[c], V[a]), sub(V[c], V[a])),
                                  dot(sub(V[c], V[b]), sub(V[c], V[b]))});
      if (!(L > 1e-12 * e2)) return set_error(TC_E_INVALID_ARG, "triangle " + std::to_string(f) + " is degenerate");
      fn[f] = {cr[0] / L, cr[1] / L, cr[2] / L};
      vol6 += dot(V[a], cross(V[b], V[c]));
      for (int i = 0; i < 3; ++i) {
        cen[f][i] = (V[a][i] + V[b][i] + V[c][i]) / 3.0;
        box[f][i] = std::min({V[a][i], V[b][i], V[c][i]});
        box[f][3 + i] = std::max({V[a][i], V[b][i], V[c][i]});
      }
    }
    for (const auto& e : directed)
      if (!directed.count({e.first.second, e.first.first}))
        return set_error(TC_E_INVALID_ARG, "mesh is not closed (an edge has one triangle)");
    if (!(vol6 > 0)) return set_error(TC_E_INVALID_ARG, "mesh normals must point outward (enclosed volume <= 0)");
    // edge ids and pseudonormals
    std::map<std::pair<int, int>, int> edge_id;
    std::vector<int32_t> tid(6 * (size_t)n_tris);
    std::vector<Vec3> en, vn(n_verts, Vec3{0, 0, 0});
    for (int f = 0; f < n_tris; ++f) {
      const int t[3] = {tris[3 * f], tris[3 * f + 1], tris[3 * f + 2]};
      for (int k = 0; k < 3; ++k) {
        const std::pair<int, int> key{std::min(t[k], t[(k + 1) % 3]), std::max(t[k], t[(k + 1) % 3])};
        auto it = edge_id.find(key);
        if (it == edge_id.end()) {
          it = edge_id.emplace(key, (int)en.size()).first;
          en.push_back(Vec3{0, 0, 0});
        }
        for (int i = 0; i < 3; ++i) en[it->second][i] += fn[f][i];
        tid[6 * (size_t)f + k] = t[k];
        tid[6 * (size_t)f + 3 + k] = it->second;
        // interior angle at corner k
        const Vec3 u = sub(V[t[(k + 1) % 3]], V[t[k]]), w = sub(V[t[(k + 2) % 3]], V[t[k]]);
        const double ang = std::acos(std::max(-1.0, std::min(1.0, dot(u, w) / (norm(u) * norm(w)))));
        for (int i = 0; i < 3; ++i) vn[t[k]][i] += ang * fn[f][i];
      }
    }
    // hierarchy; triangles stored in leaf order
    Tree tree;
    tree.order.resize(n_tris);
    std::iota(tree.order.begin(), tree.order.end(), 0);
    build(tree, 0, n_tris, cen, box);
    std::vector<double> tv(9 * (size_t)n_tris), tn(3 * (size_t)n_tris);
    std::vector<int32_t> tid_l(6 * (size_t)n_tris);
    for (int s = 0; s < n_tris; ++s) {
      const int f = tree.order[s];
      for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) tv[9 * (size_t)s + 3 * k + i] = V[tris[3 * f + k]][i];
      for (int i = 0; i < 3; ++i) tn[3 * (size_t)s + i] = fn[f][i];
      for (int j = 0; j < 6; ++j) tid_l[6 * (size_t)s + j] = tid[6 * (size_t)f + j];
    }
    std::vector<double> enf(3 * en.size()), vnf(3 * (size_t)n_verts);
    for (size_t e = 0; e < en.size(); ++e)
      for (int i = 0; i < 3; ++i) enf[3 * e + i] = en[e][i];
    for (int v = 0; v < n_verts; ++v)
      for (int i = 0; i < 3; ++i) vnf[3 * (size_t)v + i] = vn[v][i];
    std::vector<double> mv(3 * (size_t)n_verts), va(n_verts, 0.0), mel(en.size());
    std::vector<int32_t> me(2 * en.size());
    for (int v = 0; v < n_verts; ++v)
      for (int i = 0; i < 3; ++i) mv[3 * (size_t)v + i] = V[v][i];
    for (int f = 0; f < n_tris; ++f) {
      const Vec3 cr = cross(sub(V[tris[3 * f + 1]], V[tris[3 * f]]), sub(V[tris[3 * f + 2]], V[tris[3 * f]]));
      for (int k = 0; k < 3; ++k) va[tris[3 * f + k]] += 0.5 * norm(cr) / 3.0;
    }
    for (const auto& kv : edge_id) {
      me[2 * (size_t)kv.second] = kv.first.first;
      me[2 * (size_t)kv.second + 1] = kv.first.second;
      mel[kv.second] = norm(sub(V[kv.first.second], V[kv.first.first]));
    }
    std::vector<uint8_t> own(n_tris, 0), v_seen(n_verts, 0), e_seen(en.size(), 0);
    for (int s = 0; s < n_tris; ++s)
      for (int k = 0; k < 3; ++k) {
        const int v = tid_l[6 * (size_t)s + k], e = tid_l[6 * (size_t)s + 3 + k];
        if (!v_seen[v]) { v_seen[v] = 1; own[s] |= (uint8_t)(1u << k); }
        if (!e_seen[e]) { e_seen[e] = 1; own[s] |= (uint8_t)(1u << (3 + k)); }
      }
    out.mv = std::move(mv);
    out.va = std::move(va);
    out.mel = std::move(mel);
    out.me = std::move(me);
    out.own = std::move(own);
    out.convex = surface_is_convex(V, tris, n_tris, fn);
    out.tree = std::move(tree);
    out.tv = std::move(tv);
    out.tn = std::move(tn);
    out.tid_l = std::move(tid_l);
    out.enf = std::move(enf);
    out.vnf = std::move(vnf);
  }
  return TC_OK;
}

}  // namespace

extern "C" {

tc_status tc_validate_rigid_mesh(int32_t n_verts, const double* verts, int32_t n_tris, const int32_t* tris) {
  try {
    Tables t;
    return mesh_tables(n_verts, verts, n_tris, tris, t);
  } catch (const std::bad_alloc&) {
    return set_error(TC_E_NO_MEMORY, "host allocation failed");
  }
}

tc_status tc_rigid_mesh_create(tc_context* ctx, int32_t n_verts, const double* verts, int32_t n_tris,
                               const int32_t* tris, int32_t* id) {
  if (!ctx || !id) return set_error(TC_E_INVALID_ARG, "null argument");
  *id = -1;
  try {
    Tables tb;
    tc_status vs = mesh_tables(n_verts, verts, n_tris, tris, tb);
    if (vs) return vs;
    const Tree& tree = tb.tree;
    const std::vector<double>& tv = tb.tv;
    const std::vector<double>& tn = tb.tn;
    const std::vector<int32_t>& tid_l = tb.tid_l;
    const std::vector<double>& enf = tb.enf;
    const std::vector<double>& vnf = tb.vnf;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    int slot = -1;
    {
      std::lock_guard<std::mutex> ml(ctx->mesh_mu);
      for (int k = 0; k < (int)ctx->mesh_slots.size(); ++k)
        if (!ctx->mesh_slots[k].live && !ctx->mesh_slots[k].mem) { slot = k; break; }
      // reserve the slot while the tables upload (mem set, not yet live)
      if (slot >= 0) ctx->mesh_slots[slot].mem = reinterpret_cast<void*>(1);
    }
    if (slot < 0) return set_error(TC_E_NO_MEMORY, "all TC_MAX_MESHES mesh slots are in use");
    auto unreserve = [&] {
      std::lock_guard<std::mutex> ml(ctx->mesh_mu);
      ctx->mesh_slots[slot] = tc_context::MeshSlot{};
    };
    if (hipSetDevice(ctx->device) != hipSuccess) { unreserve(); return set_error(TC_E_HIP, "hipSetDevice"); }
    const size_t b_nodes = a256(sizeof(BvhNode) * tree.nodes.size()), b_tv = a256(8 * tv.size()),
                 b_tn = a256(8 * tn.size()), b_tid = a256(4 * tid_l.size()), b_en = a256(8 * enf.size()),
                 b_vn = a256(8 * vnf.size()), b_mv = a256(8 * tb.mv.size()), b_va = a256(8 * tb.va.size()),
                 b_me = a256(4 * tb.me.size()), b_mel = a256(8 * tb.mel.size()), b_own = a256(tb.own.size());
    const size_t total = b_nodes + b_tv + b_tn + b_tid + b_en + b_vn + b_mv + b_va + b_me + b_mel + b_own;
    tc_status st;
    char* mem = static_cast<char*>(ctx->dev_alloc(total, &st));
    if (!mem) { unreserve(); return st; }
    DevMesh dm{};
    dm.n_tri = n_tris;
    dm.n_node = (int)tree.nodes.size();
    dm.convex = tb.convex ? 1 : 0;
    dm.n_vert = n_verts;
    char* p = mem;
    dm.nodes = reinterpret_cast<const BvhNode*>(p); p += b_nodes;
    dm.tv = reinterpret_cast<const double*>(p); p += b_tv;
    dm.tn = reinterpret_cast<const double*>(p); p += b_tn;
    dm.tid = reinterpret_cast<const int32_t*>(p); p += b_tid;
    dm.en = reinterpret_cast<const double*>(p); p += b_en;
    dm.vn = reinterpret_cast<const double*>(p); p += b_vn;
    dm.mv = reinterpret_cast<const double*>(p); p += b_mv;
    dm.va = reinterpret_cast<const double*>(p); p += b_va;
    dm.me = reinterpret_cast<const int32_t*>(p); p += b_me;
    dm.mel = reinterpret_cast<const double*>(p); p += b_mel;
    dm.own = reinterpret_cast<const uint8_t*>(p);
    hipError_t e = hipMemcpy((void*)dm.nodes, tree.nodes.data(), sizeof(BvhNode) * tree.nodes.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)dm.tv, tv.data(), 8 * tv.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)dm.tn, tn.data(), 8 * tn.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)dm.tid, tid_l.data(), 4 * tid_l.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)dm.en, enf.data(), 8 * enf.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)dm.vn, vnf.data(), 8 * vnf.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)dm.mv, tb.mv.data(), 8 * tb.mv.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)dm.va, tb.va.data(), 8 * tb.va.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)dm.me, tb.me.data(), 4 * tb.me.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)dm.mel, tb.mel.data(), 8 * tb.mel.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)dm.own, tb.own.data(), tb.own.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_meshes + slot, &dm, sizeof(DevMesh), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      ctx->dev_free(mem, total);
      unreserve();
      return hip_fail(e, "mesh upload");
    }
    {
      std::lock_guard<std::mutex> ml(ctx->mesh_mu);
      ctx->mesh_slots[slot] = tc_context::MeshSlot{true, mem, total, tb.mv};
    }
    *id = slot;
    return TC_OK;
  } catch (const std::bad_alloc&) {
    return set_error(TC_E_NO_MEMORY, "host allocation failed");
  }
}

tc_status tc_rigid_mesh_destroy(tc_context* ctx, int32_t id) {
  if (!ctx) return set_error(TC_E_INVALID_ARG, "ctx is null");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  {
    std::lock_guard<std::mutex> ml(ctx->mesh_mu);
    if (id < 0 || id >= (int)ctx->mesh_slots.size() || !ctx->mesh_slots[id].live)
      return set_error(TC_E_INVALID_ARG, "unknown mesh id");
  }
  for (const tc_pad* p : ctx->pads)
    if (p->busy.load()) return set_error(TC_E_BUSY, "a pad has a request on a server");
  TC_HIP(hipSetDevice(ctx->device));
  TC_HIP(hipStreamSynchronize(ctx->stream));
  tc_context::MeshSlot m;
  {
    // not live from here on: new requests naming it are rejected
    std::lock_guard<std::mutex> ml(ctx->mesh_mu);
    m = ctx->mesh_slots[id];
    ctx->mesh_slots[id].live = false;
  }
  const DevMesh zero{};
  const hipError_t e = hipMemcpy(ctx->d_meshes + id, &zero, sizeof(DevMesh), hipMemcpyHostToDevice);
  ctx->dev_free(m.mem, m.bytes);
  {
    std::lock_guard<std::mutex> ml(ctx->mesh_mu);
    ctx->mesh_slots[id] = tc_context::MeshSlot{};
  }
  if (e != hipSuccess) return hip_fail(e, "mesh table update");
  return TC_OK;
}

}  // extern "C"
