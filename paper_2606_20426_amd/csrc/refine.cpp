// Conforming adaptive refinement of a tet mesh by terminal-edge bisection,
// driven by the contact sizing field of Sec. III-A (host setup code; see
// tc_refine_mesh in tacauchy.h for the field and the procedure, whose order
// fixes the result).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <string>
#include <unordered_map>
#include <vector>

#include "runtime.h"

// every sum and product is rounded on its own (no fused multiply-add), so the
// result is reproducible across compilers and equal to a plain FP64 reading
#pragma clang fp contract(off)

namespace {

using tc::set_error;

struct Field {
  int k = 2, u = 0, v = 1, side = 1;
  double lo[3], hi[3], half[3], H = 0, cu = 0, cv = 0;
  double band = 0.15, inner = 0.4, trans = 0.2, lc = 0.8e-3, lg = 3.2e-3;

  double h(const double* p) const {
    const double depth = side > 0 ? hi[k] - p[k] : p[k] - lo[k];
    if (depth > band * H) return lg;
    const double du = (p[u] - cu) / half[u];
    const double dv = (p[v] - cv) / half[v];
    const double rho = std::sqrt(du * du + dv * dv);
    if (rho <= inner) return lc;
    if (rho >= inner + trans) return lg;
    const double w = 0.5 * (1.0 + std::cos(M_PI * (rho - inner) / trans));
    return lg + (lc - lg) * w;
  }
};

constexpr int kPairs[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

struct Refiner {
  std::vector<std::array<double, 3>> X;
  std::vector<std::array<int32_t, 4>> T;
  std::vector<int32_t> M;
  std::unordered_map<uint64_t, std::vector<int32_t>> around;
  const Field* f = nullptr;

  static uint64_t ekey(int32_t a, int32_t b) {
    if (a > b) std::swap(a, b);
    return ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
  }
  static int32_t ea(uint64_t e) { return (int32_t)(e >> 32); }
  static int32_t eb(uint64_t e) { return (int32_t)(e & 0xffffffffu); }

  double len2(uint64_t e) const {
    const auto& a = X[ea(e)];
    const auto& b = X[eb(e)];
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return dx * dx + dy * dy + dz * dz;
  }
  // order: squared length, then smaller id, then larger id
  bool less(uint64_t p, uint64_t q) const {
    const double lp = len2(p), lq = len2(q);
    if (lp != lq) return lp < lq;
    return p < q;
  }
  void edges(int32_t t, uint64_t out[6]) const {
    for (int j = 0; j < 6; ++j) out[j] = ekey(T[t][kPairs[j][0]], T[t][kPairs[j][1]]);
  }
  uint64_t longest(int32_t t) const {
    uint64_t e[6];
    edges(t, e);
    uint64_t best = e[0];
    for (int j = 1; j < 6; ++j)
      if (less(best, e[j])) best = e[j];
    return best;
  }
  bool too_long(uint64_t e) const {
    const auto& a = X[ea(e)];
    const auto& b = X[eb(e)];
    const double m[3] = {0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1]), 0.5 * (a[2] + b[2])};
    const double h = f->h(m);
    return len2(e) > 3.0 * h * h;
  }
  bool needs(int32_t t) const {
    uint64_t e[6];
    edges(t, e);
    for (int j = 0; j < 6; ++j)
      if (too_long(e[j])) return true;
    return false;
  }
  void add(int32_t t) {
    uint64_t e[6];
    edges(t, e);
    for (int j = 0; j < 6; ++j) around[e[j]].push_back(t);
  }
  void remove(int32_t t) {
    uint64_t e[6];
    edges(t, e);
    for (int j = 0; j < 6; ++j) {
      auto it = around.find(e[j]);
      auto& v = it->second;
      v.erase(std::find(v.begin(), v.end(), t));
      if (v.empty()) around.erase(it);
    }
  }

  tc_status run(int64_t max_tets) {
    for (int32_t t = 0; t < (int32_t)T.size(); ++t) add(t);
    std::deque<int32_t> queue;
    for (int32_t t = 0; t < (int32_t)T.size(); ++t) queue.push_back(t);
    while (!queue.empty()) {
      const int32_t t = queue.front();
      queue.pop_front();
      while (needs(t)) {
        uint64_t e = longest(t);
        for (;;) {
          uint64_t nxt = e;
          for (int32_t s : around[e]) {
            const uint64_t ls = longest(s);
            if (less(nxt, ls)) nxt = ls;
          }
          if (nxt == e) break;
          e = nxt;
        }
        const int32_t a = ea(e), b = eb(e);
        const auto pa = X[a], pb = X[b];
        X.push_back({0.5 * (pa[0] + pb[0]), 0.5 * (pa[1] + pb[1]), 0.5 * (pa[2] + pb[2])});
        const int32_t m = (int32_t)X.size() - 1;
        std::vector<int32_t> ring = around[e];
        std::sort(ring.begin(), ring.end());
        for (int32_t s : ring) {
          if ((int64_t)T.size() >= max_tets) return set_error(TC_E_INVALID_ARG, "refinement exceeds max_tets");
          remove(s);
          const std::array<int32_t, 4> old = T[s];
          std::array<int32_t, 4> keep = old, fresh = old;
          for (int j = 0; j < 4; ++j) {
            if (old[j] == b) keep[j] = m;
            if (old[j] == a) fresh[j] = m;
          }
          T[s] = keep;
          T.push_back(fresh);
          M.push_back(M[s]);
          const int32_t n = (int32_t)T.size() - 1;
          add(s);
          add(n);
          queue.push_back(s);
          queue.push_back(n);
        }
      }
    }
    return TC_OK;
  }
};

}  // namespace

extern "C" {

tc_status tc_sizing_default(tc_sizing* out) {
  if (!out) return set_error(TC_E_INVALID_ARG, "out is null");
  std::memset(out, 0, sizeof *out);
  out->axis = -1;
  out->side = 1;
  out->band = 0.15;
  out->inner = 0.4;
  out->transition = 0.2;
  out->l_contact = 0.8e-3;
  out->l_global = 3.2e-3;
  out->centre[0] = NAN;
  out->centre[1] = NAN;
  out->max_tets = 1 << 24;
  return TC_OK;
}

tc_status tc_refine_mesh(const tc_mesh* in, const tc_sizing* s, int32_t cap_verts, int32_t cap_tets,
                         double* xyz_out, int32_t* tets_out, int32_t* mat_out, int32_t* n_verts_out,
                         int32_t* n_tets_out) {
  if (!in || !s || !n_verts_out || !n_tets_out) return set_error(TC_E_INVALID_ARG, "null argument");
  std::string err;
  tc_status st = tc::validate_mesh(in, TC_MAX_MATERIALS, err);
  if (st) return set_error(st, err);
  if (s->axis < -1 || s->axis > 2 || (s->side != 1 && s->side != -1))
    return set_error(TC_E_INVALID_ARG, "sizing: axis in -1..2, side +1 or -1");
  const double pos[] = {s->band, s->inner, s->transition, s->l_contact, s->l_global};
  for (double v : pos)
    if (!std::isfinite(v) || !(v > 0)) return set_error(TC_E_INVALID_ARG, "sizing: band, inner, transition, l_contact, l_global must be > 0");
  if (s->max_tets < in->n_tets || s->max_tets > ((int64_t)1 << 30))
    return set_error(TC_E_INVALID_ARG, "sizing: max_tets must be in [n_tets, 2^30]");
  try {
    Refiner r;
    const int V = in->n_verts, T = in->n_tets;
    r.X.resize(V);
    for (int i = 0; i < V; ++i)
      for (int c = 0; c < 3; ++c) r.X[i][c] = in->rest_xyz[3 * i + c];
    r.T.resize(T);
    r.M.resize(T);
    for (int t = 0; t < T; ++t) {
      for (int j = 0; j < 4; ++j) r.T[t][j] = in->tets[4 * t + j];
      r.M[t] = in->tet_material ? in->tet_material[t] : 0;
    }
    Field f;
    for (int c = 0; c < 3; ++c) { f.lo[c] = INFINITY; f.hi[c] = -INFINITY; }
    for (int i = 0; i < V; ++i)
      for (int c = 0; c < 3; ++c) {
        f.lo[c] = std::min(f.lo[c], r.X[i][c]);
        f.hi[c] = std::max(f.hi[c], r.X[i][c]);
      }
    double ext[3];
    for (int c = 0; c < 3; ++c) {
      ext[c] = f.hi[c] - f.lo[c];
      f.half[c] = 0.5 * ext[c];
    }
    if (s->axis < 0) {
      f.k = 0;
      for (int c = 1; c < 3; ++c)
        if (ext[c] < ext[f.k]) f.k = c;
    } else {
      f.k = s->axis;
    }
    f.u = f.k == 0 ? 1 : 0;
    f.v = f.k == 2 ? 1 : 2;
    f.side = s->side;
    f.H = ext[f.k];
    f.cu = std::isnan(s->centre[0]) ? 0.5 * (f.lo[f.u] + f.hi[f.u]) : s->centre[0];
    f.cv = std::isnan(s->centre[1]) ? 0.5 * (f.lo[f.v] + f.hi[f.v]) : s->centre[1];
    f.band = s->band;
    f.inner = s->inner;
    f.trans = s->transition;
    f.lc = s->l_contact;
    f.lg = s->l_global;
    if (!(f.half[f.u] > 0) || !(f.half[f.v] > 0)) return set_error(TC_E_INVALID_ARG, "mesh is flat in the contact plane");
    r.f = &f;
    if ((st = r.run(s->max_tets))) return st;
    *n_verts_out = (int32_t)r.X.size();
    *n_tets_out = (int32_t)r.T.size();
    if (cap_verts < (int64_t)r.X.size() || cap_tets < (int64_t)r.T.size())
      return set_error(TC_E_INVALID_ARG, "output capacity too small (sizes reported)");
    if (!xyz_out || !tets_out) return set_error(TC_E_INVALID_ARG, "output arrays are null");
    for (size_t i = 0; i < r.X.size(); ++i)
      for (int c = 0; c < 3; ++c) xyz_out[3 * i + c] = r.X[i][c];
    for (size_t t = 0; t < r.T.size(); ++t) {
      for (int j = 0; j < 4; ++j) tets_out[4 * t + j] = r.T[t][j];
      if (mat_out) mat_out[t] = r.M[t];
    }
    return TC_OK;
  } catch (const std::bad_alloc&) {
    return set_error(TC_E_NO_MEMORY, "host allocation failed");
  }
}

}  // extern "C"
