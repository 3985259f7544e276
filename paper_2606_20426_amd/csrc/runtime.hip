// Runtime behind the C ABI: context, scratch arena, pads, batch plans and the
// Newton driver that sequences the kernels of kernels.hip.
#include "runtime.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>

namespace tc {

namespace {
thread_local std::string g_last_error;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

tc_status set_error(tc_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

tc_status hip_fail(hipError_t e, const char* what) {
  return set_error(e == hipErrorOutOfMemory ? TC_E_NO_MEMORY : TC_E_HIP,
                   std::string(what) + ": " + hipGetErrorString(e));
}

const std::string& last_error() { return g_last_error; }

// ------------------------------------------------------------------ arena

void* Arena::take(size_t bytes) {
  bytes = align256(bytes);
  for (auto& c : chunks) {
    for (auto it = c.free_.begin(); it != c.free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        c.free_.erase(it);
        if (len > bytes) c.free_[off + bytes] = len - bytes;
        return c.base + off;
      }
    }
  }
  return nullptr;
}

void Arena::give(void* p, size_t bytes) {
  bytes = align256(bytes);
  char* cp = static_cast<char*>(p);
  for (auto& c : chunks) {
    if (cp < c.base || cp >= c.base + c.size) continue;
    size_t off = (size_t)(cp - c.base), len = bytes;
    auto next = c.free_.lower_bound(off);
    if (next != c.free_.end() && off + len == next->first) {
      len += next->second;
      next = c.free_.erase(next);
    }
    if (next != c.free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    c.free_[off] = len;
    return;
  }
}

bool Arena::add_chunk(char* base, size_t size) {
  Chunk c{base, size, {}};
  c.free_[0] = size;
  chunks.push_back(std::move(c));
  return true;
}

std::vector<std::pair<char*, size_t>> Arena::drop_empty() {
  std::vector<std::pair<char*, size_t>> out;
  for (auto it = chunks.begin(); it != chunks.end();) {
    if (it->free_.size() == 1 && it->free_.begin()->first == 0 && it->free_.begin()->second == it->size) {
      out.push_back({it->base, it->size});
      it = chunks.erase(it);
    } else {
      ++it;
    }
  }
  return out;
}

size_t Arena::held() const {
  size_t s = 0;
  for (auto& c : chunks) s += c.size;
  return s;
}

BatchPlan::~BatchPlan() {
  // the graph's kernel nodes hold the tile and descriptor pointers below:
  // the executable graph goes first
  if (cg_exec) (void)hipGraphExecDestroy(cg_exec);
  if (cg_graph) (void)hipGraphDestroy(cg_graph);
  if (d_ctiles) (void)hipFree(d_ctiles);
  if (h_ctiles) (void)hipHostFree(h_ctiles);
  if (d_desc) (void)hipFree(d_desc);
  if (d_tiles) (void)hipFree(d_tiles);
  if (h_stage) (void)hipHostFree(h_stage);
}

// Descriptor versions are unique across all pads of the process: a plan
// built for a pad that was destroyed can never match a later pad that
// happens to reuse its address and scratch.
uint64_t next_desc_version() {
  static std::atomic<uint64_t> counter{0};
  return counter.fetch_add(1, std::memory_order_relaxed) + 1;
}

}  // namespace tc

using namespace tc;

void* tc_context::dev_alloc(size_t bytes, tc_status* st) {
  bytes = align256(bytes == 0 ? 256 : bytes);
  if (budget && used + bytes > budget) {
    *st = set_error(TC_E_NO_MEMORY, "HBM budget exceeded (" + std::to_string(used + bytes) + " > " +
                                        std::to_string(budget) + " bytes)");
    return nullptr;
  }
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    *st = hip_fail(e, "hipMalloc");
    return nullptr;
  }
  used += bytes;
  *st = TC_OK;
  return p;
}

void tc_context::dev_free(void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  used -= align256(bytes == 0 ? 256 : bytes);
}

namespace tc {

// --------------------------------------------------------------- slot pool

tc_status pool_reserve(tc_context* ctx, SlotPool& p, int cap) {
  (void)ctx;
  if (cap <= p.cap) return TC_OK;
  cap = std::max(cap, 64);
  pool_free(p);
  TC_HIP(hipMalloc(&p.d_state, sizeof(EnvState) * cap));
  TC_HIP(hipMalloc(&p.d_pose, sizeof(EnvPose) * cap));
  TC_HIP(hipHostMalloc(&p.h_state, sizeof(EnvState) * cap, hipHostMallocDefault));
  TC_HIP(hipHostMalloc(&p.h_pose, sizeof(EnvPose) * cap, hipHostMallocDefault));
  p.cap = cap;
  return TC_OK;
}

void pool_free(SlotPool& p) {
  if (p.d_state) (void)hipFree(p.d_state);
  if (p.d_pose) (void)hipFree(p.d_pose);
  if (p.h_state) (void)hipHostFree(p.h_state);
  if (p.h_pose) (void)hipHostFree(p.h_pose);
  p = SlotPool{};
}

void init_state(EnvState& S, EnvPose& Q, int mode, int n_ind, const tc_indenter* ind, const tc_pad* pad) {
  std::memset(&S, 0, sizeof S);
  S.mode = mode;
  S.phase = mode == 0 ? PH_INIT : PH_FINISH;
  S.status = TC_OK;
  std::memset(&Q, 0, sizeof Q);
  Q.n_ind = n_ind;
  const bool has_prev = pad && pad->n_prev == n_ind;
  for (int m = 0; m < n_ind; ++m) {
    std::memcpy(&Q.ind[m], &ind[m], sizeof(DevIndenter));
    std::memcpy(&Q.prev[m], has_prev ? &pad->prev[m] : &ind[m], sizeof(DevIndenter));
  }
  // vertex-face / edge-edge pairs: on with mesh_contact 2 and a mesh
  // indenter; the feasible start looks for features carried through the
  // pad surface within each mesh's travel since the previous pose
  if (!pad || pad->params.mesh_contact != 2 || pad->Se == 0) return;
  for (int m = 0; m < n_ind; ++m) {
    if (ind[m].shape != TC_MESH) continue;
    Q.pairs = 1;
    const int id = ind[m].reserved;
    const auto& slots = pad->ctx->mesh_slots;
    if (!has_prev || id < 0 || id >= (int)slots.size()) continue;
    const std::vector<double>& V = slots[id].verts;
    const DevIndenter& A = Q.ind[m];
    const DevIndenter& B = Q.prev[m];
    double t2 = 0.0;
    for (size_t v = 0; v + 2 < V.size(); v += 3) {
      double d2 = 0.0;
      for (int i = 0; i < 3; ++i) {
        const double a = A.R[3 * i] * V[v] + A.R[3 * i + 1] * V[v + 1] + A.R[3 * i + 2] * V[v + 2] + A.c[i];
        const double b = B.R[3 * i] * V[v] + B.R[3 * i + 1] * V[v + 1] + B.R[3 * i + 2] * V[v + 2] + B.c[i];
        d2 += (a - b) * (a - b);
      }
      t2 = std::max(t2, d2);
    }
    Q.travel[m] = std::sqrt(t2);
  }
}

void remember_pose(tc_pad* pad, const EnvPose& Q) {
  pad->n_prev = Q.n_ind;
  for (int m = 0; m < Q.n_ind; ++m) std::memcpy(&pad->prev[m], &Q.ind[m], sizeof(tc_indenter));
}

void fill_stats(tc_step_stats& o, const EnvState& S, double ms) {
  o.status = S.status;
  o.newton_iters = S.newton_iters;
  o.cg_iters = S.cg_total;
  o.ls_halvings = S.ls_total;
  o.final_step_inf = S.final_step_inf;
  o.energy = S.E_cur;
  for (int c = 0; c < 3; ++c) o.reaction[c] = S.reaction[c];
  o.ms = ms;
}

}  // namespace tc

namespace tc {

// ---------------------------------------------------------------- timing

static hipEvent_t get_event(tc_context* ctx) {
  if (!ctx->free_events.empty()) {
    hipEvent_t e = ctx->free_events.back();
    ctx->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Launch; while timing is on, every timing_stride-th launch of the
// self-timed CG kernels (launched tens of thousands of times per run) and
// every launch of the other kernels is timed: events recorded by the
// dispatch, or the blocks' own clock cells in the slice of the stream that
// launches.  Streams driven by different host threads each have a slice.
static hipError_t timed_launch(tc_context* ctx, TimingSlice& ts, KernelId k, bool fp64, const LaunchArgs& a) {
  if (!ctx->timing) return launch_kernel(k, fp64, a);
  bool sample;
  {
    std::lock_guard<std::mutex> lk(ctx->tmu);
    const int stride = self_timed(k) ? ctx->timing_stride : 1;
    sample = ctx->timers[(int)k].launches++ % stride == 0;
  }
  if (!sample) return launch_kernel(k, fp64, a);
  LaunchArgs b = a;
  const int blocks = ((a.ntiles + 7) / 8) * 8;   // the launch's grid
  const size_t cap = ts.cap ? ts.cap : ctx->clock_cap;
  if (self_timed(k) && a.ntiles > 0 && ts.used + 2 * (size_t)blocks <= cap) {
    // every block stamps its own start and end
    const size_t cell = ts.base + ts.used;
    ts.used += 2 * (size_t)blocks;
    b.clock = ctx->clock_cells + cell;
    const hipError_t e = launch_kernel(k, fp64, b);
    ts.pending.push_back({k, nullptr, nullptr, cell - ts.base, blocks});
    return e;
  }
  if (self_timed(k)) return launch_kernel(k, fp64, a);   // no room: not timed
  {
    std::lock_guard<std::mutex> lk(ctx->tmu);
    b.ev0 = get_event(ctx);
    b.ev1 = get_event(ctx);
  }
  const hipError_t e = launch_kernel(k, fp64, b);
  ts.pending.push_back({k, b.ev0, b.ev1, 0, -1});
  return e;
}

// Called after `stream`, the one the slice's launches went to, has been
// synchronised.  Events are read at every call; the clock cells (one more
// copy and synchronisation) only when `all` is set or the slice is half
// full, so the readbacks inside a step do not pay for them.
static void resolve_timing(tc_context* ctx, TimingSlice& ts, hipStream_t stream, bool all) {
  std::vector<unsigned long long> clk;
  const size_t cap = ts.cap ? ts.cap : ctx->clock_cap;
  const bool cells = all || 2 * ts.used > cap;
  if (cells && ts.used > 0) {
    clk.resize(ts.used);
    if (hipMemcpyAsync(clk.data(), ctx->clock_cells + ts.base, 8 * clk.size(), hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      clk.clear();
    (void)hipMemsetAsync(ctx->clock_cells + ts.base, 0, 8 * ts.used, stream);
    ts.used = 0;
  }
  std::lock_guard<std::mutex> lk(ctx->tmu);
  std::vector<Pending> keep;
  for (auto& p : ts.pending) {
    if (p.blocks >= 0) {
      if (!cells) {
        keep.push_back(p);
        continue;
      }
      if (p.cell + 2 * (size_t)p.blocks <= clk.size()) {
        // blocks past the tile list store nothing (zero cells)
        unsigned long long t0 = ~0ull, t1 = 0;
        for (int b = 0; b < p.blocks; ++b) {
          const unsigned long long s0 = clk[p.cell + 2 * b], s1 = clk[p.cell + 2 * b + 1];
          if (s0 == 0 || s1 == 0) continue;
          t0 = std::min(t0, s0);
          t1 = std::max(t1, s1);
        }
        if (t1 >= t0 && t0 != ~0ull) {
          ctx->timers[(int)p.k].ms += (double)(t1 - t0) / ctx->clock_khz;
          ctx->timers[(int)p.k].timed += 1;
        }
      }
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->timers[(int)p.k].ms += ms;
      ctx->timers[(int)p.k].timed += 1;
    }
    ctx->free_events.push_back(p.a);
    ctx->free_events.push_back(p.b);
  }
  ts.pending.swap(keep);
}

static void resolve_timing(tc_context* ctx) { resolve_timing(ctx, ctx->tslice, ctx->stream, true); }

// ------------------------------------------------------------ scratch layout

struct ScratchLayout {
  size_t Ke, A, xn, xhat, g, d, r, z, p0, p1, q, Pinv, gb, Hb, fric;
  size_t prz, ppq, pg2, pe, pdir, pfilt, pc3, ps3, prec, pflag;
  size_t total;
};

// Surface primitives with pair records (mesh_contact 2), else 0.
static size_t pair_prims(const tc_pad* p) {
  return p->params.mesh_contact == 2 ? (size_t)p->S + p->Se : 0;
}

static ScratchLayout scratch_layout(const tc_pad* p) {
  ScratchLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) { const size_t r = o; o += align256(b == 0 ? 8 : b); return r; };
  const size_t R = (size_t)p->rsize, V = p->V, T = p->T, C = std::max(p->C, 1), S = p->S;
  L.Ke = take(10 * T * KC * R);
  L.A = take((size_t)p->W * 9 * V * R);
  L.xn = take(24 * V);
  L.xhat = take(24 * V);
  L.g = take(24 * V);
  L.d = take(3 * V * R);
  L.r = take(24 * V);
  L.z = take(3 * V * R);
  L.p0 = take(3 * V * R);
  L.p1 = take(3 * V * R);
  L.q = take(3 * V * R);
  L.Pinv = take(6 * V * R);
  L.gb = take(24 * C);
  L.Hb = take(48 * C);
  L.fric = take(p->params.friction > 0 ? 8 * FRIC_STRIDE * MAX_IND * C : 0);
  const size_t nv = cdiv(V, 64), nt = cdiv(T, 64), nc = cdiv(C, 64), ns = cdiv(std::max<size_t>(S, 1), 64);
  const size_t NP = pair_prims(p), np = cdiv(NP, 64);
  L.prz = take(8 * nv);
  L.ppq = take(8 * ((size_t)cdiv(V, 2) + 1));
  L.pg2 = take(8 * nv);
  L.pe = take(8 * (nt + nv + nc + np));
  L.pdir = take(16 * nv);
  L.pfilt = take(8 * (nc + np));
  L.pc3 = take(24 * nc);
  L.ps3 = take(24 * ns);
  L.prec = take(8 * PREC * NP);
  L.pflag = take(4 * NP);
  L.total = o;
  return L;
}

static void bind_scratch_desc(tc_pad* p) {
  const ScratchLayout L = scratch_layout(p);
  // plans copy the descriptor: a rebinding (even at the same address, with
  // another layout) invalidates them
  p->desc_version = next_desc_version();
  char* b = static_cast<char*>(p->scratch);
  EnvDesc& E = p->desc;
  E.Ke = b + L.Ke;
  E.A = b + L.A;
  E.xn = (double*)(b + L.xn);
  E.xhat = (double*)(b + L.xhat);
  E.g = (double*)(b + L.g);
  E.d = b + L.d;
  E.r = (double*)(b + L.r);
  E.z = b + L.z;
  E.p0 = b + L.p0;
  E.p1 = b + L.p1;
  E.q = b + L.q;
  E.Pinv = b + L.Pinv;
  E.gb = (double*)(b + L.gb);
  E.Hb = (double*)(b + L.Hb);
  E.fric = (double*)(b + L.fric);
  E.part_rz = (double*)(b + L.prz);
  E.part_pq = (double*)(b + L.ppq);
  E.part_g2 = (double*)(b + L.pg2);
  E.part_e = (double*)(b + L.pe);
  E.part_dir = (double*)(b + L.pdir);
  E.part_filt = (double*)(b + L.pfilt);
  E.part_c3 = (double*)(b + L.pc3);
  E.part_s3 = (double*)(b + L.ps3);
  const bool pairs = pair_prims(p) > 0;
  E.prec = pairs ? (double*)(b + L.prec) : nullptr;
  E.pflag = pairs ? (int32_t*)(b + L.pflag) : nullptr;
}

tc_status ensure_scratch(tc_pad* p) {
  if (p->scratch) return TC_OK;
  tc_context* ctx = p->ctx;
  const size_t need = scratch_layout(p).total;
  void* s = ctx->arena.take(need);
  if (!s) {
    // grow the pool by a chunk (at least 256 MiB) within the budget
    const size_t chunk = std::max(align256(need), (size_t)256 << 20);
    size_t want = chunk;
    if (ctx->budget && ctx->used + want > ctx->budget) want = align256(need);
    tc_status st;
    void* base = ctx->dev_alloc(want, &st);
    if (!base) return st;
    ctx->arena.add_chunk(static_cast<char*>(base), want);
    s = ctx->arena.take(need);
    if (!s) return set_error(TC_E_NO_MEMORY, "scratch arena fragmentation");
  }
  p->scratch = s;
  p->scratch_bytes = need;
  bind_scratch_desc(p);
  return TC_OK;
}

tc_status ensure_scratch_evicting(tc_pad* p, const std::vector<tc_pad*>& keep) {
  tc_status s = ensure_scratch(p);
  if (s != TC_E_NO_MEMORY) return s;
  tc_context* ctx = p->ctx;
  std::vector<tc_pad*> idle;
  for (tc_pad* q : ctx->pads)
    if (q != p && q->scratch && !q->in_flight.load() && std::find(keep.begin(), keep.end(), q) == keep.end())
      idle.push_back(q);
  std::sort(idle.begin(), idle.end(), [](tc_pad* a, tc_pad* b) { return a->scratch_bytes > b->scratch_bytes; });
  if (!idle.empty()) (void)hipStreamSynchronize(ctx->stream);   // no kernel may still use it
  for (tc_pad* q : idle) {
    release_scratch(q);
    ctx->evictions++;
    if ((s = ensure_scratch(p)) != TC_E_NO_MEMORY) return s;
  }
  // fragmentation: hand completely free chunks back and allocate anew
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& c : ctx->arena.drop_empty()) ctx->dev_free(c.first, c.second);
  return ensure_scratch(p);
}

void release_scratch(tc_pad* p) {
  if (!p->scratch) return;
  p->ctx->arena.give(p->scratch, p->scratch_bytes);
  p->scratch = nullptr;
  p->scratch_bytes = 0;
  drop_plans(p->ctx);   // plans hold scratch pointers
}

// ------------------------------------------------------------- batch plan

tc_status get_lane(tc_context* ctx, int g) {
  while ((int)ctx->lanes.size() <= g) {
    auto L = std::make_unique<Lane>();
    TC_HIP(hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking));
    L->plan = &L->own_plan;
    L->pool = &L->own_pool;
    L->ts = &L->own_ts;
    ctx->lanes.push_back(std::move(L));
  }
  return TC_OK;
}

void drop_plans(tc_context* ctx) {
  ctx->plan.reset();
  for (auto& L : ctx->lanes) L->own_plan.reset();
}

void free_lanes(tc_context* ctx) {
  for (auto& L : ctx->lanes) {
    (void)hipStreamSynchronize(L->stream);
    L->own_plan.reset();
    pool_free(L->own_pool);
    for (auto& p : L->own_ts.pending) {
      if (p.blocks < 0) {
        ctx->free_events.push_back(p.a);
        ctx->free_events.push_back(p.b);
      }
    }
    (void)hipStreamDestroy(L->stream);
  }
  ctx->lanes.clear();
}

tc_status build_plan(tc_context* ctx, int n, tc_pad* const* pads, const int* slots, const SlotPool& pool,
                     std::unique_ptr<BatchPlan>& out, hipStream_t stream) {
  if (!stream) stream = ctx->stream;
  std::unique_ptr<BatchPlan> old = std::move(out);
  auto P = std::make_unique<BatchPlan>();
  P->slots.assign(slots, slots + n);
  P->BV = ctx->cg_block;
  P->BT = ctx->el_block;
  P->BS = ctx->spmv_block;
  P->fp64 = pads[0]->fp64;
  P->pads.assign(pads, pads + n);
  P->h_desc.resize(n);
  int Wmax = 0;
  int64_t blocks = 0, rows = 0;
  for (int i = 0; i < n; ++i) {
    Wmax = std::max(Wmax, pads[i]->W);
    blocks += pads[i]->nnz_blocks;
    rows += pads[i]->V;
  }
  // SpMV lanes per row: 16 while the rows hold 16 blocks or fewer on
  // average (a lane then takes every 16th slot of a wider row), else 32;
  // one thread per row beyond 64 slots
  const double fill = rows ? (double)blocks / (double)rows : 0.0;
  P->lpr = Wmax > 64 ? 0 : (Wmax <= 16 || fill <= 16.0) ? 16 : 32;
  const int rows_spmv = P->lpr ? (ctx->spmv_block / P->lpr) * SPMV_ROWS_PER_GROUP : P->BV;
  std::vector<Tile> tiles;
  const int BV = P->BV, BT = P->BT;
  for (int i = 0; i < n; ++i) {
    tc_pad* p = pads[i];
    P->scratch.push_back(p->scratch);
    P->versions.push_back(p->desc_version);
    EnvDesc E = p->desc;
    E.n_vt = cdiv(p->V, BV);
    E.n_tt = cdiv(p->T, BT);
    E.n_ct = p->C > 0 ? cdiv(p->C, BV) : 0;
    E.n_st = cdiv(p->S, BV);
    E.n_at = cdiv((int64_t)E.V_E, BV);
    E.n_te = cdiv(p->T, BV);
    E.n_spt = cdiv(p->V, rows_spmv);
    E.n_pt = E.prec ? cdiv((int64_t)p->S + p->Se, BV) : 0;
    E.st = pool.d_state + slots[i];
    E.pose = pool.d_pose + slots[i];
    P->h_desc[i] = E;
  }
  auto add_cls = [&](BatchPlan::Cls c, auto count_of) {
    P->off[c] = (int)tiles.size();
    for (int i = 0; i < n; ++i) {
      const int k = count_of(P->h_desc[i]);
      for (int t = 0; t < k; ++t) tiles.push_back(Tile{i, t});
    }
    P->cnt[c] = (int)tiles.size() - P->off[c];
  };
  add_cls(BatchPlan::VERT, [](const EnvDesc& E) { return E.n_vt; });
  add_cls(BatchPlan::TET, [](const EnvDesc& E) { return E.n_tt; });
  add_cls(BatchPlan::CAND, [](const EnvDesc& E) { return E.n_ct; });
  add_cls(BatchPlan::SURF, [](const EnvDesc& E) { return E.n_st; });
  add_cls(BatchPlan::ASM, [](const EnvDesc& E) { return E.n_at; });
  add_cls(BatchPlan::ENERGY, [](const EnvDesc& E) { return E.n_te + E.n_vt + E.n_ct; });
  add_cls(BatchPlan::SPMV, [](const EnvDesc& E) { return E.n_spt; });
  add_cls(BatchPlan::PAIR, [](const EnvDesc& E) { return E.n_pt; });
  // buffers of the replaced plan are taken over when large enough (its graph
  // executable, which holds their addresses, is destroyed with it below);
  // new ones get 25 % headroom
  const int nt = std::max<int>((int)tiles.size(), 1);
  const int ring = 4 * (int)tiles.size() + 64;
  if (old && old->desc_cap >= n) {
    std::swap(P->d_desc, old->d_desc);
    P->desc_cap = old->desc_cap;
  } else {
    P->desc_cap = n + n / 4 + 1;
    TC_HIP(hipMalloc(&P->d_desc, sizeof(EnvDesc) * P->desc_cap));
  }
  if (old && old->tiles_cap >= nt) {
    std::swap(P->d_tiles, old->d_tiles);
    P->tiles_cap = old->tiles_cap;
  } else {
    P->tiles_cap = nt + nt / 4;
    TC_HIP(hipMalloc(&P->d_tiles, sizeof(Tile) * P->tiles_cap));
  }
  if (old && old->ctiles_cap >= ring) {
    std::swap(P->d_ctiles, old->d_ctiles);
    std::swap(P->h_ctiles, old->h_ctiles);
    P->ctiles_cap = old->ctiles_cap;
  } else {
    P->ctiles_cap = ring + ring / 4;
    TC_HIP(hipMalloc(&P->d_ctiles, sizeof(Tile) * P->ctiles_cap));
    TC_HIP(hipHostMalloc(&P->h_ctiles, sizeof(Tile) * P->ctiles_cap, hipHostMallocDefault));
  }
  // the uploads go through pinned staging, asynchronously; a staging buffer
  // taken over may still feed the last rebuild's copies only if that call
  // ended early (every step, tick and probe ends with a readback), so the
  // stream, normally idle here, is waited for first
  const size_t stage_need = sizeof(EnvDesc) * n + sizeof(Tile) * tiles.size();
  if (old && old->stage_cap >= stage_need) {
    TC_HIP(hipStreamSynchronize(stream));
    std::swap(P->h_stage, old->h_stage);
    P->stage_cap = old->stage_cap;
  } else {
    P->stage_cap = stage_need + stage_need / 4 + 64;
    TC_HIP(hipHostMalloc(&P->h_stage, P->stage_cap, hipHostMallocDefault));
  }
  old.reset();
  std::memcpy(P->h_stage, P->h_desc.data(), sizeof(EnvDesc) * n);
  std::memcpy(P->h_stage + sizeof(EnvDesc) * n, tiles.data(), sizeof(Tile) * tiles.size());
  TC_HIP(hipMemcpyAsync(P->d_desc, P->h_stage, sizeof(EnvDesc) * n, hipMemcpyHostToDevice, stream));
  TC_HIP(hipMemcpyAsync(P->d_tiles, P->h_stage + sizeof(EnvDesc) * n, sizeof(Tile) * tiles.size(),
                        hipMemcpyHostToDevice, stream));
  P->d_state = pool.d_state;
  out = std::move(P);
  return TC_OK;
}

bool plan_matches(const BatchPlan* P, tc_context* ctx, int n, tc_pad* const* pads, const int* slots,
                  const SlotPool& pool) {
  if (!P || (int)P->pads.size() != n || P->BV != ctx->cg_block || P->BT != ctx->el_block || P->BS != ctx->spmv_block ||
      P->d_state != pool.d_state)
    return false;
  for (int i = 0; i < n; ++i)
    if (P->pads[i] != pads[i] || P->scratch[i] != pads[i]->scratch || P->slots[i] != slots[i] ||
        P->versions[i] != pads[i]->desc_version)
      return false;
  return true;
}

// ----------------------------------------------------------------- driver

void Runner::launch(KernelId k, int cls, int parity, int mode) {
  LaunchArgs a;
  a.envs = P->d_desc;
  a.n_env = n;
  a.parity = parity;
  a.mode = mode;
  a.stream = strm();
  if (cls != BatchPlan::NCLS) {
    a.tiles = P->d_tiles + P->off[cls];
    a.ntiles = P->cnt[cls];
    a.block = cls == BatchPlan::TET ? P->BT : (cls == BatchPlan::SPMV && P->lpr) ? P->BS : P->BV;
    a.lpr = P->lpr;
  }
  (void)timed_launch(ctx, slice(), k, P->fp64, a);
}

void Runner::launch_tiles(KernelId k, const Tile* tiles, int ntiles, int block, int parity, int mode) {
  LaunchArgs a;
  a.envs = P->d_desc;
  a.n_env = n;
  a.parity = parity;
  a.mode = mode;
  a.stream = strm();
  a.tiles = tiles;
  a.ntiles = ntiles;
  a.block = block;
  a.lpr = P->lpr;
  (void)timed_launch(ctx, slice(), k, P->fp64, a);
}

Runner::View Runner::view(bool (*pred)(const EnvState&), unsigned mask, bool copy) {
  View v{};
  int nm = 0;
  for (int i = 0; i < n; ++i) nm += pred(state(i));
  v.full = nm == n;
  if (v.full) {
    for (int c = 0; c < BatchPlan::NCLS; ++c) {
      v.t[c] = P->d_tiles + P->off[c];
      v.c[c] = P->cnt[c];
    }
    return v;
  }
  // compacted lists go to the next free part of the ring; the ring is only
  // rewritten after a host sync, when every earlier copy and launch is done
  const int base = P->ctiles_off;
  for (int c = 0; c < BatchPlan::NCLS; ++c) {
    const int start = P->ctiles_off;
    v.t[c] = P->d_ctiles + start;
    v.c[c] = 0;
    if (!(mask >> c & 1u)) continue;
    int k = start;
    for (int i = 0; i < n; ++i) {
      if (!pred(state(i))) continue;
      const EnvDesc& E = P->h_desc[i];
      const int cnt = c == BatchPlan::VERT ? E.n_vt : c == BatchPlan::TET ? E.n_tt : c == BatchPlan::CAND ? E.n_ct
                    : c == BatchPlan::SURF ? E.n_st : c == BatchPlan::ASM ? E.n_at
                    : c == BatchPlan::ENERGY ? E.n_te + E.n_vt + E.n_ct
                    : c == BatchPlan::PAIR ? E.n_pt : E.n_spt;
      if (k + cnt > P->ctiles_cap) {   // cannot happen (4x capacity); never launch a truncated list
        ring_overflow = true;
        break;
      }
      for (int t = 0; t < cnt; ++t) P->h_ctiles[k++] = Tile{i, t};
    }
    v.c[c] = k - start;
    P->ctiles_off = k;
  }
  if (unflushed < 0) unflushed = base;
  if (copy) flush_views();
  return v;
}

void Runner::flush_views() {
  if (unflushed < 0) return;
  const int len = P->ctiles_off - unflushed;
  if (len > 0)
    (void)hipMemcpyAsync(P->d_ctiles + unflushed, P->h_ctiles + unflushed, sizeof(Tile) * len,
                         hipMemcpyHostToDevice, strm());
  unflushed = -1;
}

void Runner::launch_v(KernelId k, const View& v, int cls, int parity, int mode) {
  const int block = cls == BatchPlan::TET ? P->BT : (cls == BatchPlan::SPMV && P->lpr) ? P->BS : P->BV;
  launch_tiles(k, v.t[cls], v.c[cls], block, parity, mode);
}

tc_status Runner::readback() {
  TC_HIP(hipGetLastError());
  if (ring_overflow) return set_error(TC_E_HIP, "compacted tile lists overflowed their ring");
  TC_HIP(hipMemcpyAsync(pool->h_state, pool->d_state, sizeof(EnvState) * span, hipMemcpyDeviceToHost, strm()));
  TC_HIP(hipStreamSynchronize(strm()));
  P->ctiles_off = 0;
  unflushed = -1;
  if (ctx->timing) resolve_timing(ctx, slice(), strm(), false);
  return TC_OK;
}

bool Runner::any(bool (*pred)(const EnvState&)) const {
  for (int i = 0; i < n; ++i)
    if (pred(state(i))) return true;
  return false;
}

bool Runner::any_pairs(bool (*pred)(const EnvState&)) const {
  for (int i = 0; i < n; ++i)
    if (pred(state(i)) && P->h_desc[i].n_pt > 0 && pool->h_pose[P->slots[i]].pairs) return true;
  return false;
}

tc_status Runner::cg_chunk(int M, const View& v) {
  if (v.full && ctx->use_graphs && !ctx->timing) {
    if (!P->cg_exec || P->graph_M != M) {
      if (P->cg_exec) { (void)hipGraphExecDestroy(P->cg_exec); P->cg_exec = nullptr; }
      if (P->cg_graph) { (void)hipGraphDestroy(P->cg_graph); P->cg_graph = nullptr; }
      TC_HIP(hipStreamBeginCapture(strm(), hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < M; ++k) {
        launch_v(KernelId::cg_spmv, v, BatchPlan::SPMV, k & 1);
        launch_v(KernelId::cg_update, v, BatchPlan::VERT, k & 1);
      }
      TC_HIP(hipStreamEndCapture(strm(), &P->cg_graph));
      TC_HIP(hipGraphInstantiate(&P->cg_exec, P->cg_graph, nullptr, nullptr, 0));
      P->graph_M = M;
    }
    TC_HIP(hipGraphLaunch(P->cg_exec, strm()));
  } else {
    for (int k = 0; k < M; ++k) {
      launch_v(KernelId::cg_spmv, v, BatchPlan::SPMV, k & 1);
      launch_v(KernelId::cg_update, v, BatchPlan::VERT, k & 1);
    }
  }
  return TC_OK;
}

// Predict, feasible start and E(x0) of the pads being initialised.
void Runner::init_launches() {
  const View vi = view(is_init);
  launch_v(KernelId::predict, vi, BatchPlan::VERT);
  launch_v(KernelId::project, vi, BatchPlan::CAND, 0, 0);
  if (any_pairs(is_init)) {
    // pads with vertex-face / edge-edge pairs: vertex rounds alternate
    // with the surface primitives' pushes, then both checks
    for (int r = 0; r < 8; ++r) {
      launch_v(KernelId::project, vi, BatchPlan::CAND, 0, 1);
      launch_v(KernelId::pair_push, vi, BatchPlan::PAIR, 0, 0);
      launch_v(KernelId::pair_apply, vi, BatchPlan::CAND);
    }
    launch_v(KernelId::project, vi, BatchPlan::CAND, 0, 2);
    launch_v(KernelId::pair_push, vi, BatchPlan::PAIR, 0, 1);
  }
  launch_v(KernelId::energy, vi, BatchPlan::ENERGY, 0, 0);
  if (any_pairs(is_init)) launch_v(KernelId::pairs, vi, BatchPlan::PAIR, 0, 4);
  launch(KernelId::env_ls, BatchPlan::NCLS, 0, 0);
}

// Extraction and commit of the pads whose Newton solve has ended.
void Runner::finish_launches() {
  const View vf = view(is_finish);
  launch_v(KernelId::sigma, vf, BatchPlan::TET);
  launch_v(KernelId::traction, vf, BatchPlan::SURF);
  if (any_pairs(is_finish)) launch_v(KernelId::pairs, vf, BatchPlan::PAIR, 0, 1);
  launch_v(KernelId::contact, vf, BatchPlan::CAND);
  launch_v(KernelId::commit, vf, BatchPlan::VERT);
  launch(KernelId::env_extract, BatchPlan::NCLS);
}

tc_status Runner::finish() {
  if (!any(is_finish)) return TC_OK;
  finish_launches();
  return readback();
}

// Lockstep schedule: one Newton iteration for every pad in PH_RUN (pads in
// PH_INIT are initialised first and join it; pads that end up in PH_FINISH
// get their extraction).  Launches cover only the tiles of the pads
// concerned.
tc_status Runner::tick(bool init) {
  tc_status st;
  static const bool debug = std::getenv("TC_DEBUG") != nullptr;
  if (init) init_launches();
  if (any(init ? init_or_run : is_run)) {
    const View v = view(init ? init_or_run : is_run);
    launch(KernelId::newton_begin, BatchPlan::NCLS);
    launch_v(KernelId::element, v, BatchPlan::TET);
    if (any_pairs(init ? init_or_run : is_run)) launch_v(KernelId::pairs, v, BatchPlan::PAIR, 0, 0);
    launch_v(KernelId::barrier, v, BatchPlan::CAND);
    launch_v(KernelId::asm_diag, v, BatchPlan::VERT);
    launch_v(KernelId::asm_off, v, BatchPlan::ASM);
    int max_cg = 0;
    for (int i = 0; i < n; ++i) max_cg = std::max(max_cg, P->pads[i]->params.max_cg);
    const int M = std::max(2, ctx->cg_per_replay & ~1);
    View vc = v;
    int n_cur = -1;
    for (int done = 0; done <= max_cg + M; done += M) {
      if ((st = cg_chunk(M, vc))) return st;
      if ((st = readback())) return st;
      int n_act = 0;
      for (int i = 0; i < n; ++i) n_act += cg_pending(state(i));
      if (n_act == 0) break;
      if (n_cur < 0) {
        n_cur = 0;
        for (int i = 0; i < n; ++i) n_cur += is_run(state(i));
      }
      if (n_act * 4 <= n_cur * 3 || !vc.full) {
        vc = view(cg_pending);   // shrink the launches to the pads still iterating
        n_cur = n_act;
      }
    }
    // the views are rebuilt after the sync: pads may have failed meanwhile
    const View vr = view(is_run);
    launch_v(KernelId::newton_dir, vr, BatchPlan::VERT);
    launch_v(KernelId::filter, vr, BatchPlan::CAND);
    if (any_pairs(is_run)) launch_v(KernelId::pairs, vr, BatchPlan::PAIR, 0, 3);
    launch(KernelId::env_dir, BatchPlan::NCLS);
    if (debug) {
      if ((st = readback())) return st;
      for (int i = 0; i < n; ++i) {
        const EnvState& S = state(i);
        std::fprintf(stderr, "[tc] pad %d newton %d cg %d rz0 %.3e |d| %.3e g.d %.3e amax %.3e E %.12e conv %d\n", i,
                     S.newton_iters, S.cg_iters, S.rz0, S.final_step_inf, S.gTd, S.alpha_max, S.E_cur, S.dir_conv);
      }
    }
    int max_h = 0;
    for (int i = 0; i < n; ++i)
      max_h = std::max(max_h, P->pads[i]->params.max_halvings + P->pads[i]->params.ls_expand);
    // first line-search round without waiting for the direction's flags
    // (pads that converged skip it on the device)
    View vl = debug ? view(ls_pending) : vr;
    const bool ls_pairs = any_pairs(is_run);
    for (int r = 0; r <= max_h + 1; ++r) {
      launch_v(KernelId::energy, vl, BatchPlan::ENERGY, 0, 1);
      if (ls_pairs) launch_v(KernelId::pairs, vl, BatchPlan::PAIR, 0, 2);
      launch(KernelId::env_ls, BatchPlan::NCLS, 0, 1);
      if ((st = readback())) return st;
      if (debug)
        for (int i = 0; i < n; ++i) {
          const EnvState& S = state(i);
          std::fprintf(stderr, "[tc]   ls pad %d done %d halv %d alpha %.3e E_next %.12e status %d\n", i, S.ls_done,
                       S.ls_halv, S.ls_alpha, S.E_next, S.status);
        }
      if (!any(ls_pending)) break;
      vl = view(ls_pending);
    }
    const View vu = view(is_run);
    launch_v(KernelId::update, vu, BatchPlan::VERT);
    launch(KernelId::env_update, BatchPlan::NCLS);
    if ((st = readback())) return st;
  } else if (init) {
    if ((st = readback())) return st;
  }
  return finish();
}

// One round of the staged schedule, from the stages the last readback saw.
// Pads whose CG ended get their direction, step bound and K trial energies
// of the line search; pads whose search ends within the round are updated,
// and those that go on start their next Newton iteration (Hessians,
// assembly); then every pad in CG, those just assembled included, runs M CG
// iterations (M even: every pad enters its CG at parity 0).  A launch also
// covers pads that may reach the kernel's stage only within the round; the
// kernels pass over pads at another stage.  One readback ends the round.
tc_status Runner::round(int M, int K, bool serve) {
  static const bool debug = std::getenv("TC_DEBUG") != nullptr;
  using B = BatchPlan;
  const bool init = serve && any(is_init);
  const bool fin = serve && any(is_finish);
  // pads being initialised join the first Newton iteration's launches; the
  // kernels pass over any that the feasible start fails
  auto starting = init ? may_start_or_init : may_start;
  auto cg_pads = init ? run_or_init : is_run;
  if (init) init_launches();
  const unsigned mD = 1u << B::VERT | 1u << B::CAND | 1u << B::PAIR;
  const unsigned mL = 1u << B::ENERGY | 1u << B::PAIR | 1u << B::VERT;
  const unsigned mA = 1u << B::TET | 1u << B::PAIR | 1u << B::CAND | 1u << B::VERT | 1u << B::ASM;
  const unsigned mC = 1u << B::SPMV | 1u << B::VERT;
  const bool anyD = any(dir_pending), anyL = any(turning), anyA = any(starting);
  std::vector<char> was_dir;
  if (debug)
    for (int i = 0; i < n; ++i) was_dir.push_back(dir_pending(state(i)));
  View vD{}, vL{}, vA{};
  if (anyD) vD = view(dir_pending, mD, false);
  if (anyL) vL = view(turning, mL, false);
  if (anyA) vA = view(starting, mA, false);
  const View vC = view(cg_pads, mC, false);
  flush_views();
  if (anyD) {
    launch_v(KernelId::newton_dir, vD, B::VERT);
    launch_v(KernelId::filter, vD, B::CAND);
    if (any_pairs(dir_pending)) launch_v(KernelId::pairs, vD, B::PAIR, 0, 3);
    launch(KernelId::env_dir, B::NCLS);
  }
  if (anyL) {
    const bool pairs = any_pairs(turning);
    for (int k = 0; k < K; ++k) {
      launch_v(KernelId::energy, vL, B::ENERGY, 0, 1);
      if (pairs) launch_v(KernelId::pairs, vL, B::PAIR, 0, 2);
      launch(KernelId::env_ls, B::NCLS, 0, 1);
    }
    launch_v(KernelId::update, vL, B::VERT);
    launch(KernelId::env_update, B::NCLS);
  }
  if (anyA) {
    launch(KernelId::newton_begin, B::NCLS);
    launch_v(KernelId::element, vA, B::TET);
    if (any_pairs(starting)) launch_v(KernelId::pairs, vA, B::PAIR, 0, 0);
    launch_v(KernelId::barrier, vA, B::CAND);
    launch_v(KernelId::asm_diag, vA, B::VERT);
    launch_v(KernelId::asm_off, vA, B::ASM);
  }
  tc_status st;
  // no CG chunk when no pad can be in CG (all others still searching)
  if ((anyA || any(in_cg)) && (st = cg_chunk(M, vC))) return st;
  if (fin) finish_launches();    // (the pads that had ended before this round)
  if ((st = readback())) return st;
  if (debug)
    for (int i = 0; i < n; ++i) {
      if (!was_dir[i]) continue;
      const EnvState& S = state(i);
      std::fprintf(stderr, "[tc] pad %d newton %d cg %d rz0 %.3e |d| %.3e g.d %.3e amax %.3e E %.12e conv %d\n", i,
                   S.newton_iters, S.cg_iters, S.rz0, S.final_step_inf, S.gTd, S.alpha_max, S.E_cur, S.dir_conv);
    }
  return TC_OK;
}

tc_status Runner::staged(int M, int K) {
  tc_status st;
  init_launches();
  if ((st = readback())) return st;
  // a Newton iteration takes at most this many rounds: its CG chunks, its
  // line search's trial energies K per round, one round to start
  int limit = 2;
  for (int i = 0; i < n; ++i) {
    const tc_params& q = P->pads[i]->params;
    const int per_it = (q.max_cg + M) / M + (q.max_halvings + q.ls_expand + 1 + K - 1) / K + 1;
    limit = std::max(limit, (q.max_newton + 1) * per_it + 2);
  }
  for (int r = 0; any(is_run); ++r) {
    if (r >= limit) return set_error(TC_E_HIP, "staged Newton driver did not terminate");
    if ((st = round(M, K))) return st;
  }
  return finish();
}

// Algorithmic HBM bytes of one launch's work on one pad (each array element
// read or written once; gathers of shared vertex data counted once).
static double kernel_bytes(KernelId k, const tc_pad* p) {
  const double R = p->rsize, V = p->V, T = p->T, C = p->C, S = p->S;
  const double nnzb = (double)p->nnz_blocks;
  switch (k) {
    case KernelId::cg_spmv: return nnzb * (9 * R + 4) + V * 12 * R;
    case KernelId::cg_update: return V * (21 * R + 48);
    case KernelId::element: return T * (56 + 100 * R) + V * 48;
    case KernelId::asm_diag: return T * (36 * R) + V * (97 + 24 * R);
    case KernelId::asm_off: return T * (54 * R) + p->n_edges * (14 + 18 * R);
    case KernelId::energy:   // friction: x_t and one indenter's lag record per contact vertex
      return T * (16 + 10 * R) + V * (56 + 3 * R) + C * 40 + (p->params.friction > 0 ? C * 88 : 0);
    case KernelId::sigma: return T * (16 + 15 * R) + V * 24;
    case KernelId::traction: return S * (17 + 24 + 6 * R + 9 * R) + V * 24;
    default: return 0.0;
  }
}

void account_bytes(tc_context* ctx, const tc_pad* pad, const EnvState& S) {
  const double nt = S.newton_iters, cg = S.cg_total;
  auto add = [&](KernelId k, double count) { ctx->timers[(int)k].bytes += count * kernel_bytes(k, pad); };
  add(KernelId::cg_spmv, cg);
  add(KernelId::cg_update, cg);
  add(KernelId::element, nt);
  add(KernelId::asm_diag, nt);
  add(KernelId::asm_off, nt);
  add(KernelId::energy, 1 + nt + S.ls_total);
  add(KernelId::sigma, 1);
  add(KernelId::traction, 1);
}

tc_status run_batch(tc_context* ctx, int n, tc_pad* const* pads, const int32_t* n_ind,
                    const tc_indenter* ind, tc_step_stats* stats, int mode) {
  const double t0 = now_ms();
  std::string err;
  if (n < 1 || !pads) return set_error(TC_E_INVALID_ARG, "need at least one pad");
  if (!n_ind) return set_error(TC_E_INVALID_ARG, "n_ind is null");
  int off = 0;
  for (int i = 0; i < n; ++i) {
    if (!pads[i] || pads[i]->ctx != ctx) return set_error(TC_E_INVALID_ARG, "pad is null or from another context");
    if (pads[i]->fp64 != pads[0]->fp64) return set_error(TC_E_INVALID_ARG, "pads of one batch must share the precision");
    for (int j = 0; j < i; ++j)
      if (pads[j] == pads[i]) return set_error(TC_E_INVALID_ARG, "a pad appears twice in the batch");
    if (pads[i]->busy.load()) return set_error(TC_E_BUSY, "pad has a request in flight on a server");
    tc_status s = validate_indenters(n_ind[i], ind ? ind + off : nullptr, err);
    if (s) return set_error(s, "pad " + std::to_string(i) + ": " + err);
    if ((s = check_meshes(ctx, n_ind[i], ind ? ind + off : nullptr))) return s;
    off += n_ind[i];
  }
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  TC_HIP(hipSetDevice(ctx->device));
  {
    const std::vector<tc_pad*> keep(pads, pads + n);
    for (int i = 0; i < n; ++i) {
      tc_status s = ensure_scratch_evicting(pads[i], keep);
      if (s) return s;
    }
  }
  // pads split into groups, each stepped on its own stream by its own host
  // thread (the first group on this one): one group's CG tail and host
  // round trips overlap with the other groups' launches
  const int G = mode == 0 ? std::max(1, std::min(ctx->n_lanes, n / 2)) : 1;
  std::vector<std::vector<int>> groups(G);
  if (G == 1) {
    for (int i = 0; i < n; ++i) groups[0].push_back(i);
  } else {
    // the pads that iterated longest in their last step, up to a quarter of
    // the batch's tets, get the first stream: their long chains of small
    // launches run beside the other groups' large launches instead of
    // lengthening steps that also carry bulk work.  The rest are split into
    // groups of about equal cost, a pad's cost being its tets times its
    // Newton iterations, largest first to the group with the least; each
    // group keeps the batch order
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return pads[x]->last_newton > pads[y]->last_newton; });
    int64_t total = 0, slow = 0;
    for (int i = 0; i < n; ++i) total += pads[i]->T;
    auto cost = [&](int i) { return (int64_t)pads[i]->T * std::max(1, pads[i]->last_newton); };
    std::vector<int> rest;
    for (int i : order) {
      // (at least one pad left for each of the other groups)
      const int left = n - (int)groups[0].size() - (int)rest.size();
      if (slow < total / 4 && left > G - 1) {
        groups[0].push_back(i);
        slow += pads[i]->T;
      } else {
        rest.push_back(i);
      }
    }
    std::stable_sort(rest.begin(), rest.end(), [&](int x, int y) { return cost(x) > cost(y); });
    std::vector<int64_t> load(G, 0);
    for (int i : rest) {
      const int g = 1 + (int)(std::min_element(load.begin() + 1, load.end()) - load.begin() - 1);
      groups[g].push_back(i);
      load[g] += cost(i);
    }
    for (auto& gr : groups) std::sort(gr.begin(), gr.end());
  }
  std::vector<int> first_of(n, 0);   // index of each pad's first pose
  off = 0;
  for (int i = 0; i < n; ++i) {
    first_of[i] = off;
    off += n_ind[i];
  }
  struct Job {
    Lane* lane;
    std::vector<tc_pad*> pads;
    std::vector<int> idx;
    tc_status st = TC_OK;
    std::string err;
  };
  std::vector<Job> jobs(G);
  for (int g = 0; g < G; ++g) {
    Job& J = jobs[g];
    if (G == 1) {
      J.lane = &ctx->lane0;
    } else {
      tc_status s = get_lane(ctx, g);
      if (s) return s;
      J.lane = ctx->lanes[g].get();
    }
    J.idx = groups[g];
    for (int i : J.idx) J.pads.push_back(pads[i]);
    Lane& L = *J.lane;
    const int m = (int)J.pads.size();
    tc_status s = pool_reserve(ctx, *L.pool, m);
    if (s) return s;
    std::vector<int> slots(m);
    for (int i = 0; i < m; ++i) slots[i] = i;
    if (!plan_matches(L.plan->get(), ctx, m, J.pads.data(), slots.data(), *L.pool)) {
      if ((s = build_plan(ctx, m, J.pads.data(), slots.data(), *L.pool, *L.plan, L.stream))) return s;
    }
    for (int k = 0; k < m; ++k) {
      const int i = J.idx[k];
      init_state(L.pool->h_state[k], L.pool->h_pose[k], mode, n_ind[i], ind ? ind + first_of[i] : nullptr, pads[i]);
    }
    static_assert(sizeof(DevIndenter) == sizeof(tc_indenter), "indenter layout");
    TC_HIP(hipMemcpyAsync(L.pool->d_state, L.pool->h_state, sizeof(EnvState) * m, hipMemcpyHostToDevice, L.stream));
    TC_HIP(hipMemcpyAsync(L.pool->d_pose, L.pool->h_pose, sizeof(EnvPose) * m, hipMemcpyHostToDevice, L.stream));
    if (G > 1) {
      // every lane's slice of the clock cells
      L.ts->base = (size_t)g * (ctx->clock_cap / G);
      L.ts->cap = ctx->clock_cap / G;
    }
  }
  auto drive = [ctx, mode](Job& J) {
    Lane& L = *J.lane;
    const int m = (int)J.pads.size();
    Runner run{ctx, L.plan->get(), m, L.pool, m, L.stream, L.ts};
    int max_newton = 0;
    for (tc_pad* p : J.pads) max_newton = std::max(max_newton, p->params.max_newton);
    tc_status st = TC_OK;
    if (mode == 1) {
      st = run.tick(false);
    } else if (ctx->staged) {
      st = run.staged(std::max(2, ctx->cg_per_replay & ~1), ctx->ls_per_round);
    } else {
      bool init = true;
      for (int guard = 0;; ++guard) {
        if ((st = run.tick(init))) break;
        init = false;
        if (!run.any(Runner::not_done)) break;
        if (guard > max_newton + 2) {
          st = set_error(TC_E_HIP, "Newton driver did not terminate");
          break;
        }
      }
    }
    // the step's remaining clock cells (the stream is synchronised: every
    // tick ends with a readback)
    if (ctx->timing) resolve_timing(ctx, *L.ts, L.stream, true);
    J.st = st;
    if (st) J.err = last_error();
  };
  if (G == 1) {
    drive(jobs[0]);
  } else {
    std::vector<std::thread> th;
    for (int g = 1; g < G; ++g)
      th.emplace_back([&, g] {
        if (hipSetDevice(ctx->device) != hipSuccess) {
          jobs[g].st = set_error(TC_E_HIP, "hipSetDevice in a lane thread");
          jobs[g].err = last_error();
          return;
        }
        drive(jobs[g]);
      });
    drive(jobs[0]);
    for (auto& t : th) t.join();
    for (int g = 0; g < G; ++g) {
      jobs[g].lane->ts->base = 0;
      jobs[g].lane->ts->cap = 0;
    }
  }
  for (auto& J : jobs)
    if (J.st) return set_error(J.st, J.err);
  tc_status first = TC_OK;
  const double ms = now_ms() - t0;
  for (auto& J : jobs) {
    for (size_t k = 0; k < J.pads.size(); ++k) {
      const int i = J.idx[k];
      const EnvState& S = J.lane->pool->h_state[k];
      if (S.status == TC_OK && mode == 0) {
        pads[i]->step_count++;
        pads[i]->last_newton = S.newton_iters;
        remember_pose(pads[i], J.lane->pool->h_pose[k]);
      }
      if (S.status != TC_OK && first == TC_OK) first = S.status;
      if (stats) fill_stats(stats[i], S, ms);
      if (ctx->timing) account_bytes(ctx, pads[i], S);
    }
  }
  if (first != TC_OK) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "step failed: %s", tc_status_string(first));
    set_error(first, buf);
  }
  return first;
}

// One Newton direction at the committed positions (inspection).
tc_status newton_direction(tc_pad* pad, int n_ind, const tc_indenter* ind, double* dir, double* grad) {
  tc_context* ctx = pad->ctx;
  std::string err;
  tc_status s = validate_indenters(n_ind, ind, err);
  if (s) return set_error(s, err);
  if ((s = check_meshes(ctx, n_ind, ind))) return s;
  if (!dir) return set_error(TC_E_INVALID_ARG, "dir is null");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  TC_HIP(hipSetDevice(ctx->device));
  if ((s = ensure_scratch(pad))) return s;
  SlotPool& pool = ctx->pool;
  if ((s = pool_reserve(ctx, pool, 1))) return s;
  int slot = 0;
  tc_pad* pads[1] = {pad};
  if (!plan_matches(ctx->plan.get(), ctx, 1, pads, &slot, pool)) {
    if ((s = build_plan(ctx, 1, pads, &slot, pool, ctx->plan))) return s;
  }
  BatchPlan* P = ctx->plan.get();
  init_state(pool.h_state[0], pool.h_pose[0], 0, n_ind, ind, pad);
  pool.h_state[0].force_tight = 1;   // CG straight to the convergence tolerance
  TC_HIP(hipMemcpyAsync(pool.d_state, pool.h_state, sizeof(EnvState), hipMemcpyHostToDevice, ctx->stream));
  TC_HIP(hipMemcpyAsync(pool.d_pose, pool.h_pose, sizeof(EnvPose), hipMemcpyHostToDevice, ctx->stream));
  Runner run{ctx, P, 1, &pool, 1};
  const Runner::View v = run.view(Runner::not_done);
  run.launch_v(KernelId::predict, v, BatchPlan::VERT);
  run.launch_v(KernelId::energy, v, BatchPlan::ENERGY, 0, 0);
  if (run.any_pairs(Runner::not_done)) run.launch_v(KernelId::pairs, v, BatchPlan::PAIR, 0, 4);
  run.launch(KernelId::env_ls, BatchPlan::NCLS, 0, 0);
  run.launch(KernelId::newton_begin, BatchPlan::NCLS);
  run.launch_v(KernelId::element, v, BatchPlan::TET);
  if (run.any_pairs(Runner::init_or_run)) run.launch_v(KernelId::pairs, v, BatchPlan::PAIR, 0, 0);
  run.launch_v(KernelId::barrier, v, BatchPlan::CAND);
  run.launch_v(KernelId::asm_diag, v, BatchPlan::VERT);
  run.launch_v(KernelId::asm_off, v, BatchPlan::ASM);
  const int M = std::max(2, ctx->cg_per_replay & ~1);
  for (int done = 0; done <= pad->params.max_cg + M; done += M) {
    if ((s = run.cg_chunk(M, v))) return s;
    if ((s = run.readback())) return s;
    if (pool.h_state[0].status != TC_OK) return set_error(pool.h_state[0].status, "probe failed");
    if (pool.h_state[0].cg_done) break;
  }
  const size_t n3 = 3 * (size_t)pad->V;
  if (pad->fp64) {
    TC_HIP(hipMemcpy(dir, pad->desc.d, 8 * n3, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> tmp(n3);
    TC_HIP(hipMemcpy(tmp.data(), pad->desc.d, 4 * n3, hipMemcpyDeviceToHost));
    for (size_t k = 0; k < n3; ++k) dir[k] = tmp[k];
  }
  if (grad) TC_HIP(hipMemcpy(grad, pad->desc.g, 8 * n3, hipMemcpyDeviceToHost));
  return TC_OK;
}

}  // namespace tc

// =================================================================== C ABI

namespace {

template <class F>
tc_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return set_error(TC_E_NO_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(TC_E_INVALID_ARG, e.what());
  } catch (...) {
    return set_error(TC_E_INVALID_ARG, "unknown exception");
  }
}

tc_status field_layout(const tc_pad* p, int field, int* dtype, int64_t* count, int* comps, const void** src) {
  const int R = p->fp64 ? TC_DT_F64 : TC_DT_F32;
  const EnvDesc& E = p->desc;
  struct F { int dt; int64_t n; int c; const void* ptr; };
  F f{};
  switch (field) {
    case TC_F_POSITIONS: f = {TC_DT_F64, p->V, 3, E.x}; break;
    case TC_F_VELOCITIES: f = {TC_DT_F64, p->V, 3, E.v}; break;
    case TC_F_REST: f = {TC_DT_F64, p->V, 3, E.X}; break;
    case TC_F_SIGMA: f = {R, p->T, 6, E.sigma}; break;
    case TC_F_TRACTION: f = {R, p->S, 3, E.traction}; break;
    case TC_F_PRESSURE: f = {R, p->S, 1, E.pressure}; break;
    case TC_F_TANGENTIAL: f = {R, p->S, 3, E.tangential}; break;
    case TC_F_TRI_AREA: f = {R, p->S, 1, E.tri_area}; break;
    case TC_F_TRI_NORMAL: f = {R, p->S, 3, E.tri_normal}; break;
    case TC_F_CONTACT_FORCE: f = {TC_DT_F64, p->C, 3, E.c_force}; break;
    case TC_F_CONTACT_NORMAL: f = {TC_DT_F64, p->C, 3, E.c_normal}; break;
    case TC_F_CONTACT_AREA: f = {TC_DT_F64, p->C, 1, E.c_area}; break;
    case TC_F_CONTACT_FN: f = {TC_DT_F64, p->C, 3, E.c_fn}; break;
    case TC_F_CONTACT_FT: f = {TC_DT_F64, p->C, 3, E.c_ft}; break;
    case TC_F_CONTACT_PRESSURE: f = {TC_DT_F64, p->C, 1, E.c_press}; break;
    case TC_F_REACTION: f = {TC_DT_F64, 1, 3, E.reaction}; break;
    case TC_F_TRACTION_SUM: f = {TC_DT_F64, 1, 3, E.traction_sum}; break;
    case TC_F_SURFACE_TRIS: f = {TC_DT_I32, p->S, 3, E.tris}; break;
    case TC_F_SURFACE_PARENT: f = {TC_DT_I32, p->S, 1, E.parent}; break;
    case TC_F_SURFACE_IS_TOP: f = {TC_DT_U8, p->S, 1, E.is_top}; break;
    case TC_F_CANDIDATES: f = {TC_DT_I32, p->C, 1, E.cand}; break;
    case TC_F_CAND_REST_AREA: f = {TC_DT_F64, p->C, 1, E.cand_area}; break;
    case TC_F_MASS: f = {TC_DT_F64, p->V, 1, E.mass}; break;
    case TC_F_FIXED: f = {TC_DT_U8, p->V, 1, E.fixed}; break;
    case TC_F_TETS: f = {TC_DT_I32, p->T, 4, E.tets}; break;
    default: return set_error(TC_E_INVALID_ARG, "unknown field " + std::to_string(field));
  }
  if (dtype) *dtype = f.dt;
  if (count) *count = f.n;
  if (comps) *comps = f.c;
  if (src) *src = f.ptr;
  return TC_OK;
}

size_t dtype_size(int dt) { return dt == TC_DT_F64 ? 8 : dt == TC_DT_U8 ? 1 : 4; }

tc_status upload(tc_context* ctx, void* dst, const void* src, size_t bytes) {
  TC_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
  return TC_OK;
}

}  // namespace

extern "C" {

const char* tc_version(void) { return "tacauchy-mi355x 0.1 (gfx950)"; }

const char* tc_status_string(tc_status s) {
  switch (s) {
    case TC_OK: return "TC_OK";
    case TC_E_INVALID_ARG: return "TC_E_INVALID_ARG";
    case TC_E_BAD_MESH: return "TC_E_BAD_MESH";
    case TC_E_NO_MEMORY: return "TC_E_NO_MEMORY";
    case TC_E_HIP: return "TC_E_HIP";
    case TC_E_INFEASIBLE: return "TC_E_INFEASIBLE";
    case TC_E_NOT_CONVERGED: return "TC_E_NOT_CONVERGED";
    case TC_E_LINESEARCH: return "TC_E_LINESEARCH";
    case TC_E_NO_DEVICE: return "TC_E_NO_DEVICE";
    case TC_E_BUSY: return "TC_E_BUSY";
    default: return "TC_E_UNKNOWN";
  }
}

const char* tc_last_error(void) { return tc::last_error().c_str(); }

tc_status tc_params_default(tc_params* out) {
  if (!out) return set_error(TC_E_INVALID_ARG, "out is null");
  std::memset(out, 0, sizeof *out);
  out->dt = 1.0 / 60.0;
  out->dhat = 1e-4;
  out->kappa = 1e3;
  out->newton_tol = 1e-6;
  out->cg_rel_tol = 1e-4;
  out->max_newton = 1024;
  out->max_cg = 4000;
  out->quasi_static = 0;
  out->precision = TC_PREC_MIXED;
  out->literal_alpha = 0;
  out->precond = TC_PRECOND_BLOCK_JACOBI;
  out->max_halvings = 40;
  out->cg_forcing = 1;
  out->hess_proj = 0;
  out->init_guess = 0;
  out->cg_conv_tol = 0.0;
  out->cg_eta_max = 0.5;
  out->ls_expand = 0;
  out->mesh_contact = 0;
  out->friction = 0.0;
  out->eps_v = 0.01;
  return TC_OK;
}

tc_status tc_validate_mesh(const tc_mesh* mesh, int32_t n_materials) {
  return guarded([&] {
    std::string err;
    tc_status s = validate_mesh(mesh, n_materials, err);
    return s ? set_error(s, err) : TC_OK;
  });
}

tc_status tc_validate_materials(int32_t n, const tc_material* m) {
  std::string err;
  tc_status s = validate_materials(n, m, err);
  return s ? set_error(s, err) : TC_OK;
}

tc_status tc_validate_params(const tc_params* p) {
  std::string err;
  tc_status s = validate_params(p, err);
  return s ? set_error(s, err) : TC_OK;
}

tc_status tc_validate_indenters(int32_t n, const tc_indenter* ind) {
  std::string err;
  tc_status s = validate_indenters(n, ind, err);
  return s ? set_error(s, err) : TC_OK;
}

tc_status tc_mesh_surface(const tc_mesh* mesh, int32_t* n_tris, int32_t* n_candidates, int32_t* tris,
                          int32_t* parent, uint8_t* is_top, int32_t* candidates, int32_t tris_capacity,
                          int32_t cand_capacity) {
  return guarded([&]() -> tc_status {
    std::string err;
    tc_status s = validate_mesh(mesh, 1 << 30, err);
    if (s) return set_error(s, err);
    if (!n_tris || !n_candidates) return set_error(TC_E_INVALID_ARG, "count outputs are null");
    Topology t;
    build_surface(mesh, t);
    const int S = (int)t.parent.size(), C = (int)t.cand.size();
    *n_tris = S;
    *n_candidates = C;
    if (!tris) return TC_OK;
    if (tris_capacity < S || cand_capacity < C || !parent || !is_top || !candidates)
      return set_error(TC_E_INVALID_ARG, "output capacity too small or null output");
    std::memcpy(tris, t.tris.data(), sizeof(int32_t) * 3 * S);
    std::memcpy(parent, t.parent.data(), sizeof(int32_t) * S);
    std::memcpy(is_top, t.is_top.data(), S);
    std::memcpy(candidates, t.cand.data(), sizeof(int32_t) * C);
    return TC_OK;
  });
}

tc_status tc_context_create(int32_t device, void* hip_stream, uint64_t hbm_budget, tc_context** out) {
  return guarded([&]() -> tc_status {
    if (!out) return set_error(TC_E_INVALID_ARG, "out is null");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return set_error(TC_E_NO_DEVICE, "no HIP device");
    if (device < 0 || device >= count) return set_error(TC_E_INVALID_ARG, "device ordinal out of range");
    hipDeviceProp_t prop;
    TC_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return set_error(TC_E_NO_DEVICE, std::string("library is built for gfx950, device is ") + prop.gcnArchName);
    TC_HIP(hipSetDevice(device));
    {
      const tc_status ns = noalloc_init(device);
      if (ns) return ns;
    }
    auto* ctx = new tc_context();
    ctx->device = device;
    ctx->budget = hbm_budget;
    if (hip_stream) {
      ctx->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      hipError_t e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
      if (e != hipSuccess) { delete ctx; return hip_fail(e, "hipStreamCreate"); }
      ctx->own_stream = true;
    }
    ctx->lane0.stream = ctx->stream;
    ctx->lane0.plan = &ctx->plan;
    ctx->lane0.pool = &ctx->pool;
    ctx->lane0.ts = &ctx->tslice;
    {
      const size_t tb = sizeof(DevMesh) * MAX_MESHES;
      hipError_t e = hipMalloc(&ctx->d_meshes, tb);
      if (e == hipSuccess) e = hipMemset(ctx->d_meshes, 0, tb);
      if (e != hipSuccess) {
        if (ctx->d_meshes) (void)hipFree(ctx->d_meshes);
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return hip_fail(e, "mesh table");
      }
      ctx->mesh_slots.resize(MAX_MESHES);
    }
    *out = ctx;
    return TC_OK;
  });
}

tc_status tc_context_destroy(tc_context* ctx) {
  if (!ctx) return TC_OK;
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    // pads and servers keep a pointer to the context and lock its mutex
    // when they are destroyed: they must go first
    if (!ctx->pads.empty() || ctx->n_servers.load() > 0)
      return set_error(TC_E_BUSY, "context still has " + std::to_string(ctx->pads.size()) + " pads and " +
                                      std::to_string(ctx->n_servers.load()) + " servers");
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    free_lanes(ctx);
    ctx->plan.reset();
    for (auto& c : ctx->arena.chunks) (void)hipFree(c.base);
    ctx->arena.chunks.clear();
    resolve_timing(ctx);
    for (auto e : ctx->free_events) (void)hipEventDestroy(e);
    if (ctx->clock_cells) (void)hipFree(ctx->clock_cells);
    free_meshes(ctx);
    if (ctx->d_meshes) (void)hipFree(ctx->d_meshes);
    pool_free(ctx->pool);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
  return TC_OK;
}

tc_status tc_context_memory(const tc_context* ctx, uint64_t* used, uint64_t* budget) {
  if (!ctx) return set_error(TC_E_INVALID_ARG, "ctx is null");
  if (used) *used = ctx->used;
  if (budget) *budget = ctx->budget;
  return TC_OK;
}

tc_status tc_context_set_timing(tc_context* ctx, int32_t enable) {
  if (!ctx) return set_error(TC_E_INVALID_ARG, "ctx is null");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (enable < 0) return set_error(TC_E_INVALID_ARG, "enable must be >= 0");
  if (enable > 0 && !ctx->clock_cells) {
    TC_HIP(hipSetDevice(ctx->device));
    int khz = 0;
    TC_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device));
    if (khz <= 0) return set_error(TC_E_HIP, "device reports no wall clock rate");
    ctx->clock_khz = khz;
    ctx->clock_cap = (size_t)4 << 20;   // 32 MiB of cells
    TC_HIP(hipMalloc(&ctx->clock_cells, 8 * ctx->clock_cap));
    TC_HIP(hipMemsetAsync(ctx->clock_cells, 0, 8 * ctx->clock_cap, ctx->stream));
    TC_HIP(hipStreamSynchronize(ctx->stream));   // other streams use the cells too
    ctx->tslice.used = 0;
  }
  ctx->timing = enable != 0;
  if (enable > 0) ctx->timing_stride = enable;
  return TC_OK;
}

tc_status tc_context_reset_timing(tc_context* ctx) {
  if (!ctx) return set_error(TC_E_INVALID_ARG, "ctx is null");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  resolve_timing(ctx);
  for (auto& t : ctx->timers) t = KernelTimer{};
  return TC_OK;
}

tc_status tc_context_timing(tc_context* ctx, int32_t cap, int32_t* n, char (*names)[TC_TIMER_NAME_LEN],
                            double* avg_ms, int64_t* launches, double* bytes_per_launch) {
  if (!ctx || !n) return set_error(TC_E_INVALID_ARG, "ctx or n is null");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  resolve_timing(ctx);
  int k = 0;
  for (int i = 0; i < (int)KernelId::count && k < cap; ++i) {
    const KernelTimer& t = ctx->timers[i];
    if (t.launches == 0 || t.timed == 0) continue;
    if (names) {
      std::strncpy(names[k], kernel_name((KernelId)i), TC_TIMER_NAME_LEN - 1);
      names[k][TC_TIMER_NAME_LEN - 1] = 0;
    }
    if (avg_ms) avg_ms[k] = t.ms / t.timed;
    if (launches) launches[k] = t.launches;
    if (bytes_per_launch) bytes_per_launch[k] = t.bytes / t.launches;
    ++k;
  }
  *n = k;
  return TC_OK;
}

tc_status tc_set_launch(tc_context* ctx, int32_t cg_block, int32_t elem_block, int32_t spmv_block,
                        int32_t cg_per_replay, int32_t use_graphs) {
  if (!ctx) return set_error(TC_E_INVALID_ARG, "ctx is null");
  auto okb = [](int b) { return b == 0 || (b >= 64 && b <= 1024 && b % 64 == 0); };
  if (!okb(cg_block) || !okb(elem_block) || !okb(spmv_block) || elem_block > 256)
    return set_error(TC_E_INVALID_ARG, "block sizes: multiples of 64 up to 1024 (element up to 256)");
  if (cg_per_replay < 0 || (cg_per_replay && (cg_per_replay < 2 || cg_per_replay % 2)))
    return set_error(TC_E_INVALID_ARG, "CG iterations per replay must be even and >= 2");
  if (use_graphs < -1 || use_graphs > 1) return set_error(TC_E_INVALID_ARG, "use_graphs must be -1, 0 or 1");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (cg_block) ctx->cg_block = cg_block;
  if (elem_block) ctx->el_block = elem_block;
  if (spmv_block) ctx->spmv_block = spmv_block;
  if (cg_per_replay) ctx->cg_per_replay = cg_per_replay;
  if (use_graphs >= 0) ctx->use_graphs = use_graphs != 0;
  drop_plans(ctx);
  return TC_OK;
}

tc_status tc_set_streams(tc_context* ctx, int32_t n_streams) {
  if (!ctx) return set_error(TC_E_INVALID_ARG, "ctx is null");
  if (n_streams < 1 || n_streams > TC_MAX_STREAMS) return set_error(TC_E_INVALID_ARG, "n_streams must be 1..4");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->n_lanes = n_streams;
  return TC_OK;
}

tc_status tc_set_schedule(tc_context* ctx, int32_t staged, int32_t line_search_evals) {
  if (!ctx) return set_error(TC_E_INVALID_ARG, "ctx is null");
  if (staged < 0 || staged > 1) return set_error(TC_E_INVALID_ARG, "staged must be 0 or 1");
  if (line_search_evals < 0 || line_search_evals > 8)
    return set_error(TC_E_INVALID_ARG, "line_search_evals must be 0..8");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->staged = staged != 0;
  if (line_search_evals) ctx->ls_per_round = line_search_evals;
  return TC_OK;
}

tc_status tc_pad_create(tc_context* ctx, const tc_mesh* mesh, int32_t n_materials, const tc_material* materials,
                        const tc_params* params, tc_pad** out) {
  return guarded([&]() -> tc_status {
    if (!ctx || !out) return set_error(TC_E_INVALID_ARG, "ctx or out is null");
    *out = nullptr;
    std::string err;
    tc_status s;
    if ((s = validate_materials(n_materials, materials, err))) return set_error(s, err);
    if ((s = validate_params(params, err))) return set_error(s, err);
    if ((s = validate_mesh(mesh, n_materials, err))) return set_error(s, err);
    Topology t;
    build_surface(mesh, t);
    build_sparsity(mesh, t);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    TC_HIP(hipSetDevice(ctx->device));
    auto* p = new tc_pad();
    std::unique_ptr<tc_pad, void (*)(tc_pad*)> guard(p, [](tc_pad* q) {
      for (auto& a : q->allocs) q->ctx->dev_free(a.first, a.second);
      delete q;
    });
    p->ctx = ctx;
    p->id = ctx->next_pad_id++;
    p->V = mesh->n_verts;
    p->T = mesh->n_tets;
    p->S = (int)t.parent.size();
    p->C = (int)t.cand.size();
    p->S_top = 0;
    for (auto v : t.is_top) p->S_top += v;
    p->W = t.W;
    p->nnz_blocks = t.nnz_blocks;
    p->n_edges = (int64_t)(t.eitem.size() / 2);
    p->fp64 = params->precision == TC_PREC_FP64;
    p->rsize = p->fp64 ? 8 : 4;
    p->params = *params;
    p->n_mat = n_materials;
    for (int k = 0; k < MAX_MAT; ++k) { p->mu[k] = p->lam[k] = p->alpha[k] = p->rho[k] = 0; }
    for (int k = 0; k < n_materials; ++k) {
      // Eq. 1 Lame parameters; rest shift alpha = 1 + mu / lambda (P(I) = 0)
      // unless the literal alpha = 1 of Eq. 2 is requested
      const tc_material& m = materials[k];
      p->mu[k] = m.E / (2.0 * (1.0 + m.nu));
      p->lam[k] = m.E * m.nu / ((1.0 + m.nu) * (1.0 - 2.0 * m.nu));
      p->alpha[k] = params->literal_alpha ? 1.0 : 1.0 + p->mu[k] / p->lam[k];
      p->rho[k] = m.density;
    }
    if (n_materials > 1 || mesh->tet_material) {
      for (int k = 0; k < n_materials; ++k)
        if (!(p->lam[k] > 0)) return set_error(TC_E_INVALID_ARG, "nu must be > 0 for the rest-stable shift");
    } else if (!(p->lam[0] > 0) && !params->literal_alpha) {
      return set_error(TC_E_INVALID_ARG, "nu must be > 0 for the rest-stable shift mu / lambda");
    }
    p->bbox_diag = t.bbox_diag;
    auto alloc = [&](size_t bytes, tc_status* st) -> void* {
      void* q = ctx->dev_alloc(bytes, st);
      if (q) { p->allocs.push_back({q, bytes}); p->resident_bytes += align256(bytes); }
      return q;
    };
    const size_t V = p->V, T = p->T, S = p->S, C = std::max(p->C, 1), R = p->rsize;
    EnvDesc& E = p->desc;
    std::memset(&E, 0, sizeof E);
    E.V = p->V; E.T = p->T; E.C = p->C; E.S = p->S; E.W = p->W;
#define ALLOC(ptr, type, bytes)                     \
  do {                                              \
    ptr = (type)alloc(bytes, &s);                   \
    if (!ptr) return s;                             \
  } while (0)
    double *X, *x, *v, *mass, *carea;
    int32_t *tets, *cand, *cov, *tris, *parent, *ctp, *cti, *col, *cptr;
    uint32_t* clist;
    int32_t *cpos, *dptr, *eptr, *eitem;
    uint8_t *fixed, *istop;
    int8_t* mat = nullptr;
    void *Dminv, *vol;
    ALLOC(X, double*, 24 * V);
    ALLOC(x, double*, 24 * V);
    ALLOC(v, double*, 24 * V);
    ALLOC(tets, int32_t*, 16 * T);
    ALLOC(Dminv, void*, 9 * T * R);
    ALLOC(vol, void*, T * R);
    if (n_materials > 1 || mesh->tet_material) ALLOC(mat, int8_t*, T);
    ALLOC(mass, double*, 8 * V);
    ALLOC(fixed, uint8_t*, V);
    ALLOC(cand, int32_t*, 4 * C);
    ALLOC(cov, int32_t*, 4 * V);
    ALLOC(carea, double*, 8 * C);
    ALLOC(tris, int32_t*, 12 * S);
    ALLOC(parent, int32_t*, 4 * S);
    ALLOC(istop, uint8_t*, S);
    ALLOC(ctp, int32_t*, 4 * (C + 1));
    ALLOC(cti, int32_t*, 4 * std::max<size_t>(t.ctri_idx.size(), 1));
    ALLOC(col, int32_t*, 4 * t.col.size());
    ALLOC(cptr, int32_t*, 4 * t.cptr.size());
    ALLOC(clist, uint32_t*, 4 * t.clist.size());
    ALLOC(cpos, int32_t*, 4 * t.cpos.size());
    ALLOC(dptr, int32_t*, 4 * t.dptr.size());
    ALLOC(eptr, int32_t*, 4 * t.eptr.size());
    ALLOC(eitem, int32_t*, 4 * std::max<size_t>(t.eitem.size(), 1));
    ALLOC(E.sigma, void*, 6 * T * R);
    ALLOC(E.traction, void*, 3 * S * R);
    ALLOC(E.pressure, void*, S * R);
    ALLOC(E.tangential, void*, 3 * S * R);
    ALLOC(E.tri_area, void*, S * R);
    ALLOC(E.tri_normal, void*, 3 * S * R);
    ALLOC(E.tri_cross, double*, 24 * S);
    ALLOC(E.c_force, double*, 24 * C);
    ALLOC(E.c_normal, double*, 24 * C);
    ALLOC(E.c_area, double*, 8 * C);
    ALLOC(E.c_fn, double*, 24 * C);
    ALLOC(E.c_ft, double*, 24 * C);
    ALLOC(E.c_press, double*, 8 * C);
    ALLOC(E.reaction, double*, 24);
    ALLOC(E.traction_sum, double*, 24);
    // surface edges and the incidence tables of the vertex-face / edge-edge
    // pairs against rigid meshes (mesh_contact 2)
    {
      std::map<std::pair<int, int>, int> key;
      for (size_t j = 0; j < S; ++j)
        for (int k = 0; k < 3; ++k) {
          const int a = t.tris[3 * j + k], b = t.tris[3 * j + (k + 1) % 3];
          key.emplace(std::make_pair(std::min(a, b), std::max(a, b)), 0);
        }
      std::vector<int32_t> sedge, sadj, esed, vptr, vidx;
      std::vector<double> slen;
      int Se = 0;
      for (auto& kv : key) {
        kv.second = Se++;
        sedge.push_back(kv.first.first);
        sedge.push_back(kv.first.second);
        const double* A = mesh->rest_xyz + 3 * (size_t)kv.first.first;
        const double* B = mesh->rest_xyz + 3 * (size_t)kv.first.second;
        slen.push_back(std::sqrt((B[0] - A[0]) * (B[0] - A[0]) + (B[1] - A[1]) * (B[1] - A[1]) +
                                 (B[2] - A[2]) * (B[2] - A[2])));
      }
      sadj.assign(2 * (size_t)Se, -1);
      std::vector<std::vector<int32_t>> vl(V);
      for (size_t j = 0; j < S; ++j)
        for (int k = 0; k < 3; ++k) {
          const int a = t.tris[3 * j + k], b = t.tris[3 * j + (k + 1) % 3];
          const int f = key.at({std::min(a, b), std::max(a, b)});
          int32_t* slot = &sadj[2 * (size_t)f];
          const int32_t code = (int32_t)((j << 3) | (3 + k));
          if (slot[0] < 0) slot[0] = code;
          else if (slot[1] < 0) slot[1] = code;
          vl[a].push_back((int32_t)((j << 2) | k));
        }
      for (int f = 0; f < Se; ++f)
        for (int e = 0; e < 2; ++e) vl[sedge[2 * f + e]].push_back((int32_t)(((S + f) << 2) | e));
      const size_t VE = t.eitem.size() / 2;
      esed.assign(std::max<size_t>(VE, 1), -1);
      for (size_t k = 0; k < VE; ++k) {
        const int i = t.eitem[2 * k] / p->W, j = t.eitem[2 * k + 1] / p->W;
        auto it = key.find({std::min(i, j), std::max(i, j)});
        if (it != key.end()) esed[k] = it->second;
      }
      vptr.push_back(0);
      for (int c = 0; c < p->C; ++c) {
        std::vector<int32_t>& l = vl[t.cand[c]];
        std::sort(l.begin(), l.end());
        vidx.insert(vidx.end(), l.begin(), l.end());
        vptr.push_back((int32_t)vidx.size());
      }
      p->Se = Se;
      int32_t *d_sedge, *d_sadj, *d_esed, *d_vptr, *d_vidx;
      double* d_slen;
      ALLOC(d_sedge, int32_t*, 4 * std::max<size_t>(sedge.size(), 1));
      ALLOC(d_slen, double*, 8 * std::max<size_t>(slen.size(), 1));
      ALLOC(d_sadj, int32_t*, 4 * std::max<size_t>(sadj.size(), 1));
      ALLOC(d_esed, int32_t*, 4 * esed.size());
      ALLOC(d_vptr, int32_t*, 4 * vptr.size());
      ALLOC(d_vidx, int32_t*, 4 * std::max<size_t>(vidx.size(), 1));
      if (Se > 0) {
        if ((s = upload(ctx, d_sedge, sedge.data(), 4 * sedge.size()))) return s;
        if ((s = upload(ctx, d_slen, slen.data(), 8 * slen.size()))) return s;
        if ((s = upload(ctx, d_sadj, sadj.data(), 4 * sadj.size()))) return s;
      }
      if ((s = upload(ctx, d_esed, esed.data(), 4 * esed.size()))) return s;
      if ((s = upload(ctx, d_vptr, vptr.data(), 4 * vptr.size()))) return s;
      if (!vidx.empty() && (s = upload(ctx, d_vidx, vidx.data(), 4 * vidx.size()))) return s;
      E.Se = Se;
      E.sedge = d_sedge;
      E.sedge_len0 = d_slen;
      E.sedge_adj = d_sadj;
      E.edge_sedge = d_esed;
      E.vp_ptr = d_vptr;
      E.vp_idx = d_vidx;
    }
#undef ALLOC
    if ((s = upload(ctx, X, mesh->rest_xyz, 24 * V))) return s;
    if ((s = upload(ctx, x, mesh->rest_xyz, 24 * V))) return s;
    TC_HIP(hipMemsetAsync(v, 0, 24 * V, ctx->stream));
    if ((s = upload(ctx, tets, mesh->tets, 16 * T))) return s;
    std::vector<int8_t> hmat;
    if (mat) {
      hmat.resize(T, 0);
      if (mesh->tet_material)
        for (size_t e = 0; e < T; ++e) hmat[e] = (int8_t)mesh->tet_material[e];
      if ((s = upload(ctx, mat, hmat.data(), T))) return s;
    }
    if ((s = upload(ctx, fixed, t.fixed.data(), V))) return s;
    if (p->C > 0 && (s = upload(ctx, cand, t.cand.data(), 4 * p->C))) return s;
    if ((s = upload(ctx, cov, t.cand_of_vert.data(), 4 * V))) return s;
    if ((s = upload(ctx, tris, t.tris.data(), 12 * S))) return s;
    if ((s = upload(ctx, parent, t.parent.data(), 4 * S))) return s;
    if ((s = upload(ctx, istop, t.is_top.data(), S))) return s;
    if ((s = upload(ctx, ctp, t.ctri_ptr.data(), 4 * t.ctri_ptr.size()))) return s;
    if (!t.ctri_idx.empty() && (s = upload(ctx, cti, t.ctri_idx.data(), 4 * t.ctri_idx.size()))) return s;
    if ((s = upload(ctx, col, t.col.data(), 4 * t.col.size()))) return s;
    if ((s = upload(ctx, cptr, t.cptr.data(), 4 * t.cptr.size()))) return s;
    if ((s = upload(ctx, clist, t.clist.data(), 4 * t.clist.size()))) return s;
    if ((s = upload(ctx, cpos, t.cpos.data(), 4 * t.cpos.size()))) return s;
    if ((s = upload(ctx, dptr, t.dptr.data(), 4 * t.dptr.size()))) return s;
    if ((s = upload(ctx, eptr, t.eptr.data(), 4 * t.eptr.size()))) return s;
    if (!t.eitem.empty() && (s = upload(ctx, eitem, t.eitem.data(), 4 * t.eitem.size()))) return s;
    TC_HIP(hipMemsetAsync(E.reaction, 0, 24, ctx->stream));
    TC_HIP(hipMemsetAsync(E.traction_sum, 0, 24, ctx->stream));
    E.X = X; E.x = x; E.v = v; E.tets = tets; E.Dminv = Dminv; E.vol = vol; E.mat = mat;
    E.mass = mass; E.fixed = fixed; E.cand = cand; E.cand_of_vert = cov; E.cand_area = carea;
    E.tris = tris; E.parent = parent; E.is_top = istop; E.ctri_ptr = ctp; E.ctri_idx = cti;
    E.col = col; E.cptr = cptr; E.clist = clist; E.cpos = cpos;
    E.dptr = dptr; E.eptr = eptr; E.eitem = eitem;
    E.V_E = (int32_t)(t.eitem.size() / 2);
    E.meshes = ctx->d_meshes;
    for (int k = 0; k < MAX_MAT; ++k) {
      E.mu[k] = p->mu[k]; E.lam[k] = p->lam[k]; E.alpha[k] = p->alpha[k]; E.rho[k] = p->rho[k];
      E.cshift[k] = (k < n_materials && !params->literal_alpha) ? p->mu[k] : 0.0;
    }
    tc_pad_set_params(p, params);
    // setup kernels (a1): Dm^-1 and V_e, lumped mass, rest contact areas
    {
      const int B = 256;
      EnvDesc Ed = E;
      Ed.n_vt = cdiv(p->V, B);
      Ed.n_tt = cdiv(p->T, B);
      Ed.n_ct = p->C > 0 ? cdiv(p->C, B) : 0;
      std::vector<Tile> tiles;
      for (int k = 0; k < Ed.n_tt; ++k) tiles.push_back({0, k});
      for (int k = 0; k < Ed.n_vt; ++k) tiles.push_back({0, k});
      for (int k = 0; k < Ed.n_ct; ++k) tiles.push_back({0, k});
      EnvDesc* dd = nullptr;
      Tile* dt = nullptr;
      TC_HIP(hipMalloc(&dd, sizeof(EnvDesc)));
      TC_HIP(hipMalloc(&dt, sizeof(Tile) * tiles.size()));
      TC_HIP(hipMemcpyAsync(dd, &Ed, sizeof(EnvDesc), hipMemcpyHostToDevice, ctx->stream));
      TC_HIP(hipMemcpyAsync(dt, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, ctx->stream));
      LaunchArgs a;
      a.envs = dd;
      a.n_env = 1;
      a.block = B;
      a.stream = ctx->stream;
      a.tiles = dt; a.ntiles = Ed.n_tt;
      TC_HIP(launch_kernel(KernelId::setup_tets, p->fp64, a));
      a.tiles = dt + Ed.n_tt; a.ntiles = Ed.n_vt; a.out = mass;
      TC_HIP(launch_kernel(KernelId::setup_mass, p->fp64, a));
      a.tiles = dt + Ed.n_tt + Ed.n_vt; a.ntiles = Ed.n_ct; a.out = carea;
      TC_HIP(launch_kernel(KernelId::setup_area, p->fp64, a));
      TC_HIP(hipGetLastError());
      TC_HIP(hipStreamSynchronize(ctx->stream));
      (void)hipFree(dd);
      (void)hipFree(dt);
    }
    p->scratch_need = scratch_layout(p).total;
    ctx->pads.push_back(p);
    *out = guard.release();
    return TC_OK;
  });
}

tc_status tc_pad_destroy(tc_pad* pad) {
  if (!pad) return TC_OK;
  tc_context* ctx = pad->ctx;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (pad->busy.load()) return set_error(TC_E_BUSY, "pad has a request in flight on a server");
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  release_scratch(pad);
  drop_plans(ctx);
  for (auto& a : pad->allocs) ctx->dev_free(a.first, a.second);
  ctx->pads.erase(std::remove(ctx->pads.begin(), ctx->pads.end(), pad), ctx->pads.end());
  delete pad;
  return TC_OK;
}

tc_status tc_pad_get_info(const tc_pad* pad, tc_pad_info* out) {
  if (!pad || !out) return set_error(TC_E_INVALID_ARG, "pad or out is null");
  out->n_verts = pad->V;
  out->n_tets = pad->T;
  out->n_surface_tris = pad->S;
  out->n_top_tris = pad->S_top;
  out->n_candidates = pad->C;
  out->ell_width = pad->W;
  out->precision = pad->fp64 ? TC_PREC_FP64 : TC_PREC_MIXED;
  out->n_materials = pad->n_mat;
  out->resident_bytes = pad->resident_bytes;
  out->scratch_bytes = pad->scratch_need;
  out->bbox_diag = pad->bbox_diag;
  return TC_OK;
}

tc_status tc_pad_set_params(tc_pad* pad, const tc_params* params) {
  if (!pad) return set_error(TC_E_INVALID_ARG, "pad is null");
  std::string err;
  tc_status s = validate_params(params, err);
  if (s) return set_error(s, err);
  if ((params->precision == TC_PREC_FP64) != pad->fp64) return set_error(TC_E_INVALID_ARG, "precision is fixed at pad creation");
  std::lock_guard<std::recursive_mutex> lk(pad->ctx->mu);
  if (pad->busy.load()) return set_error(TC_E_BUSY, "pad has a request in flight on a server");
  const bool fric_layout = (pad->params.friction > 0) != (params->friction > 0) ||
                           (pad->params.mesh_contact == 2) != (params->mesh_contact == 2);
  pad->params = *params;
  if (fric_layout) {
    // the step scratch holds the friction lag only while friction is on,
    // the pair records only with mesh_contact 2
    (void)hipStreamSynchronize(pad->ctx->stream);
    release_scratch(pad);
    pad->scratch_need = scratch_layout(pad).total;
  }
  EnvDesc& E = pad->desc;
  E.h = params->dt;
  E.dhat = params->dhat;
  E.kappa = params->kappa;
  E.tol_abs = params->newton_tol * pad->bbox_diag;
  E.noise = 1e-12;
  E.cg_rel_tol = params->cg_rel_tol;
  E.cg_forcing = params->cg_forcing;
  E.hess_proj = params->hess_proj;
  E.cg_conv_tol = params->cg_conv_tol > 0 ? params->cg_conv_tol : params->cg_rel_tol;
  E.cg_eta_max = params->cg_eta_max;
  E.init_guess = params->init_guess;
  E.ls_expand = params->ls_expand;
  E.cg_warm = params->cg_warm;
  E.fr_mu = params->friction;
  E.fr_eps = params->eps_v * params->dt;
  E.mesh_pairs = params->mesh_contact;
  for (int c = 0; c < 3; ++c) E.gravity[c] = params->gravity[c];
  E.quasi_static = params->quasi_static;
  E.max_cg = params->max_cg;
  E.max_newton = params->max_newton;
  E.max_halvings = params->max_halvings;
  E.precond = params->precond;
  pad->desc_version = next_desc_version();
  drop_plans(pad->ctx);
  return TC_OK;
}

tc_status tc_pad_reset(tc_pad* pad) {
  if (!pad) return set_error(TC_E_INVALID_ARG, "pad is null");
  tc_context* ctx = pad->ctx;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (pad->busy.load()) return set_error(TC_E_BUSY, "pad has a request in flight on a server");
  TC_HIP(hipSetDevice(ctx->device));
  TC_HIP(hipMemcpyAsync(pad->desc.x, pad->desc.X, 24 * (size_t)pad->V, hipMemcpyDeviceToDevice, ctx->stream));
  TC_HIP(hipMemsetAsync(pad->desc.v, 0, 24 * (size_t)pad->V, ctx->stream));
  TC_HIP(hipStreamSynchronize(ctx->stream));
  pad->step_count = 0;
  pad->last_newton = 0;
  pad->n_prev = 0;
  return TC_OK;
}

tc_status tc_pad_release_scratch(tc_pad* pad) {
  if (!pad) return set_error(TC_E_INVALID_ARG, "pad is null");
  std::lock_guard<std::recursive_mutex> lk(pad->ctx->mu);
  if (pad->busy.load()) return set_error(TC_E_BUSY, "pad has a request in flight on a server");
  (void)hipStreamSynchronize(pad->ctx->stream);
  release_scratch(pad);
  return TC_OK;
}

tc_status tc_step(tc_pad* pad, int32_t n_ind, const tc_indenter* ind, tc_step_stats* stats) {
  if (!pad) return set_error(TC_E_INVALID_ARG, "pad is null");
  return guarded([&] { return run_batch(pad->ctx, 1, &pad, &n_ind, ind, stats, 0); });
}

tc_status tc_step_batch(tc_context* ctx, int32_t n, tc_pad* const* pads, const int32_t* n_ind,
                        const tc_indenter* ind, tc_step_stats* stats) {
  if (!ctx) return set_error(TC_E_INVALID_ARG, "ctx is null");
  return guarded([&] { return run_batch(ctx, n, pads, n_ind, ind, stats, 0); });
}

tc_status tc_extract(tc_pad* pad, int32_t n_ind, const tc_indenter* ind) {
  if (!pad) return set_error(TC_E_INVALID_ARG, "pad is null");
  return guarded([&] { return run_batch(pad->ctx, 1, &pad, &n_ind, ind, nullptr, 1); });
}

tc_status tc_pad_newton_direction(tc_pad* pad, int32_t n_ind, const tc_indenter* ind, double* dir, double* grad) {
  if (!pad) return set_error(TC_E_INVALID_ARG, "pad is null");
  if (pad->busy.load()) return set_error(TC_E_BUSY, "pad has a request in flight on a server");
  return guarded([&] { return newton_direction(pad, n_ind, ind, dir, grad); });
}

tc_status tc_field_info(const tc_pad* pad, int32_t field, int32_t* dtype, int64_t* count, int32_t* components) {
  if (!pad) return set_error(TC_E_INVALID_ARG, "pad is null");
  return field_layout(pad, field, dtype, count, components, nullptr);
}

tc_status tc_pad_read(const tc_pad* pad, int32_t field, void* dst, size_t bytes, int32_t dst_is_device) {
  if (!pad || !dst) return set_error(TC_E_INVALID_ARG, "pad or dst is null");
  int dt, comps;
  int64_t count;
  const void* src;
  tc_status s = field_layout(pad, field, &dt, &count, &comps, &src);
  if (s) return s;
  const size_t need = (size_t)count * comps * dtype_size(dt);
  if (bytes < need) return set_error(TC_E_INVALID_ARG, "destination too small: need " + std::to_string(need) + " bytes");
  if (need == 0) return TC_OK;
  tc_context* ctx = pad->ctx;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  TC_HIP(hipSetDevice(ctx->device));
  TC_HIP(hipMemcpyAsync(dst, src, need, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
  TC_HIP(hipStreamSynchronize(ctx->stream));
  return TC_OK;
}

tc_status tc_pad_write(tc_pad* pad, int32_t field, const void* src, size_t bytes, int32_t src_is_device) {
  if (!pad || !src) return set_error(TC_E_INVALID_ARG, "pad or src is null");
  if (field != TC_F_POSITIONS && field != TC_F_VELOCITIES) return set_error(TC_E_INVALID_ARG, "only POSITIONS and VELOCITIES are writable");
  const size_t need = 24 * (size_t)pad->V;
  if (bytes != need) return set_error(TC_E_INVALID_ARG, "size must be exactly " + std::to_string(need) + " bytes");
  tc_context* ctx = pad->ctx;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (pad->busy.load()) return set_error(TC_E_BUSY, "pad has a request in flight on a server");
  TC_HIP(hipSetDevice(ctx->device));
  void* dst = field == TC_F_POSITIONS ? (void*)pad->desc.x : (void*)pad->desc.v;
  TC_HIP(hipMemcpyAsync(dst, src, need, src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
  TC_HIP(hipStreamSynchronize(ctx->stream));
  return TC_OK;
}

// state buffer: magic, version, V, T, step count, then x and v; version 2
// appends the number of previous indenter poses and TC_MAX_INDENTERS poses
static const uint64_t kStateMagic = 0x5441434155434859ULL;
static const size_t kPoseBytes = 8 + sizeof(tc_indenter) * TC_MAX_INDENTERS;

tc_status tc_pad_save_state(const tc_pad* pad, void* buf, size_t* bytes) {
  if (!pad || !bytes) return set_error(TC_E_INVALID_ARG, "pad or bytes is null");
  const size_t xv = 48 * (size_t)pad->V;
  const size_t need = 40 + xv + kPoseBytes;
  if (!buf) { *bytes = need; return TC_OK; }
  if (*bytes < need) return set_error(TC_E_INVALID_ARG, "buffer too small");
  uint64_t head[5] = {kStateMagic, 2, (uint64_t)pad->V, (uint64_t)pad->T, (uint64_t)pad->step_count};
  std::memcpy(buf, head, 40);
  char* b = static_cast<char*>(buf) + 40;
  tc_status s = tc_pad_read(pad, TC_F_POSITIONS, b, 24 * (size_t)pad->V, 0);
  if (s) return s;
  s = tc_pad_read(pad, TC_F_VELOCITIES, b + 24 * (size_t)pad->V, 24 * (size_t)pad->V, 0);
  if (s) return s;
  const uint64_t np = (uint64_t)pad->n_prev;
  std::memcpy(b + xv, &np, 8);
  std::memset(b + xv + 8, 0, kPoseBytes - 8);
  std::memcpy(b + xv + 8, pad->prev, sizeof(tc_indenter) * pad->n_prev);
  *bytes = need;
  return TC_OK;
}

tc_status tc_pad_load_state(tc_pad* pad, const void* buf, size_t bytes) {
  if (!pad || !buf) return set_error(TC_E_INVALID_ARG, "pad or buf is null");
  const size_t xv = 48 * (size_t)pad->V;
  if (bytes < 40 + xv) return set_error(TC_E_INVALID_ARG, "buffer too small");
  uint64_t head[5];
  std::memcpy(head, buf, 40);
  if (head[0] != kStateMagic || (head[1] != 1 && head[1] != 2)) return set_error(TC_E_INVALID_ARG, "not a pad state buffer");
  if (head[2] != (uint64_t)pad->V || head[3] != (uint64_t)pad->T) return set_error(TC_E_INVALID_ARG, "state is for a different mesh");
  if (head[1] == 2 && bytes < 40 + xv + kPoseBytes) return set_error(TC_E_INVALID_ARG, "buffer too small");
  const char* b = static_cast<const char*>(buf) + 40;
  uint64_t np = 0;
  if (head[1] == 2) {
    std::memcpy(&np, b + xv, 8);
    if (np > TC_MAX_INDENTERS) return set_error(TC_E_INVALID_ARG, "corrupt pose count in state buffer");
  }
  tc_status s = tc_pad_write(pad, TC_F_POSITIONS, b, 24 * (size_t)pad->V, 0);
  if (s) return s;
  s = tc_pad_write(pad, TC_F_VELOCITIES, b + 24 * (size_t)pad->V, 24 * (size_t)pad->V, 0);
  if (s) return s;
  pad->step_count = (int64_t)head[4];
  pad->n_prev = (int)np;
  if (np) std::memcpy(pad->prev, b + xv + 8, sizeof(tc_indenter) * np);
  return TC_OK;
}

tc_status tc_autotune(tc_context* ctx, int32_t n, tc_pad* const* pads, const int32_t* n_ind,
                      const tc_indenter* ind, int32_t* chosen) {
  if (!ctx || n < 1 || !pads || !n_ind) return set_error(TC_E_INVALID_ARG, "bad autotune arguments");
  return guarded([&]() -> tc_status {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    TC_HIP(hipSetDevice(ctx->device));
    const int blk_cands[] = {128, 256, 512, 1024};
    const int el_cands[] = {64, 128, 256};
    const bool old_timing = ctx->timing;
    const int old_stride = ctx->timing_stride;
    const bool old_graphs = ctx->use_graphs;
    ctx->timing = true;
    ctx->timing_stride = 1;
    ctx->use_graphs = false;
    // probe: one step per candidate on saved state, restored afterwards
    auto probe = [&](int vb, int eb, int sb, double* t_spmv, double* t_upd, double* t_el) -> tc_status {
      ctx->cg_block = vb;
      ctx->el_block = eb;
      ctx->spmv_block = sb;
      drop_plans(ctx);
      for (auto& t : ctx->timers) t = KernelTimer{};
      std::vector<std::vector<char>> saved(n);
      std::vector<int64_t> steps(n);
      for (int i = 0; i < n; ++i) {
        size_t b = 0;
        tc_pad_save_state(pads[i], nullptr, &b);
        saved[i].resize(b);
        tc_status s = tc_pad_save_state(pads[i], saved[i].data(), &b);
        if (s) return s;
        steps[i] = pads[i]->step_count;
      }
      std::vector<tc_step_stats> st(n);
      tc_status s = run_batch(ctx, n, pads, n_ind, ind, st.data(), 0);
      for (int i = 0; i < n; ++i) {
        tc_pad_load_state(pads[i], saved[i].data(), saved[i].size());
        pads[i]->step_count = steps[i];
      }
      if (s && s != TC_E_NOT_CONVERGED && s != TC_E_LINESEARCH) return s;
      resolve_timing(ctx);
      int64_t cgit = 0;
      for (auto& x : st) cgit += x.cg_iters;
      const KernelTimer& ts = ctx->timers[(int)KernelId::cg_spmv];
      const KernelTimer& tu = ctx->timers[(int)KernelId::cg_update];
      const KernelTimer& te = ctx->timers[(int)KernelId::element];
      *t_spmv = cgit ? ts.ms / (double)cgit : 1e30;
      *t_upd = cgit ? tu.ms / (double)cgit : 1e30;
      *t_el = te.timed ? te.ms / te.timed : 1e30;
      return TC_OK;
    };
    int bcg = ctx->cg_block, bel = ctx->el_block, bsp = ctx->spmv_block;
    double best_u = 1e30, best_s = 1e30, best_e = 1e30;
    for (int b : blk_cands) {
      double ts, tu, te;
      tc_status s = probe(b, 128, b, &ts, &tu, &te);
      if (s) return s;
      if (tu < best_u) { best_u = tu; bcg = b; }
      if (ts < best_s) { best_s = ts; bsp = b; }
    }
    for (int eb : el_cands) {
      double ts, tu, te;
      tc_status s = probe(bcg, eb, bsp, &ts, &tu, &te);
      if (s) return s;
      if (te < best_e) { best_e = te; bel = eb; }
    }
    ctx->cg_block = bcg;
    ctx->el_block = bel;
    ctx->spmv_block = bsp;
    // second phase, by the wall time of whole probe steps with timing off:
    // streams the batch is split over, then CG iterations between host
    // checks (best of two probes each; the probes repeat identical work)
    ctx->timing = false;
    auto wall = [&](double* ms) -> tc_status {
      double best = 1e30;
      for (int rep = 0; rep < 2; ++rep) {
        std::vector<std::vector<char>> saved(n);
        std::vector<int64_t> steps(n);
        for (int i = 0; i < n; ++i) {
          size_t b = 0;
          tc_pad_save_state(pads[i], nullptr, &b);
          saved[i].resize(b);
          tc_status s = tc_pad_save_state(pads[i], saved[i].data(), &b);
          if (s) return s;
          steps[i] = pads[i]->step_count;
        }
        const double t0 = now_ms();
        tc_status s = run_batch(ctx, n, pads, n_ind, ind, nullptr, 0);
        const double dt = now_ms() - t0;
        for (int i = 0; i < n; ++i) {
          tc_pad_load_state(pads[i], saved[i].data(), saved[i].size());
          pads[i]->step_count = steps[i];
        }
        if (s && s != TC_E_NOT_CONVERGED && s != TC_E_LINESEARCH) return s;
        best = std::min(best, dt);
      }
      *ms = best;
      return TC_OK;
    };
    int best_lanes = ctx->n_lanes;
    double best_ms = 1e30;
    for (int nl = 1; nl <= TC_MAX_STREAMS && nl <= std::max(1, n / 2); ++nl) {
      ctx->n_lanes = nl;
      double ms;
      tc_status s = wall(&ms);
      if (s) return s;
      if (ms < best_ms * 0.98) { best_ms = ms; best_lanes = nl; }
    }
    ctx->n_lanes = best_lanes;
    int best_chunk = ctx->cg_per_replay;
    best_ms = 1e30;
    for (int ch : {8, 12, 16, 24}) {
      ctx->cg_per_replay = ch;
      double ms;
      tc_status s = wall(&ms);
      if (s) return s;
      if (ms < best_ms * 0.98) { best_ms = ms; best_chunk = ch; }
    }
    ctx->cg_per_replay = best_chunk;
    ctx->timing = old_timing;
    ctx->timing_stride = old_stride;
    ctx->use_graphs = old_graphs;
    drop_plans(ctx);
    for (auto& t : ctx->timers) t = KernelTimer{};
    if (chosen) {
      chosen[0] = bcg; chosen[1] = bel; chosen[2] = bsp; chosen[3] = ctx->cg_per_replay;
      chosen[4] = ctx->n_lanes;
    }
    return TC_OK;
  });
}

}  // extern "C"
