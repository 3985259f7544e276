// Internal runtime objects behind the C ABI (context, pads, batch plans).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tacauchy.h"
#include "tc_device.h"
#include "tc_launch.h"
#include "topology.h"

namespace tc {

tc_status set_error(tc_status s, const std::string& msg);
tc_status hip_fail(hipError_t e, const char* what);

#define TC_HIP(expr)                                        \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return ::tc::hip_fail(e_, #expr); \
  } while (0)

// First-fit sub-allocator of step scratch over device chunks of the context.
class Arena {
 public:
  struct Chunk {
    char* base;
    size_t size;
    std::map<size_t, size_t> free_;  // offset -> length
  };
  void* take(size_t bytes);          // nullptr if nothing fits
  void give(void* p, size_t bytes);
  bool add_chunk(char* base, size_t size);
  // removes the chunks that are entirely free; returns them (base, size)
  std::vector<std::pair<char*, size_t>> drop_empty();
  size_t held() const;
  std::vector<Chunk> chunks;
};

struct KernelTimer {
  double ms = 0.0;          // summed over the timed launches
  int64_t timed = 0;        // launches bracketed by events
  int64_t launches = 0;     // every launch while timing was on
  double bytes = 0.0;       // algorithmic bytes of all those launches
};

struct BatchPlan;

// A timed launch: its events, or (self-timed kernels) its blocks' clock
// cells at offset `cell` of its slice.
struct Pending {
  KernelId k;
  hipEvent_t a, b;
  size_t cell;
  int blocks;          // -1: events
};

// The clock cells [base, base + cap) of the context's array that one stream
// uses for its self-timed launches (cap 0: the whole array), and the timed
// launches of that stream not yet read back.
struct TimingSlice {
  std::vector<Pending> pending;
  size_t base = 0, cap = 0, used = 0;
};

// Device array of per-step states and poses with pinned host mirrors; a pad
// in a batch occupies one slot.
struct SlotPool {
  int cap = 0;
  EnvState* d_state = nullptr;
  EnvPose* d_pose = nullptr;
  EnvState* h_state = nullptr;
  EnvPose* h_pose = nullptr;
};

// A stream that steps a group of a batch's pads, with its own batch plan,
// state slots and timing slice.  The context's lane 0 points at the
// context's own stream, plan, pool and slice; the lanes of a batch split
// into groups own theirs.
struct Lane {
  hipStream_t stream = nullptr;
  std::unique_ptr<BatchPlan>* plan = nullptr;
  SlotPool* pool = nullptr;
  TimingSlice* ts = nullptr;
  std::unique_ptr<BatchPlan> own_plan;
  SlotPool own_pool;
  TimingSlice own_ts;
};

}  // namespace tc

struct tc_pad;

struct tc_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint64_t budget = 0;
  uint64_t used = 0;                 // resident + scratch chunks + plans
  tc::Arena arena;
  // launch shape
  int cg_block = 256;
  int spmv_block = 256;
  int el_block = 128;
  int cg_per_replay = 12;
  bool use_graphs = false;
  bool staged = true;                // batch schedule: staged (else lockstep)
  int ls_per_round = 3;              // trial energies per round of the staged schedule
  // timing
  bool timing = false;
  int timing_stride = 1;             // time every k-th launch of each kernel
  // clock cells of self-timed launches since the last sync (device, zeroed)
  unsigned long long* clock_cells = nullptr;
  size_t clock_cap = 0;              // in cells (u64)
  double clock_khz = 0.0;
  tc::TimingSlice tslice;            // launches on the context stream
  std::mutex tmu;                    // timers and the event pool (streams of several host threads)
  std::vector<hipEvent_t> free_events;
  tc::KernelTimer timers[(int)tc::KernelId::count];
  // per-step algorithmic byte counts are added when the step finishes
  std::unique_ptr<tc::BatchPlan> plan;
  tc::SlotPool pool;                 // slots of synchronous steps
  tc::Lane lane0;                    // the context's stream, plan, pool, slice
  int n_lanes = 1;                   // streams a batch is split over
  std::vector<std::unique_ptr<tc::Lane>> lanes;   // lanes of split batches
  std::recursive_mutex mu;           // serialises device work of API calls and the server
  int next_pad_id = 1;
  std::vector<tc_pad*> pads;         // every live pad of the context
  std::atomic<int64_t> evictions{0}; // step scratch released to make room
  std::atomic<int> n_servers{0};     // live servers of the context
  // rigid meshes (TC_MESH indenters): device table [MAX_MESHES], zeroed
  // slots are free; each live slot owns one device allocation
  tc::DevMesh* d_meshes = nullptr;
  struct MeshSlot {
    bool live = false;
    void* mem = nullptr;
    size_t bytes = 0;
    std::vector<double> verts;   // host copy of the vertices (local frame): a pose change's travel
  };
  std::vector<MeshSlot> mesh_slots;
  // guards mesh_slots' live flags: request submission checks them without
  // waiting for the device mutex (held by the server for a whole tick)
  mutable std::mutex mesh_mu;

  void* dev_alloc(size_t bytes, tc_status* st);
  void dev_free(void* p, size_t bytes);
};

struct tc_pad {
  tc_context* ctx = nullptr;
  int id = 0;
  int V = 0, T = 0, C = 0, S = 0, S_top = 0, W = 0;
  int Se = 0;                        // surface edges
  int64_t nnz_blocks = 0;
  int64_t n_edges = 0;               // unique edges (off-diagonal block pairs)
  bool fp64 = false;
  int rsize = 4;
  tc_params params{};
  int n_mat = 1;
  double mu[tc::MAX_MAT], lam[tc::MAX_MAT], alpha[tc::MAX_MAT], rho[tc::MAX_MAT];
  double bbox_diag = 0.0;
  int64_t step_count = 0;
  int last_newton = 0;               // Newton iterations of the last completed step (batch grouping)
  // indenter poses of the last completed step (friction lag), n_prev = 0: none
  int n_prev = 0;
  tc_indenter prev[TC_MAX_INDENTERS];
  uint64_t desc_version = 0;         // new (process-unique) value whenever the descriptor changes
  std::atomic<int> busy{0};
  std::atomic<int> in_flight{0};     // a step of this pad is on the device (server slot)
  // resident device arrays (one allocation each, tracked for free)
  std::vector<std::pair<void*, size_t>> allocs;
  uint64_t resident_bytes = 0;
  tc::EnvDesc desc{};                // resident and output pointers
  // step scratch (one arena block)
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  size_t scratch_need = 0;
};

namespace tc {

// Device-side data of a fixed list of pads with their scratch bound.
struct BatchPlan {
  std::vector<tc_pad*> pads;
  std::vector<int> slots;            // state/pose slot of each pad
  std::vector<void*> scratch;
  std::vector<uint64_t> versions;    // desc_version of each pad at build time
  int BV = 0, BT = 0, BS = 0;
  bool fp64 = false;
  EnvDesc* d_desc = nullptr;
  EnvState* d_state = nullptr;
  EnvState* h_state = nullptr;      // pinned
  Tile* d_tiles = nullptr;
  size_t dev_bytes = 0;
  // PAIR: surface triangles and edges (mesh_contact 2)
  enum Cls { VERT, TET, CAND, SURF, ASM, ENERGY, SPMV, PAIR, NCLS };
  int lpr = 0;                       // SpMV lanes per row
  int off[NCLS] = {0}, cnt[NCLS] = {0};
  std::vector<EnvDesc> h_desc;
  int desc_cap = 0, tiles_cap = 0;   // allocated lengths of d_desc and d_tiles
  char* h_stage = nullptr;           // pinned staging of the descriptor and tile uploads
  size_t stage_cap = 0;
  Tile* d_ctiles = nullptr;          // ring of compacted tile lists
  Tile* h_ctiles = nullptr;          // pinned staging of the ring
  int ctiles_cap = 0;
  int ctiles_off = 0;                // reset at every host sync
  hipGraphExec_t cg_exec = nullptr;
  hipGraph_t cg_graph = nullptr;
  int graph_M = 0;
  ~BatchPlan();
};

// Runs one step (mode 0) or extraction only (mode 1) for the pads.
tc_status run_batch(tc_context* ctx, int n, tc_pad* const* pads, const int32_t* n_ind,
                    const tc_indenter* ind, tc_step_stats* stats, int mode);

tc_status newton_direction(tc_pad* pad, int n_ind, const tc_indenter* ind, double* dir, double* grad);
tc_status ensure_scratch(tc_pad* pad);
uint64_t next_desc_version();
// Looks up this device's no-alloc scratch array (device current); once per
// device, at context creation.
tc_status noalloc_init(int device);
// The same, making room within the context budget when it is short: step
// scratch of pads not in `keep` and not in flight is released (largest
// first), then arena chunks left entirely free go back to the device.
tc_status ensure_scratch_evicting(tc_pad* pad, const std::vector<tc_pad*>& keep);
void release_scratch(tc_pad* pad);
tc_status pool_reserve(tc_context* ctx, SlotPool& p, int cap);
void pool_free(SlotPool& p);
// Builds the plan into `out`.  A plan already there is replaced; its device
// and pinned buffers are taken over when large enough (its stream must be
// idle), so that rebuilding a plan for a changed set of pads (the serving
// loop, between ticks) allocates nothing in the common case.
tc_status build_plan(tc_context* ctx, int n, tc_pad* const* pads, const int* slots, const SlotPool& pool,
                     std::unique_ptr<BatchPlan>& out, hipStream_t stream = nullptr);
// Lane g of split batches (created on first use, default-priority stream).
tc_status get_lane(tc_context* ctx, int g);
// Drops every cached batch plan of the context (lanes' streams idle).
void drop_plans(tc_context* ctx);
// Frees the split-batch lanes (streams idle).
void free_lanes(tc_context* ctx);
const std::string& last_error();
bool plan_matches(const BatchPlan* P, tc_context* ctx, int n, tc_pad* const* pads, const int* slots,
                  const SlotPool& pool);
void account_bytes(tc_context* ctx, const tc_pad* pad, const EnvState& s);
// Step-start state and poses of one slot; the friction lag takes the pad's
// previous poses when it has as many, else the current ones.
void init_state(EnvState& S, EnvPose& Q, int mode, int n_ind, const tc_indenter* ind, const tc_pad* pad);
// After a completed step: its poses become the pad's previous poses.
void remember_pose(tc_pad* pad, const EnvPose& Q);
// Every TC_MESH indenter names a live mesh of the context.
tc_status check_meshes(const tc_context* ctx, int n_ind, const tc_indenter* ind);
// Release every mesh of a context (context destruction).
void free_meshes(tc_context* ctx);
void fill_stats(tc_step_stats& o, const EnvState& S, double ms);

// Sequences the kernels of one Newton iteration over a plan.  Pad i of the
// plan uses state slot P->slots[i]; readbacks copy slots [0, span).
struct Runner {
  tc_context* ctx;
  BatchPlan* P;
  int n;
  SlotPool* pool;
  int span;
  // the stream the launches go to and its timing slice (null: the
  // context's own)
  hipStream_t stream = nullptr;
  TimingSlice* ts = nullptr;

  hipStream_t strm() const { return stream ? stream : ctx->stream; }
  TimingSlice& slice() const { return ts ? *ts : ctx->tslice; }

  const EnvState& state(int i) const { return pool->h_state[P->slots[i]]; }
  void launch(KernelId k, int cls, int parity = 0, int mode = 0);
  tc_status readback();
  bool any(bool (*pred)(const EnvState&)) const;
  // some pad matching pred has vertex-face / edge-edge pairs this step
  bool any_pairs(bool (*pred)(const EnvState&)) const;
  // tile lists of the kernel classes restricted to the pads matching a
  // predicate (the plan's own lists when every pad matches)
  struct View {
    const Tile* t[BatchPlan::NCLS];
    int c[BatchPlan::NCLS];
    bool full;
  };
  // mask: bit c set for each kernel class c to list (the others stay
  // empty); copy false: the lists are copied to the device by the next
  // flush_views, which must come before the first launch that reads them
  View view(bool (*pred)(const EnvState&), unsigned mask = ~0u, bool copy = true);
  void flush_views();
  int unflushed = -1;               // ring start of lists built but not yet copied
  bool ring_overflow = false;       // a view did not fit the ring (reported at the next readback)
  void launch_v(KernelId k, const View& v, int cls, int parity = 0, int mode = 0);
  tc_status cg_chunk(int M, const View& v);
  void launch_tiles(KernelId k, const Tile* tiles, int ntiles, int block, int parity, int mode = 0);
  // lockstep schedule: one Newton iteration of every running pad (pads
  // being initialised first)
  tc_status tick(bool init);
  // staged schedule: the whole step, each pad through the stages of its
  // Newton iterations at its own pace, in rounds of launches
  tc_status staged(int M, int K);
  // serve: pads admitted since the last readback are initialised within the
  // round, and pads that had ended at its start are extracted within it, so
  // the round's readback is its only host round trip
  tc_status round(int M, int K, bool serve = false);
  void init_launches();
  void finish_launches();
  tc_status finish();

  static bool is_run(const EnvState& s) { return s.phase == PH_RUN && s.status == TC_OK; }
  static bool cg_pending(const EnvState& s) { return is_run(s) && !s.cg_done; }
  static bool ls_pending(const EnvState& s) { return is_run(s) && !s.ls_done; }
  static bool is_finish(const EnvState& s) { return s.phase == PH_FINISH; }
  static bool not_done(const EnvState& s) { return s.phase != PH_DONE && s.phase != PH_IDLE; }
  static bool is_init(const EnvState& s) { return s.phase == PH_INIT && s.status == TC_OK; }
  static bool init_or_run(const EnvState& s) { return is_init(s) || is_run(s); }
  // stages of running pads as the last readback saw them
  static bool in_cg(const EnvState& s) {
    return is_run(s) && (s.stage == ST_ASM || s.stage == ST_CG) && !s.cg_done;
  }
  static bool dir_pending(const EnvState& s) { return is_run(s) && s.stage == ST_CG && s.cg_done; }
  static bool turning(const EnvState& s) { return dir_pending(s) || (is_run(s) && s.stage == ST_LS); }
  static bool may_start(const EnvState& s) { return is_run(s) && (s.stage == ST_START || turning(s)); }
  // the same with the pads admitted since the last readback (serving)
  static bool may_start_or_init(const EnvState& s) { return may_start(s) || is_init(s); }
  static bool run_or_init(const EnvState& s) { return is_run(s) || is_init(s); }
};

}  // namespace tc
