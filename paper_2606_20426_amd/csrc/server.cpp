// Continuous-batching step server: one host thread drives a running batch
// of pad steps; requests join at Newton-iteration boundaries and leave when
// their step completes (see tc_server_create in tacauchy.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "runtime.h"

using namespace tc;

struct tc_server {
  struct Req {
    uint64_t ticket = 0;
    tc_pad* pad = nullptr;
    int tag = 0;
    int n_ind = 0;
    tc_indenter ind[TC_MAX_INDENTERS];
    double t_arrive = 0;
    double t_admit = 0;
  };
  tc_context* ctx = nullptr;
  int max_slots = 1;
  std::thread th;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::deque<Req> queue;
  std::vector<tc_result> done;
  std::vector<int> slot_used;
  std::vector<Req> slot_req;
  SlotPool pool;
  std::unique_ptr<BatchPlan> plan;
  uint64_t next_ticket = 1;
  tc_server_stats stats{};
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  tc_status fatal = TC_OK;

  double now() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  void loop();
  bool admit(std::vector<int>& fresh);
};

// Admit queued requests (FIFO, a pad's requests in order) while slots are
// free and their step scratch fits the context budget; when memory runs
// short, the step scratch of pads without a step on the device is released
// first.
bool tc_server::admit(std::vector<int>& fresh) {
  std::vector<tc_pad*> running;
  for (int s = 0; s < max_slots; ++s)
    if (slot_used[s]) running.push_back(slot_req[s].pad);
  bool blocked = false;
  for (auto it = queue.begin(); it != queue.end() && !blocked;) {
    int slot = -1;
    for (int s = 0; s < max_slots; ++s)
      if (!slot_used[s]) { slot = s; break; }
    if (slot < 0) break;
    tc_pad* p = it->pad;
    if (std::find(running.begin(), running.end(), p) != running.end()) { ++it; continue; }
    bool earlier_same_pad = false;
    for (auto jt = queue.begin(); jt != it; ++jt)
      if (jt->pad == p) earlier_same_pad = true;
    if (earlier_same_pad) { ++it; continue; }
    // running requests keep their scratch; any other pad's may go
    tc_status s = ensure_scratch_evicting(p, running);
    // short of memory: wait for running requests to finish; with none
    // running the request can never fit and is rejected
    if (s == TC_E_NO_MEMORY && !running.empty()) { blocked = true; break; }
    Req r = *it;
    it = queue.erase(it);
    if (s != TC_OK) {
      tc_result res{};
      res.ticket = r.ticket;
      res.status = s;
      res.pad_index = r.tag;
      res.t_arrive_ms = r.t_arrive;
      res.t_admit_ms = res.t_done_ms = now();
      res.stats.status = s;
      r.pad->busy.store(0);
      done.push_back(res);
      stats.rejected++;
      continue;
    }
    r.t_admit = now();
    p->in_flight.store(1);
    slot_used[slot] = 1;
    slot_req[slot] = r;
    running.push_back(p);
    fresh.push_back(slot);
    stats.admitted++;
  }
  return !fresh.empty();
}

void tc_server::loop() {
  for (;;) {
    std::vector<int> fresh;
    {
      std::unique_lock<std::mutex> lk(m);
      cv_work.wait(lk, [&] {
        if (stop) return true;
        for (int s = 0; s < max_slots; ++s)
          if (slot_used[s]) return true;
        return !queue.empty();
      });
      int nrun = 0;
      for (int s = 0; s < max_slots; ++s) nrun += slot_used[s];
      if (stop && nrun == 0) break;
      std::lock_guard<std::recursive_mutex> dl(ctx->mu);
      if (!stop) admit(fresh);
      nrun = 0;
      for (int s = 0; s < max_slots; ++s) nrun += slot_used[s];
      stats.running = nrun;
      stats.queued = (int)queue.size();
      stats.max_running_seen = std::max(stats.max_running_seen, nrun);
      if (nrun == 0) {
        // nothing admissible (memory): wait for a submit or stop
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(200));
        continue;
      }
    }
    std::lock_guard<std::recursive_mutex> dl(ctx->mu);
    (void)hipSetDevice(ctx->device);
    std::vector<tc_pad*> pads;
    std::vector<int> slots;
    for (int s = 0; s < max_slots; ++s)
      if (slot_used[s]) { pads.push_back(slot_req[s].pad); slots.push_back(s); }
    const int n = (int)pads.size();
    for (int s : fresh) {
      const Req& r = slot_req[s];
      init_state(pool.h_state[s], pool.h_pose[s], 0, r.n_ind, r.ind, r.pad);
      (void)hipMemcpyAsync(pool.d_state + s, pool.h_state + s, sizeof(EnvState), hipMemcpyHostToDevice, ctx->stream);
      (void)hipMemcpyAsync(pool.d_pose + s, pool.h_pose + s, sizeof(EnvPose), hipMemcpyHostToDevice, ctx->stream);
    }
    tc_status st = TC_OK;
    if (!plan_matches(plan.get(), ctx, n, pads.data(), slots.data(), pool)) {
      st = build_plan(ctx, n, pads.data(), slots.data(), pool, plan);
    }
    if (st == TC_OK) {
      Runner run{ctx, plan.get(), n, &pool, max_slots};
      // one tick: a lockstep Newton iteration, or a staged round that also
      // initialises the admitted requests and extracts the ended ones
      st = ctx->staged ? run.round(std::max(2, ctx->cg_per_replay & ~1), ctx->ls_per_round, true)
                       : run.tick(!fresh.empty());
    }
    std::lock_guard<std::mutex> lk(m);
    stats.ticks++;
    const double t = now();
    for (int i = 0; i < n; ++i) {
      const int s = slots[i];
      const EnvState& S = pool.h_state[s];
      if (st == TC_OK && S.phase != PH_DONE) continue;
      Req& r = slot_req[s];
      tc_result res{};
      res.ticket = r.ticket;
      res.status = st != TC_OK ? st : S.status;
      res.pad_index = r.tag;
      res.t_arrive_ms = r.t_arrive;
      res.t_admit_ms = r.t_admit;
      res.t_done_ms = t;
      fill_stats(res.stats, S, t - r.t_admit);
      res.stats.status = res.status;
      if (res.status == TC_OK) {
        r.pad->step_count++;
        remember_pose(r.pad, pool.h_pose[s]);
      }
      if (ctx->timing) account_bytes(ctx, r.pad, S);
      r.pad->in_flight.store(0);
      r.pad->busy.store(0);
      done.push_back(res);
      slot_used[s] = 0;
      stats.completed++;
    }
    if (st != TC_OK) fatal = st;
    cv_done.notify_all();
  }
  std::lock_guard<std::mutex> lk(m);
  for (auto& r : queue) {
    tc_result res{};
    res.ticket = r.ticket;
    res.status = TC_E_BUSY;
    res.pad_index = r.tag;
    res.t_arrive_ms = r.t_arrive;
    res.t_admit_ms = res.t_done_ms = now();
    res.stats.status = TC_E_BUSY;
    r.pad->busy.store(0);
    done.push_back(res);
  }
  queue.clear();
  cv_done.notify_all();
}

extern "C" {

tc_status tc_server_create(tc_context* ctx, int32_t max_slots, tc_server** out) {
  if (!ctx || !out || max_slots < 1 || max_slots > 4096) return set_error(TC_E_INVALID_ARG, "bad server arguments");
  *out = nullptr;
  auto* s = new tc_server();
  s->ctx = ctx;
  s->max_slots = max_slots;
  s->slot_used.assign(max_slots, 0);
  s->slot_req.resize(max_slots);
  {
    std::lock_guard<std::recursive_mutex> dl(ctx->mu);
    (void)hipSetDevice(ctx->device);
    tc_status st = pool_reserve(ctx, s->pool, max_slots);
    if (st) { delete s; return st; }
    for (int k = 0; k < s->pool.cap; ++k) {
      std::memset(&s->pool.h_state[k], 0, sizeof(EnvState));
      s->pool.h_state[k].phase = PH_IDLE;
    }
    hipError_t e = hipMemcpy(s->pool.d_state, s->pool.h_state, sizeof(EnvState) * s->pool.cap, hipMemcpyHostToDevice);
    if (e != hipSuccess) { pool_free(s->pool); delete s; return hip_fail(e, "server state upload"); }
  }
  ctx->n_servers++;
  s->th = std::thread([s] { s->loop(); });
  *out = s;
  return TC_OK;
}

tc_status tc_server_submit(tc_server* srv, tc_pad* pad, int32_t tag, int32_t n_ind, const tc_indenter* ind,
                           uint64_t* ticket) {
  if (!srv || !pad) return set_error(TC_E_INVALID_ARG, "server or pad is null");
  if (pad->ctx != srv->ctx) return set_error(TC_E_INVALID_ARG, "pad belongs to another context");
  std::string err;
  tc_status s = validate_indenters(n_ind, ind, err);
  if (s) return set_error(s, err);
  if ((s = check_meshes(srv->ctx, n_ind, ind))) return s;
  std::lock_guard<std::mutex> lk(srv->m);
  if (srv->stop) return set_error(TC_E_BUSY, "server is stopping");
  tc_server::Req r;
  r.ticket = srv->next_ticket++;
  r.pad = pad;
  r.tag = tag;
  r.n_ind = n_ind;
  for (int k = 0; k < n_ind; ++k) r.ind[k] = ind[k];
  r.t_arrive = srv->now();
  pad->busy.store(1);
  srv->queue.push_back(r);
  srv->stats.submitted++;
  if (ticket) *ticket = r.ticket;
  srv->cv_work.notify_one();
  return TC_OK;
}

tc_status tc_server_poll(tc_server* srv, tc_result* out, int32_t cap, int32_t* n, int32_t wait_us) {
  if (!srv || !n || (cap > 0 && !out)) return set_error(TC_E_INVALID_ARG, "bad poll arguments");
  std::unique_lock<std::mutex> lk(srv->m);
  if (srv->done.empty() && wait_us > 0)
    srv->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return !srv->done.empty(); });
  const int k = std::min<int>(cap, (int)srv->done.size());
  for (int i = 0; i < k; ++i) out[i] = srv->done[i];
  srv->done.erase(srv->done.begin(), srv->done.begin() + k);
  *n = k;
  if (srv->fatal != TC_OK) return set_error(srv->fatal, "server device error");
  return TC_OK;
}

tc_status tc_server_get_stats(tc_server* srv, tc_server_stats* out) {
  if (!srv || !out) return set_error(TC_E_INVALID_ARG, "server or out is null");
  std::lock_guard<std::mutex> lk(srv->m);
  *out = srv->stats;
  out->queued = (int)srv->queue.size();
  uint64_t sc = 0;
  for (int s = 0; s < srv->max_slots; ++s)
    if (srv->slot_used[s]) sc += srv->slot_req[s].pad->scratch_bytes;
  out->scratch_in_use = sc;
  out->evictions = srv->ctx->evictions.load();
  return TC_OK;
}

tc_status tc_server_destroy(tc_server* srv) {
  if (!srv) return TC_OK;
  {
    std::lock_guard<std::mutex> lk(srv->m);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->th.joinable()) srv->th.join();
  {
    std::lock_guard<std::recursive_mutex> dl(srv->ctx->mu);
    srv->plan.reset();
    pool_free(srv->pool);
    srv->ctx->n_servers--;
  }
  delete srv;
  return TC_OK;
}

}  // extern "C"
