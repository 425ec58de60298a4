// Serving (continuous batching), in two forms over one caller-provided arena:
// whole calls -- worker threads with their own streams each run one request's call at
// a time in a block of the arena; or steps -- step engines (stepped.hip), each with a
// scheduler thread and stream of its own, advance their resident requests together,
// sweep by sweep, admitting new requests between steps.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "mgcd.h"
#include "stepped.hpp"

namespace {

constexpr size_t ALIGN = 256;
// Streams on which a stepped server's engine runs the phase work of many requests at
// once.
constexpr int STEP_PHASE_LANES = 4;
// Step engines of a stepped server: each takes half the resident places and half the
// shared region and runs on a stream and scheduler thread of its own, so that one
// engine's sweeps overlap the other's phase work (host round trips).
constexpr int STEP_ENGINES = 2;

struct Request {
  int64_t ticket = 0;
  mgcd_csr g{};
  int32_t *out = nullptr;
  size_t need = 0;
  int state = 0;  // 0 waiting, 1 running, 2 done
  int rc = MGCD_OK;
  std::string err;
  mgcd_stats stats{};
  double t_submit = 0, t_start = 0, t_end = 0;
  size_t off = 0;       // its block in the arena
  mgcd::StepJob job;    // step-level serving
  int eng = 0;          // step-level serving: its engine
};

// One step engine of a stepped server and the requests resident in it.
struct EngineSlot {
  std::unique_ptr<mgcd::StepEngine> engine;
  char *shared = nullptr;  // its slice of the shared region
  size_t shared_bytes = 0;
  int64_t max_resident = 0;
  std::unordered_map<Request *, std::shared_ptr<Request>> resident;
  int64_t res_N = 0, res_E = 0;
  std::multiset<int32_t> res_n;
  std::multiset<int64_t> res_nnz;
  mgcd_step_stats stats{};  // the engine's counters, copied under the server's lock
};

// First-fit allocator over [0, cap) with coalescing of free neighbours.
struct BlockAllocator {
  std::map<size_t, size_t> free_;  // offset -> size
  size_t used = 0, peak = 0;
  explicit BlockAllocator(size_t cap) {
    if (cap) free_[0] = cap;
  }
  bool take(size_t bytes, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used += bytes;
      if (used > peak) peak = used;
      return true;
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    used -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
};

int run_call(int32_t algo, const mgcd_csr *g, const mgcd_params *p, int32_t *out, void *ws,
             size_t bytes, mgcd_stats *stats, hipStream_t st) {
  switch (algo) {
    case MGCD_ALGO_LPA: return lpa_run(g, p, out, ws, bytes, stats, st);
    case MGCD_ALGO_LOUVAIN: return louvain_run(g, p, out, ws, bytes, stats, st);
    default: return leiden_run(g, p, out, ws, bytes, stats, st);
  }
}

}  // namespace

struct mgcd_server {
  char *arena = nullptr;
  int32_t algo = 0;
  mgcd_params params{};
  int device = 0;
  BlockAllocator blocks{0};
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::mutex mu;
  std::condition_variable cv_admit, cv_done;
  std::deque<std::shared_ptr<Request>> waiting;
  std::unordered_map<int64_t, std::shared_ptr<Request>> tickets;
  int64_t next_ticket = 1;
  int64_t running = 0;
  bool stopping = false;
  // step-level serving: the shared region [0, shared) of the arena (one slice per
  // engine), blocks after it
  bool stepped = false;
  size_t shared = 0;
  std::vector<EngineSlot> engs;
  uint64_t admit_gen = 0;  // changes whenever a request arrives or a block is freed
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // The oldest waiting request can start: a free block exists for it.
  bool head_fits(size_t *off) {
    return !waiting.empty() && blocks.take(waiting.front()->need, off);
  }

  void work(int slot) {
    (void)hipSetDevice(device);
    hipStream_t st = streams[slot];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      size_t off = 0;
      cv_admit.wait(lk, [&] { return (stopping && waiting.empty()) || head_fits(&off); });
      if (waiting.empty()) break;  // stopping and drained
      std::shared_ptr<Request> r = waiting.front();
      waiting.pop_front();
      r->state = 1;
      r->t_start = now();
      ++running;
      lk.unlock();
      const int rc = run_call(algo, &r->g, &params, r->out, arena + off, r->need, &r->stats, st);
      std::string err = rc == MGCD_OK ? std::string() : std::string(mgcd_last_error());
      lk.lock();
      blocks.give(off, r->need);
      r->rc = rc;
      r->err = std::move(err);
      r->t_end = now();
      r->state = 2;
      --running;
      cv_done.notify_all();
      cv_admit.notify_all();  // freed memory may admit the next request
    }
  }

  // Step-level serving: the oldest waiting requests join engine e while it has a
  // resident place, its shared slice holds its union with them and their block fits
  // (in arrival order; a request that does not fit waits for others to finish).
  void admit_waiting(int e, std::vector<std::shared_ptr<Request>> &adm) {
    EngineSlot &E = engs[(size_t)e];
    while (!waiting.empty() && (int64_t)E.resident.size() < E.max_resident) {
      std::shared_ptr<Request> r = waiting.front();
      const int32_t n = (int32_t)r->g.n;
      const int64_t nnz = r->g.nnz;
      const int32_t mx_n = std::max(n, E.res_n.empty() ? 0 : *E.res_n.rbegin());
      const int64_t mx_e = std::max(nnz, E.res_nnz.empty() ? (int64_t)0 : *E.res_nnz.rbegin());
      const size_t need = mgcd::StepEngine::shared_need(algo, params, (int64_t)E.resident.size() + 1,
                                                        E.res_N + n, E.res_E + nnz, mx_n, mx_e);
      size_t off = 0;
      if (need > E.shared_bytes || !blocks.take(r->need, &off)) break;
      waiting.pop_front();
      r->off = off;
      r->eng = e;
      r->job.g = r->g;
      r->job.out = r->out;
      r->job.block = arena + shared + off;
      r->job.user = r.get();
      r->state = 1;
      r->t_start = now();
      E.resident[r.get()] = r;
      E.res_N += n;
      E.res_E += nnz;
      E.res_n.insert(n);
      E.res_nnz.insert(nnz);
      ++running;
      adm.push_back(r);
    }
  }

  void complete(Request *r) {
    EngineSlot &E = engs[(size_t)r->eng];
    blocks.give(r->off, r->need);
    ++admit_gen;
    E.res_N -= r->g.n;
    E.res_E -= r->g.nnz;
    E.res_n.erase(E.res_n.find((int32_t)r->g.n));
    E.res_nnz.erase(E.res_nnz.find(r->g.nnz));
    r->rc = r->job.rc;
    r->err = r->job.err;
    r->stats = r->job.stats;
    r->t_end = now();
    r->state = 2;
    --running;
    E.resident.erase(r);
  }

  bool all_idle() const {
    for (const EngineSlot &E : engs)
      if (!E.resident.empty()) return false;
    return true;
  }

  void run_steps(int e) {
    (void)hipSetDevice(device);
    EngineSlot &E = engs[(size_t)e];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      std::vector<std::shared_ptr<Request>> adm;
      const uint64_t gen = admit_gen;
      admit_waiting(e, adm);
      if (adm.empty() && E.resident.empty()) {
        if (waiting.empty()) {
          if (stopping) break;
          cv_admit.wait(lk, [&] { return stopping || !waiting.empty(); });
          continue;
        }
        if (all_idle() && blocks.used == 0) {
          // nothing resident anywhere and the oldest request does not fit: it never will
          std::shared_ptr<Request> r = waiting.front();
          waiting.pop_front();
          r->rc = MGCD_E_WORKSPACE;
          r->err = "request does not fit the server's arena";
          r->t_start = r->t_end = now();
          r->state = 2;
          cv_done.notify_all();
          continue;
        }
        // the other engine holds the memory the oldest request needs: wait until a
        // request arrives or a block is freed (also when stopping: the queue drains)
        cv_admit.wait(lk, [&] { return admit_gen != gen; });
        continue;
      }
      lk.unlock();
      std::vector<mgcd::StepJob *> fin;
      auto fail = [&](int code, const std::string &msg) {
        E.engine->fail_all(code, msg, fin);
        for (auto &r : adm)
          if (!r->job.done) {
            r->job.rc = code;
            r->job.err = msg;
            r->job.done = true;
            fin.push_back(&r->job);
          }
      };
      try {
        std::vector<mgcd::StepJob *> js;
        for (auto &r : adm) js.push_back(&r->job);
        E.engine->admit(js, fin);
        E.engine->step(fin);
      } catch (const mgcd::Error &ex) {
        fail(ex.code, ex.what());
      } catch (const std::exception &ex) {
        fail(MGCD_E_ARG, ex.what());
      }
      lk.lock();
      E.stats = E.engine->counters();
      for (mgcd::StepJob *j : fin) complete((Request *)j->user);
      if (!fin.empty()) {
        cv_done.notify_all();
        cv_admit.notify_all();  // freed memory may admit requests into the other engine
      }
    }
  }
};

static int fail(int code, const char *msg) {
  mgcd::set_last_error(msg);
  return code;
}

extern "C" {

int mgcd_server_create(void *arena, size_t arena_bytes, int32_t slots, int32_t algo,
                       const mgcd_params *p, mgcd_server **out) {
  if (!out) return fail(MGCD_E_ARG, "out is null");
  *out = nullptr;
  if (!arena || arena_bytes == 0) return fail(MGCD_E_ARG, "arena is empty");
  if (((uintptr_t)arena % ALIGN) != 0) return fail(MGCD_E_ARG, "arena must be 256-byte aligned");
  if (slots < 1 || slots > 64) return fail(MGCD_E_ARG, "slots must be in [1, 64]");
  if (algo < MGCD_ALGO_LPA || algo > MGCD_ALGO_LEIDEN) return fail(MGCD_E_UNSUPPORTED, "unknown algorithm");
  auto s = std::make_unique<mgcd_server>();
  s->arena = (char *)arena;
  s->algo = algo;
  if (p)
    s->params = *p;
  else
    mgcd_default_params(algo, &s->params);
  s->blocks = BlockAllocator(arena_bytes / ALIGN * ALIGN);
  if (hipGetDevice(&s->device) != hipSuccess) return fail(MGCD_E_HIP, "hipGetDevice failed");
  mgcd::set_last_error("");
  for (int q = 0; q < slots; ++q) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      return fail(MGCD_E_HIP, "hipStreamCreateWithFlags failed");
    }
    s->streams.push_back(st);
  }
  for (int q = 0; q < slots; ++q) s->workers.emplace_back([srv = s.get(), q] { srv->work(q); });
  *out = s.release();
  return MGCD_OK;
}

int mgcd_server_create_stepped(void *arena, size_t arena_bytes, size_t shared_bytes, int32_t max_resident,
                               int32_t sweeps_per_step, int32_t algo, const mgcd_params *p, mgcd_server **out) {
  if (!out) return fail(MGCD_E_ARG, "out is null");
  *out = nullptr;
  if (!arena || arena_bytes == 0) return fail(MGCD_E_ARG, "arena is empty");
  if (((uintptr_t)arena % ALIGN) != 0) return fail(MGCD_E_ARG, "arena must be 256-byte aligned");
  if (max_resident < 1 || max_resident > (1 << 16)) return fail(MGCD_E_ARG, "max_resident must be in [1, 65536]");
  if (sweeps_per_step < 0) return fail(MGCD_E_ARG, "sweeps_per_step must be >= 0");
  if (algo < MGCD_ALGO_LPA || algo > MGCD_ALGO_LEIDEN) return fail(MGCD_E_UNSUPPORTED, "unknown algorithm");
  const size_t cap = arena_bytes / ALIGN * ALIGN;
  if (shared_bytes == 0) shared_bytes = cap / 20 * 9;  // 45%
  shared_bytes = shared_bytes / ALIGN * ALIGN;
  if (shared_bytes == 0 || shared_bytes >= cap) return fail(MGCD_E_ARG, "shared_bytes must leave room for blocks");
  auto s = std::make_unique<mgcd_server>();
  s->arena = (char *)arena;
  s->algo = algo;
  try {
    mgcd_params d;
    if (!p) {
      mgcd_default_params(algo, &d);
      p = &d;
    }
    s->params = mgcd::checked_params(p);
    if (algo != MGCD_ALGO_LPA && s->params.one_scan)
      throw mgcd::Error(MGCD_E_UNSUPPORTED, "one_scan is defined for LPA only");
  } catch (const mgcd::Error &e) {
    return fail(e.code, e.what());
  }
  s->stepped = true;
  s->shared = shared_bytes;
  s->blocks = BlockAllocator(cap - shared_bytes);
  if (hipGetDevice(&s->device) != hipSuccess) return fail(MGCD_E_HIP, "hipGetDevice failed");
  mgcd::set_last_error("");
  const int ne = max_resident < STEP_ENGINES ? max_resident : STEP_ENGINES;
  const size_t slice = shared_bytes / (size_t)ne / ALIGN * ALIGN;
  s->engs.resize((size_t)ne);
  for (int e = 0; e < ne; ++e) {
    EngineSlot &E = s->engs[(size_t)e];
    E.shared = s->arena + (size_t)e * slice;
    E.shared_bytes = slice;
    E.max_resident = max_resident / ne + (e < max_resident % ne ? 1 : 0);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      return fail(MGCD_E_HIP, "hipStreamCreateWithFlags failed");
    }
    s->streams.push_back(st);
    try {
      E.engine = std::make_unique<mgcd::StepEngine>(algo, s->params, sweeps_per_step, E.shared, slice, st,
                                                    STEP_PHASE_LANES);
    } catch (const mgcd::Error &ex) {
      s->engs.clear();
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      return fail(ex.code, ex.what());
    }
  }
  for (int e = 0; e < ne; ++e) s->workers.emplace_back([srv = s.get(), e] { srv->run_steps(e); });
  *out = s.release();
  return MGCD_OK;
}

int mgcd_server_submit(mgcd_server *s, const mgcd_csr *g, int32_t *communities_out,
                       int64_t *ticket) {
  if (!s || !g || !ticket) return fail(MGCD_E_ARG, "null argument");
  if (g->n < 0 || g->nnz < 0) return fail(MGCD_E_ARG, "negative size");
  if (g->n > 0 && !communities_out) return fail(MGCD_E_ARG, "communities_out is null");
  auto r = std::make_shared<Request>();
  r->g = *g;
  r->out = communities_out;
  const size_t need = s->stepped ? mgcd::StepEngine::block_bytes(s->algo, s->params, g->n, g->nnz)
                                 : mgcd_workspace_bytes(s->algo, g->n, g->nnz, &s->params);
  r->need = need < ALIGN ? ALIGN : (need + ALIGN - 1) / ALIGN * ALIGN;
  std::lock_guard<std::mutex> lk(s->mu);
  size_t cap = 0;
  for (auto &b : s->blocks.free_) cap += b.second;
  cap += s->blocks.used;
  if (r->need > cap) return fail(MGCD_E_WORKSPACE, "request needs more than the whole arena");
  if (s->stepped &&
      mgcd::StepEngine::shared_need(s->algo, s->params, 1, g->n, g->nnz, (int32_t)g->n, g->nnz) >
          s->engs[0].shared_bytes)
    return fail(MGCD_E_WORKSPACE, "request needs more than a step engine's share of the shared region");
  if (s->stopping) return fail(MGCD_E_ARG, "server is shutting down");
  r->ticket = s->next_ticket++;
  ++s->admit_gen;
  r->t_submit = s->now();
  s->tickets[r->ticket] = r;
  s->waiting.push_back(r);
  *ticket = r->ticket;
  s->cv_admit.notify_all();
  return MGCD_OK;
}

int mgcd_server_poll(mgcd_server *s, int64_t ticket, int32_t *state) {
  if (!s || !state) return fail(MGCD_E_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(MGCD_E_ARG, "unknown ticket");
  *state = it->second->state;
  return MGCD_OK;
}

int mgcd_server_wait(mgcd_server *s, int64_t ticket, mgcd_stats *stats, double *times) {
  if (!s) return fail(MGCD_E_ARG, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(MGCD_E_ARG, "unknown ticket");
  std::shared_ptr<Request> r = it->second;
  s->cv_done.wait(lk, [&] { return r->state == 2; });
  s->tickets.erase(ticket);
  if (stats) *stats = r->stats;
  if (times) {
    times[0] = r->t_submit;
    times[1] = r->t_start;
    times[2] = r->t_end;
  }
  if (r->rc != MGCD_OK) mgcd::set_last_error(r->err);
  return r->rc;
}

int mgcd_server_info(mgcd_server *s, int64_t *waiting, int64_t *running, size_t *bytes_in_use,
                     size_t *peak_bytes) {
  if (!s) return fail(MGCD_E_ARG, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (waiting) *waiting = (int64_t)s->waiting.size();
  if (running) *running = s->running;
  if (bytes_in_use) *bytes_in_use = s->blocks.used;
  if (peak_bytes) *peak_bytes = s->blocks.peak;
  return MGCD_OK;
}

int mgcd_server_step_stats(mgcd_server *s, mgcd_step_stats *out) {
  if (!s || !out) return fail(MGCD_E_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  mgcd_step_stats t{};
  for (const EngineSlot &E : s->engs) {
    t.steps += E.stats.steps;
    t.sweeps += E.stats.sweeps;
    t.sweeps_moving += E.stats.sweeps_moving;
    t.packs += E.stats.packs;
    t.transitions += E.stats.transitions;
    t.rows_swept += E.stats.rows_swept;
    t.rows_moving += E.stats.rows_moving;
    t.s_pack += E.stats.s_pack;
    t.s_sweep += E.stats.s_sweep;
    t.s_phase += E.stats.s_phase;
    t.s_admit += E.stats.s_admit;
  }
  *out = t;
  return MGCD_OK;
}

int mgcd_server_destroy(mgcd_server *s) {
  if (!s) return MGCD_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv_admit.notify_all();
  for (auto &t : s->workers) t.join();
  int rc = MGCD_OK;
  for (hipStream_t st : s->streams)
    if (hipStreamDestroy(st) != hipSuccess) rc = fail(MGCD_E_HIP, "hipStreamDestroy failed");
  delete s;
  return rc;
}

}  // extern "C"
