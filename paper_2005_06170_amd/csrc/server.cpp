// Continuous-batching server for catalogs of uneven sizes (mps_server_*).
//
// Requests enter a FIFO.  Worker threads, each owning one HIP stream, admit
// the oldest request whose device footprint fits the remaining HBM budget
// and whose grid shape has a resident (or creatable) plan; a worker that
// admits a small request also takes the other queued small requests of the
// same grid shape (up to its batch size) and launches all their stages
// back to back on its stream.  Requests that arrive while others are on the
// device are admitted as soon as a worker and memory free up, and their
// kernels run concurrently with the others' on separate streams.  Plans
// (grids, twiddles, tables, particle workspace) stay resident between
// requests and are evicted least-recently-used only when a new shape needs
// the memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace mps {
namespace {

constexpr int kMaxBatch = 16;

struct Request {
  uint64_t ticket = 0;
  mps_catalog cat{};
  std::vector<double> edges;
  int n_grid = 0;
  mps_precision prec = MPS_F32;
  mps_result* out = nullptr;
  size_t bytes = 0;           // footprint of a plan serving it
  bool done = false;
  int status = MPS_OK;
};

struct PooledPlan {
  mps_plan* plan = nullptr;
  int n_grid = 0;
  mps_precision prec = MPS_F32;
  int64_t cap = 0;            // particles reserved
  int64_t host_cap = 0;       // particles of host-catalog staging reserved
  size_t bytes = 0;
  bool busy = false;
  uint64_t last_use = 0;
};

}  // namespace

struct Server {
  size_t budget = 0;
  size_t used = 0;             // bytes held by pooled plans
  int max_inflight = 1;
  int64_t small = 0;
  int device = 0;
  uint64_t next_ticket = 1;
  uint64_t clock = 0;
  bool stop = false;

  std::mutex mu;
  std::condition_variable cv_work;   // queue or memory changed
  std::condition_variable cv_done;   // a request finished
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
  std::list<PooledPlan> pool;
  std::vector<std::thread> workers;
};

namespace {

// Evict idle plans (least recently used first, never `keep`) until `need`
// more bytes fit the budget.  Returns false if running requests hold too much.
bool make_room(Server* s, size_t need, const PooledPlan* keep) {
  while (s->used + need > s->budget) {
    auto victim = s->pool.end();
    for (auto it = s->pool.begin(); it != s->pool.end(); ++it)
      if (!it->busy && &*it != keep && (victim == s->pool.end() || it->last_use < victim->last_use)) victim = it;
    if (victim == s->pool.end()) return false;
    mps_plan_destroy(victim->plan);
    s->used -= victim->bytes;
    s->pool.erase(victim);
  }
  return true;
}

size_t plan_bytes(int n_grid, mps_precision prec, int64_t cap, int64_t host_cap) {
  return mps_footprint(n_grid, prec, cap) + kHostStageBytes * static_cast<size_t>(host_cap);
}

// An idle pooled plan of this shape with room for np particles (and, for a
// host-resident catalog, np particles of staging): reuse one that is large
// enough, else grow the largest idle one of the shape, else create one.
// Called with mu held; returns nullptr if the budget cannot host it right
// now (*status stays MPS_OK) or never can / creation failed.
PooledPlan* acquire_plan(Server* s, int n_grid, mps_precision prec, int64_t np, bool host, int* status) {
  *status = MPS_OK;
  const int64_t hp = host ? np : 0;
  if (plan_bytes(n_grid, prec, np, hp) > s->budget) {
    *status = MPS_E_TOOBIG;
    return nullptr;
  }
  PooledPlan* fit = nullptr;
  PooledPlan* grow = nullptr;
  for (auto& pp : s->pool) {
    if (pp.busy || pp.n_grid != n_grid || pp.prec != prec) continue;
    if (pp.cap >= np && pp.host_cap >= hp) {
      if (!fit || pp.cap < fit->cap) fit = &pp;
    } else if (!grow || pp.cap > grow->cap) {
      grow = &pp;
    }
  }
  if (fit) {
    fit->busy = true;
    fit->last_use = ++s->clock;
    return fit;
  }
  if (grow) {
    const int64_t cap = std::max(grow->cap, np), hcap = std::max(grow->host_cap, hp);
    const size_t need = plan_bytes(n_grid, prec, cap, hcap);
    if (!make_room(s, need - grow->bytes, grow)) return nullptr;
    int st = mps_plan_reserve(grow->plan, cap);
    if (st == MPS_OK && hcap > 0) st = ensure_host_stage(reinterpret_cast<Plan*>(grow->plan), hcap);
    if (st != MPS_OK) {
      *status = st;
      return nullptr;
    }
    s->used += need - grow->bytes;
    grow->bytes = need;
    grow->cap = cap;
    grow->host_cap = hcap;
    grow->busy = true;
    grow->last_use = ++s->clock;
    return grow;
  }
  const size_t need = plan_bytes(n_grid, prec, np, hp);
  if (!make_room(s, need, nullptr)) return nullptr;
  mps_plan* plan = nullptr;
  int st = mps_plan_create(&plan, n_grid, prec);
  if (st == MPS_OK) st = mps_plan_reserve(plan, np);
  if (st == MPS_OK && hp > 0) st = ensure_host_stage(reinterpret_cast<Plan*>(plan), hp);
  if (st != MPS_OK) {
    if (plan) mps_plan_destroy(plan);
    *status = st;
    return nullptr;
  }
  PooledPlan pp;
  pp.plan = plan;
  pp.n_grid = n_grid;
  pp.prec = prec;
  pp.cap = np;
  pp.host_cap = hp;
  pp.bytes = need;
  pp.busy = true;
  pp.last_use = ++s->clock;
  s->used += need;
  s->pool.push_back(pp);
  return &s->pool.back();
}

void finish(Server* s, const std::shared_ptr<Request>& r, int status) {
  r->status = status;
  r->done = true;
  (void)s;
}

void worker_main(Server* s) {
  (void)hipSetDevice(s->device);
  hipStream_t stream = nullptr;
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    std::vector<std::shared_ptr<Request>> batch;
    std::vector<PooledPlan*> plans;
    // admit: the oldest request that fits; small requests pull same-shape peers
    while (batch.empty()) {
      if (s->stop && s->queue.empty()) {
        lk.unlock();
        if (stream) (void)hipStreamDestroy(stream);
        return;
      }
      for (auto it = s->queue.begin(); it != s->queue.end();) {
        const auto r = *it;
        int st = MPS_OK;
        PooledPlan* pp = acquire_plan(s, r->n_grid, r->prec, r->cat.n_particles,
                                      (r->cat.flags & MPS_CATALOG_HOST) != 0, &st);
        if (!pp && st != MPS_OK) {  // can never run (too big, or creation failed)
          it = s->queue.erase(it);
          finish(s, r, st);
          s->cv_done.notify_all();
          continue;
        }
        if (!pp) {
          ++it;
          continue;
        }
        batch.push_back(r);
        plans.push_back(pp);
        it = s->queue.erase(it);
        if (r->cat.n_particles <= s->small) {
          for (auto jt = s->queue.begin(); jt != s->queue.end() && batch.size() < kMaxBatch;) {
            const auto q = *jt;
            if (q->n_grid != r->n_grid || q->prec != r->prec || q->cat.n_particles > s->small) {
              ++jt;
              continue;
            }
            int st2 = MPS_OK;
            PooledPlan* p2 = acquire_plan(s, q->n_grid, q->prec, q->cat.n_particles,
                                          (q->cat.flags & MPS_CATALOG_HOST) != 0, &st2);
            if (!p2) break;
            batch.push_back(q);
            plans.push_back(p2);
            jt = s->queue.erase(jt);
          }
        }
        break;
      }
      if (batch.empty()) s->cv_work.wait(lk);
    }
    lk.unlock();

    // run the batch: all stages enqueued back to back, one synchronisation
    std::vector<int> status(batch.size(), MPS_OK);
    for (size_t i = 0; i < batch.size(); ++i) {
      Plan* p = reinterpret_cast<Plan*>(plans[i]->plan);
      int st = ensure_bins(p, &batch[i]->cat);
      if (st == MPS_OK) st = ensure_particles(p, batch[i]->cat.n_particles);
      if (st == MPS_OK) st = enqueue_estimate(p, &batch[i]->cat, stream);
      status[i] = st;
    }
    const bool synced = hipStreamSynchronize(stream) == hipSuccess;
    for (size_t i = 0; i < batch.size(); ++i) {
      if (status[i] == MPS_OK)
        status[i] = synced ? unpack(reinterpret_cast<Plan*>(plans[i]->plan), &batch[i]->cat, batch[i]->out)
                           : MPS_E_HIP;
    }

    lk.lock();
    for (size_t i = 0; i < batch.size(); ++i) {
      plans[i]->busy = false;
      finish(s, batch[i], status[i]);
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

}  // namespace
}  // namespace mps

using namespace mps;

extern "C" {

int mps_server_create(mps_server** out, size_t hbm_budget_bytes, int max_inflight, int64_t small_particles) {
  if (!out || hbm_budget_bytes == 0 || max_inflight < 1 || max_inflight > 64 || small_particles < 0)
    return MPS_E_ARG;
  *out = nullptr;
  Server* s = new (std::nothrow) Server();
  if (!s) return MPS_E_NOMEM;
  s->budget = hbm_budget_bytes;
  s->max_inflight = max_inflight;
  s->small = small_particles;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return MPS_E_HIP;
  }
  try {
    for (int i = 0; i < max_inflight; ++i) s->workers.emplace_back(worker_main, s);
  } catch (...) {
    {
      std::lock_guard<std::mutex> g(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    delete s;
    return MPS_E_NOMEM;
  }
  *out = reinterpret_cast<mps_server*>(s);
  return MPS_OK;
}

int mps_submit(mps_server* srv, const mps_catalog* cat, int n_grid, mps_precision prec, mps_result* out,
               uint64_t* ticket) {
  if (!srv || !cat || !out || !ticket) return MPS_E_ARG;
  Server* s = reinterpret_cast<Server*>(srv);
  if (n_grid < 8 || n_grid > 1024 || (n_grid & (n_grid - 1)) || (prec != MPS_F32 && prec != MPS_F64))
    return MPS_E_ARG;
  const int st = validate_catalog(nullptr, cat);
  if (st != MPS_OK) return st;
  auto r = std::make_shared<Request>();
  r->cat = *cat;
  if (cat->k_edges) {
    r->edges.assign(cat->k_edges, cat->k_edges + cat->n_bins + 1);
    r->cat.k_edges = r->edges.data();
  }
  r->n_grid = n_grid;
  r->prec = prec;
  r->out = out;
  r->bytes = mps_footprint(n_grid, prec, cat->n_particles) + host_stage_bytes(cat);
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return MPS_E_ARG;
    if (r->bytes > s->budget) return MPS_E_TOOBIG;
    if (s->queue.size() >= 4096) return MPS_E_BUSY;
    r->ticket = s->next_ticket++;
    s->queue.push_back(r);
    s->tickets[r->ticket] = r;
    *ticket = r->ticket;
  }
  s->cv_work.notify_one();
  return MPS_OK;
}

int mps_wait(mps_server* srv, uint64_t ticket, double timeout_s) {
  if (!srv) return MPS_E_ARG;
  Server* s = reinterpret_cast<Server*>(srv);
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return MPS_E_ARG;
  const auto r = it->second;
  const auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::microseconds(static_cast<int64_t>(std::max(0.0, timeout_s) * 1e6));
  while (!r->done) {
    if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !r->done) return MPS_E_TIMEOUT;
  }
  s->tickets.erase(ticket);
  return r->status;
}

int mps_server_destroy(mps_server* srv) {
  if (!srv) return MPS_E_ARG;
  Server* s = reinterpret_cast<Server*>(srv);
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& pp : s->pool) mps_plan_destroy(pp.plan);
  delete s;
  return MPS_OK;
}

}  // extern "C"
