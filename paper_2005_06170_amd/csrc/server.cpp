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
// A queued request may be passed over by later ones at most this many times;
// after that, nothing behind it is admitted until it fits.
constexpr int kMaxPassed = 8;

struct Request {
  uint64_t ticket = 0;
  mps_catalog cat{};
  std::vector<double> edges;
  int n_grid = 0;
  mps_precision prec = MPS_F32;
  mps_result* out = nullptr;
  size_t bytes = 0;           // footprint of a plan serving it
  hipEvent_t ready = nullptr; // recorded on the submitter's stream
  int passed = 0;             // later requests admitted while this one waited
  bool done = false;
  int status = MPS_OK;
};

// Scatter buffers a plan holds beyond its grids, tables and records: the
// halo form's halo buffer, the paired deposits' job scratch.
constexpr unsigned kExtraHalo = 1, kExtraPairs = 2;

struct PooledPlan {
  mps_plan* plan = nullptr;   // nullptr while a worker creates it
  int n_grid = 0;
  mps_precision prec = MPS_F32;
  int64_t cap = 0;            // particles reserved
  int64_t host_cap = 0;       // particles of host-catalog staging reserved
  unsigned extras = 0;        // kExtra* buffers it holds
  size_t bytes = 0;
  bool busy = false;
  uint64_t last_use = 0;
};

// What a worker must do, outside the server lock, before it can run a
// request on `pp`: destroy the evicted plans (their bytes are still counted
// until then), then create the plan or grow its reservation.
struct Admission {
  PooledPlan* pp = nullptr;
  enum { kReady, kGrow, kCreate } action = kReady;
  int64_t cap = 0, host_cap = 0;          // reservation to make (grow, create)
  unsigned extras = 0;                    // kExtra* buffers the plan must hold
  std::vector<std::pair<mps_plan*, size_t>> victims;
};

}  // namespace

struct Server {
  size_t budget = 0;
  size_t used = 0;             // bytes held by pooled plans (and dying ones)
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
  std::vector<hipEvent_t> free_events;
  std::vector<std::thread> workers;
};

namespace {

// Take idle plans (least recently used first, never `keep`) out of the pool
// until `need` more bytes fit the budget.  Their bytes stay in s->used until
// the caller has destroyed them outside the lock.  Returns false (and puts
// nothing back) if running requests hold too much.
bool make_room(Server* s, size_t need, const PooledPlan* keep, Admission* adm) {
  size_t freed = 0;
  std::vector<std::list<PooledPlan>::iterator> take;
  while (s->used - freed + need > s->budget) {
    auto victim = s->pool.end();
    for (auto it = s->pool.begin(); it != s->pool.end(); ++it) {
      if (it->busy || &*it == keep) continue;
      if (std::find(take.begin(), take.end(), it) != take.end()) continue;
      if (victim == s->pool.end() || it->last_use < victim->last_use) victim = it;
    }
    if (victim == s->pool.end()) return false;
    take.push_back(victim);
    freed += victim->bytes;
  }
  for (auto it : take) {
    adm->victims.emplace_back(it->plan, it->bytes);
    s->pool.erase(it);
  }
  return true;
}

// Device bytes of a pooled plan: grids and tables, cap particles' records,
// host_cap particles' staging, and the `extras` buffers it holds (the
// footprint counts those a catalog of cap particles would take instead).
size_t plan_bytes(int n_grid, mps_precision prec, int64_t cap, int64_t host_cap, unsigned extras) {
  const int64_t nt = n_grid / tile_for(n_grid, prec);
  const size_t pairs = pair_scratch_bytes(nt * nt * nt, kPairBlocks);
  size_t b = mps_footprint(n_grid, prec, cap);
  if (scatter_form_for(n_grid, prec, cap) == kFormHalo) b -= halo_bytes(n_grid, prec);
  if (pairs_reachable(n_grid, prec, cap)) b -= pairs;
  if (extras & kExtraHalo) b += halo_bytes(n_grid, prec);
  if (extras & kExtraPairs) b += pairs;
  return b + kHostStageBytes * static_cast<size_t>(host_cap);
}

// The scatter buffers the request's plan needs: the halo form's, or the
// paired deposits' (truncated BL3 kernel).
unsigned needs_extras(const mps_catalog& c, int n_grid, mps_precision prec) {
  if (kernel_id(c.flags) != 0) return 0u;
  unsigned e = 0u;
  if (scatter_form_for(n_grid, prec, c.n_particles) == kFormHalo) e |= kExtraHalo;
  if (pairs_reachable(n_grid, prec, c.n_particles)) e |= kExtraPairs;
  return e;
}

// Under the lock: choose an idle pooled plan of this shape with room for np
// particles (and, for a host-resident catalog, np particles of staging; and
// the `extras` buffers), else one to grow, else a new one, and reserve
// its bytes.  Returns false if the budget cannot host it right now (*status
// stays MPS_OK) or never can (*status = MPS_E_TOOBIG).
bool admit_plan(Server* s, int n_grid, mps_precision prec, int64_t np, bool host, unsigned extras,
                Admission* adm, int* status) {
  *status = MPS_OK;
  const int64_t hp = host ? np : 0;
  if (plan_bytes(n_grid, prec, np, hp, extras) > s->budget) {
    *status = MPS_E_TOOBIG;
    return false;
  }
  PooledPlan* fit = nullptr;
  PooledPlan* grow = nullptr;
  for (auto& pp : s->pool) {
    if (pp.busy || pp.n_grid != n_grid || pp.prec != prec) continue;
    if (pp.cap >= np && pp.host_cap >= hp && (pp.extras & extras) == extras) {
      if (!fit || pp.cap < fit->cap) fit = &pp;
    } else if (!grow || pp.cap > grow->cap) {
      grow = &pp;
    }
  }
  if (fit) {
    fit->busy = true;
    fit->last_use = ++s->clock;
    adm->pp = fit;
    adm->action = Admission::kReady;
    return true;
  }
  if (grow) {
    const int64_t cap = std::max(grow->cap, np), hcap = std::max(grow->host_cap, hp);
    const unsigned h = grow->extras | extras;
    const size_t need = plan_bytes(n_grid, prec, cap, hcap, h);
    if (!make_room(s, need - grow->bytes, grow, adm)) return false;
    adm->pp = grow;
    adm->action = Admission::kGrow;
    adm->cap = cap;
    adm->host_cap = hcap;
    adm->extras = h;
    s->used += need - grow->bytes;
    grow->bytes = need;
    grow->busy = true;
    grow->last_use = ++s->clock;
    return true;
  }
  const size_t need = plan_bytes(n_grid, prec, np, hp, extras);
  if (!make_room(s, need, nullptr, adm)) return false;
  PooledPlan pp;
  pp.n_grid = n_grid;
  pp.prec = prec;
  pp.bytes = need;
  pp.busy = true;
  pp.last_use = ++s->clock;
  s->used += need;
  s->pool.push_back(pp);
  adm->pp = &s->pool.back();
  adm->action = Admission::kCreate;
  adm->cap = np;
  adm->host_cap = hp;
  adm->extras = extras;
  return true;
}

// Outside the lock: destroy the victims, then create or grow the plan.
// Re-locks to settle the byte counts; returns the status of the reservation.
int carry_out(Server* s, Admission* adm, std::unique_lock<std::mutex>& lk) {
  lk.unlock();
  size_t freed = 0;
  for (auto& v : adm->victims) {
    mps_plan_destroy(v.first);
    freed += v.second;
  }
  int st = MPS_OK;
  PooledPlan* pp = adm->pp;
  mps_plan* created = nullptr;
  if (adm->action == Admission::kCreate) {
    st = mps_plan_create(&created, pp->n_grid, pp->prec);
    // the records, and the scatter buffers the admitted request needs
    // (mps_plan_reserve would allocate them for any plan that could use
    // them), here rather than in the worker's first estimate
    if (st == MPS_OK && adm->cap > 0) st = ensure_particles(reinterpret_cast<Plan*>(created), adm->cap);
    if (st == MPS_OK && adm->host_cap > 0) st = ensure_host_stage(reinterpret_cast<Plan*>(created), adm->host_cap);
    if (st == MPS_OK && (adm->extras & kExtraHalo)) st = ensure_halo(reinterpret_cast<Plan*>(created));
    if (st == MPS_OK && (adm->extras & kExtraPairs)) st = ensure_pair_scratch(reinterpret_cast<Plan*>(created));
    if (st != MPS_OK && created) {
      mps_plan_destroy(created);
      created = nullptr;
    }
  } else if (adm->action == Admission::kGrow) {
    if (adm->cap > 0) st = ensure_particles(reinterpret_cast<Plan*>(pp->plan), adm->cap);
    if (st == MPS_OK && adm->host_cap > 0) st = ensure_host_stage(reinterpret_cast<Plan*>(pp->plan), adm->host_cap);
    if (st == MPS_OK && (adm->extras & kExtraHalo)) st = ensure_halo(reinterpret_cast<Plan*>(pp->plan));
    if (st == MPS_OK && (adm->extras & kExtraPairs)) st = ensure_pair_scratch(reinterpret_cast<Plan*>(pp->plan));
  }
  lk.lock();
  s->used -= freed;
  if (adm->action == Admission::kCreate) {
    if (st == MPS_OK) {
      pp->plan = created;
      pp->cap = adm->cap;
      pp->host_cap = adm->host_cap;
      pp->extras = adm->extras;
    } else {
      s->used -= pp->bytes;
      for (auto it = s->pool.begin(); it != s->pool.end(); ++it)
        if (&*it == pp) {
          s->pool.erase(it);
          break;
        }
      adm->pp = nullptr;
    }
  } else if (adm->action == Admission::kGrow) {
    if (st == MPS_OK) {
      pp->cap = adm->cap;
      pp->host_cap = adm->host_cap;
      pp->extras = adm->extras;
    } else {  // a failed reservation may have dropped part of the old one
      mps_plan* dead = pp->plan;
      s->used -= pp->bytes;
      for (auto it = s->pool.begin(); it != s->pool.end(); ++it)
        if (&*it == pp) {
          s->pool.erase(it);
          break;
        }
      adm->pp = nullptr;
      lk.unlock();
      mps_plan_destroy(dead);
      lk.lock();
    }
  }
  if (freed > 0 || st != MPS_OK) s->cv_work.notify_all();
  return st;
}

// A worker's particle workspace (sorted records and host-catalog staging),
// lent to the plan of each large request it runs, so that plans of large
// requests hold only their grids and tables and a plan pool does not keep
// one catalog-sized buffer per plan.  Grows (never shrinks); its bytes count
// against the budget from the moment they are reserved.
struct ParticleSpace {
  float4* sorted = nullptr;
  int64_t cap = 0;
  float* host = nullptr;
  int64_t host_cap = 0;
  size_t bytes = 0;             // allocated
  size_t reserved = 0;          // counted in the budget (>= bytes)
  int64_t want_cap = 0, want_host = 0;
  static size_t size_of(int64_t cap, int64_t host_cap) {
    return static_cast<size_t>(cap) * 2 * sizeof(float4) + kHostStageBytes * static_cast<size_t>(host_cap);
  }
};

// Round a particle count up so that a workspace is not regrown for every
// slightly larger catalog: to a multiple of 2^20, and at least 1.5x the old
// capacity when it must grow.
int64_t grown(int64_t need, int64_t old) {
  if (need <= old) return old;
  int64_t c = need > old + old / 2 ? need : old + old / 2;
  c = (c + (1 << 20) - 1) & ~static_cast<int64_t>((1 << 20) - 1);
  return c < 0x7fffffffll ? c : 0x7fffffffll;
}

void finish(Server* s, const std::shared_ptr<Request>& r, int status) {
  r->status = status;
  r->done = true;
  if (r->ready) {
    s->free_events.push_back(r->ready);
    r->ready = nullptr;
  }
}

void worker_main(Server* s) {
  (void)hipSetDevice(s->device);
  hipStream_t stream = nullptr;
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
  hipEvent_t fork = nullptr;
  if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) fork = nullptr;
  BatchWorkspace ws;  // this worker's multi-catalog scatter buffers
  ParticleSpace wp;   // this worker's particle workspace for large requests
  std::vector<std::pair<mps_plan*, size_t>> dead;  // evicted plans not yet freed
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    std::vector<std::shared_ptr<Request>> batch;
    std::vector<Admission> adms;
    // admit: the oldest request that fits, unless an older one has been
    // passed over kMaxPassed times; small requests pull same-shape peers
    while (batch.empty()) {
      if (s->stop && s->queue.empty()) {
        lk.unlock();
        if (stream) (void)hipStreamDestroy(stream);
        if (fork) (void)hipEventDestroy(fork);
        if (ws.d_cats) (void)hipFree(ws.d_cats);
        if (ws.d_starts) (void)hipFree(ws.d_starts);
        if (ws.d_queue) (void)hipFree(ws.d_queue);
        if (ws.h_cats) (void)hipHostFree(ws.h_cats);
        if (ws.h_starts) (void)hipHostFree(ws.h_starts);
        for (hipEvent_t e : ws.done)
          if (e) (void)hipEventDestroy(e);
        if (wp.sorted) (void)hipFree(wp.sorted);
        if (wp.host) (void)hipFree(wp.host);
        lk.lock();
        s->used -= wp.reserved;
        return;
      }
      for (auto it = s->queue.begin(); it != s->queue.end();) {
        const auto r = *it;
        int st = MPS_OK;
        Admission adm;
        const bool large = r->cat.n_particles > s->small;
        const bool host = (r->cat.flags & MPS_CATALOG_HOST) != 0;
        const unsigned extras = needs_extras(r->cat, r->n_grid, r->prec);
        if (large) {
          // the plan holds its grids only; the records live in this worker's
          // workspace, reserved (and grown if needed) first
          const int64_t np = r->cat.n_particles;
          if (plan_bytes(r->n_grid, r->prec, 0, 0, extras) + ParticleSpace::size_of(np, host ? np : 0) > s->budget) {
            it = s->queue.erase(it);
            finish(s, r, MPS_E_TOOBIG);
            s->cv_done.notify_all();
            continue;
          }
          const int64_t cap = grown(np, wp.want_cap > wp.cap ? wp.want_cap : wp.cap);
          const int64_t hcap = host ? grown(np, wp.want_host > wp.host_cap ? wp.want_host : wp.host_cap)
                                    : (wp.want_host > wp.host_cap ? wp.want_host : wp.host_cap);
          size_t need = ParticleSpace::size_of(cap, hcap);
          if (need + plan_bytes(r->n_grid, r->prec, 0, 0, extras) > s->budget)
            need = ParticleSpace::size_of(np, host ? np : 0);  // no headroom: exactly what it needs
          if (need > wp.reserved) {
            Admission wadm;
            if (!make_room(s, need - wp.reserved, nullptr, &wadm)) {
              if (r->passed >= kMaxPassed) break;
              ++it;
              continue;
            }
            s->used += need - wp.reserved;
            wp.reserved = need;
            wp.want_cap = need == ParticleSpace::size_of(cap, hcap) ? cap : np;
            wp.want_host = need == ParticleSpace::size_of(cap, hcap) ? hcap : (host ? np : 0);
            for (auto& v : wadm.victims) adm.victims.push_back(v);  // destroyed with the plan's victims
          }
        }
        Admission padm;
        if (!admit_plan(s, r->n_grid, r->prec, large ? 0 : r->cat.n_particles, !large && host, extras, &padm, &st)) {
          // plans a workspace reservation evicted are freed before this
          // worker waits (their bytes stay counted until then)
          for (auto& v : adm.victims) dead.push_back(v);
          adm.victims.clear();
          if (st != MPS_OK) {  // can never run
            it = s->queue.erase(it);
            finish(s, r, st);
            s->cv_done.notify_all();
            continue;
          }
          if (r->passed >= kMaxPassed) break;  // its turn: wait until it fits
          ++it;
          continue;
        }
        for (auto& v : adm.victims) padm.victims.push_back(v);
        adm = std::move(padm);
        // every older request still queued has been passed over once more
        for (auto jt = s->queue.begin(); jt != it; ++jt) ++(*jt)->passed;
        batch.push_back(r);
        adms.push_back(std::move(adm));
        it = s->queue.erase(it);
        if (r->cat.n_particles <= s->small) {
          for (auto jt = it; jt != s->queue.end() && batch.size() < kMaxBatch;) {
            const auto q = *jt;
            if (q->n_grid != r->n_grid || q->prec != r->prec || q->cat.n_particles > s->small) {
              ++jt;
              continue;
            }
            int st2 = MPS_OK;
            Admission a2;
            if (!admit_plan(s, q->n_grid, q->prec, q->cat.n_particles, (q->cat.flags & MPS_CATALOG_HOST) != 0,
                            needs_extras(q->cat, q->n_grid, q->prec), &a2, &st2))
              break;
            batch.push_back(q);
            adms.push_back(std::move(a2));
            jt = s->queue.erase(jt);
          }
        }
        break;
      }
      if (batch.empty()) {
        if (!dead.empty()) {
          std::vector<std::pair<mps_plan*, size_t>> d;
          d.swap(dead);
          lk.unlock();
          size_t freed = 0;
          for (auto& v : d) {
            mps_plan_destroy(v.first);
            freed += v.second;
          }
          lk.lock();
          s->used -= freed;
          s->cv_work.notify_all();
          continue;
        }
        s->cv_work.wait(lk);
      }
    }
    if (!dead.empty()) {  // freed outside the lock with the first admission's victims
      for (auto& v : dead) adms[0].victims.push_back(v);
      dead.clear();
    }
    // plan creation, growth and eviction run outside the lock
    std::vector<int> status(batch.size(), MPS_OK);
    for (size_t i = 0; i < batch.size(); ++i)
      if (!adms[i].victims.empty() || adms[i].action != Admission::kReady) status[i] = carry_out(s, &adms[i], lk);
    lk.unlock();

    // a large request borrows the worker's particle workspace (allocated or
    // grown here, outside the lock)
    struct Lent {
      Plan* p;
      float4* sorted;
      int64_t cap;
      float* host;
      int64_t host_cap;
    };
    std::vector<Lent> lent;
    for (size_t i = 0; i < batch.size(); ++i) {
      if (status[i] != MPS_OK || batch[i]->cat.n_particles <= s->small) continue;
      if (wp.cap < wp.want_cap || wp.host_cap < wp.want_host) {
        if (wp.sorted) (void)hipFree(wp.sorted);
        if (wp.host) (void)hipFree(wp.host);
        wp.sorted = nullptr;
        wp.host = nullptr;
        wp.cap = wp.host_cap = 0;
        wp.bytes = 0;
        bool ok = hipMalloc(reinterpret_cast<void**>(&wp.sorted),
                            static_cast<size_t>(wp.want_cap) * 2 * sizeof(float4)) == hipSuccess;
        if (ok && wp.want_host > 0)
          ok = hipMalloc(reinterpret_cast<void**>(&wp.host), kHostStageBytes * static_cast<size_t>(wp.want_host)) ==
               hipSuccess;
        if (ok) {
          wp.cap = wp.want_cap;
          wp.host_cap = wp.want_host;
          wp.bytes = ParticleSpace::size_of(wp.cap, wp.host_cap);
        } else {
          if (wp.sorted) (void)hipFree(wp.sorted);
          wp.sorted = nullptr;
          wp.host = nullptr;
          status[i] = MPS_E_NOMEM;
          continue;
        }
      }
      Plan* p = reinterpret_cast<Plan*>(adms[i].pp->plan);
      lent.push_back({p, p->sorted, p->sorted_cap, p->host_stage, p->host_cap});
      p->sorted = wp.sorted;
      p->sorted_cap = wp.cap;
      p->host_stage = wp.host;
      p->host_cap = wp.host_cap;
    }

    // run the batch: each request's stages start after its catalog is ready
    // on the submitter's stream; the requests go through the multi-catalog
    // path together (one scatter launch over all their tiles), one
    // synchronisation
    std::vector<Plan*> run_plans;
    std::vector<mps_catalog> run_cats;
    std::vector<size_t> run_idx;
    for (size_t i = 0; i < batch.size(); ++i) {
      if (status[i] != MPS_OK) continue;
      Plan* p = reinterpret_cast<Plan*>(adms[i].pp->plan);
      int st = MPS_OK;
      if (batch[i]->ready && hipStreamWaitEvent(stream, batch[i]->ready, 0) != hipSuccess) st = MPS_E_HIP;
      if (st == MPS_OK) st = ensure_bins(p, &batch[i]->cat);
      if (st == MPS_OK) st = ensure_scatter_space(p, &batch[i]->cat);
      status[i] = st;
      if (st == MPS_OK) {
        run_plans.push_back(p);
        run_cats.push_back(batch[i]->cat);
        run_idx.push_back(i);
      }
    }
    if (!run_plans.empty()) {
      const int st = fork ? enqueue_batch(run_plans.data(), run_cats.data(), static_cast<int>(run_plans.size()),
                                          &stream, 1, &fork, &ws, nullptr)
                          : MPS_E_HIP;
      if (st != MPS_OK)
        for (size_t i : run_idx) status[i] = st;
    }
    const bool synced = hipStreamSynchronize(stream) == hipSuccess;
    for (size_t i = 0; i < batch.size(); ++i) {
      if (status[i] == MPS_OK)
        status[i] = synced ? unpack(reinterpret_cast<Plan*>(adms[i].pp->plan), &batch[i]->cat, batch[i]->out)
                           : MPS_E_HIP;
    }
    for (const Lent& l : lent) {  // the plans get their own buffers back
      l.p->sorted = l.sorted;
      l.p->sorted_cap = l.cap;
      l.p->host_stage = l.host;
      l.p->host_cap = l.host_cap;
    }

    lk.lock();
    for (size_t i = 0; i < batch.size(); ++i) {
      if (adms[i].pp) adms[i].pp->busy = false;
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
               hipStream_t stream, uint64_t* ticket) {
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
    // the request's kernels wait for what is already enqueued on `stream`
    // (the producer of the catalog)
    if (!s->free_events.empty()) {
      r->ready = s->free_events.back();
      s->free_events.pop_back();
    } else if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess) {
      r->ready = nullptr;
      return MPS_E_HIP;
    }
    if (hipEventRecord(r->ready, stream) != hipSuccess) {
      s->free_events.push_back(r->ready);
      r->ready = nullptr;
      return MPS_E_HIP;
    }
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
  for (auto& pp : s->pool)
    if (pp.plan) mps_plan_destroy(pp.plan);
  for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
  delete s;
  return MPS_OK;
}

}  // extern "C"
