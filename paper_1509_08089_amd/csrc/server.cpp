// Estimation server: continuous batching over resident graphs.
//
// A worker thread repeats one scheduling iteration:
//   1. admission: while a slot is free, take the waiting requests oldest first; make
//      sure each one's graph has the tables for its k, evicting the tables of idle
//      graphs (the largest first) to stay within the memory budget; a request
//      whose tables can never fit fails with MOSS_E_ADMISSION, one that must wait for
//      running requests to finish stays queued (and so do the ones behind it).  The
//      tables of an idle graph are built by a second thread while the launches go on
//      (the request joins once they are in, its reserved bytes counted meanwhile); a
//      graph with running requests gets its missing sets between two launches;
//   2. one batched launch runs the next samples of the admitted requests (requests
//      that arrived during the previous launch are in it): about iteration_samples in
//      all, the requests with the fewest samples left first, every request at least a
//      sixteenth of that and at most chunk_samples, so a short request is done after
//      the next launch while long ones take what is left;
//   3. finished requests get their finals and wake their waiters.
// Requests of at most express_samples samples skip the iterations: once their graph's
// tables are in, an express thread with a runner of its own launches all of them that
// wait, whole, beside the iteration under way (the persistent kernels leave block
// slots free), so a small request does not wait for a long launch to end.
// Each request's samples keep their global indices, so its result does not depend on
// how its work was chunked or what ran beside it.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"

using Clock = std::chrono::steady_clock;

namespace {

struct Req {
  uint64_t ticket = 0;
  int32_t graph_id = 0;
  int32_t k = 4;
  uint64_t n = 0, seed = 0;
  uint32_t flags = 0;
  uint64_t K[2] = {0, 0};
  uint64_t next[2] = {0, 0};
  uint64_t hits[2][22] = {};
  bool done = false, cancelled = false;
  moss_status status = MOSS_OK;
  moss_result result{};
  Clock::time_point t_submit, t_done;
};

struct GraphEntry {
  moss_graph* g = nullptr;
  uint64_t last_use = 0;
  int active = 0;
  bool building = false;          // the builder thread owns g until it is done
  uint64_t bytes_before = 0;      // g's table bytes when its build started
  uint64_t build_need = 0;        // bytes the build adds (reserved meanwhile)
};

struct BuildJob {
  int32_t graph_id;
  uint32_t mask;
};

}  // namespace

struct moss_server {
  moss_server_config cfg{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_build, cv_express;
  std::thread worker, builder, express;
  bool stop = false;
  std::deque<BuildJob> jobs;
  uint64_t arrivals = 0, builds_done = 0, cancels = 0;  // what wakes an idle worker
  std::deque<std::shared_ptr<Req>> pending;
  std::vector<std::shared_ptr<Req>> active;
  std::unordered_map<uint64_t, std::shared_ptr<Req>> by_ticket;
  std::vector<GraphEntry> graphs;
  uint64_t next_ticket = 1;
  uint64_t iterations = 0, completed = 0, samples_done = 0, evictions = 0, express_launches = 0;
  uint64_t express_running = 0;  // requests in the express launch under way
  std::vector<double> latencies_ms;
  bool have_first = false;
  Clock::time_point t_first, t_last;
  std::unique_ptr<moss::BatchRunner> runner, express_runner;

  void finish(const std::shared_ptr<Req>& r, moss_status st) {
    r->status = st;
    r->done = true;
    r->t_done = Clock::now();
    if (st == MOSS_OK) {
      ++completed;
      samples_done += r->n;
      latencies_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
      t_last = r->t_done;
    }
  }

  // Table bytes held, a graph under construction at what it will hold.
  uint64_t resident_bytes() const {
    uint64_t b = 0;
    for (const GraphEntry& e : graphs) b += e.building ? e.bytes_before + e.build_need : e.g->table_bytes;
    return b;
  }

  // A request the express thread takes (when its graph's tables are in).
  bool express_size(const Req& r) const { return !cfg.express_off && r.n <= cfg.express_samples; }

  // The table sets of r's request, and whether they are resident and usable now.
  static uint32_t tables_of(const Req& r) {
    moss::EstimatePlan plan;
    (void)moss::plan_estimate(r.k, r.n, r.flags, &plan);  // checked at submission
    return plan.tables;
  }
  bool tables_ready(const Req& r) const {
    const GraphEntry& ge = graphs[(size_t)r.graph_id];
    const uint32_t mask = tables_of(r);
    return !ge.building && (ge.g->built & mask) == mask;
  }

  enum class Room { kOk, kWait, kNever };

  // Makes room within the memory budget for building `mask` on ge's graph, with mu
  // held: evicts the tables of idle graphs other than ge's (the largest first, least
  // recently used among equal sizes: one large eviction frees what several small ones
  // would, and the small graphs it spares are cheap to keep), then, if ge's graph is
  // idle, its own table sets that `mask` does not name.  kOk: the tables now fit.
  // kWait: what still stands in the way is held by running requests, by a build under
  // way, or by a call of another caller on an idle graph (its claim failed), and will
  // be released.  kNever: nothing left to evict.
  Room make_room(GraphEntry& ge, uint32_t mask) {
    const uint64_t budget = cfg.mem_budget_bytes;
    if (!budget) return Room::kOk;
    std::vector<char> held(graphs.size(), 0);  // idle graphs whose claim failed
    bool waiting = false;
    for (;;) {
      if (resident_bytes() + moss::table_bytes_needed(ge.g, mask) <= budget) return Room::kOk;
      GraphEntry* victim = nullptr;
      for (size_t i = 0; i < graphs.size(); ++i) {
        GraphEntry& e = graphs[i];
        if (&e != &ge && !held[i] && !e.building && e.active == 0 && e.g->built &&
            (!victim || e.g->table_bytes > victim->g->table_bytes ||
             (e.g->table_bytes == victim->g->table_bytes && e.last_use < victim->last_use)))
          victim = &e;
      }
      uint32_t drop = MOSS_TABLES_K4 | MOSS_TABLES_K5 | MOSS_TABLES_K4MIN;
      if (!victim && ge.active == 0 && (ge.g->built & ~mask)) {
        victim = &ge;
        drop = ge.g->built & ~mask;  // the sets this request needs stay
      }
      if (!victim) break;
      moss::GraphClaim claim(victim->g);
      if (!claim.ok()) {
        held[(size_t)(victim - graphs.data())] = 1;
        waiting = true;
        if (victim == &ge) break;
        continue;
      }
      moss::free_graph_tables(victim->g, drop);
      ++evictions;
    }
    for (const GraphEntry& e : graphs)  // running requests, and builds, end
      if (e.building || (e.active > 0 && e.g->table_bytes)) waiting = true;
    return waiting ? Room::kWait : Room::kNever;
  }

  void loop();
  void build_loop();
  void express_loop();
};

void moss_server::loop() {
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] { return stop || !pending.empty() || !active.empty(); });
    if (stop) {
      for (auto& r : pending) finish(r, MOSS_E_CANCELLED);
      for (auto& r : active) finish(r, MOSS_E_CANCELLED);
      pending.clear();
      active.clear();
      cv_done.notify_all();
      return;
    }
    // 1. admission
    bool blocked = false;  // a waiting request waits for memory to be released
    for (auto it = pending.begin(); it != pending.end() && active.size() < cfg.max_slots;) {
      std::shared_ptr<Req> r = *it;
      if (r->cancelled) {
        finish(r, MOSS_E_CANCELLED);
        it = pending.erase(it);
        continue;
      }
      GraphEntry& ge = graphs[(size_t)r->graph_id];
      if (ge.building) {  // joins once its graph's tables are in
        ++it;
        continue;
      }
      const uint32_t mask = tables_of(*r);
      const bool small = express_size(*r);
      if (small && (ge.g->built & mask) == mask) {  // the express thread takes it
        ++it;
        continue;
      }
      if ((ge.g->built & mask) != mask) {
        const uint64_t need = moss::table_bytes_needed(ge.g, mask);
        if (cfg.mem_budget_bytes && need > cfg.mem_budget_bytes) {
          finish(r, MOSS_E_ADMISSION);
          it = pending.erase(it);
          continue;
        }
        const Room room = make_room(ge, mask);
        if (room == Room::kNever) {
          finish(r, MOSS_E_ADMISSION);
          it = pending.erase(it);
          continue;
        }
        if (room == Room::kWait) {  // running requests, builds (or another caller) will release memory
          blocked = true;
          break;
        }
        if (ge.active == 0) {  // an idle graph: its tables are built beside the launches
          ge.building = true;
          ge.bytes_before = ge.g->table_bytes;
          ge.build_need = need;
          jobs.push_back({r->graph_id, mask});
          cv_build.notify_one();
          ++it;
          continue;
        }
        moss_status st;  // a graph with running requests: its missing sets go in now
        {
          moss::GraphClaim claim(ge.g);
          st = claim.ok() ? moss::build_tables(ge.g, mask) : MOSS_E_BUSY;
        }
        if (st != MOSS_OK) {
          finish(r, st);
          it = pending.erase(it);
          continue;
        }
        if (small) {  // its tables are in: the express thread takes it
          cv_express.notify_one();
          ++it;
          continue;
        }
      }
      it = pending.erase(it);
      moss_result hdr;
      moss::result_header(ge.g, r->k, r->n, r->flags, &hdr);
      r->K[0] = hdr.K[0];
      r->K[1] = hdr.K[1];
      ge.active += 1;
      active.push_back(r);
    }
    cv_done.notify_all();
    if (active.empty()) {
      if (blocked) {
        // only a call of another caller on an idle graph (or a build) holds the memory;
        // the former's end is not signalled here, so look again shortly (the wait
        // releases mu)
        cv_work.wait_for(lk, std::chrono::milliseconds(1), [&] { return stop; });
      } else {
        // nothing admissible: wait for a new arrival, a finished build, a cancel, an
        // express launch (its graphs went idle; a waiting request may need their
        // tables rebuilt or their memory) or a stop
        const uint64_t a0 = arrivals, b0 = builds_done, c0 = cancels, x0 = express_launches;
        cv_work.wait(lk, [&] {
          return stop || arrivals != a0 || builds_done != b0 || cancels != c0 || express_launches != x0;
        });
      }
      continue;
    }
    // 2. the next samples of the admitted requests, fewest left first
    std::vector<moss::WorkItem> work;
    std::vector<std::shared_ptr<Req>> batch = active;
    std::vector<uint64_t> upto(batch.size() * 2);
    std::vector<uint64_t> left_of(batch.size());
    std::vector<size_t> order(batch.size());
    for (size_t i = 0; i < batch.size(); ++i) {
      const Req& r = *batch[i];
      left_of[i] = (r.K[0] - r.next[0]) + (r.K[1] - r.next[1]);
      order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return left_of[x] < left_of[y]; });
    uint64_t budget = cfg.iteration_samples;
    const uint64_t floor_share = std::max<uint64_t>(1, cfg.iteration_samples / 16);
    for (size_t i : order) {
      Req& r = *batch[i];
      moss_graph* g = graphs[(size_t)r.graph_id].g;
      moss::EstimatePlan plan;
      (void)moss::plan_estimate(r.k, r.n, r.flags, &plan);
      const uint64_t left = left_of[i];
      const uint64_t give = std::min({left, cfg.chunk_samples, std::max(budget, floor_share)});
      budget -= std::min(budget, give);
      // the two samplers advance in proportion to what each has left
      const uint64_t left0 = r.K[0] - r.next[0];
      uint64_t g0 = left ? (uint64_t)(((unsigned __int128)give * left0 + left - 1) / left) : 0;
      g0 = std::min(g0, left0);
      const uint64_t g1 = std::min(r.K[1] - r.next[1], give - std::min(give, g0));
      const uint64_t add[2] = {g0, g1};
      for (int s = 0; s < 2; ++s) {
        const uint64_t b = s < plan.count ? r.next[s] + add[s] : r.next[s];
        upto[2 * i + s] = b;
        if (b > r.next[s]) work.push_back({g, plan.sampler[s], r.seed, r.next[s], b, (uint32_t)(2 * i + s)});
      }
    }
    lk.unlock();
    std::vector<uint64_t> bins(batch.size() * 2 * 22, 0);
    // large chunks on large graphs go sorted by group, as in moss_estimate_batch
    moss_status st = work.empty() ? MOSS_OK
                                  : runner->run(work, (uint32_t)(batch.size() * 2), bins.data(), nullptr, nullptr, 0,
                                                0, true);
    lk.lock();
    ++iterations;
    // 3. account and complete
    std::vector<std::shared_ptr<Req>> still;
    for (size_t i = 0; i < batch.size(); ++i) {
      std::shared_ptr<Req>& r = batch[i];
      GraphEntry& ge = graphs[(size_t)r->graph_id];
      ge.last_use = iterations;
      bool finished = false;
      if (st != MOSS_OK) {
        finish(r, st);
        finished = true;
      } else {
        for (int s = 0; s < 2; ++s) {
          for (int c = 0; c < 22; ++c) r->hits[s][c] += bins[(2 * i + s) * 22 + c];
          r->next[s] = upto[2 * i + s];
        }
        if (r->cancelled) {
          finish(r, MOSS_E_CANCELLED);
          finished = true;
        } else if (r->next[0] >= r->K[0] && r->next[1] >= r->K[1]) {
          moss_result res;
          moss::result_header(ge.g, r->k, r->n, r->flags, &res);
          std::memcpy(res.hits, r->hits, sizeof(res.hits));
          moss_status fs = moss_finals(&res);
          r->result = res;
          finish(r, fs);
          finished = true;
        }
      }
      if (finished) ge.active -= 1;
      else still.push_back(r);
    }
    active.swap(still);
    cv_done.notify_all();
  }
}

// The builder thread: builds the tables of an idle graph (claimed meanwhile) while the
// worker's launches go on, then lets the worker admit the requests that waited for them;
// a failed build fails them with its status.
void moss_server::build_loop() {
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_build.wait(lk, [&] { return stop || !jobs.empty(); });
    if (stop) return;  // builds not started are dropped: the worker cancelled their requests
    const BuildJob job = jobs.front();
    jobs.pop_front();
    moss_graph* g = graphs[(size_t)job.graph_id].g;
    lk.unlock();
    moss_status st;
    {
      moss::GraphClaim claim(g);
      st = claim.ok() ? moss::build_tables(g, job.mask) : MOSS_E_BUSY;
    }
    lk.lock();
    graphs[(size_t)job.graph_id].building = false;
    ++builds_done;
    if (st != MOSS_OK) {
      for (auto it = pending.begin(); it != pending.end();) {
        moss::EstimatePlan plan;
        (void)moss::plan_estimate((*it)->k, (*it)->n, (*it)->flags, &plan);
        if ((*it)->graph_id == job.graph_id && (plan.tables & job.mask)) {
          finish(*it, st);
          it = pending.erase(it);
        } else {
          ++it;
        }
      }
      cv_done.notify_all();
    }
    cv_work.notify_all();
    cv_express.notify_one();
  }
}

// The express thread: launches every waiting request of at most express_samples
// samples whose tables are in, each whole, with a runner of its own; the graphs it
// uses count as active meanwhile, so their tables are not evicted under it.
void moss_server::express_loop() {
  std::unique_lock<std::mutex> lk(mu);
  auto ready = [&](const Req& r) { return !r.cancelled && express_size(r) && tables_ready(r); };
  for (;;) {
    cv_express.wait(lk, [&] {
      if (stop) return true;
      for (const auto& r : pending)
        if (ready(*r)) return true;
      return false;
    });
    if (stop) return;  // the worker cancels what is still pending
    std::vector<std::shared_ptr<Req>> batch;
    for (auto it = pending.begin(); it != pending.end() && batch.size() < cfg.max_slots;) {
      const std::shared_ptr<Req> r = *it;
      if (!ready(*r)) {
        ++it;
        continue;
      }
      it = pending.erase(it);
      GraphEntry& ge = graphs[(size_t)r->graph_id];
      moss_result hdr;
      moss::result_header(ge.g, r->k, r->n, r->flags, &hdr);
      r->K[0] = hdr.K[0];
      r->K[1] = hdr.K[1];
      ge.active += 1;
      batch.push_back(r);
    }
    std::vector<moss::WorkItem> work;
    for (size_t i = 0; i < batch.size(); ++i) {
      const Req& r = *batch[i];
      moss::EstimatePlan plan;
      (void)moss::plan_estimate(r.k, r.n, r.flags, &plan);
      for (int s = 0; s < plan.count; ++s)
        if (r.K[s]) work.push_back({graphs[(size_t)r.graph_id].g, plan.sampler[s], r.seed, 0, r.K[s], (uint32_t)(2 * i + s)});
    }
    express_running = batch.size();
    lk.unlock();
    std::vector<uint64_t> bins(batch.size() * 2 * 22, 0);
    // all in the persistent kernel: at these sizes the grouping passes do not pay
    const moss_status st = work.empty() ? MOSS_OK
                                        : express_runner->run(work, (uint32_t)(batch.size() * 2), bins.data(),
                                                              nullptr, nullptr, 0, 0, false);
    lk.lock();
    ++express_launches;
    express_running = 0;
    for (size_t i = 0; i < batch.size(); ++i) {
      const std::shared_ptr<Req>& r = batch[i];
      GraphEntry& ge = graphs[(size_t)r->graph_id];
      ge.last_use = iterations;
      ge.active -= 1;
      if (st != MOSS_OK) {
        finish(r, st);
      } else if (r->cancelled) {
        finish(r, MOSS_E_CANCELLED);
      } else {
        moss_result res;
        moss::result_header(ge.g, r->k, r->n, r->flags, &res);
        for (int s = 0; s < 2; ++s)
          for (int c = 0; c < 22; ++c) res.hits[s][c] = bins[(2 * i + s) * 22 + c];
        r->result = res;
        finish(r, moss_finals(&r->result));
      }
    }
    cv_done.notify_all();
    cv_work.notify_all();  // graphs went idle: their memory may be what a request waits for
  }
}

using namespace moss;

extern "C" {

moss_status moss_server_create(const moss_server_config* cfg, void* hip_stream, moss_server** out) {
  (void)hip_stream;
  if (!out) return MOSS_E_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MOSS_E_DEVICE;
  moss_status st = ensure_device(dev);
  if (st != MOSS_OK) return st;
  moss_server* s = new (std::nothrow) moss_server();
  if (!s) return MOSS_E_NOMEM;
  if (cfg) s->cfg = *cfg;
  if (!s->cfg.max_slots) s->cfg.max_slots = 256;
  if (!s->cfg.chunk_samples) s->cfg.chunk_samples = 1ull << 25;
  if (!s->cfg.iteration_samples) s->cfg.iteration_samples = 1ull << 25;
  if (!s->cfg.express_samples) s->cfg.express_samples = 1ull << 22;
  s->device = dev;
  s->runner = std::make_unique<BatchRunner>(dev);
  s->express_runner = std::make_unique<BatchRunner>(dev);
  s->worker = std::thread([s] {
    DeviceScope scope(s->device);
    s->loop();
  });
  s->builder = std::thread([s] {
    DeviceScope scope(s->device);
    s->build_loop();
  });
  s->express = std::thread([s] {
    DeviceScope scope(s->device);
    s->express_loop();
  });
  *out = s;
  return MOSS_OK;
}

moss_status moss_server_add_graph(moss_server* s, moss_graph* g, int32_t* graph_id) {
  if (!s || !g || !graph_id) return MOSS_E_ARG;
  if (g->device != s->device) return MOSS_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  GraphEntry e;
  e.g = g;
  s->graphs.push_back(e);
  *graph_id = (int32_t)s->graphs.size() - 1;
  return MOSS_OK;
}

moss_status moss_server_submit(moss_server* s, int32_t graph_id, int32_t k, uint64_t n_samples, uint64_t seed,
                               uint32_t flags, uint64_t* ticket) {
  moss::EstimatePlan plan;
  if (!s || !ticket || moss::plan_estimate(k, n_samples, flags, &plan) != MOSS_OK) return MOSS_E_ARG;
  auto r = std::make_shared<Req>();
  r->graph_id = graph_id;
  r->k = k;
  r->n = n_samples;
  r->seed = seed;
  r->flags = flags;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return MOSS_E_CANCELLED;
    if (graph_id < 0 || (size_t)graph_id >= s->graphs.size()) return MOSS_E_ARG;
    r->ticket = s->next_ticket++;
    if (!s->have_first) {
      s->have_first = true;
      s->t_first = r->t_submit;
    }
    s->pending.push_back(r);
    s->by_ticket[r->ticket] = r;
    *ticket = r->ticket;
    ++s->arrivals;
  }
  s->cv_work.notify_one();
  s->cv_express.notify_one();
  return MOSS_OK;
}

moss_status moss_server_wait(moss_server* s, uint64_t ticket, int64_t timeout_ms, moss_result* out) {
  if (!s || !out) return MOSS_E_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return MOSS_E_ARG;
  std::shared_ptr<Req> r = it->second;
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, [&] { return r->done; });
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return r->done; })) {
    return MOSS_E_TIMEOUT;
  }
  s->by_ticket.erase(ticket);
  if (r->status == MOSS_OK) *out = r->result;
  return r->status;
}

moss_status moss_server_cancel(moss_server* s, uint64_t ticket) {
  if (!s) return MOSS_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return MOSS_E_ARG;
  it->second->cancelled = true;
  ++s->cancels;
  s->cv_work.notify_one();
  return MOSS_OK;
}

moss_status moss_server_stats_get(moss_server* s, moss_server_stats* out) {
  if (!s || !out) return MOSS_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  moss_server_stats r{};
  r.completed = s->completed;
  r.samples = s->samples_done;
  r.iterations = s->iterations;
  r.queued = s->pending.size();
  r.active = s->active.size() + s->express_running;
  r.evictions = s->evictions;
  r.express_launches = s->express_launches;
  r.table_bytes = s->resident_bytes();
  if (!s->latencies_ms.empty()) {
    std::vector<double> v = s->latencies_ms;
    std::sort(v.begin(), v.end());
    auto q = [&](double f) {
      size_t i = (size_t)std::min<double>((double)v.size() - 1, std::max(0.0, f * (double)v.size() - 1e-9));
      return v[i];
    };
    r.p50_ms = q(0.50);
    r.p99_ms = q(0.99);
    const double secs = std::chrono::duration<double>(s->t_last - s->t_first).count();
    r.samples_per_s = secs > 0 ? (double)s->samples_done / secs : 0.0;
  }
  *out = r;
  return MOSS_OK;
}

moss_status moss_server_destroy(moss_server* s) {
  if (!s) return MOSS_E_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_build.notify_all();
  s->cv_express.notify_all();
  if (s->worker.joinable()) s->worker.join();
  if (s->express.joinable()) s->express.join();  // a launch under way finishes first
  if (s->builder.joinable()) s->builder.join();  // and so does a build
  s->runner->release();
  s->express_runner->release();
  delete s;
  return MOSS_OK;
}

}  // extern "C"
