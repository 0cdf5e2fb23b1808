// Batched estimation: many (graph, k, budget, seed) requests drained by one
// persistent kernel launch, replayed from a captured hipGraph.
#include "batch.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

namespace moss {

namespace {
std::mutex g_tune_mu;
Tuning g_tuning;

std::mutex g_runner_mu;
std::map<int, std::unique_ptr<BatchRunner>> g_runners;

constexpr uint32_t kDefaultTile = 4096;

// Batched items drawn by grouped launches of their own: at least 2^20 samples on a graph
// whose sampled bytes are past 32 MB (the tuning's schedule overrides: PLAIN never, XCD
// always).
constexpr uint64_t kBatchSortMinSamples = 1ull << 20;
constexpr uint64_t kBatchSortMinFootprint = 32ull << 20;
constexpr uint64_t kBatchSortChunk = 1ull << 25;

bool batch_sorted(const moss_graph* g, uint64_t n, const Tuning& t) {
  if (t.schedule == MOSS_SCHEDULE_PLAIN) return false;
  if (t.schedule == MOSS_SCHEDULE_XCD) return n > 0;
  const uint64_t min_n = t.group_min_samples_log2 ? 1ull << t.group_min_samples_log2 : kBatchSortMinSamples;
  const uint64_t min_fp = t.group_min_footprint_mb ? (uint64_t)t.group_min_footprint_mb << 20 : kBatchSortMinFootprint;
  return n >= min_n && sampling_footprint(g) >= min_fp;
}
}  // namespace

Tuning current_tuning() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tuning;
}

uint32_t sort_window_for(const moss_graph* g) {
  const uint32_t w = current_tuning().sort_window;
  return w ? w : sort_window(sampling_footprint(g));
}

BatchRunner* batch_runner(int device) {
  std::lock_guard<std::mutex> lk(g_runner_mu);
  auto it = g_runners.find(device);
  if (it != g_runners.end()) return it->second.get();
  auto r = std::make_unique<BatchRunner>(device);
  BatchRunner* p = r.get();
  g_runners[device] = std::move(r);
  return p;
}

void result_header(const moss_graph* g, int32_t k, uint64_t n_samples, uint32_t flags, moss_result* r) {
  std::memset(r, 0, sizeof(*r));
  r->k = k;
  r->flags = flags;
  r->n_samples = n_samples;
  EstimatePlan plan;
  (void)plan_estimate(k, n_samples, flags, &plan);  // callers checked the request
  r->K[0] = plan.K[0];
  r->K[1] = plan.K[1];
  if (k == 4) {
    r->n_motifs = 6;
    r->gamma[0] = g->total[0];
    r->gamma[1] = plan.count == 2 ? g->total[3] : 0;
    r->lambda = g->lambda3;
  } else {
    r->n_motifs = 21;
    r->gamma[0] = g->total[1];
    r->gamma[1] = g->total[2];
    r->lambda = g->lambda4;
  }
}

BatchRunner::BatchRunner(int device) : device_(device) {}

BatchRunner::~BatchRunner() {
  // The per-device runners live until process exit, when the runtime may already be
  // gone; owners that end earlier (servers) call release() first.
}

void BatchRunner::release() {
  DeviceScope scope(device_);
  if (stream_) (void)hipStreamSynchronize(stream_);
  if (exec_) (void)hipGraphExecDestroy(exec_);
  if (graph_) (void)hipGraphDestroy(graph_);
  exec_ = nullptr;
  graph_ = nullptr;
  graph_grid_ = graph_block_ = 0;
  if (d_views_) (void)hipFree(d_views_);
  if (d_items_) (void)hipFree(d_items_);
  if (d_ctl_) (void)hipFree(d_ctl_);
  if (d_bins_) (void)hipFree(d_bins_);
  d_views_ = nullptr;
  d_items_ = nullptr;
  d_ctl_ = nullptr;
  d_bins_ = nullptr;
  cap_views_ = cap_items_ = cap_slots_ = 0;
  if (h_in_) (void)hipHostFree(h_in_);
  if (h_bins_) (void)hipHostFree(h_bins_);
  h_in_ = nullptr;
  h_bins_ = nullptr;
  cap_in_ = 0;
  if (ev0_) (void)hipEventDestroy(ev0_);
  if (ev1_) (void)hipEventDestroy(ev1_);
  if (ev_wait_) (void)hipEventDestroy(ev_wait_);
  if (ev_clear_) (void)hipEventDestroy(ev_clear_);
  for (int j = 0; j < 2; ++j) {
    if (ev_side_[j]) (void)hipEventDestroy(ev_side_[j]);
    ev_side_[j] = nullptr;
    if (side_[j]) {
      (void)hipStreamSynchronize(side_[j]);
      (void)hipStreamDestroy(side_[j]);
    }
    side_[j] = nullptr;
  }
  ev0_ = ev1_ = ev_wait_ = ev_clear_ = nullptr;
  if (stream_) (void)hipStreamDestroy(stream_);
  stream_ = nullptr;
}

moss_status BatchRunner::reserve(size_t views, size_t items, size_t slots) {
  bool changed = false;
  auto grow = [&](size_t need, size_t& cap, auto** ptr, size_t elem) -> moss_status {
    if (need <= cap) return MOSS_OK;
    size_t c = std::max<size_t>(need, cap * 2);
    if (*ptr) (void)hipFree((void*)*ptr);
    *ptr = nullptr;
    if (hipMalloc((void**)ptr, c * elem) != hipSuccess) {
      *ptr = nullptr;
      cap = 0;
      return MOSS_E_NOMEM;
    }
    cap = c;
    changed = true;
    return MOSS_OK;
  };
  moss_status st = grow(std::max<size_t>(views, 64), cap_views_, &d_views_, sizeof(SamplerView));
  if (st == MOSS_OK) st = grow(std::max<size_t>(items, 512), cap_items_, &d_items_, sizeof(BatchItem));
  if (st == MOSS_OK) {
    const size_t old = cap_slots_;
    st = grow(std::max<size_t>(slots, 512), cap_slots_, &d_bins_, 22 * sizeof(unsigned long long));
    if (st == MOSS_OK && cap_slots_ != old) {
      if (h_bins_) (void)hipHostFree(h_bins_);
      h_bins_ = nullptr;
      if (hipHostMalloc((void**)&h_bins_, cap_slots_ * 22 * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess) {
        h_bins_ = nullptr;
        return MOSS_E_NOMEM;
      }
    }
  }
  if (st != MOSS_OK) return st;
  if (!d_ctl_) {
    if (hipMalloc((void**)&d_ctl_, 4 * sizeof(uint32_t)) != hipSuccess) {
      d_ctl_ = nullptr;
      return MOSS_E_NOMEM;
    }
    changed = true;
  }
  const size_t in_bytes = cap_views_ * sizeof(SamplerView) + cap_items_ * sizeof(BatchItem) + 64;
  if (in_bytes > cap_in_) {
    if (h_in_) (void)hipHostFree(h_in_);
    h_in_ = nullptr;
    if (hipHostMalloc((void**)&h_in_, in_bytes, hipHostMallocDefault) != hipSuccess) {
      h_in_ = nullptr;
      cap_in_ = 0;
      return MOSS_E_NOMEM;
    }
    cap_in_ = in_bytes;
  }
  if (changed && exec_) {
    (void)hipGraphExecDestroy(exec_);
    (void)hipGraphDestroy(graph_);
    exec_ = nullptr;
    graph_ = nullptr;
  }
  return MOSS_OK;
}

// Captures: clear the tile counter (a fill kernel), then the persistent kernel.  Its
// arguments are the fixed buffers above, so one capture serves every batch until a
// buffer is reallocated or the launch shape changes.  (The histogram slots are cleared
// before the graph, so that the grouped launches on the side stream can start with it.)
moss_status BatchRunner::capture(int grid, int block) {
  if (exec_ && grid == graph_grid_ && block == graph_block_) return MOSS_OK;
  if (exec_) {
    (void)hipGraphExecDestroy(exec_);
    (void)hipGraphDestroy(graph_);
    exec_ = nullptr;
    graph_ = nullptr;
  }
  hipError_t e = hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return status_of(e);
  hipError_t e1 = launch_fill_u32(d_ctl_ + kCtlCounter, 0, 1, stream_);
  if (e1 == hipSuccess) e1 = launch_batch(d_views_, d_items_, d_ctl_, d_bins_, grid, block, stream_);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(stream_, &g);
  if (e1 != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return status_of(e1 != hipSuccess ? e1 : e);
  }
  e = hipGraphInstantiate(&exec_, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    exec_ = nullptr;
    return status_of(e);
  }
  graph_ = g;
  graph_grid_ = grid;
  graph_block_ = block;
  return MOSS_OK;
}

moss_status BatchRunner::run(const std::vector<WorkItem>& work, uint32_t n_slots, uint64_t* bins_out,
                             double* device_ms, hipStream_t wait_on, uint32_t tile_samples, uint32_t blocks_per_cu,
                             bool sort_large) {
  DeviceScope scope(device_);
  if (!scope.ok()) return MOSS_E_DEVICE;
  if (!stream_) {
    if (hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking) != hipSuccess) return MOSS_E_DEVICE;
    if (hipEventCreate(&ev0_) != hipSuccess || hipEventCreate(&ev1_) != hipSuccess ||
        hipEventCreateWithFlags(&ev_wait_, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev_clear_, hipEventDisableTiming) != hipSuccess)
      return MOSS_E_DEVICE;
  }
  const Tuning tune = current_tuning();
  uint32_t T = tile_samples ? tile_samples : (tune.tile_samples ? tune.tile_samples : kDefaultTile);
  const int block = tune.threads_per_block ? (int)tune.threads_per_block : 256;
  int bpc = blocks_per_cu ? (int)blocks_per_cu : (int)tune.blocks_per_cu;
  if (bpc == 0) {  // by the largest graph of the batch (its tiles run together)
    uint64_t most = 0;
    for (const WorkItem& w : work) most = std::max(most, sampling_footprint(w.g));
    const int cap = std::max(1, std::min(8, sample_kernel_blocks_per_cu(0, block)));
    bpc = std::max(1, std::min(cap, sampling_waves_per_cu(most) / (block / 64)));
  }
  const int grid = device_cus(device_) * bpc;

  // views: one per distinct (graph, sampler)
  std::vector<SamplerView> views;
  std::vector<const moss_graph*> view_graph;  // the graph of each view
  std::map<std::pair<const moss_graph*, int>, uint32_t> view_of;
  std::vector<BatchItem> items;
  std::vector<uint64_t> item_cost;
  // large items on large graphs run as grouped launches of their own after the
  // persistent kernel (the plain path's grouping passes and sorted sampling kernel, in
  // two chains of chunks, each chain one chunk at a time through a scratch block of its
  // own), adding into their histogram slots
  struct SortChunk {
    int sampler;
    uint64_t seed, a, n;
    uint32_t slot, window;
    int grid, block;
    SamplerView view;
  };
  std::vector<SortChunk> chunks;
  uint64_t max_chunk = 0;
  for (const WorkItem& w : work) {
    if (!sort_large || w.k1 <= w.k0 || w.g->total[sampler_slot(w.sampler)] == 0) continue;
    if (!batch_sorted(w.g, w.k1 - w.k0, tune)) continue;
    const SamplerView view = sampler_view(w.g, w.sampler);
    const uint32_t window = sort_window_for(w.g);
    for (uint64_t a = w.k0; a < w.k1; a += kBatchSortChunk) {
      const uint64_t n = std::min<uint64_t>(kBatchSortChunk, w.k1 - a);
      SortChunk c{w.sampler, w.seed, a, n, w.slot, window, 0, 0, view};
      plain_launch_shape(w.g, w.sampler, n, &c.grid, &c.block);
      chunks.push_back(c);
      max_chunk = std::max(max_chunk, n);
    }
  }
  // the costliest chunks first (samples times the Philox blocks a sample of the sampler
  // takes), each to the chain with less cost so far: the two chains then end together
  // (in request order by samples, one ended 0.8 ms after the other; 20.19 -> 19.91 ms on
  // a 256-request batch)
  auto chunk_cost = [](const SortChunk& c) {
    return c.n * ((c.sampler == kMoss4 || c.sampler == kMoss4Min) ? 2u : 3u);
  };
  std::stable_sort(chunks.begin(), chunks.end(),
                   [&](const SortChunk& x, const SortChunk& y) { return chunk_cost(x) > chunk_cost(y); });
  void* sort_scratch_block[2] = {nullptr, nullptr};
  struct Release {  // the blocks go back to the cache once the stream's work has finished
    hipStream_t s;
    void* (&a)[2];
    ~Release() {
      if (!a[0] && !a[1]) return;
      (void)hipStreamSynchronize(s);
      for (void*& p : a) device_block_free(s, p);
    }
  } release{stream_, sort_scratch_block};
  const int chains = chunks.size() > 1 ? 2 : 1;
  // the side streams exist once a run has needed them (a process holds few hardware
  // queues, and streams beyond them share one, so a runner without grouped launches,
  // such as the server's express path, keeps to its one stream)
  for (int j = 0; j < (chunks.empty() ? 0 : chains); ++j) {
    if (!side_[j] && hipStreamCreateWithFlags(&side_[j], hipStreamNonBlocking) != hipSuccess) {
      side_[j] = nullptr;
      return MOSS_E_DEVICE;
    }
    if (!ev_side_[j] && hipEventCreateWithFlags(&ev_side_[j], hipEventDisableTiming) != hipSuccess) {
      ev_side_[j] = nullptr;
      return MOSS_E_DEVICE;
    }
  }
  for (int j = 0; j < chains && max_chunk > 0; ++j)
    if (device_block_alloc(stream_, &sort_scratch_block[j], (size_t)grouped_scratch_bytes(max_chunk)) != MOSS_OK)
      return MOSS_E_NOMEM;
  for (const WorkItem& w : work) {
    if (w.k1 <= w.k0 || w.g->total[sampler_slot(w.sampler)] == 0) continue;
    if (sort_large && batch_sorted(w.g, w.k1 - w.k0, tune)) continue;  // a grouped launch
    auto key = std::make_pair((const moss_graph*)w.g, w.sampler);
    auto it = view_of.find(key);
    uint32_t vi;
    if (it == view_of.end()) {
      vi = (uint32_t)views.size();
      views.push_back(sampler_view(w.g, w.sampler));
      view_graph.push_back(w.g);
      view_of[key] = vi;
    } else {
      vi = it->second;
    }
    BatchItem b{};
    b.view = vi;
    b.sampler = (uint32_t)w.sampler;
    b.out = w.slot;
    b.seed = w.seed;
    b.k0 = w.k0;
    b.k1 = w.k1;
    items.push_back(b);
    item_cost.push_back((w.k1 - w.k0) * ((w.sampler == kMoss4 || w.sampler == kMoss4Min) ? 2 : 3));
  }
  // Graph-major order: the items of one (graph, sampler) view run together, so at any
  // moment the chip works on one graph's tables and they stay in L2 and the MALL
  // (interleaving the graphs of a batch measured about 15% slower per sample).  The
  // views of the graphs with the largest sampled footprint go first, then those with
  // the most work, and the largest items first within a view: the large graphs' items
  // then run while the grouped launches on the side stream read the same tables (0.8%
  // faster on a 256-request batch than most work first; smallest graphs first was 1%
  // slower).  The kernel cuts each item into tiles itself; the host hands over the
  // item list only.
  std::vector<uint64_t> view_cost(views.size(), 0), view_fp(views.size(), 0);
  for (size_t i = 0; i < items.size(); ++i) view_cost[items[i].view] += item_cost[i];
  for (size_t vi = 0; vi < views.size(); ++vi) view_fp[vi] = sampling_footprint(view_graph[vi]);
  std::vector<size_t> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
    const uint32_t vx = items[x].view, vy = items[y].view;
    if (vx != vy) {
      if (view_fp[vx] != view_fp[vy]) return view_fp[vx] > view_fp[vy];
      return view_cost[vx] != view_cost[vy] ? view_cost[vx] > view_cost[vy] : vx < vy;
    }
    return item_cost[x] > item_cost[y];
  });
  // A batch too small to give every block of the grid a tile gets smaller tiles (a
  // multiple of the block's threads, about its samples over the blocks): otherwise a
  // few blocks draw their lanes' samples one after another while the rest idle, and
  // a 10^4-sample request took 0.1-0.2 ms of kernel time instead of a few tens of µs.
  // The tiling does not change which samples are drawn, only which lanes draw them.
  uint64_t persistent = 0, tiles_at_T = 0;
  for (const BatchItem& b : items) {
    persistent += b.k1 - b.k0;
    tiles_at_T += (b.k1 - b.k0 + T - 1) / T;
  }
  if (tiles_at_T < (uint64_t)grid) {
    const uint64_t per_block = (persistent + (uint64_t)grid - 1) / (uint64_t)grid;
    const uint64_t t = std::max<uint64_t>((uint64_t)block, (per_block + block - 1) / block * block);
    if (t < T) T = (uint32_t)t;
  }
  uint64_t n_tiles = 0;
  for (size_t i : order) {
    items[i].first_tile = (uint32_t)n_tiles;
    n_tiles += (items[i].k1 - items[i].k0 + T - 1) / T;
    if (n_tiles >= 0xFFFFFFFFull) return MOSS_E_ARG;
  }
  moss_status st = reserve(views.size(), items.size(), n_slots);
  if (st != MOSS_OK) return st;
  st = capture(grid, block);
  if (st != MOSS_OK) return st;

  // stage views | items | control words in pinned memory and copy in one transfer each
  unsigned char* p = h_in_;
  const size_t vbytes = views.size() * sizeof(SamplerView), ibytes = items.size() * sizeof(BatchItem);
  std::memcpy(p, views.data(), vbytes);
  BatchItem* ip = (BatchItem*)(p + vbytes);
  for (size_t i = 0; i < order.size(); ++i) ip[i] = items[order[i]];
  uint32_t* np = (uint32_t*)(p + vbytes + ibytes);
  np[kCtlTiles] = (uint32_t)n_tiles;
  np[kCtlCounter] = 0;
  np[kCtlItems] = (uint32_t)items.size();
  np[kCtlTileSize] = T;

  hipError_t e = hipSuccess;
  if (wait_on) {
    e = hipEventRecord(ev_wait_, wait_on);
    if (e == hipSuccess) e = hipStreamWaitEvent(stream_, ev_wait_, 0);
  }
  if (e == hipSuccess && vbytes) e = hipMemcpyAsync(d_views_, p, vbytes, hipMemcpyHostToDevice, stream_);
  if (e == hipSuccess && ibytes) e = hipMemcpyAsync(d_items_, p + vbytes, ibytes, hipMemcpyHostToDevice, stream_);
  if (e == hipSuccess) e = hipMemcpyAsync(d_ctl_, np, 4 * sizeof(uint32_t), hipMemcpyHostToDevice, stream_);
  if (e == hipSuccess) e = hipEventRecord(ev0_, stream_);
  if (e == hipSuccess) e = launch_fill_u64((uint64_t*)d_bins_, 0, (int64_t)n_slots * 22, stream_);
  // the grouped launches run on the side streams, beside the persistent kernel (whose
  // latency-bound waves leave block slots and memory bandwidth free), from the clear on;
  // each chunk goes to the chain with less cost so far.  Two chains measured 1%
  // faster than one on a 256-request batch: one chain's passes had outlasted the
  // persistent kernel by 2.5 ms.
  const int side = chunks.empty() ? 0 : chains;
  if (e == hipSuccess && side) e = hipEventRecord(ev_clear_, stream_);
  for (int j = 0; j < side && e == hipSuccess; ++j) e = hipStreamWaitEvent(side_[j], ev_clear_, 0);
  if (e == hipSuccess) e = hipGraphLaunch(exec_, stream_);
  uint64_t load[2] = {0, 0};
  for (const SortChunk& c : chunks) {
    if (e != hipSuccess) break;
    const int j = chains == 2 && load[1] < load[0] ? 1 : 0;
    load[j] += chunk_cost(c);
    e = launch_group_chunk(c.sampler, c.seed, c.a, c.n, sort_scratch_block[j], max_chunk, side_[j]);
    if (e == hipSuccess)
      e = launch_sample_chunk(c.sampler, c.view, c.seed, c.a, c.n, sort_scratch_block[j], max_chunk, c.window,
                              d_bins_ + (uint64_t)c.slot * 22, nullptr, c.grid, c.block, side_[j]);
  }
  for (int j = 0; j < side && e == hipSuccess; ++j) {
    e = hipEventRecord(ev_side_[j], side_[j]);
    if (e == hipSuccess) e = hipStreamWaitEvent(stream_, ev_side_[j], 0);
  }
  if (e == hipSuccess) e = hipEventRecord(ev1_, stream_);
  if (e == hipSuccess && n_slots)
    e = hipMemcpyAsync(h_bins_, d_bins_, (size_t)n_slots * 22 * sizeof(uint64_t), hipMemcpyDeviceToHost, stream_);
  if (e == hipSuccess) e = hipStreamSynchronize(stream_);
  if (e != hipSuccess) {
    for (int j = 0; j < side; ++j) (void)hipStreamSynchronize(side_[j]);  // nothing of this batch left running
    return status_of(e);
  }
  std::memcpy(bins_out, h_bins_, (size_t)n_slots * 22 * sizeof(uint64_t));
  if (device_ms) {
    float ms = 0.f;
    *device_ms = hipEventElapsedTime(&ms, ev0_, ev1_) == hipSuccess ? (double)ms : 0.0;
  }
  return MOSS_OK;
}

namespace {

std::mutex g_batch_mu;  // one batch at a time per process (the runner is shared)

moss_status batch_impl(const moss_request* reqs, int32_t n, moss_result* out, hipStream_t wait_on,
                       uint32_t tile_samples, uint32_t blocks_per_cu, double* device_ms) {
  if (n < 0 || (n > 0 && (!reqs || !out))) return MOSS_E_ARG;
  if (n == 0) return MOSS_OK;
  const int device = reqs[0].g ? reqs[0].g->device : -1;
  for (int32_t i = 0; i < n; ++i) {
    const moss_request& q = reqs[i];
    EstimatePlan plan;
    if (!q.g || q.g->device != device || plan_estimate(q.k, q.n_samples, q.flags, &plan) != MOSS_OK)
      return MOSS_E_ARG;
  }
  // build missing tables (each graph once)
  for (int32_t i = 0; i < n; ++i) {
    moss_graph* g = reqs[i].g;
    EstimatePlan plan;
    (void)plan_estimate(reqs[i].k, reqs[i].n_samples, reqs[i].flags, &plan);
    const uint32_t mask = plan.tables;
    if ((g->built & mask) == mask) continue;
    GraphClaim claim(g);
    if (!claim.ok()) return MOSS_E_BUSY;
    moss_status st = build_tables(g, mask);
    if (st != MOSS_OK) return st;
  }
  std::vector<WorkItem> work;
  work.reserve((size_t)n * 2);
  for (int32_t i = 0; i < n; ++i) {
    const moss_request& q = reqs[i];
    moss_result& r = out[i];
    result_header(q.g, q.k, q.n_samples, q.flags, &r);
    EstimatePlan plan;
    (void)plan_estimate(q.k, q.n_samples, q.flags, &plan);
    for (int s = 0; s < plan.count; ++s)
      work.push_back({q.g, plan.sampler[s], q.seed, 0, plan.K[s], (uint32_t)(2 * i + s)});
  }
  std::vector<uint64_t> bins((size_t)n * 2 * 22);
  std::lock_guard<std::mutex> lk(g_batch_mu);
  BatchRunner* runner = batch_runner(device);
  double ms = 0.0;
  moss_status st =
      runner->run(work, (uint32_t)(2 * n), bins.data(), &ms, wait_on, tile_samples, blocks_per_cu, true);
  if (st != MOSS_OK) return st;
  for (int32_t i = 0; i < n; ++i) {
    moss_result& r = out[i];
    std::memcpy(r.hits[0], &bins[(size_t)(2 * i) * 22], 22 * sizeof(uint64_t));
    std::memcpy(r.hits[1], &bins[(size_t)(2 * i + 1) * 22], 22 * sizeof(uint64_t));
    r.device_ms = ms;
    st = moss_finals(&r);
    if (st != MOSS_OK) return st;
  }
  if (device_ms) *device_ms = ms;
  return MOSS_OK;
}

}  // namespace
}  // namespace moss

using namespace moss;

extern "C" {

moss_status moss_estimate_batch(const moss_request* reqs, int32_t n, moss_result* out, void* hip_stream) {
  return batch_impl(reqs, n, out, (hipStream_t)hip_stream, 0, 0, nullptr);
}

moss_status moss_set_tuning(const moss_tuning* t) {
  if (!t) return MOSS_E_ARG;
  if (t->threads_per_block && (t->threads_per_block % 64 != 0 || t->threads_per_block > 256)) return MOSS_E_ARG;
  if (t->blocks_per_cu > 64 || t->schedule > MOSS_SCHEDULE_XCD) return MOSS_E_ARG;
  if (t->group_min_samples_log2 > 40 || t->group_min_footprint_mb > (1u << 20)) return MOSS_E_ARG;
  if (t->sort_window % 64 != 0 || t->sort_window > 512) return MOSS_E_ARG;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuning.tile_samples = t->tile_samples;
  g_tuning.blocks_per_cu = t->blocks_per_cu;
  g_tuning.threads_per_block = t->threads_per_block;
  g_tuning.schedule = t->schedule;
  g_tuning.group_min_samples_log2 = t->group_min_samples_log2;
  g_tuning.group_min_footprint_mb = t->group_min_footprint_mb;
  g_tuning.sort_window = t->sort_window;
  return MOSS_OK;
}

moss_status moss_get_tuning(moss_tuning* t) {
  if (!t) return MOSS_E_ARG;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  t->tile_samples = g_tuning.tile_samples;
  t->blocks_per_cu = g_tuning.blocks_per_cu;
  t->threads_per_block = g_tuning.threads_per_block;
  t->schedule = g_tuning.schedule;
  t->group_min_samples_log2 = g_tuning.group_min_samples_log2;
  t->group_min_footprint_mb = g_tuning.group_min_footprint_mb;
  t->sort_window = g_tuning.sort_window;
  return MOSS_OK;
}

moss_status moss_autotune(const moss_request* reqs, int32_t n, moss_tuning* best, double* best_ms) {
  if (!reqs || n <= 0 || !best) return MOSS_E_ARG;
  static const uint32_t kTiles[] = {2048, 4096, 16384, 65536};
  static const uint32_t kBpc[] = {2, 3, 4, 5, 6, 8};
  static const uint32_t kGroupLog2[] = {17, 18, 19, 20, 21, 22};
  static const uint32_t kGroupMb[] = {4, 8, 16, 32, 64};
  static const uint32_t kWindows[] = {128, 256, 512};
  const moss_tuning before = [] {
    moss_tuning t{};
    (void)moss_get_tuning(&t);
    return t;
  }();
  std::vector<moss_result> ref((size_t)n), cur((size_t)n);
  moss_status st = batch_impl(reqs, n, ref.data(), nullptr, kDefaultTile, 4, nullptr);  // warm-up, reference
  if (st != MOSS_OK) return st;
  // the whole call, best of two (host time included: item list, staging, copies)
  auto timed = [&](uint32_t T, uint32_t bpc, double* ms) -> moss_status {
    *ms = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
      const auto t0 = std::chrono::steady_clock::now();
      moss_status s = batch_impl(reqs, n, cur.data(), nullptr, T, bpc, nullptr);
      const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (s != MOSS_OK) return s;
      for (int32_t i = 0; i < n; ++i)
        if (std::memcmp(cur[i].hits, ref[i].hits, sizeof(ref[i].hits)) != 0) return MOSS_E_DEVICE;
      *ms = std::min(*ms, t);
    }
    return MOSS_OK;
  };
  double best_t = 1e300;
  moss_tuning b = before;
  b.threads_per_block = 256;
  // 1. tile size and occupancy of the persistent kernel, at the default grouping
  moss_tuning c = b;
  c.group_min_samples_log2 = c.group_min_footprint_mb = c.sort_window = 0;
  for (uint32_t T : kTiles) {
    for (uint32_t bpc : kBpc) {
      c.tile_samples = T;
      c.blocks_per_cu = bpc;
      if ((st = moss_set_tuning(&c)) != MOSS_OK) break;
      double ms;
      if ((st = timed(T, bpc, &ms)) != MOSS_OK) break;
      if (ms < best_t) {
        best_t = ms;
        b = c;
      }
    }
    if (st != MOSS_OK) break;
  }
  // 2. which items leave the persistent kernel for grouped launches of their own: the
  // fewest samples per item and the smallest sampled footprint of its graph
  for (uint32_t lg : kGroupLog2) {
    if (st != MOSS_OK) break;
    for (uint32_t mb : kGroupMb) {
      c = b;
      c.group_min_samples_log2 = lg;
      c.group_min_footprint_mb = mb;
      if ((st = moss_set_tuning(&c)) != MOSS_OK) break;
      double ms;
      if ((st = timed(c.tile_samples, c.blocks_per_cu, &ms)) != MOSS_OK) break;
      if (ms < best_t) {
        best_t = ms;
        b = c;
      }
    }
  }
  // 3. the window of the grouped launches' sorted kernel (by footprint, or fixed)
  for (uint32_t w : kWindows) {
    if (st != MOSS_OK) break;
    c = b;
    c.sort_window = w;
    if ((st = moss_set_tuning(&c)) != MOSS_OK) break;
    double ms;
    if ((st = timed(c.tile_samples, c.blocks_per_cu, &ms)) != MOSS_OK) break;
    if (ms < best_t) {
      best_t = ms;
      b = c;
    }
  }
  if (st != MOSS_OK) {
    (void)moss_set_tuning(&before);
    return st;
  }
  st = moss_set_tuning(&b);
  if (st != MOSS_OK) return st;
  *best = b;
  if (best_ms) *best_ms = best_t;
  return MOSS_OK;
}

}  // extern "C"
