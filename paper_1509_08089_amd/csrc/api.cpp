// C ABI: graphs, table build, plain estimation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "batch.h"
#include "internal.h"

namespace moss {

moss_status status_of(hipError_t e) {
  if (e == hipSuccess) return MOSS_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return MOSS_E_NOMEM;
  return MOSS_E_DEVICE;
}

DeviceScope::DeviceScope(int device) {
  if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
  ok_ = hipSetDevice(device) == hipSuccess;
}

DeviceScope::~DeviceScope() {
  if (prev_ >= 0) (void)hipSetDevice(prev_);
}

GraphClaim::GraphClaim(moss_graph* g) : g_(g) {
  int expected = 0;
  ok_ = g && g->busy.compare_exchange_strong(expected, 1);
}

GraphClaim::~GraphClaim() {
  if (ok_) g_->busy.store(0);
}

namespace {
std::mutex g_dev_mu;
std::vector<int> g_dev_ready;  // per device: 0 not set up, 1 ready
std::vector<int> g_dev_cus;
}  // namespace

moss_status ensure_device(int device) {
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (device < 0) return MOSS_E_DEVICE;
  if ((int)g_dev_ready.size() <= device) {
    g_dev_ready.resize(device + 1, 0);
    g_dev_cus.resize(device + 1, 0);
  }
  if (g_dev_ready[device]) return MOSS_OK;
  DeviceScope scope(device);
  if (!scope.ok()) return MOSS_E_DEVICE;
  uint8_t l4[8], lt[64], lp[64];
  class_luts(l4, lt, lp);
  hipError_t e = upload_class_luts(l4, lt, lp);
  if (e != hipSuccess) return status_of(e);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
    return MOSS_E_DEVICE;
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
    uint64_t keep = ~0ull;  // keep freed blocks for reuse instead of returning them at each sync
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  g_dev_cus[device] = cus;
  g_dev_ready[device] = 1;
  return MOSS_OK;
}

int device_cus(int device) {
  std::lock_guard<std::mutex> lk(g_dev_mu);
  return device >= 0 && device < (int)g_dev_cus.size() && g_dev_cus[device] > 0 ? g_dev_cus[device] : 256;
}

SamplerView sampler_view(const moss_graph* g, int sampler) {
  const int s = sampler_slot(sampler);
  SamplerView v{};
  v.rp = g->rp;
  v.col = g->col;
  v.acc_node = g->acc_node[s];
  v.guide = g->guide[s];
  v.acc_sigma = g->acc_sigma;
  v.acc_tau = g->acc_tau;
  v.rec = g->rec;
  v.sig_guide = g->sig_guide;
  v.tau_guide = g->tau_guide;
  v.edge_slots = g->edge_slots;
  v.edge_bits = g->edge_bits;
  v.filter = g->filter;
  v.filter_bits = g->filter_bits;
  v.rank = g->rank;
  v.col_rank = g->col_rank;
  v.acc_check = g->acc_check;
  v.check_guide = g->check_guide;
  v.total = g->total[s];
  v.n = g->n;
  v.gbits = g->gbits;
  return v;
}

// Resident waves per CU for the sampling kernels, by the bytes a graph's samples read
// at random (CSR and tables).  Measured on MI355X: a graph whose tables fit the 256 MB
// MALL samples fastest with about 20 waves per CU; one far larger than the MALL with
// 8 (more waves in flight then only add queueing and translation misses).
int sampling_waves_per_cu(uint64_t footprint_bytes) {
  const uint64_t MB = 1ull << 20;
  if (footprint_bytes <= 128 * MB) return 20;
  if (footprint_bytes <= 256 * MB) return 16;
  if (footprint_bytes <= 384 * MB) return 12;
  return 8;
}

uint64_t sampling_footprint(const moss_graph* g) {
  const uint64_t csr = ((uint64_t)g->n + 1 + (uint64_t)g->nnz) * sizeof(int32_t);
  const uint64_t edge_set = (8ull << g->edge_bits) + (8ull << g->filter_bits);
  return g->table_bytes + csr + edge_set;
}

// Whether a plain estimate on g draws its samples XCD-grouped (the tuning's schedule,
// else by size): the grouping passes pay off once the sampled tables are well beyond
// the L2 and a sampler has enough samples.  Measured per estimate (plain / grouped):
// n = 1e5, m = 1e6, MOSS-4 with 1e6 / 2e6 / 4e6 samples 0.106 / 0.171 / 0.316 ms
// against 0.140 / 0.172 / 0.253 ms, T-5 + Path-5 with 2e6 / 4e6 samples 0.283 / 0.496
// against 0.331 / 0.439 ms; n = 1e6, m = 1e7, T-5 + Path-5 with 1e6 / 2e6 / 4e6 samples
// 0.299 / 0.557 / 1.06 against 0.361 / 0.504 / 0.760 ms.  So: at least 1.5 * 2^20
// samples per sampler within the MALL, 2^19 beyond it; at n = 2e3, m = 1e4 grouping
// loses at any size.
constexpr uint64_t kGroupedMinFootprint = 32ull << 20;
constexpr uint64_t kGroupedMinSamples = 3ull << 19;
constexpr uint64_t kGroupedMinSamplesPastMall = 1ull << 19;

bool grouped_schedule(const moss_graph* g, uint64_t nsamples) {
  const uint32_t sch = current_tuning().schedule;
  if (sch == MOSS_SCHEDULE_XCD) return true;
  if (sch == MOSS_SCHEDULE_PLAIN) return false;
  const uint64_t fp = sampling_footprint(g);
  if (fp < kGroupedMinFootprint) return false;
  return nsamples >= (fp > (256ull << 20) ? kGroupedMinSamplesPastMall : kGroupedMinSamples);
}

moss_status plan_estimate(int32_t k, uint64_t n_samples, uint32_t flags, EstimatePlan* p) {
  *p = EstimatePlan{};
  if (flags & ~(MOSS_MIX_PAPER | MOSS_K4_MIN)) return MOSS_E_ARG;
  const bool with_min = (flags & MOSS_K4_MIN) != 0;
  if (k == 4 && !with_min) {
    if (n_samples < 1) return MOSS_E_ARG;
    p->count = 1;
    p->sampler[0] = kMoss4;
    p->K[0] = n_samples;
    p->tables = MOSS_TABLES_K4;
    return MOSS_OK;
  }
  if ((k != 4 && k != 5) || (k == 5 && with_min) || n_samples < 2) return MOSS_E_ARG;
  p->count = 2;
  p->sampler[0] = k == 4 ? kMoss4 : kT5;
  p->sampler[1] = k == 4 ? kMoss4Min : kPath5;
  p->K[0] = (n_samples + 1) / 2;
  p->K[1] = n_samples / 2;
  p->tables = k == 4 ? (MOSS_TABLES_K4 | MOSS_TABLES_K4MIN) : MOSS_TABLES_K5;
  return MOSS_OK;
}

void plain_launch_shape(const moss_graph* g, int sampler, uint64_t nsamples, int* grid, int* block) {
  const Tuning t = current_tuning();
  int b = t.threads_per_block ? (int)t.threads_per_block : 256;
  int per_cu = t.blocks_per_cu ? (int)t.blocks_per_cu : 0;
  if (per_cu == 0) {
    // grouped launches: 28 waves per CU (n = 1e5, m = 1e6, MOSS-4 for 1e7 samples,
    // 12 / 16 / 20 / 24 / 28 / 32 waves: 0.687 / 0.602 / 0.559 / 0.542 / 0.538 / 0.540
    // ms; n = 1e6, m = 1e7, T-5 for 5e7: 6.14 / 5.71 / 5.61 / 5.60 / 5.61 / 5.62 ms)
    const uint64_t fp = sampling_footprint(g);
    const int waves = grouped_schedule(g, nsamples) ? 28 : sampling_waves_per_cu(fp);
    const int cap = std::max(1, std::min(sample_kernel_blocks_per_cu(sampler, b), 8));
    per_cu = std::max(1, std::min(cap, waves / (b / 64)));
  }
  const uint64_t want = (nsamples + (uint64_t)b - 1) / (uint64_t)b;
  const uint64_t most = (uint64_t)device_cus(g->device) * (uint64_t)per_cu;
  *grid = (int)std::max<uint64_t>(1, std::min(want, most));
  *block = b;
}

}  // namespace moss

using namespace moss;

namespace {

// Device memory.  Each graph holds a few blocks, every array carved out of one of them
// at a 256-byte boundary.  Blocks come from the device's stream-ordered pool
// (hipMallocAsync on the graph's stream), and released blocks are kept per device for
// reuse by a later request of the same rounded size: on MI355X a hipFreeAsync call
// costs about 19 us and a hipMallocAsync call about 7 us of host time, more than the
// small kernels of a table build.  Callers release a block only once its stream has
// drained (after a synchronisation), so a cached block is idle and serves any stream.
// The cache holds at most kCacheBytes per device and drops its oldest blocks first.
constexpr size_t kCacheBytes = 1ull << 30;

size_t block_size(size_t bytes) {
  const size_t g = bytes <= (8u << 20) ? (64u << 10) : (2u << 20);
  return (std::max<size_t>(bytes, 256) + g - 1) / g * g;
}

struct BlockCache {
  std::mutex mu;
  struct Entry {
    int device;
    size_t bytes;
    void* p;
  };
  std::vector<Entry> idle;  // oldest first
  std::vector<size_t> held;  // per device
  std::map<void*, size_t> live;
};
BlockCache g_blocks;

moss_status dev_alloc_bytes(hipStream_t s, void** p, size_t bytes) {
  *p = nullptr;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return MOSS_E_DEVICE;
  const size_t sz = block_size(bytes);
  {
    std::lock_guard<std::mutex> lk(g_blocks.mu);
    for (size_t i = g_blocks.idle.size(); i-- > 0;) {
      const BlockCache::Entry& en = g_blocks.idle[i];
      if (en.device == device && en.bytes == sz) {
        *p = en.p;
        g_blocks.held[device] -= sz;
        g_blocks.idle.erase(g_blocks.idle.begin() + (std::ptrdiff_t)i);
        g_blocks.live[*p] = sz;
        return MOSS_OK;
      }
    }
  }
  hipError_t e = hipMallocAsync(p, sz, s);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return MOSS_E_NOMEM;
  }
  std::lock_guard<std::mutex> lk(g_blocks.mu);
  g_blocks.live[*p] = sz;
  return MOSS_OK;
}

// p must be idle: no work that uses it may still be queued on any stream.
void dev_free(hipStream_t s, void*& p) {
  if (!p) return;
  int device = 0;
  (void)hipGetDevice(&device);
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> lk(g_blocks.mu);
    auto it = g_blocks.live.find(p);
    const size_t sz = it != g_blocks.live.end() ? it->second : 0;
    if (it != g_blocks.live.end()) g_blocks.live.erase(it);
    if ((int)g_blocks.held.size() <= device) g_blocks.held.resize(device + 1, 0);
    if (sz > 0 && sz <= kCacheBytes) {
      g_blocks.idle.push_back({device, sz, p});
      g_blocks.held[device] += sz;
      for (size_t i = 0; g_blocks.held[device] > kCacheBytes && i < g_blocks.idle.size();) {
        if (g_blocks.idle[i].device == device) {
          g_blocks.held[device] -= g_blocks.idle[i].bytes;
          drop.push_back(g_blocks.idle[i].p);
          g_blocks.idle.erase(g_blocks.idle.begin() + (std::ptrdiff_t)i);
        } else {
          ++i;
        }
      }
    } else {
      drop.push_back(p);
    }
  }
  for (void* q : drop) (void)hipFreeAsync(q, s);
  p = nullptr;
}

struct Carve {
  size_t off = 0;
  template <typename T>
  size_t take(size_t count) {
    const size_t o = off;
    off += (count * sizeof(T) + 255) & ~(size_t)255;
    return o;
  }
};

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// per graph: word block, edge hash set and filter, items, item sums, row-guide lengths,
// scan scratch, partials, records
struct GraphLayout {
  size_t small, slots, filter, items, item_sum, guide_len, tmp[3], partials, rec, span_row, check_part, span_sums,
      span_groups, group_wrap, bytes;
};

GraphLayout graph_layout(int32_t n, int64_t nnz) {
  const int64_t cap = items_cap(n, nnz);
  GraphLayout L;
  Carve c;
  L.small = c.take<uint64_t>(kWords);
  L.slots = c.take<uint64_t>((size_t)1 << edge_hash_bits(nnz / 2));
  L.filter = c.take<uint64_t>((size_t)1 << edge_filter_bits(nnz / 2));
  L.items = c.take<uint64_t>((size_t)cap);
  L.item_sum = c.take<uint64_t>((size_t)std::max<int32_t>(1, n));
  L.guide_len = c.take<uint64_t>((size_t)n);
  for (int j = 0; j < 3; ++j) L.tmp[j] = c.take<uint64_t>((size_t)scan_tmp_elems(n));
  L.partials = c.take<uint64_t>(2 * (size_t)node_weight_blocks(n));
  L.rec = c.take<uint4>((size_t)n);
  L.span_row = c.take<int32_t>((size_t)span_count(nnz) + 1);
  L.check_part = c.take<uint64_t>((size_t)check_part_words());
  L.span_sums = c.take<uint64_t>(2 * (size_t)std::max<int64_t>(1, span_count(nnz)));
  L.span_groups = c.take<uint64_t>((size_t)std::max<int64_t>(1, span_group_count(nnz)));
  L.group_wrap = c.take<uint32_t>((size_t)std::max<int64_t>(1, span_group_count(nnz)));
  L.bytes = c.off;
  return L;
}

struct SigLayout {
  size_t acc_sigma, guide, bytes;
};

SigLayout sig_layout(const moss_graph* g) {
  SigLayout L;
  Carve c;
  L.acc_sigma = c.take<uint32_t>((size_t)g->nnz);
  L.guide = c.take<uint32_t>((size_t)g->row_guide_len);
  L.bytes = c.off;
  return L;
}

struct NodeLayout {
  size_t acc_tau, tau_guide, acc[2], guide[2], bytes;
};

// MOSS-4Min: rank pairs, rows in descending order, the row prefix of d_{v,x} d_{x,v}
// (also the rank passes' scratch) with its row guides, the node prefix and guide, and
// the counts of the mirror sort
struct MinLayout {
  size_t rank, col_rank, acc_check, check_guide, acc, guide, work, bytes;
};

MinLayout min_layout(const moss_graph* g) {
  const size_t n = (size_t)g->n, nnz = (size_t)g->nnz, G = ((size_t)1 << g->gbits) + 1;
  MinLayout L;
  Carve c;
  L.rank = c.take<uint2>(nnz);
  L.col_rank = c.take<int32_t>(nnz);
  L.acc_check = c.take<uint64_t>(nnz);
  L.check_guide = c.take<uint32_t>((size_t)g->row_guide_len);
  L.acc = c.take<uint64_t>(n);
  L.guide = c.take<uint32_t>(G);
  L.work = c.take<uint32_t>((size_t)mirror_work_words(g->nnz));
  L.bytes = c.off;
  return L;
}

// k5 = false: ACC_Gamma and its guide; true: ACC_tau, its row guides, ACC_Gamma1/2, guides
NodeLayout node_layout(const moss_graph* g, bool k5) {
  const size_t n = (size_t)g->n, G = ((size_t)1 << g->gbits) + 1;
  NodeLayout L{};
  Carve c;
  if (k5) {
    L.acc_tau = c.take<uint64_t>((size_t)g->nnz);
    L.tau_guide = c.take<uint32_t>((size_t)g->row_guide_len);
  }
  const int sets = k5 ? 2 : 1;
  for (int j = 0; j < sets; ++j) L.acc[j] = c.take<uint64_t>(n);
  for (int j = 0; j < sets; ++j) L.guide[j] = c.take<uint32_t>(G);
  L.bytes = c.off;
  return L;
}

// Small pinned host buffers for results and flags, reused across graphs.
std::mutex g_pin_mu;
std::vector<uint64_t*> g_pin_free;
constexpr size_t kPinWords = kWords;

uint64_t* pinned_chunk() {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  if (g_pin_free.empty()) {
    uint64_t* slab = nullptr;
    if (hipHostMalloc((void**)&slab, 64 * kPinWords * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess)
      return nullptr;
    for (int i = 0; i < 64; ++i) g_pin_free.push_back(slab + i * kPinWords);
  }
  uint64_t* p = g_pin_free.back();
  g_pin_free.pop_back();
  return p;
}

void pinned_release(uint64_t* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.push_back(p);
}

// Timing events, kept per device for reuse (creating and destroying them costs more
// than the small calls they time).
std::vector<std::vector<hipEvent_t>> g_events;  // guarded by g_pin_mu

hipEvent_t pooled_event(int device) {
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if ((int)g_events.size() > device && !g_events[device].empty()) {
      hipEvent_t e = g_events[device].back();
      g_events[device].pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

void event_release(int device, hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  if ((int)g_events.size() <= device) g_events.resize(device + 1);
  g_events[device].push_back(e);
}

void free_tables(moss_graph* g, uint32_t mask) {
  if (mask & MOSS_TABLES_K4) {
    dev_free(g->stream, g->mem_k4);
    g->acc_node[0] = nullptr;
    g->guide[0] = nullptr;
    g->total[0] = 0;
  }
  if (mask & MOSS_TABLES_K5) {
    dev_free(g->stream, g->mem_k5);
    g->acc_tau = nullptr;
    g->tau_guide = nullptr;
    g->acc_node[1] = g->acc_node[2] = nullptr;
    g->guide[1] = g->guide[2] = nullptr;
    g->total[1] = g->total[2] = 0;
  }
  if (mask & MOSS_TABLES_K4MIN) {
    dev_free(g->stream, g->mem_min);
    g->rank = nullptr;
    g->col_rank = nullptr;
    g->acc_check = nullptr;
    g->check_guide = nullptr;
    g->acc_node[3] = nullptr;
    g->guide[3] = nullptr;
    g->total[3] = 0;
  }
  g->built &= ~mask;
  if (!(g->built & (MOSS_TABLES_K4 | MOSS_TABLES_K5 | MOSS_TABLES_K4MIN))) {
    dev_free(g->stream, g->mem_sig);
    g->acc_sigma = nullptr;
    g->sig_guide = nullptr;
  }
  g->table_bytes = moss::table_bytes_needed(g, 0);
}

void destroy_graph(moss_graph* g) {
  if (!g) return;
  DeviceScope scope(g->device);
  (void)hipStreamSynchronize(g->stream);
  free_tables(g, MOSS_TABLES_K4 | MOSS_TABLES_K5 | MOSS_TABLES_K4MIN);
  void* csr = g->owned_rp;
  dev_free(g->stream, csr);
  dev_free(g->stream, g->mem_graph);
  pinned_release(g->h_stage);
  g->h_stage = nullptr;
  event_release(g->device, g->ev0);
  event_release(g->device, g->ev1);
  delete g;
}

int validate_error_status(uint32_t bits) {
  if (bits & kErrArg) return MOSS_E_ARG;
  if (bits & kErrSelfLoop) return MOSS_E_SELF_LOOP;
  if (bits & kErrDuplicate) return MOSS_E_DUPLICATE;
  if (bits & kErrUnsorted) return MOSS_E_UNSORTED;
  if (bits & kErrAsymmetric) return MOSS_E_ASYMMETRIC;
  if (bits & kErrOverflow) return MOSS_E_OVERFLOW;
  return MOSS_OK;
}

// Per-graph memory, events and the CSR checks shared by both creation paths: one
// pass over the nodes, one scan pair (piece counts and row-guide lengths), items and
// records, the edge hash set and filter, the column and symmetry checks, one copy
// back and one synchronisation.
moss_status finish_create(moss_graph* g) {
  const GraphLayout L = graph_layout(g->n, g->nnz);
  moss_status st = dev_alloc_bytes(g->stream, &g->mem_graph, L.bytes);
  if (st != MOSS_OK) return st;
  void* m = g->mem_graph;
  g->small = at<uint64_t>(m, L.small);
  g->edge_slots = at<uint64_t>(m, L.slots);
  g->filter = at<uint64_t>(m, L.filter);
  g->edge_bits = edge_hash_bits(g->nnz / 2);
  g->filter_bits = edge_filter_bits(g->nnz / 2);
  g->items = at<uint64_t>(m, L.items);
  g->item_sum = at<uint64_t>(m, L.item_sum);
  g->guide_len = at<uint64_t>(m, L.guide_len);
  for (int j = 0; j < 3; ++j) g->scan_tmp[j] = at<uint64_t>(m, L.tmp[j]);
  g->partials = at<uint64_t>(m, L.partials);
  g->rec = at<uint4>(m, L.rec);
  g->span_row = at<int32_t>(m, L.span_row);
  g->check_part = at<uint64_t>(m, L.check_part);
  g->span_sums = at<uint64_t>(m, L.span_sums);
  g->span_groups = at<uint64_t>(m, L.span_groups);
  g->group_wrap = at<uint32_t>(m, L.group_wrap);
  if (!(g->h_stage = pinned_chunk())) return MOSS_E_NOMEM;
  if (!(g->ev0 = pooled_event(g->device)) || !(g->ev1 = pooled_event(g->device))) return MOSS_E_DEVICE;
  hipStream_t s = g->stream;
  const int64_t cap = items_cap(g->n, g->nnz);
  uint32_t* err = (uint32_t*)(g->small + kWErr);
  FillSet f{};
  f.p[0] = g->small;
  f.count[0] = kWords;
  f.p[1] = g->edge_slots;
  f.count[1] = (int64_t)1 << g->edge_bits;
  f.value[1] = ~0ull;
  f.p[2] = g->filter;
  f.count[2] = (int64_t)1 << g->filter_bits;
  hipError_t e = launch_fill_set(f, s);
  // item_sum holds the piece counts here, scanned into each row's item end
  if (e == hipSuccess) e = launch_node_prep(g->n, g->nnz, g->rp, g->item_sum, g->guide_len, g->small, s);
  if (e == hipSuccess) {
    ScanSet set{};
    set.data[0] = g->item_sum;
    set.data[1] = g->guide_len;
    set.tmp[0] = g->scan_tmp[0];
    set.tmp[1] = g->scan_tmp[1];
    set.total[0] = g->small + kWItems;
    set.total[1] = g->small + kWGuideLen;
    set.err_bit[0] = set.err_bit[1] = kErrArg;
    set.count = 2;
    e = launch_scans(set, g->n, err, s);
  }
  if (e == hipSuccess)
    e = launch_items_records(g->n, g->nnz, g->rp, g->item_sum, g->guide_len, cap, g->items, g->rec, g->span_row,
                             g->small, s);
  if (e == hipSuccess)
    e = launch_edge_insert(g->nnz, g->span_row, g->rp, g->col, g->n, g->edge_slots, g->edge_bits, g->filter,
                           g->filter_bits, g->small, s);
  if (e == hipSuccess)
    e = launch_check_items(g->nnz, g->span_row, g->n, g->rp, g->col, !(g->flags & MOSS_TRUST_CSR), g->edge_slots,
                           g->edge_bits, g->check_part, g->small, s);
  if (e == hipSuccess) e = hipMemcpyAsync(g->h_stage, g->small, 8 * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return status_of(e);
  const uint64_t* h = g->h_stage;
  uint32_t bits = (uint32_t)(h[kWErr] & 0xFFFFFFFFu);
  if (bits) return (moss_status)validate_error_status(bits);  // a full hash set reads as overflow
  g->max_degree = (int32_t)h[kWMaxDeg];
  g->n_items = (int64_t)h[kWItems];
  g->row_guide_len = (int64_t)h[kWGuideLen];
  if (g->n_items > cap) return MOSS_E_ARG;
  if (!(g->flags & MOSS_TRUST_CSR) && 2 * h[kWUpper] != (uint64_t)g->nnz) return MOSS_E_ASYMMETRIC;
  return MOSS_OK;
}

moss_status create_common(int32_t n, int64_t nnz, uint32_t flags, void* hip_stream, moss_graph** out,
                          moss_graph** made) {
  *made = nullptr;
  if (!out || n < 0 || nnz < 0 || nnz >= (int64_t)1 << 31 || (n == 0 && nnz != 0)) return MOSS_E_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MOSS_E_DEVICE;
  moss_status st = ensure_device(dev);
  if (st != MOSS_OK) return st;
  moss_graph* g = new (std::nothrow) moss_graph();
  if (!g) return MOSS_E_NOMEM;
  g->device = dev;
  g->stream = (hipStream_t)hip_stream;
  g->n = n;
  g->nnz = nnz;
  g->flags = flags;
  int bits = 1;
  while (bits < 30 && (1ll << bits) < 2ll * (int64_t)std::max(n, 1)) ++bits;
  g->gbits = std::min(bits, 23);
  *made = g;
  return MOSS_OK;
}

}  // namespace

namespace moss {
moss_status device_block_alloc(hipStream_t s, void** p, size_t bytes) { return dev_alloc_bytes(s, p, bytes); }
void device_block_free(hipStream_t s, void*& p) { dev_free(s, p); }
}  // namespace moss

extern "C" {

const char* moss_status_string(moss_status s) {
  switch (s) {
    case MOSS_OK: return "ok";
    case MOSS_E_ARG: return "invalid argument or malformed CSR";
    case MOSS_E_UNSORTED: return "CSR row not strictly ascending";
    case MOSS_E_SELF_LOOP: return "self-loop in CSR";
    case MOSS_E_DUPLICATE: return "duplicate neighbour in CSR";
    case MOSS_E_ASYMMETRIC: return "CSR not symmetric";
    case MOSS_E_OVERFLOW: return "integer overflow in sampling tables";
    case MOSS_E_NOMEM: return "out of memory";
    case MOSS_E_DEVICE: return "HIP device error";
    case MOSS_E_NOT_BUILT: return "tables not built";
    case MOSS_E_BUSY: return "graph busy";
    case MOSS_E_TIMEOUT: return "timed out";
    case MOSS_E_CANCELLED: return "cancelled";
    case MOSS_E_ADMISSION: return "request can never be admitted";
    case MOSS_E_TOO_LARGE: return "sample range larger than the fixed scratch of the no-allocation call";
  }
  return "unknown status";
}

moss_status moss_graph_create(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, uint32_t flags,
                              void* hip_stream, moss_graph** out) {
  if (!row_ptr || (nnz > 0 && !col)) return MOSS_E_ARG;
  moss_graph* g = nullptr;
  moss_status st = create_common(n, nnz, flags, hip_stream, out, &g);
  if (st != MOSS_OK) return st;
  DeviceScope scope(g->device);
  const size_t rp_bytes = (((size_t)n + 1) * sizeof(int32_t) + 255) & ~(size_t)255;
  void* csr = nullptr;
  st = dev_alloc_bytes(g->stream, &csr, rp_bytes + (size_t)nnz * sizeof(int32_t));
  if (st == MOSS_OK) {
    g->owned_rp = at<int32_t>(csr, 0);
    g->owned_col = at<int32_t>(csr, rp_bytes);
    hipError_t e = hipMemcpyAsync(g->owned_rp, row_ptr, ((size_t)n + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                                  g->stream);
    if (e == hipSuccess && nnz > 0)
      e = hipMemcpyAsync(g->owned_col, col, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice, g->stream);
    st = status_of(e);  // the checks below end in a synchronisation before the call returns
  }
  if (st == MOSS_OK) {
    g->rp = g->owned_rp;
    g->col = g->owned_col;
    g->csr_bytes = ((uint64_t)n + 1 + (uint64_t)nnz) * sizeof(int32_t);
    st = finish_create(g);
  }
  if (st != MOSS_OK) {
    destroy_graph(g);
    return st;
  }
  *out = g;
  return MOSS_OK;
}

moss_status moss_graph_create_device(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
                                     uint32_t flags, void* hip_stream, moss_graph** out) {
  if (!d_row_ptr || (nnz > 0 && !d_col)) return MOSS_E_ARG;
  moss_graph* g = nullptr;
  moss_status st = create_common(n, nnz, flags, hip_stream, out, &g);
  if (st != MOSS_OK) return st;
  DeviceScope scope(g->device);
  g->rp = d_row_ptr;
  g->col = d_col;
  st = finish_create(g);
  if (st != MOSS_OK) {
    destroy_graph(g);
    return st;
  }
  *out = g;
  return MOSS_OK;
}

moss_status moss_graph_destroy(moss_graph* g) {
  if (!g) return MOSS_E_ARG;
  if (g->busy.load() != 0) return MOSS_E_BUSY;
  destroy_graph(g);
  return MOSS_OK;
}

moss_status moss_build_tables(moss_graph* g, uint32_t k_mask) {
  GraphClaim claim(g);
  if (!g) return MOSS_E_ARG;
  if (!claim.ok()) return MOSS_E_BUSY;
  return build_tables(g, k_mask);
}

moss_status moss_graph_get_info(const moss_graph* g, moss_graph_info* info) {
  if (!g || !info) return MOSS_E_ARG;
  moss_graph_info r{};
  r.n = g->n;
  r.max_degree = g->max_degree;
  r.nnz = g->nnz;
  r.built_mask = g->built;
  r.gamma = g->total[0];
  r.gamma1 = g->total[1];
  r.gamma2 = g->total[2];
  r.lambda3 = g->lambda3;
  r.lambda4 = g->lambda4;
  r.device_bytes = g->table_bytes + (g->owned_rp ? g->csr_bytes : 0);
  r.gamma_min = g->total[3];
  r.sampling_bytes = sampling_footprint(g);
  *info = r;
  return MOSS_OK;
}

moss_status moss_table_read(const moss_graph* g, int32_t which, void* host_out, int64_t count) {
  if (!g || !host_out) return MOSS_E_ARG;
  const void* src = nullptr;
  size_t bytes = 0;
  switch (which) {
    case MOSS_TAB_ACC_GAMMA:
    case MOSS_TAB_ACC_GAMMA1:
    case MOSS_TAB_ACC_GAMMA2: {
      if (count != g->n) return MOSS_E_ARG;
      const int s = which - MOSS_TAB_ACC_GAMMA;
      if (!(g->built & (s == 0 ? MOSS_TABLES_K4 : MOSS_TABLES_K5))) return MOSS_E_NOT_BUILT;
      src = g->acc_node[s];
      bytes = (size_t)g->n * sizeof(uint64_t);
      break;
    }
    case MOSS_TAB_ACC_SIGMA:
      if (count != g->nnz) return MOSS_E_ARG;
      if (!(g->built & (MOSS_TABLES_K4 | MOSS_TABLES_K5))) return MOSS_E_NOT_BUILT;
      src = g->acc_sigma;
      bytes = (size_t)g->nnz * sizeof(uint32_t);
      break;
    case MOSS_TAB_ACC_TAU:
      if (count != g->nnz) return MOSS_E_ARG;
      if (!(g->built & MOSS_TABLES_K5)) return MOSS_E_NOT_BUILT;
      src = g->acc_tau;
      bytes = (size_t)g->nnz * sizeof(uint64_t);
      break;
    case MOSS_TAB_ACC_GAMMA_MIN:
    case MOSS_TAB_ACC_CHECK:
    case MOSS_TAB_RANK:
    case MOSS_TAB_COL_RANK: {
      const bool nodes = which == MOSS_TAB_ACC_GAMMA_MIN;
      if (count != (nodes ? (int64_t)g->n : g->nnz)) return MOSS_E_ARG;
      if (!(g->built & MOSS_TABLES_K4MIN)) return MOSS_E_NOT_BUILT;
      src = nodes ? (const void*)g->acc_node[3]
                  : which == MOSS_TAB_ACC_CHECK ? (const void*)g->acc_check
                  : which == MOSS_TAB_RANK     ? (const void*)g->rank
                                               : (const void*)g->col_rank;
      bytes = (size_t)count * (which == MOSS_TAB_COL_RANK ? sizeof(int32_t) : sizeof(uint64_t));
      break;
    }
    case MOSS_TAB_SIGMA_GUIDE:
    case MOSS_TAB_TAU_GUIDE:
    case MOSS_TAB_CHECK_GUIDE: {
      if (count != g->row_guide_len) return MOSS_E_ARG;
      const uint32_t need = which == MOSS_TAB_SIGMA_GUIDE ? (MOSS_TABLES_K4 | MOSS_TABLES_K5)
                            : which == MOSS_TAB_TAU_GUIDE ? MOSS_TABLES_K5
                                                          : MOSS_TABLES_K4MIN;
      if (!(g->built & need)) return MOSS_E_NOT_BUILT;
      src = which == MOSS_TAB_SIGMA_GUIDE ? (const void*)g->sig_guide
            : which == MOSS_TAB_TAU_GUIDE ? (const void*)g->tau_guide
                                          : (const void*)g->check_guide;
      bytes = (size_t)count * sizeof(uint32_t);
      break;
    }
    default:
      return MOSS_E_ARG;
  }
  if (bytes == 0) return MOSS_OK;
  DeviceScope scope(g->device);
  hipError_t e = hipMemcpyAsync(host_out, src, bytes, hipMemcpyDeviceToHost, g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  return status_of(e);
}

}  // extern "C"

moss_status moss::build_tables(moss_graph* g, uint32_t k_mask) {
  if (k_mask & ~(MOSS_TABLES_K4 | MOSS_TABLES_K5 | MOSS_TABLES_K4MIN)) return MOSS_E_ARG;
  const uint32_t need = k_mask & ~g->built;
  if (!need) return MOSS_OK;
  DeviceScope scope(g->device);
  if (!scope.ok()) return MOSS_E_DEVICE;
  const bool want4 = need & MOSS_TABLES_K4, want5 = need & MOSS_TABLES_K5, want_min = need & MOSS_TABLES_K4MIN;
  // ACC_sigma and its companions come with the first MOSS-4, 5-node or MOSS-4Min set
  // (MOSS-4Min's rank passes read the neighbours' degrees from it)
  const bool want_sig = (want4 || want5 || want_min) && !g->mem_sig;
  moss_status st = MOSS_OK;
  if (want_sig) {
    const SigLayout L = sig_layout(g);
    st = dev_alloc_bytes(g->stream, &g->mem_sig, L.bytes);
    if (st == MOSS_OK) {
      g->acc_sigma = at<uint32_t>(g->mem_sig, L.acc_sigma);
      g->sig_guide = at<uint32_t>(g->mem_sig, L.guide);
    }
  }
  if (st == MOSS_OK && want4) {
    const NodeLayout L = node_layout(g, false);
    st = dev_alloc_bytes(g->stream, &g->mem_k4, L.bytes);
    if (st == MOSS_OK) {
      g->acc_node[0] = at<uint64_t>(g->mem_k4, L.acc[0]);
      g->guide[0] = at<uint32_t>(g->mem_k4, L.guide[0]);
    }
  }
  if (st == MOSS_OK && want5) {
    const NodeLayout L = node_layout(g, true);
    st = dev_alloc_bytes(g->stream, &g->mem_k5, L.bytes);
    if (st == MOSS_OK) {
      g->acc_tau = at<uint64_t>(g->mem_k5, L.acc_tau);
      g->tau_guide = at<uint32_t>(g->mem_k5, L.tau_guide);
      for (int j = 0; j < 2; ++j) {
        g->acc_node[1 + j] = at<uint64_t>(g->mem_k5, L.acc[j]);
        g->guide[1 + j] = at<uint32_t>(g->mem_k5, L.guide[j]);
      }
    }
  }
  if (st == MOSS_OK && want_min) {
    const MinLayout L = min_layout(g);
    st = dev_alloc_bytes(g->stream, &g->mem_min, L.bytes);
    if (st == MOSS_OK) {
      g->rank = at<uint2>(g->mem_min, L.rank);
      g->col_rank = at<int32_t>(g->mem_min, L.col_rank);
      g->acc_check = at<uint64_t>(g->mem_min, L.acc_check);
      g->check_guide = at<uint32_t>(g->mem_min, L.check_guide);
      g->acc_node[3] = at<uint64_t>(g->mem_min, L.acc);
      g->guide[3] = at<uint32_t>(g->mem_min, L.guide);
    }
  }
  if (st != MOSS_OK) {
    (void)hipStreamSynchronize(g->stream);  // the blocks it did get are idle before release
    free_tables(g, need);
    return st;
  }
  hipStream_t s = g->stream;
  uint32_t* err = (uint32_t*)(g->small + kWErr);
  // error bits, Lambdas and totals to zero
  FillSet f{};
  f.p[0] = g->small + kWErr;
  f.count[0] = kWLambda + 2;
  f.p[1] = g->small + kWTotal;
  f.count[1] = 4;
  hipError_t e = launch_fill_set(f, s);
  RowTables t{};
  t.rp = g->rp;
  t.col = g->col;
  t.span_row = g->span_row;
  t.acc_sigma = g->acc_sigma;
  t.span_sums = g->span_sums;
  if (g->max_degree >= kSpanGroupMinDegree) {
    t.span_groups = g->span_groups;
    t.group_wrap = g->group_wrap;
  }
  t.rec = g->rec;
  t.nnz = g->nnz;
  t.n = g->n;
  if (e == hipSuccess && want_sig) {
    t.guide = g->sig_guide;
    e = launch_row_tables(kRowSigma, t, err, s);
  }
  if (e == hipSuccess && want5) {
    t.acc_tau = g->acc_tau;
    t.guide = g->tau_guide;
    e = launch_row_tables(kRowTau, t, err, s);
  }
  if (e == hipSuccess && (want4 || want5))
    e = launch_node_weights(g->n, g->rp, g->rec, want5 ? g->acc_tau : nullptr, want4 ? g->acc_node[0] : nullptr,
                            want5 ? g->acc_node[1] : nullptr, want5 ? g->acc_node[2] : nullptr, g->partials,
                            (unsigned long long*)(g->small + kWLambda), err, s);
  ScanSet scans{};
  GuideSet guides{};
  for (int slot = 0; slot < 3; ++slot) {
    if (!(slot == 0 ? want4 : want5)) continue;
    const int j = scans.count++;
    scans.data[j] = g->acc_node[slot];
    scans.tmp[j] = g->scan_tmp[j];
    scans.err_bit[j] = slot == 0 ? kErrOverflowK4 : kErrOverflowK5;
    guides.acc[j] = g->acc_node[slot];
    guides.guide[j] = g->guide[slot];
    guides.total[j] = g->small + kWTotal + slot;
    guides.count = scans.count;
  }
  if (e == hipSuccess) e = launch_scans(scans, g->n, err, s);
  if (e == hipSuccess) e = launch_guides(guides, g->n, g->gbits, s);
  if (want_min) {
    // ranks (the row prefix array serves as their scratch), the prefix of
    // d_{v,x} d_{x,v} with its row guides, check-Gamma_v, its scan and guide
    if (e == hipSuccess) {
      RankTables rt{};
      rt.n_items = g->n_items;
      rt.items = g->items;
      rt.n = g->n;
      rt.nnz = g->nnz;
      rt.max_degree = g->max_degree;
      rt.validated = !(g->flags & MOSS_TRUST_CSR);
      rt.span_row = g->span_row;
      rt.rp = g->rp;
      rt.col = g->col;
      rt.rec = g->rec;
      rt.acc_sigma = g->acc_sigma;
      rt.scratch = g->acc_check;
      rt.work = at<uint32_t>(g->mem_min, min_layout(g).work);
      rt.rank = g->rank;
      rt.col_rank = g->col_rank;
      e = launch_rank_tables(rt, s);
    }
    if (e == hipSuccess) {
      t.rank = g->rank;
      t.acc_check = g->acc_check;
      t.guide = g->check_guide;
      e = launch_row_tables(kRowCheck, t, err, s);
    }
    if (e == hipSuccess) e = launch_row_totals(g->n, g->rp, g->acc_check, g->acc_node[3], s);
    ScanSet ms{};
    ms.data[0] = g->acc_node[3];
    ms.tmp[0] = g->scan_tmp[0];
    ms.err_bit[0] = kErrOverflowMin;
    ms.count = 1;
    GuideSet mg{};
    mg.acc[0] = g->acc_node[3];
    mg.guide[0] = g->guide[3];
    mg.total[0] = g->small + kWTotal + 3;
    mg.count = 1;
    if (e == hipSuccess) e = launch_scans(ms, g->n, err, s);
    if (e == hipSuccess) e = launch_guides(mg, g->n, g->gbits, s);
  }
  uint64_t* h = g->h_stage;
  if (e == hipSuccess) e = hipMemcpyAsync(h, g->small, kWHits * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  const hipError_t es = hipStreamSynchronize(s);  // also drains work queued before a failed launch
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) {
    free_tables(g, need);
    return status_of(e);
  }
  const uint32_t bits = (uint32_t)(h[kWErr] & 0xFFFFFFFFu);
  if ((want_sig && (bits & kErrOverflow)) || (want4 && (bits & kErrOverflowK4)) ||
      (want5 && (bits & kErrOverflowK5)) || (want_min && (bits & kErrOverflowMin))) {
    free_tables(g, need);
    return MOSS_E_OVERFLOW;
  }
  for (int slot = 0; slot < 4; ++slot)
    if (slot == 0 ? want4 : slot == 3 ? want_min : want5) g->total[slot] = g->n > 0 ? h[kWTotal + slot] : 0;
  if (want4) g->lambda3 = h[kWLambda];
  if (want5) g->lambda4 = h[kWLambda + 1];
  g->built |= need;
  g->table_bytes = table_bytes_needed(g, 0);
  return MOSS_OK;
}

void moss::free_graph_tables(moss_graph* g, uint32_t mask) {
  DeviceScope scope(g->device);
  (void)hipStreamSynchronize(g->stream);
  free_tables(g, mask & (MOSS_TABLES_K4 | MOSS_TABLES_K5 | MOSS_TABLES_K4MIN));
}

// With mask = 0: the bytes held now.  Otherwise the bytes that building `mask` adds.
uint64_t moss::table_bytes_needed(const moss_graph* g, uint32_t mask) {
  const uint64_t sig = sig_layout(g).bytes, k4 = node_layout(g, false).bytes, k5 = node_layout(g, true).bytes;
  const uint32_t have = g->built, add = mask == 0 ? have : (mask & ~have);
  const uint32_t sig_sets = MOSS_TABLES_K4 | MOSS_TABLES_K5 | MOSS_TABLES_K4MIN;  // ACC_sigma comes with any
  uint64_t b = 0;
  if ((add & sig_sets) && (mask == 0 || !(have & sig_sets))) b += sig;
  if (add & MOSS_TABLES_K4) b += k4;
  if (add & MOSS_TABLES_K5) b += k5;
  if (add & MOSS_TABLES_K4MIN) b += min_layout(g).bytes;
  return b;
}

namespace {

// Runs the samplers of one estimate on the graph's stream; hits are copied to `hits`.
// Grouped estimates go chunk by chunk (at most 2^25 samples each), the grouping passes
// and then the sampling launch of each chunk.  (Running the grouping of chunk j on a
// second stream while chunk j - 1 samples measured slower: 0.81 against 0.68 ms for
// 1e7 samples in two halves at n = 1e5, m = 1e6; no gain at n = 1e6, m = 1e7.)
// With `fixed` (a scratch of the caller's, fixed_samples samples per chunk) nothing is
// allocated.
moss_status run_samplers(moss_graph* g, const int* samplers, const uint64_t* k0, const uint64_t* k1, int count,
                         uint64_t seed, uint8_t* class_out, uint64_t hits[][22], double* device_ms,
                         void* fixed = nullptr, uint64_t fixed_samples = 0) {
  hipStream_t s = g->stream;
  unsigned long long* d_hits = (unsigned long long*)(g->small + kWHits);
  // XCD-grouped launches sort each chunk of at most 2^25 samples by group (6 bytes per
  // sample of scratch)
  void* scratch = nullptr;
  uint64_t max_n = 0;
  for (int i = 0; i < count; ++i) max_n = std::max<uint64_t>(max_n, k1[i] > k0[i] ? k1[i] - k0[i] : 0);
  if (grouped_schedule(g, max_n)) {
    if (fixed) {
      max_n = std::min<uint64_t>(max_n, fixed_samples);
      scratch = fixed;
    } else {
      max_n = std::min<uint64_t>(max_n, 1ull << 25);
      if (max_n > 0 && dev_alloc_bytes(s, &scratch, (size_t)grouped_scratch_bytes(max_n)) != MOSS_OK)
        return MOSS_E_NOMEM;
    }
  }
  // (with a scratch block, every launch below runs grouped; chunks of at most max_n)
  const uint32_t window = sort_window_for(g);
  hipError_t e = launch_fill_u64(g->small + kWHits, 0, 2 * 22, s);
  if (e == hipSuccess) e = hipEventRecord(g->ev0, s);
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    const int slot = sampler_slot(samplers[i]);
    if (g->total[slot] == 0 || k1[i] <= k0[i]) continue;
    int grid, block;
    plain_launch_shape(g, samplers[i], k1[i] - k0[i], &grid, &block);
    const SamplerView view = sampler_view(g, samplers[i]);
    if (!scratch) {
      e = launch_sample(samplers[i], view, seed, k0[i], k1[i], d_hits + 22 * i, class_out, grid, block, s);
      continue;
    }
    for (uint64_t a = k0[i]; a < k1[i] && e == hipSuccess; a += max_n) {
      const uint64_t n = std::min<uint64_t>(max_n, k1[i] - a);
      e = launch_group_chunk(samplers[i], seed, a, n, scratch, max_n, s);
      if (e == hipSuccess)
        e = launch_sample_chunk(samplers[i], view, seed, a, n, scratch, max_n, window, d_hits + 22 * i,
                                class_out ? class_out + (a - k0[i]) : nullptr, grid, block, s);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(g->ev1, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(g->h_stage, d_hits, 2 * 22 * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  const hipError_t es = hipStreamSynchronize(s);
  if (e == hipSuccess) e = es;
  if (scratch != fixed) dev_free(s, scratch);  // idle after the synchronisation
  if (e != hipSuccess) return status_of(e);
  for (int i = 0; i < count; ++i) std::memcpy(hits[i], g->h_stage + 22 * i, 22 * sizeof(uint64_t));
  float ms = 0.f;
  if (device_ms) *device_ms = hipEventElapsedTime(&ms, g->ev0, g->ev1) == hipSuccess ? (double)ms : 0.0;
  return MOSS_OK;
}

bool valid_sampler(int s) { return s == kMoss4 || s == kMoss4Min || s == kT5 || s == kPath5; }

}  // namespace

extern "C" {

moss_status moss_estimate(moss_graph* g, int32_t k, uint64_t n_samples, uint64_t seed, uint32_t flags,
                          moss_result* out) {
  EstimatePlan plan;
  if (!g || !out || plan_estimate(k, n_samples, flags, &plan) != MOSS_OK) return MOSS_E_ARG;
  GraphClaim claim(g);
  if (!claim.ok()) return MOSS_E_BUSY;
  DeviceScope scope(g->device);
  if (!scope.ok()) return MOSS_E_DEVICE;
  moss_status st = build_tables(g, plan.tables);
  if (st != MOSS_OK) return st;
  moss_result r;
  result_header(g, k, n_samples, flags, &r);
  const uint64_t k0[2] = {0, 0};
  st = run_samplers(g, plan.sampler, k0, plan.K, plan.count, seed, nullptr, r.hits, &r.device_ms);
  if (st != MOSS_OK) return st;
  st = moss_finals(&r);
  if (st != MOSS_OK) return st;
  *out = r;
  return MOSS_OK;
}

moss_status moss_estimate_to_precision(moss_graph* g, int32_t k, double eps, double delta, uint32_t motif_mask,
                                       uint64_t pilot_samples, uint64_t pilot_seed, uint64_t max_samples,
                                       uint64_t seed, uint32_t flags, moss_result* out) {
  EstimatePlan plan;
  if (!g || !out || plan_estimate(k, 2, flags, &plan) != MOSS_OK) return MOSS_E_ARG;
  const uint64_t least = plan_estimate(k, 1, flags, &plan) == MOSS_OK ? 1 : 2;
  if (pilot_samples < least || max_samples < least || !(eps > 0.0) || !(delta > 0.0) || !(delta < 1.0))
    return MOSS_E_ARG;
  moss_result pilot;
  moss_status st = moss_estimate(g, k, pilot_samples, pilot_seed, flags, &pilot);
  if (st != MOSS_OK) return st;
  uint64_t budget[21], K = 0;
  st = moss_plan_budget(&pilot, eps, delta, motif_mask, budget, &K);
  if (st != MOSS_OK) return st;
  if (K == 0) K = pilot_samples;
  K = std::min(std::max(K, least), max_samples);
  return moss_estimate(g, k, K, seed, flags, out);
}

moss_status moss_sample_range(moss_graph* g, int32_t sampler, uint64_t seed, uint64_t k0, uint64_t k1,
                              uint8_t* d_class_out, uint64_t hits[22]) {
  if (!g || !hits || !valid_sampler(sampler) || k1 < k0) return MOSS_E_ARG;
  GraphClaim claim(g);
  if (!claim.ok()) return MOSS_E_BUSY;
  DeviceScope scope(g->device);
  if (!scope.ok()) return MOSS_E_DEVICE;
  moss_status st = build_tables(g, sampler_tables(sampler));
  if (st != MOSS_OK) return st;
  uint64_t h[2][22];
  const int samplers[1] = {sampler};
  const uint64_t a[1] = {k0}, b[1] = {k1};
  if (d_class_out && g->total[sampler_slot(sampler)] == 0 && k1 > k0) {
    hipError_t e = hipMemsetAsync(d_class_out, 0, (size_t)(k1 - k0), g->stream);
    if (e != hipSuccess) return status_of(e);
  }
  st = run_samplers(g, samplers, a, b, 1, seed, d_class_out, h, nullptr);
  if (st != MOSS_OK) return st;
  std::memcpy(hits, h[0], sizeof(h[0]));
  return MOSS_OK;
}

moss_status moss_sample_range_noalloc(moss_graph* g, int32_t sampler, uint64_t seed, uint64_t k0, uint64_t k1,
                                      uint8_t* d_class_out, uint64_t hits[22]) {
  if (!g || !hits || !valid_sampler(sampler) || k1 < k0) return MOSS_E_ARG;
  if (k1 - k0 > MOSS_NOALLOC_MAX_SAMPLES) return MOSS_E_TOO_LARGE;
  static_assert(MOSS_NOALLOC_MAX_SAMPLES == kFixedScratchSamples, "the header states the fixed scratch's size");
  GraphClaim claim(g);
  if (!claim.ok()) return MOSS_E_BUSY;
  DeviceScope scope(g->device);
  if (!scope.ok()) return MOSS_E_DEVICE;
  const uint32_t need = sampler_tables(sampler);
  if ((g->built & need) != need) return MOSS_E_NOT_BUILT;
  void* fixed = nullptr;
  hipError_t e = fixed_scratch(g->device, &fixed);
  if (e != hipSuccess) return status_of(e);
  std::lock_guard<std::mutex> lk(fixed_scratch_lock(g->device));  // one user of the array at a time
  if (d_class_out && g->total[sampler_slot(sampler)] == 0 && k1 > k0) {
    e = launch_fill_u8(d_class_out, 0, (int64_t)(k1 - k0), g->stream);
    if (e != hipSuccess) return status_of(e);
  }
  uint64_t h[2][22];
  const int samplers[1] = {sampler};
  const uint64_t a[1] = {k0}, b[1] = {k1};
  moss_status st = run_samplers(g, samplers, a, b, 1, seed, d_class_out, h, nullptr, fixed, kFixedScratchSamples);
  if (st != MOSS_OK) return st;
  std::memcpy(hits, h[0], sizeof(h[0]));
  return MOSS_OK;
}

moss_status moss_sample_nodes(moss_graph* g, int32_t sampler, uint64_t seed, const uint64_t* d_index, int64_t count,
                              int32_t* d_nodes_out, uint8_t* d_class_out) {
  if (!g || !valid_sampler(sampler) || count < 0 || (count > 0 && (!d_index || !d_nodes_out))) return MOSS_E_ARG;
  GraphClaim claim(g);
  if (!claim.ok()) return MOSS_E_BUSY;
  DeviceScope scope(g->device);
  if (!scope.ok()) return MOSS_E_DEVICE;
  moss_status st = build_tables(g, sampler_tables(sampler));
  if (st != MOSS_OK) return st;
  if (g->total[sampler_slot(sampler)] == 0) return count == 0 ? MOSS_OK : MOSS_E_ARG;  // nothing can be drawn
  hipError_t e = launch_sample_nodes(sampler, sampler_view(g, sampler), seed, d_index, count, d_nodes_out,
                                     d_class_out, g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  return status_of(e);
}

}  // extern "C"
