// Library-internal declarations shared by the host sources.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "kernels.h"
#include "moss.h"

struct moss_graph {
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t n = 0;
  int64_t nnz = 0;
  int32_t max_degree = 0;
  const int32_t* rp = nullptr;
  const int32_t* col = nullptr;
  int32_t* owned_rp = nullptr;  // set when the CSR was copied from the host
  int32_t* owned_col = nullptr;
  uint32_t flags = 0;

  // Device memory comes in stream-ordered blocks: per graph (word block, edge hash set
  // and filter, work items, node records, scan scratch), and per table set (ACC_sigma
  // with its row guides; the MOSS-4 node table; the 5-node tables; the MOSS-4Min
  // tables).
  void* mem_graph = nullptr;
  void* mem_sig = nullptr;
  void* mem_k4 = nullptr;
  void* mem_k5 = nullptr;
  void* mem_min = nullptr;

  // per graph (mem_graph)
  uint64_t* small = nullptr;             // kWords words shared with the kernels
  uint64_t* items = nullptr;             // work items: rows cut into pieces of <= 256 entries
  uint64_t* item_sum = nullptr;          // n: piece counts, scanned into each row's item end (creation)
  uint64_t* guide_len = nullptr;         // n, row-guide lengths (creation only)
  uint64_t* scan_tmp[3] = {};            // block sums of up to three scans
  uint64_t* partials = nullptr;          // per-block Lambda partial sums
  uint4* rec = nullptr;                  // per node: row start, degree, S_v, row-guide offset
  int32_t* span_row = nullptr;           // per span of 256 entries: the row of its first entry
  uint64_t* check_part = nullptr;        // per-block counts of the creation check
  uint64_t* span_sums = nullptr;         // 2 per span: the row-prefix passes' span sums
  uint64_t* span_groups = nullptr;       // per 64 spans: their summed span sums
  uint32_t* group_wrap = nullptr;        // per 64 spans: whether that sum wrapped
  int64_t n_items = 0;
  int64_t row_guide_len = 0;             // entries of one row-guide array

  // sampling tables
  uint32_t* acc_sigma = nullptr;    // nnz
  uint32_t* sig_guide = nullptr;    // row guides over ACC_sigma
  uint64_t* edge_slots = nullptr;   // edge hash set for the induced-edge probes
  uint64_t* filter = nullptr;       // edge filter in front of it
  int edge_bits = 4;
  int filter_bits = 1;
  uint64_t* acc_tau = nullptr;      // nnz
  uint32_t* tau_guide = nullptr;    // row guides over ACC_tau
  uint2* rank = nullptr;            // nnz: {d_{v,x}, d_{x,v}} (MOSS-4Min)
  int32_t* col_rank = nullptr;      // nnz: rows in descending order (MOSS-4Min)
  uint64_t* acc_check = nullptr;    // nnz: row prefix of d_{v,x} d_{x,v} (MOSS-4Min)
  uint32_t* check_guide = nullptr;  // row guides over acc_check
  // n each: Gamma (MOSS-4), Gamma^(1) (T-5), Gamma^(2) (Path-5), check-Gamma (MOSS-4Min)
  uint64_t* acc_node[4] = {};
  uint32_t* guide[4] = {};          // 2^gbits + 1 each
  int gbits = 1;
  uint64_t total[4] = {};
  uint64_t lambda3 = 0, lambda4 = 0;
  uint32_t built = 0;               // MOSS_TABLES_* bits

  uint64_t* h_stage = nullptr;      // pinned host staging, kWords words
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  std::atomic<int> busy{0};
  uint64_t csr_bytes = 0;
  uint64_t table_bytes = 0;
};

namespace moss {

// index of a sampler's node distribution / tables
inline int sampler_slot(int sampler) {
  return sampler == kMoss4 ? 0 : sampler == kT5 ? 1 : sampler == kPath5 ? 2 : 3;
}

// the table sets a sampler reads
inline uint32_t sampler_tables(int sampler) {
  return sampler == kMoss4 ? MOSS_TABLES_K4 : sampler == kMoss4Min ? MOSS_TABLES_K4MIN : MOSS_TABLES_K5;
}

// The samplers of one estimate: MOSS-4 alone, MOSS-4 with MOSS-4Min (k = 4 and
// MOSS_K4_MIN) or T-5 with Path-5 (k = 5); two samplers split the budget as
// ceil(n/2), floor(n/2).
struct EstimatePlan {
  int count = 0;
  int sampler[2] = {0, 0};
  uint64_t K[2] = {0, 0};
  uint32_t tables = 0;
};
// MOSS_E_ARG for a bad k, flag or budget.
moss_status plan_estimate(int32_t k, uint64_t n_samples, uint32_t flags, EstimatePlan* p);

moss_status status_of(hipError_t e);

// Sets the device for the scope of the object and restores the previous one.
class DeviceScope {
 public:
  explicit DeviceScope(int device);
  ~DeviceScope();
  bool ok() const { return ok_; }

 private:
  int prev_ = -1;
  bool ok_ = false;
};

// Per-device one-time set-up (classification tables in constant memory).
moss_status ensure_device(int device);
int device_cus(int device);

// Classification tables (sample probe bits -> motif id), computed on the host.
void class_luts(uint8_t lut4[8], uint8_t lut5t[64], uint8_t lut5p[64]);

SamplerView sampler_view(const moss_graph* g, int sampler);
moss_status build_tables(moss_graph* g, uint32_t mask);
// Frees the tables of `mask` (waits for the graph's stream first).
void free_graph_tables(moss_graph* g, uint32_t mask);
// Device bytes that building `mask` would add to the graph.
uint64_t table_bytes_needed(const moss_graph* g, uint32_t mask);

// Launch shape of the plain sampling kernel for `nsamples` samples of graph g (the
// process-wide tuning if set, else resident waves chosen by the graph's footprint).
void plain_launch_shape(const moss_graph* g, int sampler, uint64_t nsamples, int* grid, int* block);
int sampling_waves_per_cu(uint64_t footprint_bytes);
uint64_t sampling_footprint(const moss_graph* g);
bool grouped_schedule(const moss_graph* g, uint64_t nsamples);
// Device blocks from the library's stream-ordered cache (freed blocks are kept for reuse).
moss_status device_block_alloc(hipStream_t s, void** p, size_t bytes);
void device_block_free(hipStream_t s, void*& p);

struct Tuning {
  uint32_t tile_samples = 0;
  uint32_t blocks_per_cu = 0;
  uint32_t threads_per_block = 0;
  uint32_t schedule = 0;  // MOSS_SCHEDULE_*
  uint32_t group_min_samples_log2 = 0;  // batched items drawn grouped: at least 2^x samples (0 = default)
  uint32_t group_min_footprint_mb = 0;  // ... on graphs whose sampled bytes reach x MB (0 = default)
  uint32_t sort_window = 0;             // samples per window of the sorted kernel (0 = by footprint)
};

// The sorted sampling kernel's window on g: the tuning's, else by the sampled bytes.
uint32_t sort_window_for(const moss_graph* g);
Tuning current_tuning();

// RAII claim on a graph for the duration of a call (MOSS_E_BUSY when taken).
class GraphClaim {
 public:
  explicit GraphClaim(moss_graph* g);
  ~GraphClaim();
  bool ok() const { return ok_; }

 private:
  moss_graph* g_;
  bool ok_;
};

}  // namespace moss
