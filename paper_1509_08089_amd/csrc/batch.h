// Batched execution shared by moss_estimate_batch and the server.
#pragma once
#include <cstdint>
#include <vector>

#include "internal.h"

namespace moss {

// Samples [k0, k1) of one sampler on one graph, counted into histogram slot `slot`.
struct WorkItem {
  moss_graph* g;
  int sampler;
  uint64_t seed;
  uint64_t k0, k1;
  uint32_t slot;
};

// Device-side state of batched launches on one device: tile list buffers, the
// per-slot histograms and the captured hipGraph of (clear, persistent kernel).
class BatchRunner {
 public:
  explicit BatchRunner(int device);
  ~BatchRunner();
  BatchRunner(const BatchRunner&) = delete;
  BatchRunner& operator=(const BatchRunner&) = delete;

  // Runs every work item in one persistent launch; bins_out receives n_slots x 22
  // counters.  `wait_on` (may be null) is a stream whose queued work must finish
  // first.  tile_samples / blocks_per_cu of 0 use the current tuning.  With
  // `sort_large`, items with many samples on graphs past the L2s run instead as grouped
  // launches of their own (the plain path's grouping passes and sorted sampling
  // kernel), beside the persistent kernel, adding into their histogram slots.
  moss_status run(const std::vector<WorkItem>& work, uint32_t n_slots, uint64_t* bins_out, double* device_ms,
                  hipStream_t wait_on, uint32_t tile_samples = 0, uint32_t blocks_per_cu = 0,
                  bool sort_large = false);

  int device() const { return device_; }

  // Frees the runner's device buffers, graph and stream (the runner stays usable).
  void release();

 private:
  moss_status reserve(size_t views, size_t items, size_t slots);
  moss_status capture(int grid, int block);

  int device_;
  hipStream_t stream_ = nullptr;
  hipStream_t side_[2] = {};  // the grouped launches in two chains, beside the persistent kernel
  hipEvent_t ev0_ = nullptr, ev1_ = nullptr, ev_wait_ = nullptr, ev_clear_ = nullptr, ev_side_[2] = {};
  SamplerView* d_views_ = nullptr;
  BatchItem* d_items_ = nullptr;
  uint32_t* d_ctl_ = nullptr;  // control words (kCtl*)
  unsigned long long* d_bins_ = nullptr;
  size_t cap_views_ = 0, cap_items_ = 0, cap_slots_ = 0;
  unsigned char* h_in_ = nullptr;  // pinned staging for views + items + control words
  size_t cap_in_ = 0;
  uint64_t* h_bins_ = nullptr;     // pinned, cap_slots_ x 22
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
  int graph_grid_ = 0, graph_block_ = 0;
};

// The process-wide runner of a device (created on first use).
BatchRunner* batch_runner(int device);

// Fills a moss_result's header fields (k, K, gamma, lambda, flags) for a request.
void result_header(const moss_graph* g, int32_t k, uint64_t n_samples, uint32_t flags, moss_result* r);

}  // namespace moss
