// Host-side declarations of the HIP kernels' launchers (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace moss {

// Sampler ids double as Philox key tags.
constexpr int kMoss4 = 0x4;
constexpr int kT5 = 0x51;
constexpr int kPath5 = 0x52;

// Error bits raised by the device-side checks.
constexpr uint32_t kErrArg = 1u << 0;
constexpr uint32_t kErrUnsorted = 1u << 1;
constexpr uint32_t kErrSelfLoop = 1u << 2;
constexpr uint32_t kErrDuplicate = 1u << 3;
constexpr uint32_t kErrAsymmetric = 1u << 4;
constexpr uint32_t kErrOverflow = 1u << 5;    // a row sum S_v needs more than 32 bits (all tables)
constexpr uint32_t kErrOverflowK4 = 1u << 6;  // Gamma prefix or Lambda_3 exceeds 64 bits
constexpr uint32_t kErrOverflowK5 = 1u << 7;  // a Gamma^(1)/Gamma^(2) value or prefix, or Lambda_4

// What one sampler needs of one graph.
struct SamplerView {
  const int32_t* rp;          // row_ptr[n+1]
  const int32_t* col;         // col[nnz], rows ascending
  const uint4* rec;           // per node: row start, degree, S_v, row-guide offset
  const uint64_t* acc_node;   // inclusive prefix of the node weights of this sampler
  const uint32_t* guide;      // guide[0..2^gbits]: node-draw search windows
  const uint32_t* acc_sigma;  // row-local inclusive prefix of d_x - 1
  const uint64_t* acc_tau;    // row-local inclusive prefix of the tau weights (Path-5)
  const uint32_t* sig_guide;  // row guides over ACC_sigma (rows with d >= kRowGuideMin)
  const uint32_t* tau_guide;  // row guides over ACC_tau (Path-5)
  const uint64_t* edge_slots; // edge hash set: 2^edge_bits slots, key min << 32 | max
  uint64_t total;             // sum of the node weights
  int32_t n;
  int32_t gbits;
  int32_t edge_bits;
  int32_t pad;
};

// Rows with at least this many entries get a guide table for their weighted picks.
constexpr int32_t kRowGuideMin = 64;

// One unit of batched work: samples [k0, k1) of one sampler on one graph.
struct Tile {
  uint32_t view;     // index into the SamplerView array
  uint32_t sampler;  // kMoss4 / kT5 / kPath5
  uint32_t out;      // histogram slot (22 counters each)
  uint32_t pad;
  uint64_t seed;
  uint64_t k0, k1;
};

hipError_t upload_class_luts(const uint8_t lut4[8], const uint8_t lut5t[64], const uint8_t lut5p[64]);

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t value, int64_t count, hipStream_t s);

hipError_t launch_check_rowptr(int32_t n, int64_t nnz, const int32_t* rp, uint32_t* err, hipStream_t s);
// Work items: rows cut into pieces of at most 256 entries.  item_end (n u64) receives
// the inclusive prefix of the piece counts; items (at most n + nnz/256 + 1 u64) the
// packed (row, piece) pairs; the item count is item_end[n-1].
hipError_t launch_items(int32_t n, const int32_t* rp, uint64_t* item_end, uint64_t* items, uint64_t* tmp,
                        uint32_t* err, hipStream_t s);
// n_items: device word holding the item count; max_items bounds it (grid size)
hipError_t launch_check_items(int64_t max_items, const uint64_t* n_items, const uint64_t* items, int32_t n,
                              const int32_t* rp, const int32_t* col, bool full, uint32_t* err, hipStream_t s);

// Row prefixes ACC_sigma (tau = false) or ACC_tau (tau = true, needs ACC_sigma);
// item_sum holds n_items u64, tmp scan_tmp_elems(n_items) u64.
hipError_t launch_row_prefix(bool tau, int64_t n_items, const uint64_t* items, const int32_t* rp, const int32_t* col,
                             uint32_t* acc_sigma, uint64_t* acc_tau, uint64_t* item_sum, uint64_t* tmp, uint32_t* err,
                             hipStream_t s);

// Row guides.  row_guide_sizes: per node the guide length (0, or 2^g + 1 with
// g = floor(log2 d) - 1 when d >= kRowGuideMin) into sizes (n u64, scanned in place
// afterwards by the caller into inclusive ends).  records: rec[v] = {row start,
// degree, S_v, guide offset}.  row_guides: fills the guides of ACC_sigma (tau=false)
// or ACC_tau (tau=true); goff_end is the scanned sizes array.
hipError_t launch_row_guide_sizes(int32_t n, const int32_t* rp, uint64_t* sizes, hipStream_t s);
hipError_t launch_records(int32_t n, const int32_t* rp, const uint32_t* acc_sigma, const uint64_t* goff_end,
                          uint4* rec, hipStream_t s);
hipError_t launch_row_guides(bool tau, int64_t n_items, const uint64_t* items, const int32_t* rp, const uint4* rec,
                             const uint32_t* acc_sigma, const uint64_t* acc_tau, uint32_t* guide, hipStream_t s);

// Edge hash set over the undirected edges (slots: 2^bits u64, filled with the empty
// key first); bits is chosen by the caller so that the load factor stays low.
int edge_hash_bits(int64_t m);
hipError_t launch_edge_hash(int64_t n_items, const uint64_t* items, const int32_t* rp, const int32_t* col,
                            uint64_t* slots, int bits, uint32_t* err, hipStream_t s);

// Node weights (any output may be null) and Lambda_3, Lambda_4 into lambdas[0..1];
// partials must hold 2 * node_weight_blocks(n) u64.
int node_weight_blocks(int32_t n);
hipError_t launch_node_weights(int32_t n, const int32_t* rp, const uint32_t* acc_sigma, const uint64_t* acc_tau,
                               uint64_t* w_gamma, uint64_t* w_gamma1, uint64_t* w_gamma2, uint64_t* partials,
                               unsigned long long* lambdas, uint32_t* err, hipStream_t s);

// In-place inclusive scan of u64[n]; `tmp` must hold scan_tmp_elems(n) u64; a wrap
// sets `err_bit` in *err.
int64_t scan_tmp_elems(int64_t n);
hipError_t launch_scan_inplace(uint64_t* data, int64_t n, uint64_t* tmp, uint32_t* err, uint32_t err_bit,
                               hipStream_t s);

// The total is read on the device (acc[n-1]).
hipError_t launch_guide(const uint64_t* acc, int32_t n, int gbits, uint32_t* guide, hipStream_t s);

// Plain sampling launch: samples [k0, k1) of one sampler, hits[22] accumulated.
hipError_t launch_sample(int sampler, const SamplerView& v, uint64_t seed, uint64_t k0, uint64_t k1,
                         unsigned long long* hits, uint8_t* class_out, int grid, int block, hipStream_t s);

hipError_t launch_sample_nodes(int sampler, const SamplerView& v, uint64_t seed, const uint64_t* index,
                               int64_t count, int32_t* nodes_out, uint8_t* class_out, hipStream_t s);

// Batched persistent launch over a tile list resident in device memory.
hipError_t launch_batch(const SamplerView* views, const Tile* tiles, const uint32_t* n_tiles,
                        uint32_t* tile_counter, unsigned long long* bins, int grid, int block, hipStream_t s);

// Registers/VGPR usage probe for occupancy decisions (max active blocks per CU).
int sample_kernel_blocks_per_cu(int sampler, int block);

}  // namespace moss
