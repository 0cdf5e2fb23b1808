// Host-side declarations of the HIP kernels' launchers (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

namespace moss {

// Sampler ids double as Philox key tags.
constexpr int kMoss4 = 0x4;
constexpr int kMoss4Min = 0x41;
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
constexpr uint32_t kErrOverflowMin = 1u << 8; // a row or node prefix of the MOSS-4Min weights exceeds 64 bits

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
  const uint64_t* filter;     // edge filter: 2^filter_bits words of 64 bits
  const uint2* rank;          // MOSS-4Min, per entry (v, x): {d_{v,x}, d_{x,v}}
  const int32_t* col_rank;    // MOSS-4Min: each row in descending order (N_{v,x} = its first d_{v,x})
  const uint64_t* acc_check;  // MOSS-4Min: row-local inclusive prefix of d_{v,x} d_{x,v}
  const uint32_t* check_guide;  // row guides over acc_check
  uint64_t total;             // sum of the node weights
  int32_t n;
  int32_t gbits;
  int32_t edge_bits;
  int32_t filter_bits;
};

// Per-graph block of 64-bit words shared by the kernels and the host (one copy back
// per call instead of one per value).
constexpr int kWErr = 0;       // error bits (u32, low half)
constexpr int kWLambda = 2;    // Lambda_3, Lambda_4
constexpr int kWItems = 4;     // number of work items
constexpr int kWGuideLen = 5;  // entries of one row-guide array
constexpr int kWUpper = 6;     // CSR entries (v, c) with c > v
constexpr int kWMaxDeg = 7;    // largest degree
constexpr int kWTotal = 8;     // totals of the Gamma, Gamma^(1), Gamma^(2), check-Gamma node weights
constexpr int kWHits = 16;     // 2 x 22 hit counters of a plain estimate
constexpr int kWords = 64;

// Rows with at least this many entries get a guide table for their weighted picks.
constexpr int32_t kRowGuideMin = 64;

// One item of batched work: samples [k0, k1) of one sampler on one graph, cut into tiles
// of the launch's tile size; its tiles are numbered from first_tile on (the items of a
// launch in order, each with at least one tile).
struct BatchItem {
  uint32_t view;        // index into the SamplerView array
  uint32_t sampler;     // kMoss4 / kMoss4Min / kT5 / kPath5
  uint32_t out;         // histogram slot (22 counters each)
  uint32_t first_tile;  // tiles of the items before it
  uint64_t seed;
  uint64_t k0, k1;      // sample indices
};

// Control words of a batched launch: tiles in all, the tile counter (cleared by the
// launch), items, samples per tile.
constexpr int kCtlTiles = 0, kCtlCounter = 1, kCtlItems = 2, kCtlTileSize = 3;

hipError_t upload_class_luts(const uint8_t lut4[8], const uint8_t lut5t[64], const uint8_t lut5p[64]);

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t value, int64_t count, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t value, int64_t count, hipStream_t s);

// Up to four fills of u64 ranges in one launch (unused entries: count 0).
struct FillSet {
  uint64_t* p[4];
  int64_t count[4];
  uint64_t value[4];
};
hipError_t launch_fill_set(const FillSet& f, hipStream_t s);

// In-place inclusive scans of up to three u64 arrays of length n in one set of
// launches.  tmp[j] must hold scan_tmp_elems(n) u64; a wrap sets err_bit[j] in *err;
// total[j] (may be null) receives the array's total.
struct ScanSet {
  uint64_t* data[3];
  uint64_t* tmp[3];
  uint64_t* total[3];
  uint32_t err_bit[3];
  int count;
};
int64_t scan_tmp_elems(int64_t n);
hipError_t launch_scans(const ScanSet& set, int64_t n, uint32_t* err, hipStream_t s);

// ---- graph creation (CSR validation and work items) ----
// Work items: every row cut into pieces of at most 256 entries; items_cap =
// n + nnz / 256 + 1 bounds their number for any row_ptr.
int64_t items_cap(int32_t n, int64_t nnz);
// Per node: row_ptr checks (monotone, rp[0] = 0, rp[n] = nnz: kErrArg), largest degree
// (small[kWMaxDeg]), piece count into item_cnt and row-guide length into guide_len.
hipError_t launch_node_prep(int32_t n, int64_t nnz, const int32_t* rp, uint64_t* item_cnt, uint64_t* guide_len,
                            uint64_t* small, hipStream_t s);
// Spans of CSR entries walked by the creation checks, the hash-set build and the row
// prefixes (span s starts at entry 256 s); span_row holds span_count(nnz) + 1 rows.
int64_t span_count(int64_t nnz);
int64_t span_group_count(int64_t nnz);
// Rows of at least this many entries add up their span sums by groups of 64 spans.
constexpr int32_t kSpanGroupMinDegree = 64 * 256;
// After item_end (scanned piece counts) and goff_end (scanned guide lengths): the packed
// (row, piece) items, the node records {row start, degree, 0, row-guide offset} and
// span_row[s], the row holding the span's first entry.  All do nothing once row_ptr
// has been rejected.
hipError_t launch_items_records(int32_t n, int64_t nnz, const int32_t* rp, const uint64_t* item_end,
                                const uint64_t* goff_end, int64_t cap, uint64_t* items, uint4* rec, int32_t* span_row,
                                uint64_t* small, hipStream_t s);
// The edge hash set (filled with empty keys beforehand) and the edge filter (zeroed)
// from the entries (v, c) with v < c < n; nothing once row_ptr has been rejected.
hipError_t launch_edge_insert(int64_t nnz, const int32_t* span_row, const int32_t* rp, const int32_t* col, int32_t n,
                              uint64_t* slots, int hash_bits, uint64_t* filter, int filter_bits, uint64_t* small,
                              hipStream_t s);
// Column range; with `full` also self-loops, strict ascent and, through the hash set,
// the mirror of every entry (v, c) with c < v; counts the entries with c > v into
// small[kWUpper] (through part: check_part_words() u64 of per-block counts).
int check_part_words();
hipError_t launch_check_items(int64_t nnz, const int32_t* span_row, int32_t n, const int32_t* rp, const int32_t* col,
                              bool full, const uint64_t* slots, int hash_bits, uint64_t* part, uint64_t* small,
                              hipStream_t s);

// ---- table build ----
// Row prefixes with their row guides: ACC_sigma (kRowSigma; also the node records'
// S_v), ACC_tau (kRowTau, after ACC_sigma) or the MOSS-4Min prefix of d_{v,x} d_{x,v}
// (kRowCheck, after the rank tables), over 256-entry spans of the CSR.
enum RowMode { kRowSigma = 0, kRowTau = 1, kRowCheck = 2 };
struct RowTables {
  const int32_t* rp;
  const int32_t* col;
  const int32_t* span_row;  // row of each 256-entry span's first entry (from creation)
  uint32_t* acc_sigma;
  uint64_t* acc_tau;
  const uint2* rank;
  uint64_t* acc_check;
  uint64_t* span_sums;      // 2 * span_count(nnz): per span, the open row's sum at its end,
                            // then the sum of its first row's entries in it
  uint64_t* span_groups;    // span_group_count(nnz) sums of 64 consecutive span sums, or
  uint32_t* group_wrap;     // null (rows short enough to add up their spans directly)
  uint4* rec;
  uint32_t* guide;
  int64_t nnz;
  int32_t n;
};
hipError_t launch_row_tables(int mode, const RowTables& t, uint32_t* err, hipStream_t s);

// MOSS-4Min rank tables (Section 4.2.1, order of Section 3.2): for every entry (v, x),
// rank[e] = {d_{v,x}, d_{x,v}}, and col_rank holds each row in descending order.  Needs
// the node records, the row prefix ACC_sigma (for the neighbours' degrees), the first
// row of every 256-entry span of the CSR (`span_row`, spans + 1 entries) and, for the
// per-piece passes, the work items.  `scratch` (nnz u64) and `work`
// (mirror_work_words(nnz) u32) are working memory; `validated`: the CSR passed the
// creation checks (symmetric, sorted, no repeats), which the sort-based mirror pass
// relies on.
struct RankTables {
  int64_t n_items;
  const uint64_t* items;
  int32_t n;
  int64_t nnz;
  int32_t max_degree;
  bool validated;
  const int32_t* span_row;
  const int32_t* rp;
  const int32_t* col;
  const uint4* rec;
  const uint32_t* acc_sigma;
  uint64_t* scratch;
  uint32_t* work;
  uint2* rank;
  int32_t* col_rank;
};
hipError_t launch_rank_tables(const RankTables& t, hipStream_t s);
int64_t mirror_work_words(int64_t nnz);
// w[v] = the last entry of v's row prefix `acc` (0 for an empty row).
hipError_t launch_row_totals(int32_t n, const int32_t* rp, const uint64_t* acc, uint64_t* w, hipStream_t s);

// Edge hash set size (2^bits u64 slots for m edges, load factor <= 0.4) and edge
// filter size (2^bits 64-bit words, bits >= 1).
int edge_hash_bits(int64_t m);
int edge_filter_bits(int64_t m);

// Node weights (any output may be null) from the node records' S_v and the ACC_tau row
// ends, and Lambda_3, Lambda_4 into lambdas[0..1]; partials must hold
// 2 * node_weight_blocks(n) u64.
int node_weight_blocks(int32_t n);
hipError_t launch_node_weights(int32_t n, const int32_t* rp, const uint4* rec, const uint64_t* acc_tau,
                               uint64_t* w_gamma, uint64_t* w_gamma1, uint64_t* w_gamma2, uint64_t* partials,
                               unsigned long long* lambdas, uint32_t* err, hipStream_t s);

// Node-draw guides of up to three scanned weight arrays; total[j] receives acc[j][n-1].
struct GuideSet {
  const uint64_t* acc[3];
  uint32_t* guide[3];
  uint64_t* total[3];
  int count;
};
hipError_t launch_guides(const GuideSet& set, int32_t n, int gbits, hipStream_t s);

// Plain sampling launch: samples [k0, k1) of one sampler, hits[22] accumulated.  For
// MOSS-4Min hits[7..9] also count the diamonds reached by 2, 4 and 6 ordered draws.
hipError_t launch_sample(int sampler, const SamplerView& v, uint64_t seed, uint64_t k0, uint64_t k1,
                         unsigned long long* hits, uint8_t* class_out, int grid, int block, hipStream_t s);

// The same samples drawn XCD-grouped, one chunk [a, a + n) at a time (n <= max_n <=
// 2^31): the grouping passes (group of each sample, per-block group counts, their scan,
// the sorted order) into `scratch`, which holds grouped_scratch_bytes(max_n) bytes, then
// the sampling launch that reads them.  The two may run on different streams, ordered by
// events; a scratch block serves one chunk at a time.  block must be 64, 128, 192 or 256
// threads; class_out (may be null) receives the chunk's classes at [0, n).
// `window`: sorted entries a block takes at a time (sort_window of the bytes the
// samples read at random).
int64_t grouped_scratch_bytes(uint64_t max_n);

// The no-allocation calls' fixed scratch: a device array of kFixedScratchBytes that holds
// one grouped chunk of up to kFixedScratchSamples samples.  fixed_scratch gives its
// address on `device`, which must be the current device (looked up on the first call,
// then kept); fixed_scratch_lock is held around every use of a device's copy.
constexpr uint64_t kFixedScratchSamples = 1ull << 22;
constexpr uint64_t kFixedScratchBytes = 32ull << 20;
hipError_t fixed_scratch(int device, void** out);
std::mutex& fixed_scratch_lock(int device);
uint32_t sort_window(uint64_t footprint_bytes);
hipError_t launch_group_chunk(int sampler, uint64_t seed, uint64_t a, uint64_t n, void* scratch, uint64_t max_n,
                              hipStream_t s);
hipError_t launch_sample_chunk(int sampler, const SamplerView& v, uint64_t seed, uint64_t a, uint64_t n,
                               void* scratch, uint64_t max_n, uint32_t window, unsigned long long* hits,
                               uint8_t* class_out, int grid, int block, hipStream_t s);

hipError_t launch_sample_nodes(int sampler, const SamplerView& v, uint64_t seed, const uint64_t* index,
                               int64_t count, int32_t* nodes_out, uint8_t* class_out, hipStream_t s);

// Batched persistent launch over an item list resident in device memory: blocks take
// tiles from ctl[kCtlCounter] until ctl[kCtlTiles] are drawn, each finding its item.
hipError_t launch_batch(const SamplerView* views, const BatchItem* items, uint32_t* ctl, unsigned long long* bins,
                        int grid, int block, hipStream_t s);

// Registers/VGPR usage probe for occupancy decisions (max active blocks per CU).
int sample_kernel_blocks_per_cu(int sampler, int block);

}  // namespace moss
