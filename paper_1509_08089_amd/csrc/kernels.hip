// HIP kernels of the Moss hot path for gfx950 (CDNA4, wave64).
//
// Graph creation (Section 2: an undirected simple graph as sorted CSR):
//   k_node_prep        row_ptr checks, largest degree, work-item and row-guide sizes
//   k_items_records    work items (rows cut into pieces), node records, span rows
//   k_edge_insert      the edge hash set (then k_filter_build: the edge filter)
//   k_check_items      column range, self-loops, strict ascent, symmetry
// Table build (Section 4.1.3 "Initialization", O(|E|)):
//   k_span_prefix      each 256-entry span's prefix of ACC_sigma, ACC_tau or the
//                      MOSS-4Min row weights, restarted at every row start
//   k_span_finish      adds the earlier spans' sums to rows that began before the
//                      span, writes the row guides and S_v
//   k_node_weights     Gamma_v, Gamma^(1)_v, Gamma^(2)_v, Lambda_3, Lambda_4
//   k_scan_*           node-level inclusive prefixes ACC_Gamma*
//   k_guides           search windows for the node draws
// Sampling (Algorithms 1, 3, 4):
//   k_sample<S>        grid-stride loop, one sample per lane per step,
//                      per-wave LDS histograms flushed with u64 atomics
//   k_batch            persistent kernel cutting a list of many
//                      (graph, sampler, sample range) items into tiles
//   k_sample_nodes<S>  the same draw for chosen sample indices, with nodes
//
// All counting is integer; a sample's outcome depends only on (graph, seed, sampler,
// sample index), never on which lane, block or launch draws it.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "device.h"
#include "kernels.h"

namespace moss {

__constant__ uint8_t c_lut4[8];
__constant__ uint8_t c_lut5t[64];
__constant__ uint8_t c_lut5p[64];

// ---------------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t value, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t value, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_fill_u8(uint8_t* p, uint8_t value, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// blockIdx.y selects the range
__global__ void k_fill_set(FillSet f) {
  const int j = blockIdx.y;
  uint64_t* p = f.p[j];
  const int64_t count = f.count[j];
  const uint64_t value = f.value[j];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

static int fill_grid(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(count)), dim3(256), 0, s, p, value, count);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(count)), dim3(256), 0, s, p, value, count);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint8_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u8, dim3(fill_grid(count)), dim3(256), 0, s, p, value, count);
  return hipGetLastError();
}

hipError_t launch_fill_set(const FillSet& f, hipStream_t s) {
  int64_t most = 0;
  for (int j = 0; j < 4; ++j) most = std::max(most, f.count[j]);
  if (most <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_set, dim3(fill_grid(most), 4), dim3(256), 0, s, f);
  return hipGetLastError();
}

__device__ __forceinline__ uint64_t add_wrap(uint64_t a, uint64_t b, bool& wrapped) {
  const uint64_t z = a + b;
  wrapped |= z < a;
  return z;
}

hipError_t upload_class_luts(const uint8_t lut4[8], const uint8_t lut5t[64], const uint8_t lut5p[64]) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_lut4), lut4, 8);
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_lut5t), lut5t, 64);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_lut5p), lut5p, 64);
}

// Grids of the node- and item-parallel kernels that end in one atomic per block:
// enough blocks to fill the chip, few enough that the atomics do not queue up.
static int reduce_grid(int64_t units, int64_t per_block) {
  int64_t g = (units + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 2048) g = 2048;
  return (int)g;
}

// ---------------------------------------------------------------------------------
// Work items.  Every CSR row is cut into items of at most kItem consecutive entries
// and each item is handled by one wave, so no wave walks a long row alone: the
// costliest row (a hub with tens of thousands of neighbours) becomes many items
// that run concurrently.  items[i] packs (row << 32 | piece index within the row).
// ---------------------------------------------------------------------------------
constexpr int32_t kItem = 256;
constexpr int64_t kSpan = 256;  // CSR entries per wave in the creation checks and the hash-set build

int64_t items_cap(int32_t n, int64_t nnz) { return (int64_t)n + nnz / kItem + 1; }
int64_t span_count(int64_t nnz) { return (nnz + kSpan - 1) / kSpan; }
int64_t span_group_count(int64_t nnz) { return (span_count(nnz) + 63) / 64; }

// Row guides (used by the weighted picks inside a row, see row_pick): rows with
// d >= kRowGuideMin get 2^g + 1 entries, g = floor(log2 d) - 1.
__device__ __forceinline__ int row_guide_bits(int32_t d) { return 31 - __clz(d) - 1; }

__device__ __forceinline__ uint64_t row_guide_len(int32_t d) {
  return d >= kRowGuideMin ? (1ull << row_guide_bits(d)) + 1 : 0ull;
}

__device__ __forceinline__ int row_guide_shift(uint64_t total, int g) {
  const int bl = total ? 64 - __clzll((long long)total) : 0;
  return bl > g ? bl - g : 0;
}

// ---------------------------------------------------------------------------------
// CSR validation and layout at creation.  k_node_prep checks row_ptr; the kernels
// after it read the error word first and do nothing once row_ptr is rejected, so
// no row range outside col[] is ever read and no item is written past the cap.
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_node_prep(int32_t n, int64_t nnz, const int32_t* __restrict__ rp,
                                                   uint64_t* __restrict__ item_cnt, uint64_t* __restrict__ guide_len,
                                                   uint64_t* small) {
  __shared__ uint32_t s_bad, s_max;
  if (threadIdx.x == 0) {
    s_bad = 0;
    s_max = 0;
  }
  __syncthreads();
  uint32_t bad = 0, dmax = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int64_t d = (int64_t)rp[v + 1] - (int64_t)rp[v];
    if (d < 0) {
      bad = kErrArg;
      d = 0;
    }
    if (d > nnz) d = nnz;
    dmax = max(dmax, (uint32_t)d);
    item_cnt[v] = (uint64_t)((d + kItem - 1) / kItem);
    guide_len[v] = row_guide_len((int32_t)d);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (rp[0] != 0 || (int64_t)rp[n] != nnz)) bad = kErrArg;
  bad = wave_or(bad);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dmax = max(dmax, (uint32_t)__shfl_xor((int)dmax, off, 64));
  if (lane_id() == 0) {
    if (bad) atomicOr(&s_bad, bad);
    if (dmax) atomicMax(&s_max, dmax);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_bad) atomicOr((uint32_t*)(small + kWErr), s_bad);
    if (s_max) atomicMax((unsigned long long*)(small + kWMaxDeg), (unsigned long long)s_max);
  }
}

hipError_t launch_node_prep(int32_t n, int64_t nnz, const int32_t* rp, uint64_t* item_cnt, uint64_t* guide_len,
                            uint64_t* small, hipStream_t s) {
  hipLaunchKernelGGL(k_node_prep, dim3(reduce_grid(n, 1024)), dim3(256), 0, s, n, nnz, rp, item_cnt, guide_len, small);
  return hipGetLastError();
}

__device__ __forceinline__ bool rowptr_rejected(const uint64_t* small) {
  return (*(const volatile uint32_t*)(small + kWErr) & kErrArg) != 0;
}

// item_end / goff_end: inclusive prefixes of the piece counts and guide lengths.
// span_row[s] is the row holding entry s * kSpan (each such entry lies in exactly one
// non-empty row, which writes it; a validated row_ptr keeps s below the span count),
// and span_row[spans] the last non-empty row, so that span_row[s + 1] bounds the rows
// of span s also for the last span (rows without entries after it never enter).
__global__ void k_items_records(int32_t n, int64_t nnz, const int32_t* __restrict__ rp,
                                const uint64_t* __restrict__ item_end, const uint64_t* __restrict__ goff_end,
                                int64_t cap, uint64_t* __restrict__ items, uint4* __restrict__ rec,
                                int32_t* __restrict__ span_row, const uint64_t* small) {
  if (rowptr_rejected(small)) return;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r0 = rp[v], r1 = rp[v + 1], d = r1 - r0;
    const uint64_t c = (uint64_t)((d + kItem - 1) / kItem);
    const uint64_t first = item_end[v] - c;
    for (uint64_t j = 0; j < c; ++j)
      if (first + j < (uint64_t)cap) items[first + j] = (uint64_t)v << 32 | j;
    rec[v] = make_uint4((uint32_t)r0, (uint32_t)d, 0u, (uint32_t)(goff_end[v] - row_guide_len(d)));
    for (int64_t sp = ((int64_t)r0 + kSpan - 1) / kSpan; sp * kSpan < (int64_t)r1; ++sp) span_row[sp] = (int32_t)v;
    if (d > 0 && (int64_t)r1 == nnz) span_row[(nnz + kSpan - 1) / kSpan] = (int32_t)v;
  }
}

hipError_t launch_items_records(int32_t n, int64_t nnz, const int32_t* rp, const uint64_t* item_end,
                                const uint64_t* goff_end, int64_t cap, uint64_t* items, uint4* rec, int32_t* span_row,
                                uint64_t* small, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_items_records, dim3(fill_grid(n)), dim3(256), 0, s, n, nnz, rp, item_end, goff_end, cap, items,
                     rec, span_row, small);
  return hipGetLastError();
}

static int item_grid(int64_t n_items) {
  int64_t g = (n_items + 3) / 4;  // one wave per item, 4 waves per block
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

// row start and degree of a node (the first half of its record)
__device__ __forceinline__ uint2 row_of(const uint4* __restrict__ rec, int32_t x) {
  return *reinterpret_cast<const uint2*>(rec + x);
}

struct ItemRange {
  int32_t v, r0, r1, e0, e1, piece;
};

__device__ __forceinline__ ItemRange item_range(const uint64_t* __restrict__ items, const int32_t* __restrict__ rp,
                                                int64_t i) {
  const uint64_t it = items[i];
  ItemRange r;
  r.v = (int32_t)(it >> 32);
  r.piece = (int32_t)(it & 0xFFFFFFFFu);
  r.r0 = rp[r.v];
  r.r1 = rp[r.v + 1];
  r.e0 = r.r0 + r.piece * kItem;
  r.e1 = min(r.r1, r.e0 + kItem);
  return r;
}

// The creation checks and the edge hash set go over the CSR entries in spans of kSpan
// consecutive entries, one span per wave and kSpan / 64 entries per lane (lane l takes
// entries S + l, S + l + 64, ...), so that every lane is busy whatever the degrees and
// each lane has several hash-set accesses in flight at once.
//
// The rows of a span's entries come without a dependent search: v0 = span_row[s]
// holds entry S, and the rows v0 < j <= last (last: the row of the next span's first
// entry) start inside the span, at offsets rp[j] - S in [1, kSpan].  The row of the
// entry at offset o is v0 plus the number of those rows starting at or before o, read
// from a histogram of start offsets and its prefix sum in LDS (rows without entries
// count too: they share the next row's start).  An entry is the first of its row iff
// a row starts at its offset, or, at offset 0, iff rp[v0] == S.
constexpr int kSpanPer = (int)(kSpan / 64);  // entries per lane

// LDS written by some lanes of a wave and then read by others of the same wave
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// hist: this wave's kSpan words of LDS, 16-byte aligned.  Uniform control flow.
__device__ __forceinline__ void span_rows(const int32_t* __restrict__ rp, int64_t S, int32_t v0, int32_t last,
                                          uint32_t* hist, int32_t (&row)[kSpanPer], bool (&head)[kSpanPer]) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 0; k < kSpanPer; ++k) hist[lane + 64 * k] = 0;
  wave_lds_sync();
  int64_t start0 = 0;  // rp[v0] - S, on lane 0
  for (int64_t j0 = v0; j0 <= (int64_t)last; j0 += 64) {
    const int64_t j = j0 + lane;
    if (j <= (int64_t)last) {
      const int64_t o = (int64_t)rp[j] - S;
      if (j == v0) start0 = o;
      else if (o < kSpan) atomicAdd(&hist[o], 1u);
    }
  }
  start0 = __shfl(start0, 0, 64);
  wave_lds_sync();
  static_assert(kSpan == 256, "four offsets per lane below");
  const uint4 h = reinterpret_cast<const uint4*>(hist)[lane];
  const uint32_t a = h.x, b = a + h.y, c = b + h.z, d = c + h.w;
  bool unused = false;
  const uint32_t before = (uint32_t)(wave_inclusive_scan((uint64_t)d, unused) - d);
  wave_lds_sync();
  reinterpret_cast<uint4*>(hist)[lane] =
      make_uint4((before + a) << 1 | (h.x != 0), (before + b) << 1 | (h.y != 0), (before + c) << 1 | (h.z != 0),
                 (before + d) << 1 | (h.w != 0));
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < kSpanPer; ++k) {
    const int o = lane + 64 * k;
    const uint32_t w = hist[o];
    row[k] = v0 + (int32_t)(w >> 1);
    head[k] = (w & 1) != 0 || (o == 0 && start0 == 0);
  }
  wave_lds_sync();  // the histogram is reused by the wave's next span
}

static int spans_grid(int64_t nnz) {
  const int64_t spans = (nnz + kSpan - 1) / kSpan;
  return (int)std::max<int64_t>(1, std::min<int64_t>((spans + 3) / 4, 65536));  // a span per wave, 4 waves a block
}

// The edge hash set, built at creation: every entry (v, c) with v < c < n inserts the
// key min << 32 | max (each undirected edge once, from its smaller endpoint) with a
// 64-bit compare-and-swap and linear probing.  The set has at least 1.25 slots per
// such entry, so it never fills; a full set would still be reported (kErrOverflow) and
// every probe loop is bounded.
__global__ __launch_bounds__(256) void k_edge_insert(int64_t nnz, const int32_t* __restrict__ span_row,
                                                     const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     int32_t n, unsigned long long* __restrict__ slots, int hash_bits,
                                                     uint64_t* small) {
  __shared__ __align__(16) uint32_t hist[4][kSpan];
  if (rowptr_rejected(small)) return;  // no block barrier below: waves may leave one by one
  constexpr int kPer = kSpanPer;
  const int lane = lane_id();
  uint32_t* wh = hist[threadIdx.x >> 6];
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t spans = (nnz + kSpan - 1) / kSpan;
  const uint64_t hmask = (1ull << hash_bits) - 1;
  bool full = false;
  for (int64_t sp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; sp < spans; sp += nwaves) {
    const int64_t S = sp * kSpan;
    int32_t c[kPer], row[kPer];
    bool head[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) c[k] = S + lane + 64 * k < nnz ? col[S + lane + 64 * k] : -1;
    span_rows(rp, S, span_row[sp], span_row[sp + 1], wh, row, head);
    uint64_t key[kPer], h[kPer];
    unsigned long long old[kPer];
    bool live[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      live[k] = c[k] > row[k] && c[k] < n;  // also false past nnz (c = -1)
      key[k] = edge_key(row[k], c[k]);
      h[k] = edge_slot(key[k], hash_bits);
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      old[k] = live[k] ? atomicCAS(&slots[h[k]], (unsigned long long)kEmptySlot, (unsigned long long)key[k])
                       : (unsigned long long)kEmptySlot;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (!live[k] || old[k] == kEmptySlot || old[k] == key[k]) continue;
      uint64_t hh = h[k];
      for (uint64_t probes = 1;; ++probes) {
        if (probes > hmask) {
          full = true;
          break;
        }
        hh = (hh + 1) & hmask;
        const unsigned long long o = atomicCAS(&slots[hh], (unsigned long long)kEmptySlot, (unsigned long long)key[k]);
        if (o == kEmptySlot || o == key[k]) break;
      }
    }
  }
  if (__ballot(full) != 0 && lane == 0) atomicOr((uint32_t*)(small + kWErr), kErrOverflow);
}

// The filter from the finished hash set: lane s of the grid reads slot s; the keys whose
// home slot lies in the same filter word as s (all but the few that linear probing
// carried over a word boundary) are OR-ed together across the lanes of that word, one
// atomic per word; the others set their bits with an atomic each.
__global__ __launch_bounds__(256) void k_filter_build(const uint64_t* __restrict__ slots, int hash_bits,
                                                      unsigned long long* __restrict__ filter, int filter_bits,
                                                      const uint64_t* small) {
  if (rowptr_rejected(small)) return;  // no barrier below
  const int lane = lane_id();
  const int shift = hash_bits - filter_bits;           // slots per filter word: 2^shift (>= 4 slots, see the launch)
  const int seg = shift >= 8 ? 64 : 1 << (shift - 2);  // lanes that share a word, four slots each
  const uint64_t nslots = 1ull << hash_bits;
  // each wave takes 256 consecutive slots, four per lane (a lane's four slots lie in one
  // word: a word covers at least four slots)
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; 4 * (q - lane) < nslots;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t s0 = 4 * q;
    uint64_t mine = 0;
    if (s0 < nslots) {
      const ulonglong2 a = *reinterpret_cast<const ulonglong2*>(slots + s0);
      const ulonglong2 b = *reinterpret_cast<const ulonglong2*>(slots + s0 + 2);
      const uint64_t key[4] = {a.x, a.y, b.x, b.y};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (key[j] == kEmptySlot) continue;
        const uint64_t m = filter_mask(mix64(key[j]));
        const uint64_t w = edge_slot(key[j], filter_bits);
        if (w == (s0 >> shift)) mine |= m;
        else atomicOr(&filter[w], (unsigned long long)m);
      }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1)
      if (off < seg) mine |= __shfl_xor(mine, off, 64);
    if ((lane & (seg - 1)) == 0 && mine && s0 < nslots) atomicOr(&filter[s0 >> shift], (unsigned long long)mine);
  }
}

hipError_t launch_edge_insert(int64_t nnz, const int32_t* span_row, const int32_t* rp, const int32_t* col, int32_t n,
                              uint64_t* slots, int hash_bits, uint64_t* filter, int filter_bits, uint64_t* small,
                              hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_edge_insert, dim3(spans_grid(nnz)), dim3(256), 0, s, nnz, span_row, rp, col, n,
                     (unsigned long long*)slots, hash_bits, small);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // at least four slots per filter word (the sizes below give 2^3 .. 2^6)
  if (hash_bits - filter_bits < 2) return hipErrorInvalidValue;
  const int64_t nslots = 1ll << hash_bits;
  hipLaunchKernelGGL(k_filter_build, dim3((unsigned)std::min<int64_t>((nslots / 4 + 255) / 256, 8192)), dim3(256), 0,
                     s, slots, hash_bits, (unsigned long long*)filter, filter_bits, small);
  return hipGetLastError();
}

// Column range, self-loops, strict ascent (sorted, no repeats) and symmetry, over the
// entries in spans as k_edge_insert.  Every entry (v, c) with c < v looks up its mirror
// (c, v) in the edge hash set, which holds exactly the entries with c > v; with repeats
// excluded those mirrors are distinct, so the graph is symmetric exactly when all are
// found and the entries with c > v are half of all entries (the host compares their
// count in small[kWUpper] with nnz).  Each block stores its count of those entries in
// part[block] and k_check_sum adds them up: one atomic per block on a single word
// serialises in its L2 channel (measured at n = 1e6, m = 1e7: 1.8 ms for the creation
// with 19,532 blocks adding to one word, 0.96 ms with 2,048).
constexpr int kCheckBlocks = 2048;

__global__ __launch_bounds__(256) void k_check_items(int64_t nnz, const int32_t* __restrict__ span_row, int32_t n,
                                                     const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     int full, const uint64_t* __restrict__ slots, int hash_bits,
                                                     uint64_t* __restrict__ part, uint64_t* small) {
  __shared__ uint32_t s_bad, s_skip;
  __shared__ unsigned long long s_upper;
  __shared__ __align__(16) uint32_t hist[4][kSpan];
  if (threadIdx.x == 0) {
    s_bad = 0;
    s_upper = 0;
    s_skip = rowptr_rejected(small) ? 1u : 0u;  // read once, so the whole block leaves together
  }
  __syncthreads();
  if (s_skip) return;
  constexpr int kPer = kSpanPer;
  const int lane = lane_id();
  uint32_t* wh = hist[threadIdx.x >> 6];
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t spans = (nnz + kSpan - 1) / kSpan;
  uint32_t bad = 0, upper = 0;
  for (int64_t sp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; sp < spans; sp += nwaves) {
    const int64_t S = sp * kSpan;
    int32_t c[kPer], row[kPer];
    bool head[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) c[k] = S + lane + 64 * k < nnz ? col[S + lane + 64 * k] : 0;
    const int32_t before_span = (lane == 0 && S > 0) ? col[S - 1] : 0;
    span_rows(rp, S, span_row[sp], span_row[sp + 1], wh, row, head);
    // the previous entry's column: lane l - 1's, lane 63's of the previous round, or
    // the entry before the span
    int32_t prev[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int32_t p = __shfl(c[k], (lane + 63) & 63, 64);
      const int32_t wrap = k ? __shfl(c[k > 0 ? k - 1 : 0], 63, 64) : before_span;
      prev[k] = lane ? p : wrap;
    }
    uint64_t key[kPer], h[kPer], first[kPer];
    bool probe[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t e = S + lane + 64 * k;
      const int32_t v = row[k];
      key[k] = edge_key(c[k], v);
      h[k] = edge_slot(key[k], hash_bits);
      probe[k] = false;
      if (e >= nnz) continue;
      if (c[k] < 0 || c[k] >= n) {
        bad |= kErrArg;
        continue;
      }
      if (!full) continue;
      if (c[k] == v) bad |= kErrSelfLoop;
      if (!head[k]) {
        if (prev[k] == c[k]) bad |= kErrDuplicate;
        else if (prev[k] > c[k]) bad |= kErrUnsorted;
      }
      if (c[k] > v) ++upper;
      else if (c[k] < v) probe[k] = true;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) first[k] = probe[k] ? slots[h[k]] : 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (probe[k] && !edge_hash_rest(slots, hash_bits, key[k], h[k], first[k])) bad |= kErrAsymmetric;
  }
  bad = wave_or(bad);
  const uint64_t wu = wave_sum((uint64_t)upper);
  if (lane == 0) {
    if (bad) atomicOr(&s_bad, bad);
    if (wu) atomicAdd(&s_upper, (unsigned long long)wu);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_bad) atomicOr((uint32_t*)(small + kWErr), s_bad);
    part[blockIdx.x] = s_upper;
  }
}

__global__ __launch_bounds__(256) void k_check_sum(const uint64_t* __restrict__ part, int nblocks, uint64_t* small) {
  __shared__ uint64_t wsum[4];
  uint64_t x = 0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) x += part[b];
  x = wave_sum(x);
  if (lane_id() == 0) wsum[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) small[kWUpper] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

hipError_t launch_check_items(int64_t nnz, const int32_t* span_row, int32_t n, const int32_t* rp, const int32_t* col,
                              bool full, const uint64_t* slots, int hash_bits, uint64_t* part, uint64_t* small,
                              hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  const int grid = std::min(spans_grid(nnz), kCheckBlocks);
  hipLaunchKernelGGL(k_check_items, dim3(grid), dim3(256), 0, s, nnz, span_row, n, rp, col, full ? 1 : 0, slots,
                     hash_bits, part, small);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_check_sum, dim3(1), dim3(256), 0, s, part, grid, small);
  return hipGetLastError();
}

int check_part_words() { return kCheckBlocks; }

// ---------------------------------------------------------------------------------
// Row prefixes (Section 4.1.3 ACC_sigma = ACC_mu of Section 5.1.5; the tau prefix of
// Section 5.1.2; MOSS-4Min's prefix of d_{v,x} d_{x,v}, Section 4.2.1), in two passes
// over 256-entry spans (k_span_prefix, k_span_finish below).  ACC_sigma entries are
// (d_x - 1) of the neighbours; ACC_tau entries are (d_x - 1)(S_v - (d_x - 1)) with S_v
// the row total of ACC_sigma; the MOSS-4Min entries are d_{v,x} d_{x,v} from the rank
// tables.
// ---------------------------------------------------------------------------------
// Each lane owns nb guide entries guide[goff + b0 ..) to set to val; the wave shares the
// stores out evenly (one entry of a row can own thousands of buckets while its
// neighbours own none), consecutive lanes writing consecutive entries of one owner.
// Uniform control flow.
__device__ __forceinline__ void wave_fill_guides(uint32_t* __restrict__ guide, uint32_t goff, uint32_t b0,
                                                 uint32_t nb, uint32_t val) {
  if (__ballot(nb != 0) == 0) return;  // wave-uniform
  const int lane = lane_id();
  uint32_t incl = nb;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  const uint32_t start = goff + b0 - (incl - nb);  // owner's bucket of store index t: start + t
  for (uint32_t base = 0; base < total; base += 64) {
    const uint32_t t = base + lane;
    int j = 0;  // the owner: the first lane whose inclusive count exceeds t
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
      if (__shfl(incl, j + step - 1, 64) <= t) j += step;
    const uint32_t at = __shfl(start, j & 63, 64) + t;
    const uint32_t v = __shfl(val, j & 63, 64);
    if (t < total) guide[at] = v;
  }
}

// the u64 prefix a mode writes (ACC_sigma is u32)
template <int M>
__device__ __forceinline__ uint64_t* row_out64(const RowTables& t) {
  return M == kRowTau ? t.acc_tau : t.acc_check;
}

template <int M>
__device__ __forceinline__ uint32_t row_overflow_bit() {
  return M == kRowSigma ? kErrOverflow : (M == kRowTau ? kErrOverflowK5 : kErrOverflowMin);
}

// Inclusive scan over the lanes of a wave, restarted at every lane whose `head` is set;
// on return `head` tells whether a restart lies at or before the lane.  `wrapped` is
// set on any 64-bit wrap.
__device__ __forceinline__ uint64_t wave_segmented_scan(uint64_t x, bool& head, bool& wrapped) {
  const int lane = lane_id();
  uint32_t f = head ? 1u : 0u;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_up(x, off, 64);
    const uint32_t g = __shfl_up(f, off, 64);
    if (lane >= off) {
      if (!f) x = add_wrap(y, x, wrapped);
      f |= g;
    }
  }
  head = f != 0;
  return x;
}

// Row prefixes go over the entries in 256-entry spans, one wave per span, in two passes.
// k_span_prefix: each span's entries are scanned with a restart at every row start, so
// the prefix of a row lying inside the span is final; the span records the sum of its
// last row's entries in it (span_sums[s], the row's running sum at the span's end if it
// started in the span) and the sum of its first row's entries in it
// (span_sums[spans + s]).
template <int M>
__global__ __launch_bounds__(256) void k_span_prefix(RowTables t, uint32_t* err) {
  __shared__ __align__(16) uint32_t hist[4][kSpan];
  constexpr int kPer = kSpanPer;
  const int lane = lane_id();
  uint32_t* wh = hist[threadIdx.x >> 6];
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t spans = (t.nnz + kSpan - 1) / kSpan;
  bool wrapped = false, over = false;
  for (int64_t sp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; sp < spans; sp += nwaves) {
    const int64_t S = sp * kSpan;
    const int32_t v0 = t.span_row[sp];
    uint64_t raw[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t e = S + lane + 64 * k;
      raw[k] = 0;
      if (e >= t.nnz) continue;
      if (M == kRowSigma) {
        raw[k] = (uint64_t)(uint32_t)t.col[e];
      } else if (M == kRowTau) {
        raw[k] = t.acc_sigma[e];
      } else {
        const uint2 rk = t.rank[e];
        raw[k] = (uint64_t)rk.x * (uint64_t)rk.y;
      }
    }
    const uint64_t before_span = (M == kRowTau && lane == 0 && S > 0) ? (uint64_t)t.acc_sigma[S - 1] : 0ull;
    int32_t row[kPer];
    bool head[kPer];
    span_rows(t.rp, S, v0, t.span_row[sp + 1], wh, row, head);
    uint64_t x[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const bool valid = S + lane + 64 * k < t.nnz;
      if (M == kRowSigma) {  // d_x - 1 of the neighbour x
        x[k] = valid ? (uint64_t)row_of(t.rec, (int32_t)raw[k]).y - 1 : 0ull;
      } else if (M == kRowTau) {  // (d_x - 1)(S_v - (d_x - 1)), d_x - 1 from the sigma prefix
        const uint64_t p = __shfl(raw[k], (lane + 63) & 63, 64);
        const uint64_t wrap = k ? __shfl(raw[k > 0 ? k - 1 : 0], 63, 64) : before_span;
        const uint64_t dx = head[k] ? raw[k] : raw[k] - (lane ? p : wrap);
        x[k] = valid ? dx * ((uint64_t)t.rec[row[k]].z - dx) : 0ull;
      } else {
        x[k] = valid ? raw[k] : 0ull;
      }
    }
    uint64_t carry = 0, first = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t e = S + lane + 64 * k;
      const bool valid = e < t.nnz;
      bool f = head[k];
      uint64_t v = wave_segmented_scan(x[k], f, wrapped);
      if (!f) v = add_wrap(v, carry, wrapped);
      if (valid) {
        if (M == kRowSigma) {
          over |= v > 0xFFFFFFFFull;
          t.acc_sigma[e] = (uint32_t)v;
        } else {
          row_out64<M>(t)[e] = v;
        }
      }
      carry = __shfl(v, 63, 64);
      const uint64_t in_first = __ballot(valid && row[k] == v0);
      if (in_first) first = __shfl(v, 63 - __clzll((long long)in_first), 64);
    }
    if (lane == 0) {
      t.span_sums[sp] = carry;
      t.span_sums[spans + sp] = first;
    }
  }
  // a wrap inside a tau row is a Gamma^(2)_v beyond 64 bits, inside a MOSS-4Min row a
  // check-Gamma_v beyond 64 bits; a sigma prefix beyond 32 bits does not fit ACC_sigma
  if (M != kRowSigma && __ballot(wrapped) != 0 && lane == 0) atomicOr(err, row_overflow_bit<M>());
  if (M == kRowSigma && __ballot(over) != 0 && lane == 0) atomicOr(err, kErrOverflow);
}

// Sum of the span sums tail[lo, hi) over the wave (lo, hi wave-uniform).  A long range
// (a row over hundreds of spans) goes through the sums of aligned groups of 64 spans,
// all of which lie inside the row, so a row of s spans costs about s^2 / 4096 reads in
// all instead of s^2 / 2.  `wrapped` is set on any 64-bit wrap.
__device__ __forceinline__ uint64_t span_range_sum(const uint64_t* __restrict__ tail,
                                                   const uint64_t* __restrict__ groups,
                                                   const uint32_t* __restrict__ group_wrap, int64_t lo, int64_t hi,
                                                   bool& wrapped) {
  const int lane = lane_id();
  uint64_t acc = 0;
  int64_t a = hi, b = hi;  // [a, b): whole groups
  if (groups && hi - lo >= 3 * 64) {
    a = (lo + 63) / 64 * 64;
    b = hi / 64 * 64;
    for (int64_t q = a / 64 + lane; q < b / 64; q += 64) {
      acc = add_wrap(acc, groups[q], wrapped);
      wrapped |= group_wrap[q] != 0;
    }
  }
  for (int64_t j = lo + lane; j < a; j += 64) acc = add_wrap(acc, tail[j], wrapped);
  for (int64_t j = b + lane; j < hi; j += 64) acc = add_wrap(acc, tail[j], wrapped);
  return wave_sum_wrap(acc, wrapped);
}

// groups[q] = tail[64 q] + ... + tail[64 q + 63], one wave per group; group_wrap[q]
// records a wrap (it matters only for groups inside one row, the only ones read).
__global__ __launch_bounds__(256) void k_span_groups(const uint64_t* __restrict__ tail, int64_t spans,
                                                     uint64_t* __restrict__ groups, uint32_t* __restrict__ group_wrap) {
  const int lane = lane_id();
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t ngroups = (spans + 63) / 64;
  for (int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; q < ngroups; q += nwaves) {
    const int64_t j = 64 * q + lane;
    bool wrapped = false;
    const uint64_t x = wave_sum_wrap(j < spans ? tail[j] : 0ull, wrapped);
    if (lane == 0) {
      groups[q] = x;
      group_wrap[q] = wrapped ? 1u : 0u;
    }
  }
}

// k_span_finish: a span whose first row started in an earlier span adds that row's
// sum over those spans to its first row's entries; then every entry writes its share
// of its row's guide (the row total: from this span if the row ends here, else this
// span's end plus the row's later spans) and, for ACC_sigma, the row's last entry
// records S_v.
template <int M>
__global__ __launch_bounds__(256) void k_span_finish(RowTables t, uint32_t* err) {
  __shared__ __align__(16) uint32_t hist[4][kSpan];
  __shared__ uint64_t fin[4][kSpan];
  constexpr int kPer = kSpanPer;
  const int lane = lane_id();
  uint32_t* wh = hist[threadIdx.x >> 6];
  uint64_t* fh = fin[threadIdx.x >> 6];
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t spans = (t.nnz + kSpan - 1) / kSpan;
  const uint64_t* tail = t.span_sums;
  const uint64_t* head_sum = t.span_sums + spans;
  bool wrapped = false, over = false;
  for (int64_t sp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; sp < spans; sp += nwaves) {
    const int64_t S = sp * kSpan;
    const int32_t v0 = t.span_row[sp];
    int32_t row[kPer];
    bool head[kPer];
    span_rows(t.rp, S, v0, t.span_row[sp + 1], wh, row, head);
    // the first row's sum over the earlier spans it covers
    const int64_t start0 = (int64_t)row_of(t.rec, v0).x;
    const uint64_t carry =
        start0 < S ? span_range_sum(tail, t.span_groups, t.group_wrap, start0 / kSpan, sp, wrapped) : 0ull;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int o = lane + 64 * k;
      const int64_t e = S + o;
      uint64_t v = 0;
      if (e < t.nnz) {
        v = M == kRowSigma ? (uint64_t)t.acc_sigma[e] : row_out64<M>(t)[e];
        if (carry && row[k] == v0) {
          v = add_wrap(v, carry, wrapped);
          if (M == kRowSigma) {
            over |= v > 0xFFFFFFFFull;
            t.acc_sigma[e] = (uint32_t)v;
          } else {
            row_out64<M>(t)[e] = v;
          }
        }
      }
      fh[o] = v;
    }
    wave_lds_sync();
    // total of the row that runs past the span's end, if one does
    uint64_t total_on = 0;
    if (sp + 1 < spans) {
      const int32_t rn = t.span_row[sp + 1];
      const uint2 rr = row_of(t.rec, rn);
      if ((int64_t)rr.x < S + kSpan) {
        const int64_t s1 = ((int64_t)rr.x + rr.y - 1) / kSpan;
        const uint64_t mid = span_range_sum(tail, t.span_groups, t.group_wrap, sp + 1, s1, wrapped);
        total_on = add_wrap(add_wrap(fh[kSpan - 1], mid, wrapped), head_sum[s1], wrapped);
      }
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int o = lane + 64 * k;
      const int64_t e = S + o;
      uint32_t goff = 0, b0 = 0, nb = 0, val = 0;  // this entry's guide buckets [b0, b0 + nb)
      if (e < t.nnz) {
        const int32_t r = row[k];
        const uint4 rr = t.rec[r];  // row start, degree, (S_v), guide offset
        const int64_t end = (int64_t)rr.x + rr.y;
        const uint64_t total = end - S <= kSpan ? fh[end - 1 - S] : total_on;
        const int32_t d = (int32_t)rr.y;
        if (d >= kRowGuideMin) {
          const int g = row_guide_bits(d);
          const int sh = row_guide_shift(total, g);
          const uint64_t lo = head[k] ? 0ull : (o ? fh[o - 1] : carry), hi = fh[o];
          // entry e answers the buckets whose lower bound b * 2^sh lies in [lo, hi); the
          // row's last entry also those at or above the total
          const uint64_t lim = (1ull << g) + 1;
          const uint64_t c0 = lo ? ((lo - 1) >> sh) + 1 : 0ull;
          const uint64_t c1 = e == end - 1 ? lim : (hi ? ((hi - 1) >> sh) + 1 : 0ull);
          b0 = (uint32_t)min(c0, lim);
          nb = (uint32_t)(min(c1, lim) - b0) * (c1 > c0);
          goff = rr.w;
          val = (uint32_t)(e - rr.x);
        }
        if (M == kRowSigma && e == end - 1) {
          over |= total > 0xFFFFFFFFull;
          t.rec[r].z = (uint32_t)total;
        }
      }
      wave_fill_guides(t.guide, goff, b0, nb, val);
    }
    wave_lds_sync();  // fin is reused by the wave's next span
  }
  if (M != kRowSigma && __ballot(wrapped) != 0 && lane == 0) atomicOr(err, row_overflow_bit<M>());
  if (M == kRowSigma && __ballot(over) != 0 && lane == 0) atomicOr(err, kErrOverflow);
}

template <int M>
static hipError_t row_tables_mode(const RowTables& t, uint32_t* err, hipStream_t s) {
  const dim3 grid(spans_grid(t.nnz)), block(256);
  hipLaunchKernelGGL(k_span_prefix<M>, grid, block, 0, s, t, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (t.span_groups) {
    const int64_t spans = (t.nnz + kSpan - 1) / kSpan, ngroups = (spans + 63) / 64;
    hipLaunchKernelGGL(k_span_groups, dim3((unsigned)std::min<int64_t>((ngroups + 3) / 4, 65536)), block, 0, s,
                       t.span_sums, spans, t.span_groups, t.group_wrap);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_span_finish<M>, grid, block, 0, s, t, err);
  return hipGetLastError();
}

hipError_t launch_row_tables(int mode, const RowTables& t, uint32_t* err, hipStream_t s) {
  if (t.nnz <= 0) return hipSuccess;
  switch (mode) {
    case kRowSigma: return row_tables_mode<kRowSigma>(t, err, s);
    case kRowTau: return row_tables_mode<kRowTau>(t, err, s);
    case kRowCheck: return row_tables_mode<kRowCheck>(t, err, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------
// MOSS-4Min rank tables (Section 4.2.1).  The order of Section 3.2's example ranks a
// node by degree, then id: with key(x) = d_x * 2^32 + x, x is above y exactly when
// key(x) > key(y).  d_{v,x} = |{y in N_v : y above x}| is then x's place in row v
// sorted by key, largest first, and col_rank lists the row in that order, so that
// N_{v,x} is its first d_{v,x} entries.  The passes below serve when a degree reaches
// 2^16, the CSR was not validated or ids reach 2^24 (the passes further down, which sort
// instead of searching, take every other graph); they go over the work items:
//   local    each piece ranks its entries among themselves, one wave per piece: every
//            lane compares its keys with each key of the piece, broadcast from the lane
//            that holds it; a neighbour's degree comes from the row's ACC_sigma
//            (consecutive differences, read in order) rather than its record (a bitonic sort of the piece in LDS by a block of 256 threads
//            measured slower: it spends more instructions in all, 0.87 against 0.78 ms
//            at n = 1e6, m = 1e7).  A row of one piece is finished here; a longer row's
//            piece writes its keys in descending order (scratch) and its local ranks
//   merge    one block per piece of a longer row: the row's other pieces' sorted keys
//            go through LDS, eight pieces at a time, and each thread adds the keys
//            above its entry (a binary search in LDS)
//   mirror   d_{x,v} is read at the entry (x, v): each upper entry (v, x), x > v,
//            binary-searches row x for v and writes both entries' mirror ranks.  A
//            wave takes a 256-entry span of the CSR, four entries a lane, and runs the
//            lane's four searches in step so their loads go out together (one wave per
//            row piece: 105 us at n = 1e5, m = 1e6; spans: 79 us; 1.20 ms at n = 1e6,
//            m = 1e7).  Id guides for the long rows (the bucket starts of their ids, so
//            a search in a hub row is a guide pair and a window of about four entries)
//            cut the pass to 1.05 ms at n = 1e6, m = 1e7 but cost 0.13 ms to build, so
//            they are not used; exchanging the ranks through the edge hash set's slots
//            measured 15% faster for a scratch block the size of the set.  What is left
//            is the random exchange itself, two reads and a write per pair in a
//            working set past the MALL
// Equal keys (a repeated neighbour, possible only in an unchecked CSR) are ranked by
// their place in the row, so the ranks of a row are always a permutation of 0..d-1 and
// every place of col_rank is written exactly once.  A missing mirror (also only in an
// unchecked CSR) reads as rank 0, so the entry gets weight 0.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t order_key(const uint4* __restrict__ rec, int32_t x) {
  return ((uint64_t)row_of(rec, x).y << 32) | (uint64_t)(uint32_t)x;
}

// The same key for the neighbour x at entry e of a row that starts at r0, with d_x taken
// from the row's prefix of d_x - 1 (ACC_sigma), read in order, instead of x's record.
__device__ __forceinline__ uint64_t entry_key(const uint32_t* __restrict__ sig, int32_t e, int32_t r0, int32_t x) {
  const uint32_t d1 = sig[e] - (e > r0 ? sig[e - 1] : 0u);
  return ((uint64_t)(d1 + 1u) << 32) | (uint64_t)(uint32_t)x;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(256) void k_rank_local(int64_t n_items, const uint64_t* __restrict__ items,
                                                    const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                    const uint32_t* __restrict__ sig, uint64_t* __restrict__ keys,
                                                    uint32_t* __restrict__ rank32, int32_t* __restrict__ col_rank) {
  const int lane = lane_id();
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n_items; i += nwaves) {
    const ItemRange it = item_range(items, rp, i);
    const int32_t len = it.e1 - it.e0;  // 1 .. kItem
    const bool single = it.e0 == it.r0 && it.e1 == it.r1;
    uint64_t k[kItem / 64];
    int32_t x[kItem / 64];
    uint32_t above[kItem / 64];
#pragma unroll
    for (int c = 0; c < kItem / 64; ++c) {
      const int32_t e = it.e0 + c * 64 + lane;
      x[c] = e < it.e1 ? col[e] : 0;
      k[c] = e < it.e1 ? entry_key(sig, e, it.r0, x[c]) : 0ull;
      above[c] = 0;
    }
#pragma unroll
    for (int c2 = 0; c2 < kItem / 64; ++c2) {
      if (c2 * 64 >= len) break;  // wave-uniform
      const int lim = min(64, len - c2 * 64);
      for (int j = 0; j < lim; ++j) {
        const uint64_t kj = readlane64(k[c2], j);
        const int pj = c2 * 64 + j;  // its place in the piece
#pragma unroll
        for (int c = 0; c < kItem / 64; ++c)
          above[c] += (kj > k[c] || (kj == k[c] && pj < c * 64 + lane)) ? 1u : 0u;
      }
    }
#pragma unroll
    for (int c = 0; c < kItem / 64; ++c) {
      const int32_t e = it.e0 + c * 64 + lane;
      if (e >= it.e1) continue;
      // the mirror rank is written later, by the entry's upper partner; zero meanwhile
      reinterpret_cast<uint2*>(rank32)[e] = make_uint2(above[c], 0u);
      if (single) col_rank[it.r0 + (int32_t)above[c]] = x[c];
      else keys[it.e0 + (int32_t)above[c]] = k[c];
    }
  }
}

constexpr int kMergeBatch = 8;  // pieces staged in LDS at a time

__global__ __launch_bounds__(256) void k_rank_merge(int64_t n_items, const uint64_t* __restrict__ items,
                                                    const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                    const uint32_t* __restrict__ sig, const uint64_t* __restrict__ keys,
                                                    uint32_t* __restrict__ rank32, int32_t* __restrict__ col_rank) {
  __shared__ uint64_t sk[kMergeBatch][kItem];
  const int tid = threadIdx.x;  // blockDim.x == kItem: one thread per entry of the piece
  for (int64_t i = blockIdx.x; i < n_items; i += gridDim.x) {  // block-uniform
    const ItemRange it = item_range(items, rp, i);
    if (it.e0 == it.r0 && it.e1 == it.r1) continue;  // finished by k_rank_local
    const int32_t pieces = (it.r1 - it.r0 + kItem - 1) / kItem;
    const int32_t e = it.e0 + tid;
    const bool in = e < it.e1;
    const int32_t x = in ? col[e] : 0;
    const uint64_t key = in ? entry_key(sig, e, it.r0, x) : 0ull;
    uint32_t r = in ? rank32[2 * (int64_t)e] : 0u;
    for (int32_t p0 = 0; p0 < pieces; p0 += kMergeBatch) {
      __syncthreads();  // the previous batch's searches are done
#pragma unroll
      for (int j = 0; j < kMergeBatch; ++j) {
        const int32_t q0 = it.r0 + (p0 + j) * kItem;
        if (p0 + j < pieces && q0 + tid < it.r1) sk[j][tid] = keys[q0 + tid];
      }
      __syncthreads();
      if (!in) continue;
#pragma unroll
      for (int j = 0; j < kMergeBatch; ++j) {
        const int32_t p = p0 + j;
        if (p >= pieces || p == it.piece) continue;
        const int32_t len = min(it.r1 - (it.r0 + p * kItem), kItem);
        const bool earlier = p < it.piece;  // its equal keys come first
        int32_t lo = 0, hi = len;  // first place whose key does not come before `key`
        while (lo < hi) {
          const int32_t mid = (lo + hi) >> 1;
          const uint64_t km = sk[j][mid];
          if (km > key || (earlier && km == key)) lo = mid + 1;
          else hi = mid;
        }
        r += (uint32_t)lo;
      }
    }
    if (in) {
      rank32[2 * (int64_t)e] = r;
      col_rank[it.r0 + (int32_t)r] = x;
    }
  }
}

// Mirror ranks: the entry (v, x) with x >= v finds its partner (x, v) by a binary
// search of row x and writes both entries' d_{x,v}.  A wave takes a 256-entry span of
// the CSR, four entries a lane (their rows from the span's row starts), and runs the
// lane's four searches in step, so their loads go out together.  A symmetric CSR
// always holds the partner; without it (unchecked input) the weight stays 0.
__global__ __launch_bounds__(256) void k_rank_mirror(int64_t nnz, const int32_t* __restrict__ span_row,
                                                     const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     const uint4* __restrict__ rec, uint32_t* __restrict__ rank32) {
  __shared__ __align__(16) uint32_t hist[4][kSpan];
  constexpr int kPer = kSpanPer;
  const int lane = lane_id();
  uint32_t* wh = hist[threadIdx.x >> 6];
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t spans = (nnz + kSpan - 1) / kSpan;
  for (int64_t sp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; sp < spans; sp += nwaves) {
    const int64_t S = sp * kSpan;
    int32_t c[kPer], row[kPer], lo[kPer], len[kPer], end[kPer];
    bool head[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) c[k] = S + lane + 64 * k < nnz ? col[S + lane + 64 * k] : -1;
    span_rows(rp, S, span_row[sp], span_row[sp + 1], wh, row, head);
    uint2 X[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) X[k] = row_of(rec, c[k] >= row[k] ? c[k] : 0);  // 4 loads, one wait
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const bool up = c[k] >= row[k];  // x >= v; never past nnz, where c = -1
      lo[k] = up ? (int32_t)X[k].x : 0;
      len[k] = up ? (int32_t)X[k].y : 0;
      end[k] = lo[k] + len[k];
    }
    for (;;) {  // first entry of row x not below v, four searches in step
      bool more = false;
#pragma unroll
      for (int k = 0; k < kPer; ++k) more |= len[k] > 0;
      if (!more) break;
      int32_t probe[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) probe[k] = col[len[k] > 0 ? lo[k] + (len[k] >> 1) : 0];  // 4 loads, one wait
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        if (len[k] > 0) {
          const int32_t half = len[k] >> 1;
          if (probe[k] < row[k]) {
            lo[k] += half + 1;
            len[k] -= half + 1;
          } else {
            len[k] = half;
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t e = S + lane + 64 * k;
      if (c[k] >= row[k] && lo[k] < end[k] && col[lo[k]] == row[k]) {
        rank32[2 * e + 1] = rank32[2 * (int64_t)lo[k]];
        rank32[2 * (int64_t)lo[k] + 1] = rank32[2 * e];
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// The rank passes used when every degree is below 2^16 (a degree and a place within a
// row then fit 16-bit fields).  They replace the per-piece passes above by passes that
// read each entry a fixed number of times:
//   short rows (d <= kItem)   one wave per 256-entry span ranks the rows that start in
//                             the span (at most 511 entries, staged with their keys in
//                             LDS): rows of up to kPairMax entries by counting, for each
//                             entry, the keys of its row above its own; longer ones by a
//                             bitonic sort of the row in registers (64, 128 or 256 keys)
//   long rows                 one block per row: a stable LSD radix sort of the row by
//                             degree, 8 bits a pass, over the places in descending order;
//                             rows up to kLongMid entries sort with a small block, longer
//                             ones with a full one, both in LDS (beyond kLongBig entries
//                             in the row's own scratch)
//   mirror ranks              in a validated CSR, sorting the entries stably by column
//                             puts the entry (v, x) at the index of (x, v): the entries
//                             of column x come in row order, i.e. in the order of row x,
//                             and symmetry gives column x exactly d_x places from
//                             row_ptr[x] on.  Two LSD radix passes over the column's bits
//                             (one block per 8192-entry tile: count, exclusive scan of the
//                             digit-major counts, stable scatter) carry d_{v,x} along, so
//                             the second pass writes it straight into rank[mirror].y
// Within a row, entries of equal degree rank by descending place, which is descending id
// in a sorted row (the order of Section 3.2's example); repeated neighbours (possible
// only in an unchecked CSR) get distinct ranks in some order.
// ---------------------------------------------------------------------------------
constexpr uint32_t kPairMax = 32;     // short rows up to this length rank by pairwise counts
constexpr int32_t kLongMid = 2048;    // rows up to this length sort with a 256-thread block
constexpr int32_t kLongBig = 32768;   // longer rows up to this length sort in LDS with 1024 threads

// Lanes among `act` whose `bits`-bit digit equals this lane's (uniform control flow).
__device__ __forceinline__ uint64_t wave_match(uint32_t digit, int bits, uint64_t act) {
  uint64_t m = act;
  for (int b = 0; b < bits; ++b) {
    const bool one = (digit >> b) & 1u;
    const uint64_t y = __ballot(one);
    m &= one ? y : ~y;
  }
  return m;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return (uint32_t)__popcll(m & ((1ull << lane_id()) - 1ull));
}

__device__ __forceinline__ uint32_t wave_max_exclusive(uint32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, off, 64);
    if (lane >= off) x = max(x, y);
  }
  const uint32_t e = (uint32_t)__shfl_up((int)x, 1, 64);
  return lane ? e : 0u;
}

// Ascending bitonic sort of the wave's 64 K values, lane l holding places l K .. l K + K - 1.
template <int K>
__device__ __forceinline__ void wave_bitonic(uint32_t (&a)[K]) {
  const int lane = lane_id();
#pragma unroll
  for (int size = 2; size <= 64 * K; size <<= 1) {
#pragma unroll
    for (int j = size >> 1; j > 0; j >>= 1) {
      if (j >= K) {  // the partner is in lane ^ (j / K), same slot
#pragma unroll
        for (int t = 0; t < K; ++t) {
          const int i = lane * K + t;
          const uint32_t b = (uint32_t)__shfl_xor((int)a[t], j / K, 64);
          const bool low = (i & j) == 0, asc = (i & size) == 0;
          a[t] = low == asc ? min(a[t], b) : max(a[t], b);
        }
      } else {
#pragma unroll
        for (int t = 0; t < K; ++t) {
          if (t & j) continue;
          const bool asc = ((lane * K + t) & size) == 0;
          const uint32_t x = a[t], y = a[t | j];
          a[t] = asc ? min(x, y) : max(x, y);
          a[t | j] = asc ? max(x, y) : min(x, y);
        }
      }
    }
  }
}

// One row of d <= 64 K entries whose keys (degree << 32 | id) sit at key[os ..]: sorted on
// ((0xFFFF - degree) << 8 | (255 - place)), so its q-th value is the entry of rank q.
template <int K>
__device__ void rank_row_wave(const uint64_t* key, uint32_t os, uint32_t d, int64_t r0, int zero_mirror,
                              uint32_t* __restrict__ rank32, int32_t* __restrict__ col_rank) {
  const int lane = lane_id();
  uint32_t a[K];
#pragma unroll
  for (int t = 0; t < K; ++t) {
    const uint32_t q = lane * K + t;
    a[t] = q < d ? (0xFFFFu - (uint32_t)(key[os + q] >> 32)) << 8 | (255u - q) : 0xFFFFFFFFu;
  }
  wave_bitonic<K>(a);
#pragma unroll
  for (int t = 0; t < K; ++t) {
    const uint32_t q = lane * K + t;
    if (q >= d) continue;
    const uint32_t place = 255u - (a[t] & 255u);
    const int64_t e = r0 + place;
    if (zero_mirror) reinterpret_cast<uint2*>(rank32)[e] = make_uint2(q, 0u);
    else rank32[2 * e] = q;
    col_rank[r0 + q] = (int32_t)(uint32_t)key[os + place];
  }
}

// Short rows.  seg[o] marks a row starting at offset o of the span with
// ((o + 1) << 16 | d); a running maximum over the offsets then gives every offset the
// start and length of the last row starting at or before it, and the offset belongs to
// that row iff it lies within its d entries.
constexpr int kShortWin = 2 * (int)kSpan;
constexpr int kShortSorted = 8;  // rows longer than kPairMax starting in one span (at most 256 / 33 + 1)

__global__ __launch_bounds__(256) void k_rank_short(int64_t nnz, const int32_t* __restrict__ span_row,
                                                    const uint4* __restrict__ rec, const int32_t* __restrict__ col,
                                                    const uint32_t* __restrict__ sig, int zero_mirror,
                                                    uint32_t* __restrict__ rank32, int32_t* __restrict__ col_rank) {
  __shared__ uint64_t s_key[4][kShortWin];
  __shared__ __align__(16) uint32_t s_seg[4][kShortWin];
  __shared__ uint32_t s_sorted[4][kShortSorted];
  constexpr int kPer = kShortWin / 64;
  const int lane = lane_id(), w = threadIdx.x >> 6;
  uint64_t* key = s_key[w];
  uint32_t* seg = s_seg[w];
  uint32_t* sorted = s_sorted[w];
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t spans = (nnz + kSpan - 1) / kSpan;
  for (int64_t sp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; sp < spans; sp += nwaves) {
    const int64_t S = sp * kSpan;
    const int32_t v0 = span_row[sp], last = span_row[sp + 1];
#pragma unroll
    for (int c = 0; c < kPer; ++c) seg[lane + 64 * c] = 0;
    wave_lds_sync();
    uint32_t end = 0, n_sorted = 0;  // one past the owned rows' last offset; rows to sort
    for (int64_t j0 = v0; j0 <= (int64_t)last; j0 += 64) {  // wave-uniform
      const int64_t j = j0 + lane;
      bool to_sort = false;
      uint32_t mark = 0;
      if (j <= (int64_t)last) {
        const uint2 rr = row_of(rec, (int32_t)j);
        const int64_t o = (int64_t)rr.x - S;
        if (o >= 0 && o < kSpan && rr.y >= 1u && rr.y <= (uint32_t)kItem) {
          mark = (uint32_t)(o + 1) << 16 | rr.y;
          seg[o] = mark;
          end = max(end, (uint32_t)o + rr.y);
          to_sort = rr.y > kPairMax;
        }
      }
      const uint64_t sb = __ballot(to_sort);
      if (to_sort) sorted[n_sorted + lanes_below(sb)] = mark;
      n_sorted += (uint32_t)__popcll(sb);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) end = max(end, (uint32_t)__shfl_xor((int)end, off, 64));
    if (end == 0) continue;  // wave-uniform: no short row starts here
    wave_lds_sync();
    {  // running maximum over the offsets, eight consecutive offsets a lane
      uint4 a = reinterpret_cast<const uint4*>(seg)[2 * lane], b = reinterpret_cast<const uint4*>(seg)[2 * lane + 1];
      a.y = max(a.y, a.x);
      a.z = max(a.z, a.y);
      a.w = max(a.w, a.z);
      b.x = max(b.x, a.w);
      b.y = max(b.y, b.x);
      b.z = max(b.z, b.y);
      b.w = max(b.w, b.z);
      const uint32_t before = wave_max_exclusive(b.w);
      a = make_uint4(max(a.x, before), max(a.y, before), max(a.z, before), max(a.w, before));
      b = make_uint4(max(b.x, before), max(b.y, before), max(b.z, before), max(b.w, before));
      wave_lds_sync();
      reinterpret_cast<uint4*>(seg)[2 * lane] = a;
      reinterpret_cast<uint4*>(seg)[2 * lane + 1] = b;
    }
    wave_lds_sync();
    {  // keys of the owned entries: all loads issued before the first is used
      uint32_t xs[kPer], s1[kPer], s0[kPer];
      bool own[kPer];
#pragma unroll
      for (int c = 0; c < kPer; ++c) {
        const uint32_t o = lane + 64 * c, g = seg[o], os = (g >> 16) - 1u;
        own[c] = g != 0 && o < os + (g & 0xFFFFu);
        const int64_t e = own[c] ? S + o : S;  // S itself is a real entry
        xs[c] = (uint32_t)col[e];
        s1[c] = sig[e];
        s0[c] = own[c] && o > os ? sig[e - 1] : 0u;
      }
#pragma unroll
      for (int c = 0; c < kPer; ++c)
        if (own[c]) key[lane + 64 * c] = (uint64_t)(s1[c] - s0[c] + 1u) << 32 | xs[c];
    }
    wave_lds_sync();
#pragma unroll 1
    for (int c = 0; c < kPer; ++c) {  // rows of up to kPairMax entries: pairwise counts
      if (64u * c >= end) break;  // wave-uniform
      const uint32_t o = lane + 64 * c, g = seg[o], os = (g >> 16) - 1u;
      const uint32_t d = g != 0 && o < os + (g & 0xFFFFu) && (g & 0xFFFFu) <= kPairMax ? g & 0xFFFFu : 0u;
      const bool own = d != 0;
      const uint64_t k = own ? key[o] : 0ull;
      uint32_t above = 0;
      for (uint32_t t = os, t1 = os + d; t < t1; ++t) {
        const uint64_t kt = key[t];
        above += (kt > k || (kt == k && t > o)) ? 1u : 0u;
      }
      if (own) {
        const int64_t e = S + o;
        if (zero_mirror) reinterpret_cast<uint2*>(rank32)[e] = make_uint2(above, 0u);
        else rank32[2 * e] = above;
        col_rank[S + os + above] = (int32_t)(uint32_t)k;
      }
    }
    for (uint32_t r = 0; r < n_sorted; ++r) {  // wave-uniform: the longer rows, sorted
      const uint32_t g = sorted[r], os = (g >> 16) - 1u, d = g & 0xFFFFu;
      if (d <= 64) rank_row_wave<1>(key, os, d, S + os, zero_mirror, rank32, col_rank);
      else if (d <= 128) rank_row_wave<2>(key, os, d, S + os, zero_mirror, rank32, col_rank);
      else rank_row_wave<4>(key, os, d, S + os, zero_mirror, rank32, col_rank);
    }
    wave_lds_sync();  // the LDS is reused by the wave's next span
  }
}

// One long row [r0, r0 + d) by a block of kWaves waves: kv[i] = the degree of the
// neighbour at place i (LDS, or the row's own scratch beyond the LDS size); perm holds
// the order after the first pass.  Source position j of the first pass is place d - 1 - j.
// Called by the whole block; returns synchronised.
template <int kWaves>
__device__ void rank_row_block(int32_t r0, int32_t d, int passes, const int32_t* __restrict__ col,
                               const uint32_t* __restrict__ sig, uint16_t* kv, uint16_t* perm,
                               uint32_t (*hist)[256], uint32_t* wave_tot, int zero_mirror,
                               uint32_t* __restrict__ rank32, int32_t* __restrict__ col_rank) {
  const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
#pragma unroll 8
  for (int32_t i = tid; i < d; i += kWaves * 64) {
    const uint32_t s1 = sig[r0 + i], s0 = i > 0 ? sig[r0 + i - 1] : 0u;
    kv[i] = (uint16_t)(s1 - s0 + 1u);
  }
  const int32_t iters = (d + kWaves * 64 - 1) / (kWaves * 64);  // 64-entry groups per wave
  const int32_t j0 = w * iters * 64;
  for (int p = 0; p < passes; ++p) {
    for (int i = lane; i < 256; i += 64) hist[w][i] = 0;
    __syncthreads();  // kv, or the previous pass's perm, complete
    for (int sweep = 0; sweep < 2; ++sweep) {  // 0: count, 1: scatter
      for (int32_t it = 0; it < iters; ++it) {
        const int32_t j = j0 + it * 64 + lane;
        const bool valid = j < d;
        const uint64_t act = __ballot(valid);
        if (act == 0) break;  // wave-uniform
        const int32_t i = !valid ? 0 : (p == 0 ? d - 1 - j : (int32_t)perm[j]);
        const uint32_t dg = valid ? 255u - (((uint32_t)kv[i] >> (8 * p)) & 255u) : 0u;
        if (sweep == 0) {
          if (valid) atomicAdd(&hist[w][dg], 1u);
          continue;
        }
        const uint64_t m = wave_match(dg, 8, act);
        const uint32_t below = lanes_below(m);
        const uint32_t base = valid ? hist[w][dg] : 0u;
        if (valid && below == 0) hist[w][dg] = base + (uint32_t)__popcll(m);
        const uint32_t pos = base + below;
        if (!valid || pos >= (uint32_t)d) continue;  // never, with exact counts
        if (p + 1 < passes) {
          perm[pos] = (uint16_t)i;
        } else {
          const int64_t e = (int64_t)r0 + i;
          if (zero_mirror) reinterpret_cast<uint2*>(rank32)[e] = make_uint2(pos, 0u);
          else rank32[2 * e] = pos;
        }
      }
      if (sweep == 1) break;
      __syncthreads();  // every wave's counts are in
      // digit t's first place: the counts of all smaller digits, then of the waves before
      const int t = tid;
      uint32_t tot = 0;
      if (t < 256)
        for (int q = 0; q < kWaves; ++q) tot += hist[q][t];
      bool unused = false;
      const uint32_t incl = (uint32_t)wave_inclusive_scan((uint64_t)tot, unused);
      if (t < 256 && lane == 63) wave_tot[w] = incl;
      __syncthreads();
      if (t < 256) {
        uint32_t run = incl - tot;
        for (int q = 0; q < w; ++q) run += wave_tot[q];
        for (int q = 0; q < kWaves; ++q) {
          const uint32_t c = hist[q][t];
          hist[q][t] = run;
          run += c;
        }
      }
      __syncthreads();
    }
    __syncthreads();  // this pass's perm (read by the next pass) and hist reads complete
  }
  // col_rank from the ranks just written (visible to the block after the barrier), with
  // independent loads rather than one per step of the scatter
#pragma unroll 4
  for (int32_t i = tid; i < d; i += kWaves * 64) col_rank[r0 + (int32_t)rank32[2 * ((int64_t)r0 + i)]] = col[r0 + i];
  __syncthreads();
}

// Rows longer than kItem into two lists: up to kLongMid entries (mid) and longer (big).
// Block b takes the rows [b c, (b + 1) c) in two coalesced sweeps, counting first so
// that it reserves its places with one atomic per list.  counters[0..1] must be zero.
__global__ __launch_bounds__(256) void k_long_rows(int32_t n, const int32_t* __restrict__ rp,
                                                   int32_t* __restrict__ mid, int32_t* __restrict__ big,
                                                   uint32_t* __restrict__ counters) {
  __shared__ uint32_t s_cnt[2], s_base[2];
  const int64_t chunk = ((int64_t)n + gridDim.x - 1) / gridDim.x;
  const int64_t v_begin = (int64_t)blockIdx.x * chunk, v_end = min((int64_t)n, v_begin + chunk);
  if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t v = v_begin + threadIdx.x; v < v_end; v += 256) {
    const int32_t d = rp[v + 1] - rp[v];
    if (d > kItem) atomicAdd(&s_cnt[d <= kLongMid ? 0 : 1], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    s_base[threadIdx.x] = s_cnt[threadIdx.x] ? atomicAdd(&counters[threadIdx.x], s_cnt[threadIdx.x]) : 0u;
    s_cnt[threadIdx.x] = 0;
  }
  __syncthreads();
  for (int64_t v = v_begin + threadIdx.x; v < v_end; v += 256) {
    const int32_t d = rp[v + 1] - rp[v];
    if (d <= kItem) continue;
    const int which = d <= kLongMid ? 0 : 1;
    const uint32_t at = s_base[which] + atomicAdd(&s_cnt[which], 1u);
    (which ? big : mid)[at] = (int32_t)v;
  }
}

// The rows of a list, one block a row (block b: entries b, b + G, ...), sorted by
// rank_row_block in LDS up to kCap entries.
template <int kCap, int kWaves>
__global__ __launch_bounds__(kWaves * 64) void k_rank_long(const int32_t* __restrict__ list,
                                                           const uint32_t* __restrict__ count,
                                                           const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col,
                                                           const uint32_t* __restrict__ sig, int passes,
                                                           int zero_mirror, uint32_t* __restrict__ rank32,
                                                           int32_t* __restrict__ col_rank, uint64_t* scratch) {
  __shared__ uint16_t s_kv[kCap], s_perm[kCap];
  __shared__ uint32_t hist[kWaves][256];
  __shared__ uint32_t wave_tot[4];
  const uint32_t rows = *count;
  for (uint32_t r = blockIdx.x; r < rows; r += gridDim.x) {  // block-uniform
    const int32_t v = list[r], r0 = rp[v], d = rp[v + 1] - r0;
    if (d <= kCap) {
      rank_row_block<kWaves>(r0, d, passes, col, sig, s_kv, s_perm, hist, wave_tot, zero_mirror, rank32, col_rank);
    } else {  // the row's own d words of scratch hold its 2d u16
      uint16_t* g = reinterpret_cast<uint16_t*>(scratch + r0);
      rank_row_block<kWaves>(r0, d, passes, col, sig, g, g + d, hist, wave_tot, zero_mirror, rank32, col_rank);
    }
  }
}

// Mirror sort: LSD passes of 8-bit digits over the column (three cover ids below
// 2^24).  The first pass reads the entry's column and d_{v,x} (rank[e].x) and writes
// (column >> 8) << 16 | d_{v,x}; later passes read those words, their digit being the
// word's bits 16 + 8 (p - 1) on.  The last pass writes d_{v,x} into rank[place].y: the
// entry at that place in column order is the mirror of the entry the word came from.
constexpr int kMirWaves = 8;                         // waves per block (tile)
constexpr int kMirWaveTile = 1024;                   // entries per wave: 16 groups of 64
constexpr int kMirTile = kMirWaves * kMirWaveTile;   // entries per tile
constexpr int kMirD = 256;                           // digits per pass

template <bool First>
__device__ __forceinline__ void mirror_item(const int32_t* __restrict__ col, const uint32_t* __restrict__ rank32,
                                            const uint32_t* __restrict__ in, int64_t e, int64_t e1, int shift,
                                            uint32_t& digit, uint32_t& word) {
  digit = 0;
  word = 0;
  if (e >= e1) return;
  if (First) {
    const uint32_t c = (uint32_t)col[e];
    digit = c & 255u;
    word = (c >> 8) << 16 | (rank32[2 * e] & 0xFFFFu);
  } else {
    word = in[e];
    digit = (word >> (16 + shift)) & 255u;
  }
}

// counts[tile * 256 + digit]: the tile's entries with that digit (one block a tile)
template <bool First>
__global__ __launch_bounds__(kMirWaves * 64) void k_mirror_count(int64_t nnz, const int32_t* __restrict__ col,
                                                                 const uint32_t* __restrict__ rank32,
                                                                 const uint32_t* __restrict__ in, int shift,
                                                                 uint32_t* __restrict__ counts) {
  __shared__ uint32_t s_hist[kMirD];
  constexpr int kT = kMirWaves * 64, kPer = kMirTile / kT;
  const int64_t t = blockIdx.x, e0 = t * kMirTile, e1 = min(nnz, e0 + kMirTile);
  if (threadIdx.x < kMirD) s_hist[threadIdx.x] = 0;
  uint32_t dg[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    uint32_t word;
    mirror_item<First>(col, rank32, in, e0 + u * kT + threadIdx.x, e1, shift, dg[u], word);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPer; ++u)
    if (e0 + u * kT + threadIdx.x < e1) atomicAdd(&s_hist[dg[u]], 1u);
  __syncthreads();
  if (threadIdx.x < kMirD) counts[t * kMirD + threadIdx.x] = s_hist[threadIdx.x];
}

// Stable scatter by the digit, one block a tile and each wave an eighth of it in order.
// The tile is first put in digit order in LDS (words and digits at their places within
// the tile), then written out in that order: each digit's run of a tile is about
// kMirTile / 256 = 32 consecutive places, a full line per store instead of one place
// per lane.
template <bool First, bool Last>
__global__ __launch_bounds__(kMirWaves * 64) void k_mirror_scatter(int64_t nnz, const int32_t* __restrict__ col,
                                                                   uint32_t* __restrict__ rank32,
                                                                   const uint32_t* __restrict__ in,
                                                                   uint32_t* __restrict__ out, int shift,
                                                                   const uint32_t* __restrict__ offsets) {
  __shared__ uint32_t hist[kMirWaves][kMirD];  // each wave's next place per digit
  __shared__ uint32_t delta[kMirD];            // place in the output - place in the tile
  __shared__ uint32_t tw[kMirTile];            // words in tile order
  __shared__ uint8_t td[kMirTile];             // their digits
  __shared__ uint32_t wave_tot[kMirWaves];
  constexpr int kIt = kMirWaveTile / 64, kT = kMirWaves * 64;
  const int lane = lane_id(), w = threadIdx.x >> 6, tid = threadIdx.x;
  const int64_t t = blockIdx.x, t0 = t * kMirTile, e1 = min(nnz, t0 + kMirTile);
  const int32_t n_t = (int32_t)(e1 - t0);
  const int64_t b = t0 + (int64_t)w * kMirWaveTile;  // this wave's part
  uint32_t dg[kIt], word[kIt];
#pragma unroll
  for (int u = 0; u < kIt; ++u) mirror_item<First>(col, rank32, in, b + 64 * u + lane, e1, shift, dg[u], word[u]);
  for (int i = lane; i < kMirD; i += 64) hist[w][i] = 0;
  wave_lds_sync();
#pragma unroll
  for (int u = 0; u < kIt; ++u)  // column digits are spread evenly: plain atomics rarely collide
    if (b + 64 * u + lane < e1) atomicAdd(&hist[w][dg[u]], 1u);
  __syncthreads();
  {  // places within the tile: digit-major, then wave (threads below 256: one digit each)
    const int i = tid;
    uint32_t sum = 0;
    if (i < kMirD)
      for (int q = 0; q < kMirWaves; ++q) sum += hist[q][i];
    bool unused = false;
    const uint32_t incl = (uint32_t)wave_inclusive_scan((uint64_t)sum, unused);
    if (lane == 63) wave_tot[w] = incl;
    __syncthreads();
    if (i < kMirD) {
      uint32_t run = incl - sum;
      for (int q = 0; q < w; ++q) run += wave_tot[q];
      delta[i] = offsets[t * kMirD + i] - run;
      for (int q = 0; q < kMirWaves; ++q) {
        const uint32_t c = hist[q][i];
        hist[q][i] = run;
        run += c;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kIt; ++u) {
    const bool valid = b + 64 * u + lane < e1;
    const uint64_t act = __ballot(valid);
    if (act == 0) break;  // wave-uniform
    const uint64_t m = wave_match(dg[u], 8, act);
    const uint32_t below = lanes_below(m);
    const uint32_t base = valid ? hist[w][dg[u]] : 0u;
    if (valid && below == 0) hist[w][dg[u]] = base + (uint32_t)__popcll(m);
    const uint32_t q = base + below;
    if (!valid || q >= (uint32_t)n_t) continue;  // never, with exact counts
    tw[q] = word[u];
    td[q] = (uint8_t)dg[u];
  }
  __syncthreads();
#pragma unroll 4
  for (int32_t q = tid; q < n_t; q += kT) {
    const int64_t pos = (int64_t)q + delta[td[q]];
    if (pos >= nnz) continue;  // never, with exact counts
    if (Last) rank32[2 * pos + 1] = tw[q] & 0xFFFFu;
    else out[pos] = tw[q];
  }
}

// Exclusive scan over a block of 256 threads; `total` gets the block's sum.  Uses
// wave_tot[4]; returns synchronised.
__device__ __forceinline__ uint32_t block_exclusive_256(uint32_t x, uint32_t* wave_tot, uint32_t& total) {
  const int lane = lane_id(), w = threadIdx.x >> 6;
  bool unused = false;
  const uint32_t incl = (uint32_t)wave_inclusive_scan((uint64_t)x, unused);
  if (lane == 63) wave_tot[w] = incl;
  __syncthreads();
  uint32_t before = 0;
  total = 0;
  for (int q = 0; q < 4; ++q) {
    if (q < w) before += wave_tot[q];
    total += wave_tot[q];
  }
  __syncthreads();  // wave_tot may be reused
  return before + incl - x;
}

// The mirror sort's offsets: for tile-major counts c[t D + i], replace each by
// base(i) + sum of c[t' D + i] over the tiles t' < t, base(i) being the count of all
// entries with a smaller digit (the exclusive scan in digit-major order).  Chunks of
// kCntChunk tiles: their per-digit sums S, the exclusive scan of S over the chunks of
// each digit with the digit totals, the digits' bases, then each chunk's tiles in order.
constexpr int kCntChunk = 64;

__global__ __launch_bounds__(256) void k_cnt_chunk_sums(int64_t tiles, uint32_t D, const uint32_t* __restrict__ c,
                                                        uint32_t* __restrict__ S) {
  const uint32_t i = blockIdx.y * 256 + threadIdx.x;
  if (i >= D) return;
  const int64_t t0 = (int64_t)blockIdx.x * kCntChunk, t1 = min(tiles, t0 + kCntChunk);
  uint32_t sum = 0;
#pragma unroll 8
  for (int64_t t = t0; t < t1; ++t) sum += c[t * D + i];
  S[(int64_t)blockIdx.x * D + i] = sum;
}

__global__ __launch_bounds__(256) void k_cnt_chunk_scan(int64_t chunks, uint32_t D, uint32_t* __restrict__ S,
                                                        uint32_t* __restrict__ total) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= D) return;
  uint32_t run = 0;
  for (int64_t k0 = 0; k0 < chunks; k0 += 8) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = k0 + u < chunks ? S[(k0 + u) * D + i] : 0u;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (k0 + u < chunks) S[(k0 + u) * D + i] = run;
      run += v[u];
    }
  }
  total[i] = run;
}

__global__ __launch_bounds__(256) void k_cnt_digit_base(uint32_t D, uint32_t* __restrict__ total) {
  __shared__ uint32_t wave_tot[4];
  const uint32_t per = (D + 255) / 256, i0 = min(D, threadIdx.x * per), i1 = min(D, i0 + per);
  uint32_t sum = 0;
  for (uint32_t i = i0; i < i1; ++i) sum += total[i];
  uint32_t all = 0;
  uint32_t run = block_exclusive_256(sum, wave_tot, all);
  for (uint32_t i = i0; i < i1; ++i) {
    const uint32_t v = total[i];
    total[i] = run;
    run += v;
  }
}

__global__ __launch_bounds__(256) void k_cnt_offsets(int64_t tiles, uint32_t D, uint32_t* __restrict__ c,
                                                     const uint32_t* __restrict__ S, const uint32_t* __restrict__ base) {
  const uint32_t i = blockIdx.y * 256 + threadIdx.x;
  if (i >= D) return;
  const int64_t t0 = (int64_t)blockIdx.x * kCntChunk, t1 = min(tiles, t0 + kCntChunk);
  uint32_t run = base[i] + S[(int64_t)blockIdx.x * D + i];
  for (int64_t q0 = t0; q0 < t1; q0 += 8) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = q0 + u < t1 ? c[(q0 + u) * D + i] : 0u;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (q0 + u < t1) c[(q0 + u) * D + i] = run;
      run += v[u];
    }
  }
}

// words of the mirror sort's counts and their scan: tiles x 256 counts, then S (chunks x
// 256) and the 256 totals
int64_t mirror_work_words(int64_t nnz) {
  const int64_t tiles = (nnz + kMirTile - 1) / kMirTile;
  return (tiles + (tiles + kCntChunk - 1) / kCntChunk + 1) * kMirD;
}

static hipError_t cnt_scan(int64_t tiles, uint32_t D, uint32_t* c, uint32_t* work, hipStream_t s) {
  const int64_t chunks = (tiles + kCntChunk - 1) / kCntChunk;
  uint32_t* S = work;
  uint32_t* total = work + chunks * D;
  const dim3 g2((unsigned)chunks, (D + 255) / 256);
  hipLaunchKernelGGL(k_cnt_chunk_sums, g2, dim3(256), 0, s, tiles, D, c, S);
  hipLaunchKernelGGL(k_cnt_chunk_scan, dim3((D + 255) / 256), dim3(256), 0, s, chunks, D, S, total);
  hipLaunchKernelGGL(k_cnt_digit_base, dim3(1), dim3(256), 0, s, D, total);
  hipLaunchKernelGGL(k_cnt_offsets, g2, dim3(256), 0, s, tiles, D, c, S, total);
  return hipGetLastError();
}

hipError_t launch_rank_tables(const RankTables& t, hipStream_t s) {
  if (t.nnz <= 0) return hipSuccess;
  const dim3 block(256);
  uint32_t* rank32 = reinterpret_cast<uint32_t*>(t.rank);
  const bool fast_local = t.max_degree < 65536;
  int bits = 1;  // of the largest column id
  while (bits < 31 && ((int64_t)1 << bits) < (int64_t)t.n) ++bits;
  const int passes_m = (bits + 7) / 8;
  // the words of alternate passes fill the two halves of `scratch`; they hold d_{v,x} <
  // 2^16 and the column's bits above the first digit (below 2^16 for ids below 2^24)
  const bool sort_mirror = fast_local && t.validated && passes_m <= 3;
  const int zero_mirror = sort_mirror ? 0 : 1;
  hipError_t e = hipSuccess;
  if (fast_local) {
    hipLaunchKernelGGL(k_rank_short, dim3(spans_grid(t.nnz)), block, 0, s, t.nnz, t.span_row, t.rec, t.col,
                       t.acc_sigma, zero_mirror, rank32, t.col_rank);
    const int passes = t.max_degree < 256 ? 1 : 2;
    if (t.max_degree > kItem) {  // the lists and their counters live in `work` until the mirror sort
      uint32_t* counters = t.work;
      int32_t* mid = reinterpret_cast<int32_t*>(t.work + 2);
      int32_t* big = mid + t.nnz / (kItem + 1) + 1;
      e = launch_fill_u32(counters, 0u, 2, s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_long_rows, dim3(256), block, 0, s, t.n, t.rp, mid, big, counters);
      hipLaunchKernelGGL((k_rank_long<kLongMid, 4>), dim3(2048), block, 0, s, mid, counters, t.rp, t.col,
                         t.acc_sigma, passes, zero_mirror, rank32, t.col_rank, t.scratch);
      if (t.max_degree > kLongMid) {
        hipLaunchKernelGGL((k_rank_long<kLongBig, 16>), dim3(256), dim3(1024), 0, s, big, counters + 1, t.rp, t.col,
                           t.acc_sigma, passes, zero_mirror, rank32, t.col_rank, t.scratch);
      }
    }
  } else if (t.n_items > 0) {
    hipLaunchKernelGGL(k_rank_local, dim3(item_grid(t.n_items)), block, 0, s, t.n_items, t.items, t.rp, t.col,
                       t.acc_sigma, t.scratch, rank32, t.col_rank);
    const int merge_grid = (int)std::min<int64_t>(t.n_items, 65536);
    hipLaunchKernelGGL(k_rank_merge, dim3(merge_grid), dim3(kItem), 0, s, t.n_items, t.items, t.rp, t.col,
                       t.acc_sigma, t.scratch, rank32, t.col_rank);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!sort_mirror) {
    hipLaunchKernelGGL(k_rank_mirror, dim3(spans_grid(t.nnz)), block, 0, s, t.nnz, t.span_row, t.rp, t.col, t.rec,
                       rank32);
    return hipGetLastError();
  }
  const int64_t tiles = (t.nnz + kMirTile - 1) / kMirTile;
  uint32_t* half[2] = {reinterpret_cast<uint32_t*>(t.scratch), reinterpret_cast<uint32_t*>(t.scratch) + t.nnz};
  uint32_t* counts = t.work;
  const dim3 mgrid((unsigned)tiles), mblock(kMirWaves * 64);
  for (int p = 0; p < passes_m; ++p) {
    const int shift = p ? 8 * (p - 1) : 0;
    const bool first = p == 0, last = p + 1 == passes_m;
    const uint32_t* in = first ? nullptr : half[(p - 1) & 1];
    uint32_t* out = last ? nullptr : half[p & 1];
    if (first) hipLaunchKernelGGL(k_mirror_count<true>, mgrid, mblock, 0, s, t.nnz, t.col, rank32, in, shift, counts);
    else hipLaunchKernelGGL(k_mirror_count<false>, mgrid, mblock, 0, s, t.nnz, t.col, rank32, in, shift, counts);
    e = cnt_scan(tiles, kMirD, counts, counts + tiles * kMirD, s);
    if (e != hipSuccess) return e;
    if (first && last) {
      hipLaunchKernelGGL((k_mirror_scatter<true, true>), mgrid, mblock, 0, s, t.nnz, t.col, rank32, in, out, shift,
                         counts);
    } else if (first) {
      hipLaunchKernelGGL((k_mirror_scatter<true, false>), mgrid, mblock, 0, s, t.nnz, t.col, rank32, in, out, shift,
                         counts);
    } else if (last) {
      hipLaunchKernelGGL((k_mirror_scatter<false, true>), mgrid, mblock, 0, s, t.nnz, t.col, rank32, in, out, shift,
                         counts);
    } else {
      hipLaunchKernelGGL((k_mirror_scatter<false, false>), mgrid, mblock, 0, s, t.nnz, t.col, rank32, in, out, shift,
                         counts);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ void k_row_totals(int32_t n, const int32_t* __restrict__ rp, const uint64_t* __restrict__ acc,
                             uint64_t* __restrict__ w) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r1 = rp[v + 1];
    w[v] = r1 > rp[v] ? acc[r1 - 1] : 0ull;
  }
}

hipError_t launch_row_totals(int32_t n, const int32_t* rp, const uint64_t* acc, uint64_t* w, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_totals, dim3(fill_grid(n)), dim3(256), 0, s, n, rp, acc, w);
  return hipGetLastError();
}

// Edge hash set: open addressing with linear probing, at least 2.5 slots per edge,
// so a lookup reads about 1.2-1.4 slots.
constexpr double kHashSlotsPerEdge = 2.5;

int edge_hash_bits(int64_t m) {
  int bits = 4;
  while (bits < 40 && (double)(1ll << bits) < kHashSlotsPerEdge * (double)m) ++bits;
  return bits;
}

// Edge filter: 2^bits 64-bit words, at least 8 bits per edge while that stays within
// 8 MB, else the larger of 8 MB and 4 bits per edge.  At 8.4 bits per edge about 2% of
// non-edges get through to the hash set, at 4.2 about 14%.  Measured with the grouped
// schedule: n = 1e5, m = 1e6 (MOSS-4, 1e7 samples), 0.5 MB of filter (4.2 bits) 0.560
// ms, 1 MB (8.4 bits) 0.514 ms; n = 1e6, m = 1e7 (T-5 / Path-5, 5e7 samples each), 8 MB
// (6.7 bits) 5.61 / 8.06 ms, 16 MB (13.4 bits) 6.09 / 8.39 ms, 4 MB (3.4 bits) 5.85 /
// 8.31 ms.  Past a few MB the filter no longer stays in the L2s and its own misses
// cost more than the hash-set reads it saves.
constexpr double kFilterBitsPerEdge = 8.0;
constexpr double kFilterMinBitsPerEdge = 4.0;
constexpr int kFilterCapBits = 20;  // 2^20 words = 8 MB

int edge_filter_bits(int64_t m) {
  auto bits_for = [m](double per_edge) {
    int bits = 1;
    while (bits < 34 && (double)(64ll << bits) < per_edge * (double)m) ++bits;
    return bits;
  };
  const int bits = bits_for(kFilterBitsPerEdge);
  return bits <= kFilterCapBits ? bits : std::max(kFilterCapBits, bits_for(kFilterMinBitsPerEdge));
}

// ---------------------------------------------------------------------------------
// Node weights, one thread per node, from the finished row prefixes:
//   S_v = the row total of ACC_sigma (node record);  Gamma_v = (d_v - 1) S_v  (Section 4.1.1)
//   Gamma^(1)_v = (d_v - 1)(d_v - 2) S_v                      (Section 5.1.1)
//   Gamma^(2)_v = ACC_tau at the row end = S_v^2 - sum (d_x - 1)^2 (Section 5.1.2)
//   Lambda_3 = sum C(d_v, 3), Lambda_4 = sum C(d_v, 4)        (Table 1)
// The Lambdas are reduced per block into `partials` (2 per block) and finished by
// k_lambda_final, so no two blocks update the same word.
// ---------------------------------------------------------------------------------
constexpr int kWeightThreads = 256;

__global__ __launch_bounds__(256) void k_node_weights(int32_t n, const int32_t* __restrict__ rp,
                                                      const uint4* __restrict__ rec,
                                                      const uint64_t* __restrict__ acc_tau, uint64_t* __restrict__ w_gamma,
                                                      uint64_t* __restrict__ w_gamma1, uint64_t* __restrict__ w_gamma2,
                                                      uint64_t* __restrict__ partials, uint32_t* err) {
  __shared__ uint64_t red[2][kWeightThreads / 64];
  __shared__ uint32_t red_bits;
  bool over4 = false, over5 = false;
  uint64_t l3 = 0, l4 = 0;
  if (threadIdx.x == 0) red_bits = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r0 = rp[v], r1 = rp[v + 1];
    const uint64_t d = (uint64_t)(r1 - r0);
    const uint64_t S = (uint64_t)rec[v].z;
    if (w_gamma) w_gamma[v] = d >= 1 ? (d - 1) * S : 0;
    if (w_gamma1) {
      const uint64_t dd = d >= 2 ? (d - 1) * (d - 2) : 0;
      over5 |= __umul64hi(dd, S) != 0;
      w_gamma1[v] = dd * S;
    }
    if (w_gamma2) w_gamma2[v] = d > 0 ? acc_tau[r1 - 1] : 0;
    l3 = add_wrap(l3, choose3(d, over4), over4);
    l4 = add_wrap(l4, choose4(d, over5), over5);
  }
  // block reduction of (l3, l4)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    l3 = add_wrap(l3, __shfl_xor(l3, off, 64), over4);
    l4 = add_wrap(l4, __shfl_xor(l4, off, 64), over5);
  }
  // (every lane of a wave now holds the wave total)
  const int wave = threadIdx.x >> 6;
  if (lane_id() == 0) {
    red[0][wave] = l3;
    red[1][wave] = l4;
  }
  __syncthreads();
  const uint32_t bits = (__ballot(over4) != 0 ? kErrOverflowK4 : 0u) | (__ballot(over5) != 0 ? kErrOverflowK5 : 0u);
  if (bits && lane_id() == 0) atomicOr(&red_bits, bits);
  __syncthreads();
  if (threadIdx.x == 0) {
    bool o4 = false, o5 = false;
    uint64_t a = 0, b = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      a = add_wrap(a, red[0][w], o4);
      b = add_wrap(b, red[1][w], o5);
    }
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = b;
    const uint32_t all = red_bits | (o4 ? kErrOverflowK4 : 0u) | (o5 ? kErrOverflowK5 : 0u);
    if (all) atomicOr(err, all);
  }
}

__global__ __launch_bounds__(256) void k_lambda_final(const uint64_t* __restrict__ partials, int nblocks,
                                                      unsigned long long* __restrict__ lambdas, uint32_t* err) {
  __shared__ uint64_t red[2][4];
  bool o4 = false, o5 = false;
  uint64_t a = 0, b = 0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) {
    a = add_wrap(a, partials[2 * i], o4);
    b = add_wrap(b, partials[2 * i + 1], o5);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a = add_wrap(a, __shfl_xor(a, off, 64), o4);
    b = add_wrap(b, __shfl_xor(b, off, 64), o5);
  }
  if (lane_id() == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  const uint32_t bits = (__ballot(o4) != 0 ? kErrOverflowK4 : 0u) | (__ballot(o5) != 0 ? kErrOverflowK5 : 0u);
  if (bits && lane_id() == 0) atomicOr(err, bits);
  __syncthreads();
  if (threadIdx.x == 0) {
    bool p4 = false, p5 = false;
    uint64_t x = 0, y = 0;
    for (int w = 0; w < 4; ++w) {
      x = add_wrap(x, red[0][w], p4);
      y = add_wrap(y, red[1][w], p5);
    }
    lambdas[0] = x;
    lambdas[1] = y;
    if (p4 || p5) atomicOr(err, (p4 ? kErrOverflowK4 : 0u) | (p5 ? kErrOverflowK5 : 0u));
  }
}

int node_weight_blocks(int32_t n) { return std::max(1, std::min(2048, (int)((n + 255) / 256))); }

hipError_t launch_node_weights(int32_t n, const int32_t* rp, const uint4* rec, const uint64_t* acc_tau,
                               uint64_t* w_gamma, uint64_t* w_gamma1, uint64_t* w_gamma2, uint64_t* partials,
                               unsigned long long* lambdas, uint32_t* err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nb = node_weight_blocks(n);
  hipLaunchKernelGGL(k_node_weights, dim3(nb), dim3(kWeightThreads), 0, s, n, rp, rec, acc_tau, w_gamma,
                     w_gamma1, w_gamma2, partials, err);
  hipLaunchKernelGGL(k_lambda_final, dim3(1), dim3(256), 0, s, partials, nb, lambdas, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Inclusive scans of u64 node arrays (reduce, scan of block sums, apply), blocked
// layout of 8 items per thread, wrap detection on every addition.  Up to three
// arrays of the same length go through one set of launches (blockIdx.y, or the
// block index of the middle step, selects the array).
// ---------------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int64_t kScanTile = kScanThreads * kScanItems;

// Scans one tile in place (inclusive or exclusive), starting from `offset`; returns
// the tile total.  Must be called by all 256 threads.
__device__ uint64_t block_scan_tile(uint64_t* data, int64_t base, int64_t n, uint64_t offset, bool exclusive,
                                    bool& wrapped, uint64_t* wave_tot) {
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const int64_t first = base + (int64_t)tid * kScanItems;
  uint64_t v[kScanItems];
  uint64_t t = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = first + i < n ? data[first + i] : 0;
    t = add_wrap(t, v[i], wrapped);
  }
  const uint64_t incl = wave_inclusive_scan(t, wrapped);
  if (lane == 63) wave_tot[wave] = incl;
  __syncthreads();
  uint64_t before = 0, total = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    if (w < wave) before = add_wrap(before, wave_tot[w], wrapped);
    total = add_wrap(total, wave_tot[w], wrapped);
  }
  __syncthreads();
  uint64_t run = add_wrap(offset, add_wrap(before, incl - t, wrapped), wrapped);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const uint64_t next = add_wrap(run, v[i], wrapped);
    if (first + i < n) data[first + i] = exclusive ? run : next;
    run = next;
  }
  return total;
}

__global__ __launch_bounds__(256) void k_scan_reduce(ScanSet set, int64_t n, uint32_t* err) {
  __shared__ uint64_t wave_tot[kScanThreads / 64];
  const int j = blockIdx.y;
  const uint64_t* __restrict__ in = set.data[j];
  bool wrapped = false;
  const int64_t first = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint64_t t = 0;
  for (int i = 0; i < kScanItems; ++i)
    if (first + i < n) t = add_wrap(t, in[first + i], wrapped);
  const uint64_t incl = wave_inclusive_scan(t, wrapped);
  if (lane_id() == 63) wave_tot[threadIdx.x >> 6] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t total = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) total = add_wrap(total, wave_tot[w], wrapped);
    set.tmp[j][blockIdx.x] = total;
  }
  if (__ballot(wrapped) != 0 && lane_id() == 0) atomicOr(err, set.err_bit[j]);
}

// Exclusive scan of one array's block sums by one block, tile after tile; the
// carry at the end is the array's total.
__global__ __launch_bounds__(256) void k_scan_top(ScanSet set, int64_t nb, uint32_t* err) {
  __shared__ uint64_t wave_tot[kScanThreads / 64];
  const int j = blockIdx.x;
  bool wrapped = false;
  uint64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanTile) {
    const uint64_t tot = block_scan_tile(set.tmp[j], base, nb, carry, true, wrapped, wave_tot);
    carry = add_wrap(carry, tot, wrapped);
  }
  if (threadIdx.x == 0 && set.total[j]) *set.total[j] = carry;
  if (__ballot(wrapped) != 0 && lane_id() == 0) atomicOr(err, set.err_bit[j]);
}

__global__ __launch_bounds__(256) void k_scan_apply(ScanSet set, int64_t n, uint32_t* err) {
  __shared__ uint64_t wave_tot[kScanThreads / 64];
  const int j = blockIdx.y;
  bool wrapped = false;
  block_scan_tile(set.data[j], (int64_t)blockIdx.x * kScanTile, n, set.tmp[j][blockIdx.x], false, wrapped, wave_tot);
  if (__ballot(wrapped) != 0 && lane_id() == 0) atomicOr(err, set.err_bit[j]);
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_scans(const ScanSet& set, int64_t n, uint32_t* err, hipStream_t s) {
  if (n <= 0 || set.count <= 0) return hipSuccess;
  if (set.count > 3) return hipErrorInvalidValue;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb, set.count), dim3(kScanThreads), 0, s, set, n, err);
  hipLaunchKernelGGL(k_scan_top, dim3(set.count), dim3(kScanThreads), 0, s, set, nb, err);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb, set.count), dim3(kScanThreads), 0, s, set, n, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Guide table for a node draw: guide[b] is the node drawn by the smallest word of
// bucket b (the top gbits bits of the word), guide[2^gbits] = n - 1.  The draw is
// monotone in the word, so every word of bucket b picks a node in
// [guide[b], guide[b+1]], and the search runs over that window only.
// ---------------------------------------------------------------------------------
__global__ void k_guides(GuideSet set, int32_t n, int gbits) {
  const int j = blockIdx.y;
  const uint64_t* __restrict__ acc = set.acc[j];
  uint32_t* __restrict__ guide = set.guide[j];
  const int64_t G = 1ll << gbits;
  const uint64_t total = acc[n - 1];
  if (blockIdx.x == 0 && threadIdx.x == 0 && set.total[j]) *set.total[j] = total;
  if (total == 0) return;  // nothing can be drawn; the guide is never read
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= G; b += (int64_t)gridDim.x * blockDim.x) {
    if (b == G) {
      guide[b] = (uint32_t)(n - 1);
    } else {
      const uint64_t r = bounded((uint64_t)b << (64 - gbits), total);
      guide[b] = (uint32_t)first_above(acc, 0, n - 1, r);
    }
  }
}

hipError_t launch_guides(const GuideSet& set, int32_t n, int gbits, hipStream_t s) {
  if (n <= 0 || set.count <= 0) return hipSuccess;
  if (set.count > 3) return hipErrorInvalidValue;
  const int64_t G = (1ll << gbits) + 1;
  hipLaunchKernelGGL(k_guides, dim3(fill_grid(G), set.count), dim3(256), 0, s, set, n, gbits);
  return hipGetLastError();
}

// Weighted pick in a row: the first entry i of the row whose inclusive prefix
// value(i) exceeds x (x < total = value(d-1)).
template <typename F>
__device__ __forceinline__ int32_t row_pick(F value, int32_t d, uint64_t total, uint64_t x,
                                            const uint32_t* __restrict__ guide, uint32_t goff) {
  if (d < kRowGuideMin) return first_above_by(value, 0, d - 1, x);
  const int g = row_guide_bits(d);
  const uint64_t b = x >> row_guide_shift(total, g);
  const uint2 w = load_pair(guide + goff + b);  // guide[b], guide[b + 1]
  // the window lies inside the row for any guide contents (a correct guide needs no clamp)
  const int32_t hi = min((int32_t)w.y, d - 1);
  return first_above_by(value, min((int32_t)w.x, hi), hi, x);
}

struct PrefixOf32 {
  const uint32_t* __restrict__ acc;
  __device__ uint64_t operator()(int32_t i) const { return (uint64_t)acc[i]; }
};

struct PrefixOf64 {
  const uint64_t* __restrict__ acc;
  __device__ uint64_t operator()(int32_t i) const { return acc[i]; }
};

// ---------------------------------------------------------------------------------
// The samplers.  Each returns the motif class of sample k (0 = rejected) and, when
// `nodes` is not null, writes the sampled nodes v, u, w, r, t.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ int32_t pick_node(const SamplerView& a, uint64_t x) {
  const uint64_t r = bounded(x, a.total);
  const uint32_t b = (uint32_t)(x >> (64 - a.gbits));
  const uint2 w = load_pair(a.guide + b);  // guide[b], guide[b + 1]
  return first_above(a.acc_node, (int32_t)w.x, (int32_t)w.y, r);
}

// RandomVertex(N_a - {skip}) with skip in N_a: index j uniform over the row with
// skip's slot removed; the sorted row is read at j and stepped past skip.
__device__ __forceinline__ int32_t neighbour_except(const int32_t* __restrict__ col, int32_t ra, int32_t da,
                                                    int32_t skip, uint64_t word) {
  const int32_t j = (int32_t)bounded(word, (uint64_t)(da - 1));
  const uint2 x = load_pair(col + ra + j);  // j + 1 <= da - 1: both inside the row
  return (int32_t)x.x >= skip ? (int32_t)x.y : (int32_t)x.x;
}

// Induced-edge probes of one sample (the CIS() step of Algorithms 1, 3 and 4): bit i
// of the result is set when {x[i], y[i]} is an edge.  A pair the filter turns away is
// no edge; the others are looked up in the hash set.  The pairs go one after another:
// the empty asm statement keeps the compiler from hoisting later pairs' reads above
// earlier ones, which measured a few per cent faster than issuing all of a sample's
// reads at once (the memory system is already saturated by the other waves).
template <int P>
__device__ __forceinline__ int probe_edges(const SamplerView& a, const int32_t (&x)[P], const int32_t (&y)[P]) {
  int m = 0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    asm volatile("" ::: "memory");
    const uint64_t key = edge_key(x[i], y[i]);
    const uint64_t fm = filter_mask(mix64(key));
    if ((a.filter[edge_slot(key, a.filter_bits)] & fm) != fm) continue;
    const uint64_t h = edge_slot(key, a.edge_bits);
    if (edge_hash_rest(a.edge_slots, a.edge_bits, key, h, a.edge_slots[h])) m |= 1 << i;
  }
  return m;
}

// MOSS-4 (Algorithm 1): v ~ Gamma_v, u ~ d_u - 1 over N_v, w uniform in N_v - {u},
// r uniform in N_u - {v}; rejected when r = w.  Known edges vu, vw, ur; probe bits
// b0 = u~w, b1 = v~r, b2 = w~r.
__device__ __forceinline__ int draw_moss4(const SamplerView& a, const uint8_t* lut, uint64_t seed, uint64_t k,
                                          int32_t* nodes) {
  uint64_t W[4];
  philox_block(k, 0, seed, kMoss4, W);
  const int32_t* __restrict__ col = a.col;
  const int32_t v = pick_node(a, W[0]);
  const uint4 R = a.rec[v];
  const int32_t rv = (int32_t)R.x, dv = (int32_t)R.y;
  const int32_t iu = row_pick(PrefixOf32{a.acc_sigma + rv}, dv, R.z, bounded(W[1], R.z), a.sig_guide, R.w);
  const int32_t u = col[rv + iu];
  int32_t iw = (int32_t)bounded(W[2], (uint64_t)(dv - 1));
  iw += iw >= iu;
  const int32_t w = col[rv + iw];
  const uint2 U = row_of(a.rec, u);
  const int32_t ru = (int32_t)U.x, du = (int32_t)U.y;
  const int32_t r = neighbour_except(col, ru, du, v, W[3]);
  if (nodes) {
    nodes[0] = v; nodes[1] = u; nodes[2] = w; nodes[3] = r; nodes[4] = -1;
  }
  if (r == w) return 0;
  const int32_t px[3] = {u, v, w}, py[3] = {w, r, r};
  return lut[probe_edges<3>(a, px, py)];
}

// Reach count of a MOSS-4Min sample (Section 4.2.1): the ordered draws (w, v, u, r) of
// its four nodes with edges w-v, v-u, u-r, w above u and r above v.  Nodes 0..3 are
// v, u, w, r; bit 4a + b of adj is set when nodes a and b are adjacent; k0..k3 are
// their order keys.  Each such draw has probability 1/check-Gamma, so the sample's
// set was drawn with probability (reach count)/check-Gamma.
__device__ int reach_count(uint32_t adj, uint64_t k0, uint64_t k1, uint64_t k2, uint64_t k3) {
  const uint64_t key[4] = {k0, k1, k2, k3};
  int c = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (w == v || u == w || u == v) continue;
        const int r = 6 - w - v - u;  // the fourth node
        const bool path = (adj >> (4 * w + v) & 1) && (adj >> (4 * v + u) & 1) && (adj >> (4 * u + r) & 1);
        if (path && key[w] > key[u] && key[r] > key[v]) ++c;
      }
  return c;
}

// MOSS-4Min (Algorithm 2): v ~ check-Gamma_v, u ~ d_{u,v} d_{v,u} over N_v (row prefix
// acc_check), w uniform in N_{v,u} and r uniform in N_{u,v} (the first d_{v,u} and
// d_{u,v} entries of the rows in descending order); rejected when r = w.  Known edges
// vu, vw, ur; probe bits as MOSS-4 (b0 = u~w, b1 = v~r, b2 = w~r).  A diamond (class 5)
// is reached by 2, 4 or 6 ordered draws; its count c goes out as the extra bin
// 6 + c/2 in bits 8 and up of the result.
__device__ __forceinline__ int draw_moss4min(const SamplerView& a, const uint8_t* lut, uint64_t seed, uint64_t k,
                                             int32_t* nodes) {
  uint64_t W[4];
  philox_block(k, 0, seed, kMoss4Min, W);
  const int32_t v = pick_node(a, W[0]);
  const uint4 R = a.rec[v];
  const int32_t rv = (int32_t)R.x, dv = (int32_t)R.y;
  const uint64_t* __restrict__ chk = a.acc_check + rv;
  const uint64_t T = chk[dv - 1];
  const int32_t iu = row_pick(PrefixOf64{chk}, dv, T, bounded(W[1], T), a.check_guide, R.w);
  const int32_t u = a.col[rv + iu];
  const uint2 rk = a.rank[rv + iu];  // d_{v,u}, d_{u,v}: both >= 1 for a drawn entry
  const int32_t w = a.col_rank[rv + (int32_t)bounded(W[2], (uint64_t)rk.x)];
  const uint2 U = row_of(a.rec, u);
  const int32_t r = a.col_rank[(int32_t)U.x + (int32_t)bounded(W[3], (uint64_t)rk.y)];
  if (nodes) {
    nodes[0] = v; nodes[1] = u; nodes[2] = w; nodes[3] = r; nodes[4] = -1;
  }
  if (r == w) return 0;
  const int32_t px[3] = {u, v, w}, py[3] = {w, r, r};
  const int m = probe_edges<3>(a, px, py);
  const int c = lut[m];
  if (c != 5) return c;
  // known v-u (0,1), v-w (0,2), u-r (1,3); probed u-w (1,2), v-r (0,3), w-r (2,3)
  uint32_t adj = (1u << 1) | (1u << 4) | (1u << 2) | (1u << 8) | (1u << 7) | (1u << 13);
  if (m & 1) adj |= (1u << 6) | (1u << 9);
  if (m & 2) adj |= (1u << 3) | (1u << 12);
  if (m & 4) adj |= (1u << 11) | (1u << 14);
  const uint64_t kv = ((uint64_t)R.y << 32) | (uint32_t)v, ku = ((uint64_t)U.y << 32) | (uint32_t)u;
  const uint64_t kw = ((uint64_t)row_of(a.rec, w).y << 32) | (uint32_t)w;
  const uint64_t kr = ((uint64_t)row_of(a.rec, r).y << 32) | (uint32_t)r;
  return c | ((6 + reach_count(adj, kv, ku, kw, kr) / 2) << 8);
}

// T-5 (Algorithm 3): v ~ Gamma^(1)_v, u ~ d_u - 1 over N_v, w then r uniform over
// N_v - {u} and N_v - {u, w} (excluded slots skipped in ascending order), t uniform in
// N_u - {v}; rejected when t is w or r.  Known edges vu, vw, vr, ut; probe bits
// b0 = u~w, b1 = u~r, b2 = w~r, b3 = v~t, b4 = w~t, b5 = r~t.
__device__ __forceinline__ int draw_t5(const SamplerView& a, const uint8_t* lut, uint64_t seed, uint64_t k,
                                       int32_t* nodes) {
  uint64_t W[4], X[4];
  philox_block(k, 0, seed, kT5, W);
  philox_block(k, 1, seed, kT5, X);
  const int32_t* __restrict__ col = a.col;
  const int32_t v = pick_node(a, W[0]);
  const uint4 R = a.rec[v];
  const int32_t rv = (int32_t)R.x, dv = (int32_t)R.y;
  const int32_t iu = row_pick(PrefixOf32{a.acc_sigma + rv}, dv, R.z, bounded(W[1], R.z), a.sig_guide, R.w);
  const int32_t u = col[rv + iu];
  int32_t iw = (int32_t)bounded(W[2], (uint64_t)(dv - 1));
  iw += iw >= iu;
  const int32_t w = col[rv + iw];
  const int32_t lo = min(iu, iw), hi = max(iu, iw);
  int32_t ir = (int32_t)bounded(W[3], (uint64_t)(dv - 2));
  ir += ir >= lo;
  ir += ir >= hi;
  const int32_t r = col[rv + ir];
  const uint2 U = row_of(a.rec, u);
  const int32_t ru = (int32_t)U.x, du = (int32_t)U.y;
  const int32_t t = neighbour_except(col, ru, du, v, X[0]);
  if (nodes) {
    nodes[0] = v; nodes[1] = u; nodes[2] = w; nodes[3] = r; nodes[4] = t;
  }
  if (t == w || t == r) return 0;
  const int32_t px[6] = {u, u, w, v, w, r}, py[6] = {w, r, r, t, t, t};
  return lut[probe_edges<6>(a, px, py)];
}

// Path-5 (Algorithm 4): v ~ Gamma^(2)_v, u ~ tau^(v) (row prefix ACC_tau), w ~ mu^(v,u)
// over N_v - {u} (a draw over ACC_sigma with u's block cut out, Section 5.1.5),
// r uniform in N_u - {v}, t uniform in N_w - {v}; rejected when t = u, r = w or t = r.
// Known edges vu, vw, ur, wt; probe bits b0 = v~r, b1 = v~t, b2 = u~w, b3 = u~t,
// b4 = w~r, b5 = r~t.
__device__ __forceinline__ int draw_path5(const SamplerView& a, const uint8_t* lut, uint64_t seed, uint64_t k,
                                          int32_t* nodes) {
  uint64_t W[4], X[4];
  philox_block(k, 0, seed, kPath5, W);
  philox_block(k, 1, seed, kPath5, X);
  const int32_t* __restrict__ col = a.col;
  const int32_t v = pick_node(a, W[0]);
  const uint4 R = a.rec[v];
  const int32_t rv = (int32_t)R.x, dv = (int32_t)R.y;
  const uint64_t* __restrict__ tau = a.acc_tau + rv;
  const uint64_t T = tau[dv - 1];
  const int32_t iu = row_pick(PrefixOf64{tau}, dv, T, bounded(W[1], T), a.tau_guide, R.w);
  const int32_t u = col[rv + iu];
  const uint32_t* __restrict__ sig = a.acc_sigma + rv;
  const uint64_t Sv = R.z;
  uint64_t blk_lo, blk_hi;  // u's block of ACC_sigma: [sig[iu - 1], sig[iu])
  if (iu > 0) {
    const uint2 s2 = load_pair(sig + iu - 1);
    blk_lo = s2.x;
    blk_hi = s2.y;
  } else {
    blk_lo = 0;
    blk_hi = sig[0];
  }
  const uint64_t du1 = blk_hi - blk_lo;
  uint64_t x = bounded(W[2], Sv - du1);
  x += x >= blk_lo ? du1 : 0;
  const int32_t iw = row_pick(PrefixOf32{sig}, dv, Sv, x, a.sig_guide, R.w);
  const int32_t w = col[rv + iw];
  const uint2 U = row_of(a.rec, u), Wr = row_of(a.rec, w);
  const int32_t ru = (int32_t)U.x, du = (int32_t)U.y, rw = (int32_t)Wr.x, dw = (int32_t)Wr.y;
  const int32_t r = neighbour_except(col, ru, du, v, W[3]);
  const int32_t t = neighbour_except(col, rw, dw, v, X[0]);
  if (nodes) {
    nodes[0] = v; nodes[1] = u; nodes[2] = w; nodes[3] = r; nodes[4] = t;
  }
  if (t == u || r == w || t == r) return 0;
  const int32_t px[6] = {v, v, u, u, w, r}, py[6] = {r, t, w, t, r, t};
  return lut[probe_edges<6>(a, px, py)];
}

template <int S>
__device__ __forceinline__ int draw(const SamplerView& a, const uint8_t* lut, uint64_t seed, uint64_t k,
                                    int32_t* nodes) {
  if constexpr (S == kMoss4) return draw_moss4(a, lut, seed, k, nodes);
  else if constexpr (S == kMoss4Min) return draw_moss4min(a, lut, seed, k, nodes);
  else if constexpr (S == kT5) return draw_t5(a, lut, seed, k, nodes);
  else return draw_path5(a, lut, seed, k, nodes);
}

template <int S>
__device__ __forceinline__ void load_lut(uint8_t* lut) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    if constexpr (S == kMoss4 || S == kMoss4Min) lut[tid] = tid < 8 ? c_lut4[tid] : 0;
    else if constexpr (S == kT5) lut[tid] = c_lut5t[tid];
    else lut[tid] = c_lut5p[tid];
  }
}

constexpr int kMaxWaves = 16;  // 1024 threads per block at most
constexpr int kBins = 22;

// One sample into a wave's LDS counters: its class, and for a MOSS-4Min diamond the
// reach-count bin too.
__device__ __forceinline__ void count_sample(uint32_t* bins, int c) {
  atomicAdd(&bins[c & 0xff], 1u);
  if (c >> 8) atomicAdd(&bins[c >> 8], 1u);
}

// ---------------------------------------------------------------------------------
// Lane order.  A sample's node v is monotone in its first random word W0 (the node draw
// inverts the prefix of the node weights), so samples whose first words share their
// top bits draw v from one narrow range of nodes.  A block can take its samples
// kLaneChunk at a time, counting-sort them in LDS by the top 8 bits of W0, and let its
// lanes draw them in that order: the 64 lanes of a wave then cover about 1/64 of the
// node-weight mass of the chunk, so their reads of the node prefix, guide, record, row
// prefix and row entries of v fall on a few cache lines instead of one per lane.  Each
// sample is still drawn once from its own index, so the counts are those of index
// order.
// ---------------------------------------------------------------------------------
constexpr int kLaneChunk = 4096;
constexpr int kLaneBuckets = 256;

template <int N>
struct LaneSort {
  uint16_t order[N];             // item offsets in bucket order
  uint8_t bucket[N];             // bucket of each offset
  uint32_t start[kLaneBuckets];  // bucket counts, then each bucket's next place
};

// Sorts the items j < n <= N (sample index index_of(j)) of sampler S by bits
// [shift, shift + 8) of their first word into ls.order.  Called by every thread of the
// block; returns synchronised.
template <int S, int N, typename F>
__device__ void lane_sort(LaneSort<N>& ls, uint64_t seed, F index_of, uint32_t n, int shift) {
  const int tid = threadIdx.x, bd = blockDim.x;
  for (int i = tid; i < kLaneBuckets; i += bd) ls.start[i] = 0;
  __syncthreads();
  for (uint32_t j = tid; j < n; j += bd) {
    uint64_t W[4];
    philox_block(index_of(j), 0, seed, S, W);
    const uint32_t b = (uint32_t)(W[0] >> shift) & (kLaneBuckets - 1);
    ls.bucket[j] = (uint8_t)b;
    atomicAdd(&ls.start[b], 1u);
  }
  __syncthreads();
  if (tid < kLaneBuckets / 4) {  // exclusive prefix of the counts, four per lane of wave 0
    const uint4 c = reinterpret_cast<const uint4*>(ls.start)[tid];
    const uint32_t sum = c.x + c.y + c.z + c.w;
    bool unused = false;
    const uint32_t b = (uint32_t)(wave_inclusive_scan(sum, unused) - sum);
    reinterpret_cast<uint4*>(ls.start)[tid] = make_uint4(b, b + c.x, b + c.x + c.y, b + c.x + c.y + c.z);
  }
  __syncthreads();
  for (uint32_t j = tid; j < n; j += bd) ls.order[atomicAdd(&ls.start[ls.bucket[j]], 1u)] = (uint16_t)j;
  __syncthreads();
}

// Samples [k0, k1) of sampler S drawn by the whole block in lane order (by the top 8
// bits of the first word), counted into `bins` (the calling wave's LDS counters).
// Returns synchronised.
template <int S>
__device__ void draw_lane_sorted(const SamplerView& a, const uint8_t* lut, uint64_t seed, uint64_t k0, uint64_t k1,
                                 LaneSort<kLaneChunk>& ls, uint32_t* bins) {
  for (uint64_t s0 = k0; s0 < k1; s0 += kLaneChunk) {
    const uint32_t n = (uint32_t)min((uint64_t)kLaneChunk, k1 - s0);
    lane_sort<S>(ls, seed, [&](uint32_t j) { return s0 + j; }, n, 56);
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) count_sample(bins, draw<S>(a, lut, seed, s0 + ls.order[j], nullptr));
    __syncthreads();  // the next chunk reuses ls
  }
}

// Plain sampling: block b draws chunks b, b + grid, ... of `chunk` consecutive samples
// (chunk <= kLaneChunk), each in lane order.
template <int S>
__global__ __launch_bounds__(256, 8) void k_sample(SamplerView a, uint64_t seed, uint64_t k0, uint64_t k1,
                                                uint32_t chunk, unsigned long long* __restrict__ hits,
                                                uint8_t* __restrict__ class_out) {
  __shared__ uint32_t bins[kMaxWaves][kBins + 2];
  __shared__ uint8_t lut[64];
  __shared__ LaneSort<kLaneChunk> ls;
  const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int i = tid; i < nw * (kBins + 2); i += blockDim.x) bins[i / (kBins + 2)][i % (kBins + 2)] = 0;
  load_lut<S>(lut);
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * chunk;
  for (uint64_t s0 = k0 + (uint64_t)blockIdx.x * chunk; s0 < k1; s0 += stride) {
    const uint32_t n = (uint32_t)min((uint64_t)chunk, k1 - s0);
    lane_sort<S>(ls, seed, [&](uint32_t j) { return s0 + j; }, n, 56);
    for (uint32_t j = tid; j < n; j += blockDim.x) {
      const uint64_t k = s0 + ls.order[j];
      const int c = draw<S>(a, lut, seed, k, nullptr);
      count_sample(bins[wave], c);
      if (class_out) class_out[k - k0] = (uint8_t)c;
    }
    __syncthreads();  // the next chunk reuses ls
  }
  if (tid < kBins) {
    uint64_t s = 0;
    for (int w = 0; w < nw; ++w) s += bins[w][tid];
    if (s) atomicAdd(&hits[tid], (unsigned long long)s);
  }
}

hipError_t launch_sample(int sampler, const SamplerView& v, uint64_t seed, uint64_t k0, uint64_t k1,
                         unsigned long long* hits, uint8_t* class_out, int grid, int block, hipStream_t s) {
  if (grid < 1 || block < 64 || block > 256 || block % 64) return hipErrorInvalidValue;
  // a chunk per block and round that spreads the samples over the whole grid, between
  // one sample per thread and kLaneChunk; per-wave LDS counters are 32-bit, so each
  // launch stays below 2^31 samples per wave
  const uint64_t per_round = (k1 - k0 + (uint64_t)grid - 1) / (uint64_t)grid;
  const uint32_t chunk = (uint32_t)std::min<uint64_t>(kLaneChunk, std::max<uint64_t>((uint64_t)block, per_round));
  const uint64_t max_chunk = (uint64_t)grid * (uint64_t)block * (1ull << 24);
  for (uint64_t a = k0; a < k1;) {
    const uint64_t b = k1 - a > max_chunk ? a + max_chunk : k1;
    uint8_t* co = class_out ? class_out + (a - k0) : nullptr;
    switch (sampler) {
      case kMoss4:
        hipLaunchKernelGGL(k_sample<kMoss4>, dim3(grid), dim3(block), 0, s, v, seed, a, b, chunk, hits, co);
        break;
      case kMoss4Min:
        hipLaunchKernelGGL(k_sample<kMoss4Min>, dim3(grid), dim3(block), 0, s, v, seed, a, b, chunk, hits, co);
        break;
      case kT5: hipLaunchKernelGGL(k_sample<kT5>, dim3(grid), dim3(block), 0, s, v, seed, a, b, chunk, hits, co); break;
      case kPath5:
        hipLaunchKernelGGL(k_sample<kPath5>, dim3(grid), dim3(block), 0, s, v, seed, a, b, chunk, hits, co);
        break;
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    a = b;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------------
// XCD-grouped sampling.  MI355X has 8 XCDs, each with its own 4 MB L2, and a launch's
// workgroups go to the XCDs in turn (workgroup i to XCD i mod 8).  The node draw is
// monotone in a sample's first random word, so the word's top 10 bits split the
// samples into 1024 groups of equal probability, each drawing v from one contiguous
// range of nodes.  The samples of a chunk are counting-sorted by group (count per
// block, scan, scatter), and in k_sample_sorted XCD x owns groups 128x .. 128x+127,
// one contiguous range of the sorted order, which its blocks take window after window:
// every L2 serves one eighth of the nodes, and over time a narrow node range of it.
// Blocks then help drain the other XCDs' ranges, so every sample is drawn exactly once
// wherever the workgroups actually run, and each sample's outcome is the one the
// plain kernel gives it.  Measured at n = 1e6, m = 1e7 (T-5 / Path-5): plain 10.4 /
// 14.9 ms; 32 groups found by scanning group bytes 7.0 / 11.5 ms; sorted into 256
// groups 6.8 / 10.0 ms.  With the windows and cursors below, 256 / 512 / 1024 / 2048 /
// 4096 groups: 5.61 / 5.58 / 5.61 / 5.80 / 6.27 ms (T-5), 8.06 / 7.75 / 7.62 / 7.68 /
// 8.07 ms (Path-5), and at n = 1e5, m = 1e6 (MOSS-4, 1e7 samples) 0.51 / 0.51 / 0.51 /
// 0.55 / 0.63 ms.
// ---------------------------------------------------------------------------------
constexpr int kXcds = 8;
constexpr int kSortBits = 10;
constexpr int kSortGroups = 1 << kSortBits;
using SortGroup = std::conditional_t<(kSortBits <= 8), uint8_t, uint16_t>;  // a sample's group
static_assert(kSortGroups % 256 == 0 && kSortBits <= 16, "whole groups per scatter thread");
constexpr uint32_t kSortSpan = 8192;   // samples per block of the counting passes
static_assert(kSortSpan <= 65536 && kSortSpan % 16 == 0, "16-bit local offsets, 16-byte group loads");
// Sorted entries a block takes per cursor step: 512 while the sampled tables fit the
// MALL, 256 beyond it (multiples of the 256-thread block; 128 leaves half the threads
// idle).  Smaller windows keep the blocks of an XCD closer together in the sorted
// order, so that they share more of their tables' lines in the L2, as long as the
// cursor atomics keep up.  Measured with the cursors apart (below): n = 1e6, m = 1e7,
// T-5 / Path-5 for 5e7 samples each, 5.74 / 8.31 ms at 512, 5.72 / 8.19 at 256,
// 7.31 / 10.36 at 128; n = 1e5, m = 1e6, MOSS-4 for 1e7 samples, 0.628 ms at 2048,
// 0.600 at 1024, 0.575 at 512, 0.577 at 256, 0.63 at 384, 0.78 at 128.  A cursor per
// wave instead of per block (no block barriers) measured 0.61 ms there.
uint32_t sort_window(uint64_t footprint_bytes) { return footprint_bytes > (256ull << 20) ? 256u : 512u; }

// The eight window cursors sit 256 bytes apart: packed into one line, every XCD's
// cursor atomics queued on that line (n = 1e5, m = 1e6, MOSS-4 for 1e7 samples: 0.668
// -> 0.624 ms; n = 1e6, m = 1e7, T-5 / Path-5 for 5e7 each at 256-sample windows:
// 5.84 / 8.38 -> 5.72 / 8.19 ms).
constexpr uint32_t kCursorStride = 64;  // u32
constexpr int kMaxWindow = 512;         // sorted entries a block takes at a time, at most

// The (block, group) count table is stored block-major, one 4 KB row per block, so that
// the grouping pass writes and the sorting pass reads whole rows.  Its group-major
// prefix (the place of each (block, group) run in the sorted order) is taken column by
// column: the rows are cut into at most kSortRuns runs of consecutive blocks, each run
// sums its rows per group, one wave per four groups scans those sums across the runs,
// and each run then walks its rows again writing places.  All counts fit 32 bits (a
// chunk has at most 2^31 samples).  Against a group-major table of 64-bit inclusive
// counts (one strided 8-byte store and load per (block, group), through the general
// three-kernel scan): n = 1e5, m = 1e6, MOSS-4 for 1e7 samples, sampling launch 0.493
// -> 0.476 ms; n = 1e6, m = 1e7, T-5 / Path-5 for 5e7 samples each, 5.58 / 7.57 ->
// 5.49 / 7.47 ms.
constexpr uint32_t kSortRuns = 64;  // at most one run per lane of the scanning wave
constexpr uint32_t kSortQuads = kSortGroups / 4;
static_assert(kSortQuads == 256, "one group quad per thread of a 256-thread block");

struct SortScratch {
  SortGroup* group;   // n: group of each sample
  uint32_t* order;    // n: sample offsets sorted by group
  uint32_t* counts;   // nblk rows of kSortGroups: block b's count of group g at b * kSortGroups + g
  uint32_t* place;    // same layout: where run (b, g) starts in the sorted order
  uint32_t* rsum;     // kSortRuns rows of kSortGroups: per (run, group) sums, then their exclusive prefix
  uint32_t* gtot;     // kSortGroups: samples per group
  uint32_t* gstart;   // kSortGroups + 1: start of each group in the sorted order (the last is n)
  uint32_t* cursors;  // kXcds window cursors, kCursorStride apart
  uint32_t nblk;      // blocks (rows) of this chunk
  uint32_t rows;      // rows per run
  uint32_t runs;      // runs, <= kSortRuns
};

__device__ __forceinline__ uint4* quad_at(uint32_t* table, uint32_t row, uint32_t q) {
  return reinterpret_cast<uint4*>(table + (size_t)row * kSortGroups) + q;
}

__device__ __forceinline__ void add4(uint4& a, const uint4& b) {
  a.x += b.x;
  a.y += b.y;
  a.z += b.z;
  a.w += b.w;
}

static void set_runs(SortScratch& t, uint64_t n) {
  t.nblk = (uint32_t)std::max<uint64_t>(1, (n + kSortSpan - 1) / kSortSpan);
  t.rows = (t.nblk + kSortRuns - 1) / kSortRuns;
  t.runs = (t.nblk + t.rows - 1) / t.rows;
}

static SortScratch sort_scratch(void* base, uint64_t max_n) {
  SortScratch t;
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) / 256 * 256;
    return q;
  };
  set_runs(t, max_n);
  t.group = reinterpret_cast<SortGroup*>(take(max_n * sizeof(SortGroup)));
  t.order = reinterpret_cast<uint32_t*>(take(max_n * 4));
  t.counts = reinterpret_cast<uint32_t*>(take((size_t)kSortGroups * t.nblk * 4));
  t.place = reinterpret_cast<uint32_t*>(take((size_t)kSortGroups * t.nblk * 4));
  t.rsum = reinterpret_cast<uint32_t*>(take((size_t)kSortGroups * kSortRuns * 4));
  t.gtot = reinterpret_cast<uint32_t*>(take((size_t)kSortGroups * 4));
  t.gstart = reinterpret_cast<uint32_t*>(take((size_t)(kSortGroups + 1) * 4));
  t.cursors = reinterpret_cast<uint32_t*>(take(kXcds * kCursorStride * 4));
  return t;
}

constexpr uint64_t scratch_bytes_for(uint64_t max_n) {
  const uint64_t nblk = std::max<uint64_t>(1, (max_n + kSortSpan - 1) / kSortSpan);
  auto r = [](uint64_t b) { return (b + 255) / 256 * 256; };
  return r(max_n * sizeof(SortGroup)) + r(max_n * 4) + 2 * r(kSortGroups * nblk * 4) +
         r(kSortGroups * kSortRuns * 4) + r(kSortGroups * 4) + r((kSortGroups + 1) * 4) +
         r(kXcds * kCursorStride * 4) + 256;
}

int64_t grouped_scratch_bytes(uint64_t max_n) { return (int64_t)scratch_bytes_for(max_n); }

// The fixed scratch of the no-allocation calls: one grouped chunk of up to
// kFixedScratchSamples samples (group and order of each sample, the per-block group
// counts and places, the window cursors) in a device array of the library itself.  Each
// device the library runs on holds its own copy from the module's load until the
// process ends.  Every kernel that reads a part of it writes that part first within the
// same chunk (the cursors are reset by the grouping pass), so no clearing is needed
// between calls.  In host code the array's name only stands in for it: its address on a
// device comes from the runtime, looked up once per device with that device current.
static_assert(scratch_bytes_for(kFixedScratchSamples) <= kFixedScratchBytes, "one chunk fits the fixed scratch");
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void* g_fixed_ptr[kMaxDevices] = {};
std::mutex g_fixed_use[kMaxDevices];
}  // namespace

hipError_t fixed_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  if (!g_fixed_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // callers make the device current first
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_fixed_ptr[device] = p;
  }
  *out = g_fixed_ptr[device];
  return hipSuccess;
}

std::mutex& fixed_scratch_lock(int device) { return g_fixed_use[device]; }

// Block b counts the groups of samples [b * kSortSpan, (b + 1) * kSortSpan) into row b
// of the count table.
template <int S>
__global__ __launch_bounds__(256) void k_sort_count(uint64_t seed, uint64_t k0, uint64_t n, SortScratch t) {
  __shared__ uint32_t hist[kSortGroups];
  if (blockIdx.x == 0 && threadIdx.x < kXcds) t.cursors[threadIdx.x * kCursorStride] = 0;
  for (int g = threadIdx.x; g < kSortGroups; g += blockDim.x) hist[g] = 0;
  __syncthreads();
  const uint64_t lo = (uint64_t)blockIdx.x * kSortSpan;
  const uint64_t hi = n < lo + kSortSpan ? n : lo + kSortSpan;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    uint64_t W[4];
    philox_block(k0 + i, 0, seed, S, W);
    const uint32_t g = (uint32_t)(W[0] >> (64 - kSortBits));
    t.group[i] = (SortGroup)g;
    atomicAdd(&hist[g], 1u);
  }
  __syncthreads();
  for (int g = threadIdx.x; g < kSortGroups; g += blockDim.x) t.counts[(size_t)blockIdx.x * kSortGroups + g] = hist[g];
}

// Run r sums rows [r * rows, (r + 1) * rows) of the count table per group.  The rows'
// loads go out 16 at a time.
__global__ __launch_bounds__(256) void k_sort_runsum(SortScratch t) {
  const uint32_t q = threadIdx.x;  // blockDim.x == kSortQuads
  const uint32_t b0 = blockIdx.x * t.rows, b1 = min(t.nblk, b0 + t.rows);
  uint4 s = make_uint4(0, 0, 0, 0);
  for (uint32_t b = b0; b < b1; b += 16) {
    uint4 c[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) c[k] = b + k < b1 ? *quad_at(t.counts, b + k, q) : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 16; ++k) add4(s, c[k]);
  }
  *quad_at(t.rsum, blockIdx.x, q) = s;
}

// One wave per four groups: lane r holds run r's sums and the wave scans them, leaving
// each run's exclusive prefix in place and the groups' totals in gtot.  Two 32-bit sums
// share a 64-bit lane value; neither half carries into the other, since every sum is at
// most the chunk's sample count (< 2^32).
__global__ __launch_bounds__(256) void k_sort_runscan(SortScratch t) {
  const uint32_t q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), r = (uint32_t)lane_id();
  if (q >= kSortQuads) return;  // whole waves
  const uint4 v = r < t.runs ? *quad_at(t.rsum, r, q) : make_uint4(0, 0, 0, 0);
  const uint64_t lo = (uint64_t)v.x | ((uint64_t)v.y << 32), hi = (uint64_t)v.z | ((uint64_t)v.w << 32);
  bool unused = false;
  const uint64_t ilo = wave_inclusive_scan(lo, unused), ihi = wave_inclusive_scan(hi, unused);
  const uint64_t elo = ilo - lo, ehi = ihi - hi;
  if (r < t.runs)
    *quad_at(t.rsum, r, q) = make_uint4((uint32_t)elo, (uint32_t)(elo >> 32), (uint32_t)ehi, (uint32_t)(ehi >> 32));
  if (r == t.runs - 1)
    *quad_at(t.gtot, 0, q) = make_uint4((uint32_t)ilo, (uint32_t)(ilo >> 32), (uint32_t)ihi, (uint32_t)(ihi >> 32));
}

// Each run block first turns the group totals into group starts (a block scan; block 0
// stores them, with n after the last), then walks its rows: the place of run (b, g) is
// g's start, plus the samples of g in earlier runs, plus those in the run's earlier rows.
__global__ __launch_bounds__(256) void k_sort_place(uint64_t n, SortScratch t) {
  __shared__ uint32_t wsum[4];
  const uint32_t q = threadIdx.x;  // blockDim.x == kSortQuads
  const int lane = lane_id(), wave = (int)(q >> 6);
  const uint4 tot = *quad_at(t.gtot, 0, q);
  const uint32_t mine = tot.x + tot.y + tot.z + tot.w;
  bool unused = false;
  const uint32_t incl = (uint32_t)wave_inclusive_scan((uint64_t)mine, unused);
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t off = incl - mine;
  for (int w = 0; w < wave; ++w) off += wsum[w];
  const uint4 start = make_uint4(off, off + tot.x, off + tot.x + tot.y, off + tot.x + tot.y + tot.z);
  if (blockIdx.x == 0) {
    *quad_at(t.gstart, 0, q) = start;
    if (q == 0) t.gstart[kSortGroups] = (uint32_t)n;
  }
  uint4 run = *quad_at(t.rsum, blockIdx.x, q);
  add4(run, start);
  const uint32_t b0 = blockIdx.x * t.rows, b1 = min(t.nblk, b0 + t.rows);
  for (uint32_t b = b0; b < b1; b += 16) {
    uint4 c[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) c[k] = b + k < b1 ? *quad_at(t.counts, b + k, q) : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (b + k < b1) {
        *quad_at(t.place, b + k, q) = run;
        add4(run, c[k]);
      }
    }
  }
}

// The same blocks place their samples.  A block first sorts its span by group in LDS
// (a sample of group g takes the next free slot of g's run), then writes each run to
// the block's share of g in the sorted order: consecutive threads write consecutive
// slots, so the stores coalesce (slot order within a share is immaterial).  The group
// bytes come in 16-byte loads and the local order is kept as 16-bit offsets (27 KB of
// LDS a block instead of 43 KB): 69 -> 37 us a pass on average over the n = 1e5,
// m = 1e6 and n = 1e6, m = 1e7 workloads.
__global__ __launch_bounds__(256) void k_sort_scatter(uint64_t n, SortScratch t) {
  constexpr int kPerThread = kSortGroups / 256;  // thread tid owns groups tid * kPerThread ..
  __shared__ uint32_t base[kSortGroups];   // per group: the block's share in the sorted order
  __shared__ uint32_t start[kSortGroups];  // per group: the run's start in the local order
  __shared__ uint32_t next[kSortGroups];   // per group: the run's fill cursor
  __shared__ uint32_t wsum[4];
  __shared__ uint16_t local[kSortSpan];    // span offsets sorted by group
  __shared__ __align__(16) SortGroup grp[kSortSpan];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;  // blockDim.x == 256
  const uint64_t lo = (uint64_t)blockIdx.x * kSortSpan;
  const uint32_t len = (uint32_t)(n < lo + kSortSpan ? n - lo : kSortSpan);
  // the block's share of each of this thread's groups: its place and its size
  uint32_t size[kPerThread];
  uint32_t mine = 0;
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    const uint32_t g = (uint32_t)tid * kPerThread + j;
    const size_t idx = (size_t)blockIdx.x * kSortGroups + g;
    base[g] = t.place[idx];
    size[j] = t.counts[idx];
    mine += size[j];
  }
  if (len == kSortSpan) {  // whole span: 16-byte loads
    for (uint32_t j = tid; j < kSortSpan * sizeof(SortGroup) / 16; j += blockDim.x)
      reinterpret_cast<uint4*>(grp)[j] = reinterpret_cast<const uint4*>(t.group + lo)[j];
  } else {
    for (uint32_t j = tid; j < len; j += blockDim.x) grp[j] = t.group[lo + j];
  }
  // exclusive prefix of the share sizes in group order: local run starts
  bool unused = false;
  const uint32_t incl = (uint32_t)wave_inclusive_scan((uint64_t)mine, unused);
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t off = incl - mine;
  for (int w = 0; w < wave; ++w) off += wsum[w];
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    const uint32_t g = (uint32_t)tid * kPerThread + j;
    start[g] = off;
    next[g] = off;
    off += size[j];
  }
  __syncthreads();
  for (uint32_t j = tid; j < len; j += blockDim.x) local[atomicAdd(&next[grp[j]], 1u)] = (uint16_t)j;
  __syncthreads();
  for (uint32_t j = tid; j < len; j += blockDim.x) {
    const uint32_t o = local[j];
    const uint32_t g = grp[o];
    t.order[(uint64_t)base[g] + (j - start[g])] = (uint32_t)(lo + o);
  }
}

template <int S>
__global__ __launch_bounds__(256, 8) void k_sample_sorted(SamplerView a, uint64_t seed, uint64_t k0, uint64_t n,
                                                       SortScratch t, uint32_t window,
                                                       unsigned long long* __restrict__ hits,
                                                       uint8_t* __restrict__ class_out) {
  __shared__ uint32_t bins[kMaxWaves][kBins + 2];
  __shared__ uint8_t lut[64];
  __shared__ uint32_t s_win;
  __shared__ LaneSort<kMaxWindow> ls;
  const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int i = tid; i < nw * (kBins + 2); i += blockDim.x) bins[i / (kBins + 2)][i % (kBins + 2)] = 0;
  load_lut<S>(lut);
  __syncthreads();
  // start of group g in the sorted order
  auto start = [&](uint32_t g) -> uint64_t { return g >= (uint32_t)kSortGroups ? n : (uint64_t)t.gstart[g]; };
  const uint32_t per_xcd = kSortGroups / kXcds;
  for (int step = 0; step < kXcds; ++step) {
    const uint32_t x = (uint32_t)((blockIdx.x + step) % kXcds);
    const uint64_t lo = start(x * per_xcd), hi = start((x + 1) * per_xcd);
    for (;;) {
      if (tid == 0) s_win = atomicAdd(&t.cursors[x * kCursorStride], 1u);
      __syncthreads();
      const uint64_t p = lo + (uint64_t)s_win * window;
      __syncthreads();
      if (p >= hi) break;
      const uint32_t m = (uint32_t)((hi < p + window ? hi : p + window) - p);
      // lane order inside the window: its samples share the group (the top kSortBits
      // bits of the first word); the next 8 bits order them
      lane_sort<S>(ls, seed, [&](uint32_t j) { return k0 + t.order[p + j]; }, m, 64 - kSortBits - 8);
      for (uint32_t j = tid; j < m; j += blockDim.x) {
        const uint64_t i = t.order[p + ls.order[j]];
        const int c = draw<S>(a, lut, seed, k0 + i, nullptr);
        count_sample(bins[wave], c);
        if (class_out) class_out[i] = (uint8_t)c;
      }
      __syncthreads();  // the next window reuses ls
    }
  }
  __syncthreads();
  if (tid < kBins) {
    uint64_t s = 0;
    for (int w = 0; w < nw; ++w) s += bins[w][tid];
    if (s) atomicAdd(&hits[tid], (unsigned long long)s);
  }
}

hipError_t launch_group_chunk(int sampler, uint64_t seed, uint64_t a, uint64_t n, void* scratch, uint64_t max_n,
                              hipStream_t s) {
  if (n == 0 || n > max_n || max_n > (1ull << 31)) return hipErrorInvalidValue;
  SortScratch tc = sort_scratch(scratch, max_n);
  set_runs(tc, n);
  const uint32_t nblk = tc.nblk;
  switch (sampler) {
    case kMoss4: hipLaunchKernelGGL(k_sort_count<kMoss4>, dim3(nblk), dim3(256), 0, s, seed, a, n, tc); break;
    case kMoss4Min: hipLaunchKernelGGL(k_sort_count<kMoss4Min>, dim3(nblk), dim3(256), 0, s, seed, a, n, tc); break;
    case kT5: hipLaunchKernelGGL(k_sort_count<kT5>, dim3(nblk), dim3(256), 0, s, seed, a, n, tc); break;
    case kPath5: hipLaunchKernelGGL(k_sort_count<kPath5>, dim3(nblk), dim3(256), 0, s, seed, a, n, tc); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_sort_runsum, dim3(tc.runs), dim3(kSortQuads), 0, s, tc);
  hipLaunchKernelGGL(k_sort_runscan, dim3(kSortQuads / 4), dim3(256), 0, s, tc);
  hipLaunchKernelGGL(k_sort_place, dim3(tc.runs), dim3(kSortQuads), 0, s, n, tc);
  hipLaunchKernelGGL(k_sort_scatter, dim3(nblk), dim3(256), 0, s, n, tc);
  return hipGetLastError();
}

hipError_t launch_sample_chunk(int sampler, const SamplerView& v, uint64_t seed, uint64_t a, uint64_t n,
                               void* scratch, uint64_t max_n, uint32_t window, unsigned long long* hits,
                               uint8_t* class_out, int grid, int block, hipStream_t s) {
  if (block != 64 * (block / 64) || block > 256 || block < 64 || n == 0 || n > max_n || max_n > (1ull << 31) ||
      window == 0 || window > (uint32_t)kMaxWindow)
    return hipErrorInvalidValue;
  SortScratch tc = sort_scratch(scratch, max_n);
  set_runs(tc, n);
  // no more blocks than windows (each block visits every cursor once at least), a
  // multiple of the XCD count so that every XCD gets its share of blocks
  const uint64_t wins = (n + window - 1) / window;
  const int g = (int)std::min<uint64_t>((uint64_t)grid, std::max<uint64_t>(kXcds, (wins + kXcds - 1) / kXcds * kXcds));
  switch (sampler) {
    case kMoss4:
      hipLaunchKernelGGL(k_sample_sorted<kMoss4>, dim3(g), dim3(block), 0, s, v, seed, a, n, tc, window, hits,
                         class_out);
      break;
    case kMoss4Min:
      hipLaunchKernelGGL(k_sample_sorted<kMoss4Min>, dim3(g), dim3(block), 0, s, v, seed, a, n, tc, window, hits,
                         class_out);
      break;
    case kT5:
      hipLaunchKernelGGL(k_sample_sorted<kT5>, dim3(g), dim3(block), 0, s, v, seed, a, n, tc, window, hits,
                         class_out);
      break;
    case kPath5:
      hipLaunchKernelGGL(k_sample_sorted<kPath5>, dim3(g), dim3(block), 0, s, v, seed, a, n, tc, window, hits,
                         class_out);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int S>
__global__ __launch_bounds__(256) void k_sample_nodes(SamplerView a, uint64_t seed, const uint64_t* __restrict__ index,
                                                      int64_t count, int32_t* __restrict__ nodes,
                                                      uint8_t* __restrict__ cls) {
  __shared__ uint8_t lut[64];
  load_lut<S>(lut);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    const int c = draw<S>(a, lut, seed, index[i], nodes + 5 * i);
    if (cls) cls[i] = (uint8_t)c;
  }
}

hipError_t launch_sample_nodes(int sampler, const SamplerView& v, uint64_t seed, const uint64_t* index, int64_t count,
                               int32_t* nodes_out, uint8_t* class_out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const dim3 grid((unsigned)((count + 255) / 256)), block(256);
  switch (sampler) {
    case kMoss4: hipLaunchKernelGGL(k_sample_nodes<kMoss4>, grid, block, 0, s, v, seed, index, count, nodes_out, class_out); break;
    case kMoss4Min:
      hipLaunchKernelGGL(k_sample_nodes<kMoss4Min>, grid, block, 0, s, v, seed, index, count, nodes_out, class_out);
      break;
    case kT5: hipLaunchKernelGGL(k_sample_nodes<kT5>, grid, block, 0, s, v, seed, index, count, nodes_out, class_out); break;
    case kPath5: hipLaunchKernelGGL(k_sample_nodes<kPath5>, grid, block, 0, s, v, seed, index, count, nodes_out, class_out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Persistent batched kernel: blocks take tiles from a shared counter until the list
// is drained (every block exits once the counter passes n_tiles).  Each tile's
// samples are spread over the block's lanes; its histogram is flushed to the tile's
// output slot.  The sampler is uniform within a tile, so the branch is uniform.
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(256, 8) void k_batch(const SamplerView* __restrict__ views,
                                               const BatchItem* __restrict__ items, uint32_t* ctl,
                                               unsigned long long* __restrict__ bins) {
  __shared__ uint32_t lb[kMaxWaves][kBins + 2];
  __shared__ uint8_t lut4[64], lut5t[64], lut5p[64];
  __shared__ uint32_t cur, cur_item;
  __shared__ LaneSort<kLaneChunk> ls;
  const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
  if (tid < 64) {
    lut4[tid] = tid < 8 ? c_lut4[tid] : 0;
    lut5t[tid] = c_lut5t[tid];
    lut5p[tid] = c_lut5p[tid];
  }
  const uint32_t n_tiles = ctl[kCtlTiles], n_items = ctl[kCtlItems], T = ctl[kCtlTileSize];
  uint32_t from = 0;  // tiles come in increasing order, so a block's items never go back
  for (;;) {
    if (tid == 0) {
      const uint32_t t = atomicAdd(&ctl[kCtlCounter], 1u);
      cur = t;
      if (t < n_tiles) {  // the last item whose first tile is at or before t
        uint32_t lo = from, hi = n_items - 1;
        while (lo < hi) {
          const uint32_t mid = lo + (hi - lo + 1) / 2;
          if (items[mid].first_tile <= t) lo = mid;
          else hi = mid - 1;
        }
        cur_item = lo;
      }
    }
    for (int i = tid; i < nw * (kBins + 2); i += blockDim.x) lb[i / (kBins + 2)][i % (kBins + 2)] = 0;
    __syncthreads();
    const uint32_t t = cur;
    if (t >= n_tiles) break;
    from = cur_item;
    const BatchItem it = items[from];
    const SamplerView v = views[it.view];
    const uint64_t a = it.k0 + (uint64_t)(t - it.first_tile) * T;
    const uint64_t b = it.k1 - a < T ? it.k1 : a + T;
    if (it.sampler == kMoss4) draw_lane_sorted<kMoss4>(v, lut4, it.seed, a, b, ls, lb[wave]);
    else if (it.sampler == kMoss4Min) draw_lane_sorted<kMoss4Min>(v, lut4, it.seed, a, b, ls, lb[wave]);
    else if (it.sampler == kT5) draw_lane_sorted<kT5>(v, lut5t, it.seed, a, b, ls, lb[wave]);
    else draw_lane_sorted<kPath5>(v, lut5p, it.seed, a, b, ls, lb[wave]);
    if (tid < kBins) {
      uint64_t s = 0;
      for (int w = 0; w < nw; ++w) s += lb[w][tid];
      if (s) atomicAdd(&bins[(uint64_t)it.out * kBins + tid], (unsigned long long)s);
    }
    __syncthreads();
  }
}

hipError_t launch_batch(const SamplerView* views, const BatchItem* items, uint32_t* ctl, unsigned long long* bins,
                        int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(block), 0, s, views, items, ctl, bins);
  return hipGetLastError();
}

int sample_kernel_blocks_per_cu(int sampler, int block) {
  int nb = 0;
  hipError_t e = hipSuccess;
  switch (sampler) {
    case kMoss4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sample<kMoss4>, block, 0); break;
    case kMoss4Min: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sample<kMoss4Min>, block, 0); break;
    case kT5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sample<kT5>, block, 0); break;
    case kPath5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sample<kPath5>, block, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch, block, 0); break;
  }
  return e == hipSuccess ? nb : 0;
}

}  // namespace moss
