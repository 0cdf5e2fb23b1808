// HIP kernels of the Moss hot path for gfx950 (CDNA4, wave64).
//
// Table build (Section 4.1.3 "Initialization", O(|E|)):
//   k_check_rowptr / k_check_cols   CSR validation (Section 2: undirected simple graph)
//   k_row_tables                    one wave per node: ACC_sigma, ACC_tau row prefixes,
//                                   Gamma_v, Gamma^(1)_v, Gamma^(2)_v, Lambda_3, Lambda_4
//   k_scan_*                        node-level inclusive prefixes ACC_Gamma*
//   k_guide                         search windows for the node draw
// Sampling (Algorithms 1, 3, 4):
//   k_sample<S>                     grid-stride loop, one sample per lane per step,
//                                   per-wave LDS histograms flushed with u64 atomics
//   k_batch                         persistent kernel draining a tile list of many
//                                   (graph, sampler, sample range) requests
//   k_sample_nodes<S>               the same draw for chosen sample indices, with nodes
//
// All counting is integer; a sample's outcome depends only on (graph, seed, sampler,
// sample index), never on which lane, block or launch draws it.
#include <algorithm>

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

__device__ __forceinline__ uint64_t add_wrap(uint64_t a, uint64_t b, bool& wrapped) {
  const uint64_t z = a + b;
  wrapped |= z < a;
  return z;
}

hipError_t launch_scan_inplace(uint64_t* data, int64_t n, uint64_t* tmp, uint32_t* err, uint32_t err_bit,
                               hipStream_t s);

hipError_t upload_class_luts(const uint8_t lut4[8], const uint8_t lut5t[64], const uint8_t lut5p[64]) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_lut4), lut4, 8);
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_lut5t), lut5t, 64);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_lut5p), lut5p, 64);
}

// ---------------------------------------------------------------------------------
// CSR validation.  row_ptr is checked first (its own launch), so that the column
// checks only index rows that lie inside col[].
// ---------------------------------------------------------------------------------
__global__ void k_check_rowptr(int32_t n, int64_t nnz, const int32_t* __restrict__ rp, uint32_t* err) {
  uint32_t bad = 0, dmax = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = rp[v + 1] - rp[v];
    if (d < 0) bad = kErrArg;
    else dmax = max(dmax, (uint32_t)d);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (rp[0] != 0 || (int64_t)rp[n] != nnz)) bad = kErrArg;
  bad = wave_or(bad);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dmax = max(dmax, (uint32_t)__shfl_xor((int)dmax, off, 64));
  if (lane_id() == 0) {
    if (bad) atomicOr(err, bad);
    if (dmax) atomicMax(err + 1, dmax);
  }
}

// err[0] receives error bits, err[1] the largest degree.
hipError_t launch_check_rowptr(int32_t n, int64_t nnz, const int32_t* rp, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_check_rowptr, dim3(fill_grid(n > 0 ? n : 1)), dim3(256), 0, s, n, nnz, rp, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Work items.  Every CSR row is cut into items of at most kItem consecutive entries
// and each item is handled by one wave, so no wave walks a long row alone: the
// costliest row (a hub with tens of thousands of neighbours) becomes many items
// that run concurrently.  items[i] packs (row << 32 | piece index within the row).
// Per-row quantities that span pieces are stitched with a scan over item totals.
// ---------------------------------------------------------------------------------
constexpr int32_t kItem = 256;

__global__ void k_item_count(int32_t n, const int32_t* __restrict__ rp, uint64_t* __restrict__ cnt) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    cnt[v] = (uint64_t)((rp[v + 1] - rp[v] + kItem - 1) / kItem);
}

// item_end[v] = inclusive prefix of the piece counts
__global__ void k_item_fill(int32_t n, const int32_t* __restrict__ rp, const uint64_t* __restrict__ item_end,
                            uint64_t* __restrict__ items) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t c = (uint64_t)((rp[v + 1] - rp[v] + kItem - 1) / kItem);
    const uint64_t first = item_end[v] - c;
    for (uint64_t j = 0; j < c; ++j) items[first + j] = (uint64_t)v << 32 | j;
  }
}

hipError_t launch_items(int32_t n, const int32_t* rp, uint64_t* item_end, uint64_t* items, uint64_t* tmp,
                        uint32_t* err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_count, dim3(fill_grid(n)), dim3(256), 0, s, n, rp, item_end);
  hipError_t e = launch_scan_inplace(item_end, n, tmp, err, kErrArg, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_item_fill, dim3(fill_grid(n)), dim3(256), 0, s, n, rp, item_end, items);
  return hipGetLastError();
}

static int item_grid(int64_t n_items) {
  int64_t g = (n_items + 3) / 4;  // one wave per item, 4 waves per block
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
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

// Column range, self-loops, strict ascent (sorted, no repeats) and symmetry (v must
// appear in the row of each of its neighbours).
__global__ __launch_bounds__(256) void k_check_items(const uint64_t* __restrict__ n_items_p,
                                                     const uint64_t* __restrict__ items, int32_t n,
                                                     const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     int full, uint32_t* err) {
  const int lane = lane_id();
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t n_items = (int64_t)*n_items_p;
  uint32_t bad = 0;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n_items; i += nwaves) {
    const ItemRange it = item_range(items, rp, i);
    for (int32_t e = it.e0 + lane; e < it.e1; e += 64) {
      const int32_t c = col[e];
      if (c < 0 || c >= n) {
        bad |= kErrArg;
        continue;
      }
      if (!full) continue;
      if (c == it.v) bad |= kErrSelfLoop;
      if (e > it.r0) {
        const int32_t p = col[e - 1];
        if (p == c) bad |= kErrDuplicate;
        else if (p > c) bad |= kErrUnsorted;
      }
      const int32_t rc = rp[c];
      if (!row_has(col, rc, rp[c + 1] - rc, it.v)) bad |= kErrAsymmetric;
    }
  }
  bad = wave_or(bad);
  if (lane == 0 && bad) atomicOr(err, bad);
}

hipError_t launch_check_items(int64_t max_items, const uint64_t* n_items, const uint64_t* items, int32_t n,
                              const int32_t* rp, const int32_t* col, bool full, uint32_t* err, hipStream_t s) {
  if (max_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_items, dim3(item_grid(max_items)), dim3(256), 0, s, n_items, items, n, rp, col,
                     full ? 1 : 0, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Row prefixes (Section 4.1.3 ACC_sigma = ACC_mu of Section 5.1.5; the tau prefix of
// Section 5.1.2), in three steps per table:
//   local  each item scans its own entries and writes its total to item_sum
//   scan   inclusive scan of item_sum (in place)
//   fix    every later piece of a row adds the totals of the row's earlier pieces
// ACC_sigma entries are (d_x - 1) of the neighbours; ACC_tau entries are
// (d_x - 1)(S_v - (d_x - 1)) with S_v the row total of ACC_sigma.
// ---------------------------------------------------------------------------------
template <bool TAU>
__global__ __launch_bounds__(256) void k_prefix_local(int64_t n_items, const uint64_t* __restrict__ items,
                                                      const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                      uint32_t* __restrict__ acc_sigma, uint64_t* __restrict__ acc_tau,
                                                      uint64_t* __restrict__ item_sum) {
  const int lane = lane_id();
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  bool wrapped = false;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n_items; i += nwaves) {
    const ItemRange it = item_range(items, rp, i);
    uint64_t S = 0;
    if (TAU) S = acc_sigma[it.r1 - 1];
    uint64_t carry = 0;
    for (int32_t e0 = it.e0; e0 < it.e1; e0 += 64) {
      const int32_t e = e0 + lane;
      uint64_t x = 0;
      if (e < it.e1) {
        if (TAU) {
          const uint64_t dx = (uint64_t)acc_sigma[e] - (e > it.r0 ? (uint64_t)acc_sigma[e - 1] : 0ull);
          x = dx * (S - dx);
        } else {
          const int32_t c = col[e];
          x = (uint64_t)(rp[c + 1] - rp[c] - 1);
        }
      }
      const uint64_t s = wave_inclusive_scan(x, wrapped) + carry;
      if (e < it.e1) {
        if (TAU) acc_tau[e] = s;
        else acc_sigma[e] = (uint32_t)s;
      }
      carry = __shfl(s, 63, 64);
    }
    if (lane == 0) item_sum[i] = carry;
  }
  (void)wrapped;  // row totals are checked in the fix step
}

template <bool TAU>
__global__ __launch_bounds__(256) void k_prefix_fix(int64_t n_items, const uint64_t* __restrict__ items,
                                                    const int32_t* __restrict__ rp,
                                                    const uint64_t* __restrict__ item_incl, uint32_t* __restrict__ acc_sigma,
                                                    uint64_t* __restrict__ acc_tau, uint32_t* err) {
  const int lane = lane_id();
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  bool over = false;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n_items; i += nwaves) {
    const ItemRange it = item_range(items, rp, i);
    const int64_t first = i - it.piece;  // the row's first item
    const uint64_t before_row = first > 0 ? item_incl[first - 1] : 0;
    if (it.e1 == it.r1 && !TAU) {
      // last piece: the row total S_v must fit the 32-bit ACC_sigma
      over |= item_incl[i] - before_row > 0xFFFFFFFFull;
    }
    if (it.piece == 0) continue;
    const uint64_t off = item_incl[i - 1] - before_row;
    for (int32_t e = it.e0 + lane; e < it.e1; e += 64) {
      if (TAU) acc_tau[e] += off;
      else acc_sigma[e] += (uint32_t)off;
    }
  }
  if (__ballot(over) != 0 && lane == 0) atomicOr(err, kErrOverflow);
}

hipError_t launch_row_prefix(bool tau, int64_t n_items, const uint64_t* items, const int32_t* rp, const int32_t* col,
                             uint32_t* acc_sigma, uint64_t* acc_tau, uint64_t* item_sum, uint64_t* tmp, uint32_t* err,
                             hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const dim3 grid(item_grid(n_items)), block(256);
  if (tau) hipLaunchKernelGGL(k_prefix_local<true>, grid, block, 0, s, n_items, items, rp, col, acc_sigma, acc_tau, item_sum);
  else hipLaunchKernelGGL(k_prefix_local<false>, grid, block, 0, s, n_items, items, rp, col, acc_sigma, acc_tau, item_sum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the sum of every row's tau total is Gamma^(2): a wrap there is a 5-node overflow
  e = launch_scan_inplace(item_sum, n_items, tmp, err, tau ? kErrOverflowK5 : kErrOverflow, s);
  if (e != hipSuccess) return e;
  if (tau) hipLaunchKernelGGL(k_prefix_fix<true>, grid, block, 0, s, n_items, items, rp, item_sum, acc_sigma, acc_tau, err);
  else hipLaunchKernelGGL(k_prefix_fix<false>, grid, block, 0, s, n_items, items, rp, item_sum, acc_sigma, acc_tau, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Edge hash set for the induced-edge probes (the CIS() of Algorithms 1, 3, 4): each
// undirected edge is inserted once (from its smaller endpoint's row) with a 64-bit
// compare-and-swap, linear probing.  The table has at least 2.5 slots per edge, so a
// lookup reads about 1.2-1.4 slots.  Every loop is bounded by the table size.
// ---------------------------------------------------------------------------------
int edge_hash_bits(int64_t m) {
  int bits = 4;
  while (bits < 40 && (double)(1ll << bits) < 2.5 * (double)m) ++bits;
  return bits;
}

__global__ __launch_bounds__(256) void k_edge_hash(int64_t n_items, const uint64_t* __restrict__ items,
                                                   const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   unsigned long long* __restrict__ slots, int bits, uint32_t* err) {
  const int lane = lane_id();
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t mask = (1ull << bits) - 1;
  bool full = false;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n_items; i += nwaves) {
    const ItemRange it = item_range(items, rp, i);
    for (int32_t e = it.e0 + lane; e < it.e1; e += 64) {
      const int32_t c = col[e];
      if (c <= it.v) continue;  // each edge once, from its smaller endpoint
      const uint64_t key = edge_key(it.v, c);
      uint64_t h = edge_slot(key, bits);
      uint64_t probes = 0;
      for (;;) {
        const unsigned long long old = atomicCAS(&slots[h], (unsigned long long)kEmptySlot, (unsigned long long)key);
        if (old == kEmptySlot || old == key) break;
        h = (h + 1) & mask;
        if (++probes > mask) {
          full = true;
          break;
        }
      }
    }
  }
  if (__ballot(full) != 0 && lane == 0) atomicOr(err, kErrOverflow);
}

hipError_t launch_edge_hash(int64_t n_items, const uint64_t* items, const int32_t* rp, const int32_t* col,
                            uint64_t* slots, int bits, uint32_t* err, hipStream_t s) {
  hipError_t e = launch_fill_u64(slots, kEmptySlot, 1ll << bits, s);
  if (e != hipSuccess || n_items <= 0) return e;
  hipLaunchKernelGGL(k_edge_hash, dim3(item_grid(n_items)), dim3(256), 0, s, n_items, items, rp, col,
                     (unsigned long long*)slots, bits, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Node weights, one thread per node, from the finished row prefixes:
//   S_v = ACC_sigma at the row end;  Gamma_v = (d_v - 1) S_v  (Section 4.1.1)
//   Gamma^(1)_v = (d_v - 1)(d_v - 2) S_v                      (Section 5.1.1)
//   Gamma^(2)_v = ACC_tau at the row end = S_v^2 - sum (d_x - 1)^2 (Section 5.1.2)
//   Lambda_3 = sum C(d_v, 3), Lambda_4 = sum C(d_v, 4)        (Table 1)
// The Lambdas are reduced per block into `partials` (2 per block) and finished by
// k_lambda_final, so no two blocks update the same word.
// ---------------------------------------------------------------------------------
constexpr int kWeightThreads = 256;

__global__ __launch_bounds__(256) void k_node_weights(int32_t n, const int32_t* __restrict__ rp,
                                                      const uint32_t* __restrict__ acc_sigma,
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
    const uint64_t S = d > 0 ? (uint64_t)acc_sigma[r1 - 1] : 0;
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

hipError_t launch_node_weights(int32_t n, const int32_t* rp, const uint32_t* acc_sigma, const uint64_t* acc_tau,
                               uint64_t* w_gamma, uint64_t* w_gamma1, uint64_t* w_gamma2, uint64_t* partials,
                               unsigned long long* lambdas, uint32_t* err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nb = node_weight_blocks(n);
  hipLaunchKernelGGL(k_node_weights, dim3(nb), dim3(kWeightThreads), 0, s, n, rp, acc_sigma, acc_tau, w_gamma,
                     w_gamma1, w_gamma2, partials, err);
  hipLaunchKernelGGL(k_lambda_final, dim3(1), dim3(256), 0, s, partials, nb, lambdas, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Inclusive scan of u64 node arrays (reduce, scan of block sums, apply), blocked
// layout of 8 items per thread, wrap detection on every addition.
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

__global__ __launch_bounds__(256) void k_scan_reduce(const uint64_t* __restrict__ in, int64_t n,
                                                     uint64_t* __restrict__ sums, uint32_t* err, uint32_t err_bit) {
  __shared__ uint64_t wave_tot[kScanThreads / 64];
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
    sums[blockIdx.x] = total;
  }
  if (__ballot(wrapped) != 0 && lane_id() == 0) atomicOr(err, err_bit);
}

// Exclusive scan of the block sums by one block, tile after tile.
__global__ __launch_bounds__(256) void k_scan_top(uint64_t* sums, int64_t nb, uint32_t* err, uint32_t err_bit) {
  __shared__ uint64_t wave_tot[kScanThreads / 64];
  bool wrapped = false;
  uint64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanTile) {
    const uint64_t tot = block_scan_tile(sums, base, nb, carry, true, wrapped, wave_tot);
    carry = add_wrap(carry, tot, wrapped);
  }
  if (__ballot(wrapped) != 0 && lane_id() == 0) atomicOr(err, err_bit);
}

__global__ __launch_bounds__(256) void k_scan_apply(uint64_t* data, int64_t n, const uint64_t* __restrict__ offsets,
                                                    uint32_t* err, uint32_t err_bit) {
  __shared__ uint64_t wave_tot[kScanThreads / 64];
  bool wrapped = false;
  block_scan_tile(data, (int64_t)blockIdx.x * kScanTile, n, offsets[blockIdx.x], false, wrapped, wave_tot);
  if (__ballot(wrapped) != 0 && lane_id() == 0) atomicOr(err, err_bit);
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_scan_inplace(uint64_t* data, int64_t n, uint64_t* tmp, uint32_t* err, uint32_t err_bit,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, tmp, err, err_bit);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, tmp, nb, err, err_bit);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, tmp, err, err_bit);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Guide table for a node draw: guide[b] is the node drawn by the smallest word of
// bucket b (the top gbits bits of the word), guide[2^gbits] = n - 1.  The draw is
// monotone in the word, so every word of bucket b picks a node in
// [guide[b], guide[b+1]], and the search runs over that window only.
// ---------------------------------------------------------------------------------
__global__ void k_guide(const uint64_t* __restrict__ acc, int32_t n, int gbits, uint32_t* __restrict__ guide) {
  const int64_t G = 1ll << gbits;
  const uint64_t total = acc[n - 1];
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

hipError_t launch_guide(const uint64_t* acc, int32_t n, int gbits, uint32_t* guide, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t G = (1ll << gbits) + 1;
  hipLaunchKernelGGL(k_guide, dim3(fill_grid(G)), dim3(256), 0, s, acc, n, gbits, guide);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Node records and row guides.  A weighted pick inside a row (sigma, mu, tau) is a
// search for the first entry of the row's prefix above a value x < total.  For rows
// with d >= kRowGuideMin the value range is cut into 2^g buckets of width 2^s
// (g = floor(log2 d) - 1, s = max(0, bitlen(total) - g)); guide[b] is the first
// entry above b * 2^s, and guide[2^g] = d - 1.  A value x in bucket b = x >> s has
// its answer in [guide[b], guide[b+1]], a window of about two entries.  The pick is
// the same entry as the plain binary search; only the number of reads changes.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ int row_guide_bits(int32_t d) { return 31 - __clz(d) - 1; }

__device__ __forceinline__ int row_guide_shift(uint64_t total, int g) {
  const int bl = total ? 64 - __clzll((long long)total) : 0;
  return bl > g ? bl - g : 0;
}

__global__ void k_row_guide_sizes(int32_t n, const int32_t* __restrict__ rp, uint64_t* __restrict__ sizes) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = rp[v + 1] - rp[v];
    sizes[v] = d >= kRowGuideMin ? (1ull << row_guide_bits(d)) + 1 : 0ull;
  }
}

hipError_t launch_row_guide_sizes(int32_t n, const int32_t* rp, uint64_t* sizes, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_guide_sizes, dim3(fill_grid(n)), dim3(256), 0, s, n, rp, sizes);
  return hipGetLastError();
}

// With goff_end: writes whole records (S_v = 0 when acc_sigma is null).  Without:
// only refreshes S_v of existing records.
__global__ void k_records(int32_t n, const int32_t* __restrict__ rp, const uint32_t* __restrict__ acc_sigma,
                          const uint64_t* __restrict__ goff_end, uint4* __restrict__ rec) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r0 = rp[v], r1 = rp[v + 1], d = r1 - r0;
    const uint32_t S = (acc_sigma && d > 0) ? acc_sigma[r1 - 1] : 0u;
    if (goff_end) {
      const uint64_t size = d >= kRowGuideMin ? (1ull << row_guide_bits(d)) + 1 : 0ull;
      rec[v] = make_uint4((uint32_t)r0, (uint32_t)d, S, (uint32_t)(goff_end[v] - size));
    } else {
      rec[v].z = S;
    }
  }
}

hipError_t launch_records(int32_t n, const int32_t* rp, const uint32_t* acc_sigma, const uint64_t* goff_end, uint4* rec,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_records, dim3(fill_grid(n)), dim3(256), 0, s, n, rp, acc_sigma, goff_end, rec);
  return hipGetLastError();
}

// One wave per work item: entry i of the row covers the buckets whose lower bound
// lies in [ACC[i-1], ACC[i]); the last entry also covers the buckets at or above the
// total.
template <typename T>
__global__ __launch_bounds__(256) void k_row_guides(int64_t n_items, const uint64_t* __restrict__ items,
                                                    const int32_t* __restrict__ rp, const uint4* __restrict__ rec,
                                                    const T* __restrict__ acc, uint32_t* __restrict__ guide) {
  const int lane = lane_id();
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n_items; i += nwaves) {
    const ItemRange it = item_range(items, rp, i);
    const int32_t d = it.r1 - it.r0;
    if (d < kRowGuideMin) continue;
    const int g = row_guide_bits(d);
    const uint64_t total = acc[it.r1 - 1];
    const int s = row_guide_shift(total, g);
    const uint64_t last_bucket = 1ull << g;
    uint32_t* gd = guide + rec[it.v].w;
    for (int32_t e = it.e0 + lane; e < it.e1; e += 64) {
      const uint64_t lo = e > it.r0 ? (uint64_t)acc[e - 1] : 0ull, hi = (uint64_t)acc[e];
      const uint64_t b0 = lo ? ((lo - 1) >> s) + 1 : 0ull;
      uint64_t b1 = hi ? ((hi - 1) >> s) + 1 : 0ull;
      if (e == it.r1 - 1) b1 = last_bucket + 1;
      for (uint64_t b = b0; b < b1; ++b) gd[b] = (uint32_t)(e - it.r0);
    }
  }
}

hipError_t launch_row_guides(bool tau, int64_t n_items, const uint64_t* items, const int32_t* rp, const uint4* rec,
                             const uint32_t* acc_sigma, const uint64_t* acc_tau, uint32_t* guide, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (tau)
    hipLaunchKernelGGL(k_row_guides<uint64_t>, dim3(item_grid(n_items)), dim3(256), 0, s, n_items, items, rp, rec,
                       acc_tau, guide);
  else
    hipLaunchKernelGGL(k_row_guides<uint32_t>, dim3(item_grid(n_items)), dim3(256), 0, s, n_items, items, rp, rec,
                       acc_sigma, guide);
  return hipGetLastError();
}

// Weighted pick in a row: the first entry of acc[0..d) above x (x < total = acc[d-1]).
template <typename T>
__device__ __forceinline__ int32_t row_pick(const T* __restrict__ acc, int32_t d, uint64_t total, uint64_t x,
                                            const uint32_t* __restrict__ guide, uint32_t goff) {
  if (d < kRowGuideMin) return first_above(acc, 0, d - 1, x);
  const int g = row_guide_bits(d);
  const uint64_t b = x >> row_guide_shift(total, g);
  const uint32_t* gd = guide + goff;
  return first_above(acc, (int32_t)gd[b], (int32_t)gd[b + 1], x);
}

// ---------------------------------------------------------------------------------
// The samplers.  Each returns the motif class of sample k (0 = rejected) and, when
// `nodes` is not null, writes the sampled nodes v, u, w, r, t.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ int32_t pick_node(const SamplerView& a, uint64_t x) {
  const uint64_t r = bounded(x, a.total);
  const uint32_t b = (uint32_t)(x >> (64 - a.gbits));
  return first_above(a.acc_node, (int32_t)a.guide[b], (int32_t)a.guide[b + 1], r);
}

// RandomVertex(N_a - {skip}) with skip in N_a: index j uniform over the row with
// skip's slot removed; the sorted row is read at j and stepped past skip.
__device__ __forceinline__ int32_t neighbour_except(const int32_t* __restrict__ col, int32_t ra, int32_t da,
                                                    int32_t skip, uint64_t word) {
  const int32_t j = (int32_t)bounded(word, (uint64_t)(da - 1));
  const int32_t x = col[ra + j];
  return x >= skip ? col[ra + j + 1] : x;
}

// row start and degree of a node (the first half of its record)
__device__ __forceinline__ uint2 row_of(const uint4* __restrict__ rec, int32_t x) {
  return *reinterpret_cast<const uint2*>(rec + x);
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
  const int32_t iu = row_pick(a.acc_sigma + rv, dv, R.z, bounded(W[1], R.z), a.sig_guide, R.w);
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
  const uint64_t* __restrict__ hs = a.edge_slots;
  const int hb = a.edge_bits;
  const int m = (int)edge_hash_has(hs, hb, u, w) | (int)edge_hash_has(hs, hb, v, r) << 1 |
                (int)edge_hash_has(hs, hb, w, r) << 2;
  return lut[m];
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
  const int32_t iu = row_pick(a.acc_sigma + rv, dv, R.z, bounded(W[1], R.z), a.sig_guide, R.w);
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
  const uint64_t* __restrict__ hs = a.edge_slots;
  const int hb = a.edge_bits;
  const int m = (int)edge_hash_has(hs, hb, u, w) | (int)edge_hash_has(hs, hb, u, r) << 1 |
                (int)edge_hash_has(hs, hb, w, r) << 2 | (int)edge_hash_has(hs, hb, v, t) << 3 |
                (int)edge_hash_has(hs, hb, w, t) << 4 | (int)edge_hash_has(hs, hb, r, t) << 5;
  return lut[m];
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
  const int32_t iu = row_pick(tau, dv, T, bounded(W[1], T), a.tau_guide, R.w);
  const int32_t u = col[rv + iu];
  const uint32_t* __restrict__ sig = a.acc_sigma + rv;
  const uint64_t Sv = R.z;
  const uint64_t blk_lo = iu > 0 ? sig[iu - 1] : 0;
  const uint64_t du1 = (uint64_t)sig[iu] - blk_lo;
  uint64_t x = bounded(W[2], Sv - du1);
  x += x >= blk_lo ? du1 : 0;
  const int32_t iw = row_pick(sig, dv, Sv, x, a.sig_guide, R.w);
  const int32_t w = col[rv + iw];
  const uint2 U = row_of(a.rec, u), Wr = row_of(a.rec, w);
  const int32_t ru = (int32_t)U.x, du = (int32_t)U.y, rw = (int32_t)Wr.x, dw = (int32_t)Wr.y;
  const int32_t r = neighbour_except(col, ru, du, v, W[3]);
  const int32_t t = neighbour_except(col, rw, dw, v, X[0]);
  if (nodes) {
    nodes[0] = v; nodes[1] = u; nodes[2] = w; nodes[3] = r; nodes[4] = t;
  }
  if (t == u || r == w || t == r) return 0;
  const uint64_t* __restrict__ hs = a.edge_slots;
  const int hb = a.edge_bits;
  const int m = (int)edge_hash_has(hs, hb, v, r) | (int)edge_hash_has(hs, hb, v, t) << 1 |
                (int)edge_hash_has(hs, hb, u, w) << 2 | (int)edge_hash_has(hs, hb, u, t) << 3 |
                (int)edge_hash_has(hs, hb, w, r) << 4 | (int)edge_hash_has(hs, hb, r, t) << 5;
  return lut[m];
}

template <int S>
__device__ __forceinline__ int draw(const SamplerView& a, const uint8_t* lut, uint64_t seed, uint64_t k,
                                    int32_t* nodes) {
  if constexpr (S == kMoss4) return draw_moss4(a, lut, seed, k, nodes);
  else if constexpr (S == kT5) return draw_t5(a, lut, seed, k, nodes);
  else return draw_path5(a, lut, seed, k, nodes);
}

template <int S>
__device__ __forceinline__ void load_lut(uint8_t* lut) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    if constexpr (S == kMoss4) lut[tid] = tid < 8 ? c_lut4[tid] : 0;
    else if constexpr (S == kT5) lut[tid] = c_lut5t[tid];
    else lut[tid] = c_lut5p[tid];
  }
}

constexpr int kMaxWaves = 16;  // 1024 threads per block at most
constexpr int kBins = 22;

template <int S>
__global__ __launch_bounds__(256, 8) void k_sample(SamplerView a, uint64_t seed, uint64_t k0, uint64_t k1,
                                                unsigned long long* __restrict__ hits, uint8_t* __restrict__ class_out) {
  __shared__ uint32_t bins[kMaxWaves][kBins + 2];
  __shared__ uint8_t lut[64];
  const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int i = tid; i < nw * (kBins + 2); i += blockDim.x) bins[i / (kBins + 2)][i % (kBins + 2)] = 0;
  load_lut<S>(lut);
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = k0 + (uint64_t)blockIdx.x * blockDim.x + tid; k < k1; k += stride) {
    const int c = draw<S>(a, lut, seed, k, nullptr);
    atomicAdd(&bins[wave][c], 1u);
    if (class_out) class_out[k - k0] = (uint8_t)c;
  }
  __syncthreads();
  if (tid < kBins) {
    uint64_t s = 0;
    for (int w = 0; w < nw; ++w) s += bins[w][tid];
    if (s) atomicAdd(&hits[tid], (unsigned long long)s);
  }
}

hipError_t launch_sample(int sampler, const SamplerView& v, uint64_t seed, uint64_t k0, uint64_t k1,
                         unsigned long long* hits, uint8_t* class_out, int grid, int block, hipStream_t s) {
  // per-wave LDS counters are 32-bit: keep each launch below 2^31 samples per wave
  const uint64_t max_chunk = (uint64_t)grid * (uint64_t)block * (1ull << 24);
  for (uint64_t a = k0; a < k1;) {
    const uint64_t b = k1 - a > max_chunk ? a + max_chunk : k1;
    uint8_t* co = class_out ? class_out + (a - k0) : nullptr;
    switch (sampler) {
      case kMoss4: hipLaunchKernelGGL(k_sample<kMoss4>, dim3(grid), dim3(block), 0, s, v, seed, a, b, hits, co); break;
      case kT5: hipLaunchKernelGGL(k_sample<kT5>, dim3(grid), dim3(block), 0, s, v, seed, a, b, hits, co); break;
      case kPath5: hipLaunchKernelGGL(k_sample<kPath5>, dim3(grid), dim3(block), 0, s, v, seed, a, b, hits, co); break;
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    a = b;
  }
  return hipSuccess;
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
__global__ __launch_bounds__(256, 8) void k_batch(const SamplerView* __restrict__ views, const Tile* __restrict__ tiles,
                                               const uint32_t* __restrict__ n_tiles_p, uint32_t* tile_counter,
                                               unsigned long long* __restrict__ bins) {
  __shared__ uint32_t lb[kMaxWaves][kBins + 2];
  __shared__ uint8_t lut4[64], lut5t[64], lut5p[64];
  __shared__ uint32_t cur;
  const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
  if (tid < 64) {
    lut4[tid] = tid < 8 ? c_lut4[tid] : 0;
    lut5t[tid] = c_lut5t[tid];
    lut5p[tid] = c_lut5p[tid];
  }
  const uint32_t n_tiles = *n_tiles_p;
  for (;;) {
    if (tid == 0) cur = atomicAdd(tile_counter, 1u);
    for (int i = tid; i < nw * (kBins + 2); i += blockDim.x) lb[i / (kBins + 2)][i % (kBins + 2)] = 0;
    __syncthreads();
    const uint32_t t = cur;
    if (t >= n_tiles) break;
    const Tile tile = tiles[t];
    const SamplerView v = views[tile.view];
    if (tile.sampler == kMoss4) {
      for (uint64_t k = tile.k0 + tid; k < tile.k1; k += blockDim.x)
        atomicAdd(&lb[wave][draw_moss4(v, lut4, tile.seed, k, nullptr)], 1u);
    } else if (tile.sampler == kT5) {
      for (uint64_t k = tile.k0 + tid; k < tile.k1; k += blockDim.x)
        atomicAdd(&lb[wave][draw_t5(v, lut5t, tile.seed, k, nullptr)], 1u);
    } else {
      for (uint64_t k = tile.k0 + tid; k < tile.k1; k += blockDim.x)
        atomicAdd(&lb[wave][draw_path5(v, lut5p, tile.seed, k, nullptr)], 1u);
    }
    __syncthreads();
    if (tid < kBins) {
      uint64_t s = 0;
      for (int w = 0; w < nw; ++w) s += lb[w][tid];
      if (s) atomicAdd(&bins[(uint64_t)tile.out * kBins + tid], (unsigned long long)s);
    }
    __syncthreads();
  }
}

hipError_t launch_batch(const SamplerView* views, const Tile* tiles, const uint32_t* n_tiles, uint32_t* tile_counter,
                        unsigned long long* bins, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(block), 0, s, views, tiles, n_tiles, tile_counter, bins);
  return hipGetLastError();
}

int sample_kernel_blocks_per_cu(int sampler, int block) {
  int nb = 0;
  hipError_t e = hipSuccess;
  switch (sampler) {
    case kMoss4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sample<kMoss4>, block, 0); break;
    case kT5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sample<kT5>, block, 0); break;
    case kPath5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sample<kPath5>, block, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch, block, 0); break;
  }
  return e == hipSuccess ? nb : 0;
}

}  // namespace moss
