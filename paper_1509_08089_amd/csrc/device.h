// Device helpers for the Moss sampling kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace moss {

// Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC 2011).  Each round
// takes the 128-bit products of words 0 and 2 with two odd multipliers; the next
// state is (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0)); the key
// advances by two Weyl increments between rounds.
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

// The 128-bit product a * b as four 32 x 32 -> 64-bit partial products, each one
// multiply-add (v_mad_u64_u32); none of the partial sums exceeds 64 bits.  Spelled out
// because the high half written as __umul64hi next to a 64-bit low product compiles to
// about a third more multiplies (the Philox rounds are what the grouping pass spends
// its time on).
__device__ __forceinline__ void mul_wide(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p = (uint64_t)a0 * b0;
  const uint64_t t = (uint64_t)a1 * b0 + (p >> 32);
  const uint64_t u = (uint64_t)a0 * b1 + (uint32_t)t;
  hi = (uint64_t)a1 * b1 + (t >> 32) + (u >> 32);
  lo = (u << 32) | (uint32_t)p;
}

// Random words of block `blk` of sample `k`: counter (k, blk, 0, 0), key (seed, tag).
__device__ __forceinline__ void philox_block(uint64_t k, uint64_t blk, uint64_t seed, uint64_t tag,
                                             uint64_t out[4]) {
  uint64_t x0 = k, x1 = blk, x2 = 0, x3 = 0;
  uint64_t k0 = seed, k1 = tag;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mul_wide(x0, kPhiloxM0, hi0, lo0);
    mul_wide(x2, kPhiloxM1, hi1, lo1);
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

// Two consecutive 32-bit words p[0], p[1] in one 8-byte load (dword alignment is enough
// for global loads on gfx950), so a guide window or a pair of row entries costs one
// memory request instead of two.
template <typename T>
__device__ __forceinline__ uint2 load_pair(const T* p) {
  static_assert(sizeof(T) == 4, "32-bit words");
  uint2 v;
  __builtin_memcpy(&v, p, sizeof(v));
  return v;
}

// floor(x * n / 2^64): a uniform index in [0, n) from one 64-bit word.
__device__ __forceinline__ uint64_t bounded(uint64_t x, uint64_t n) { return __umul64hi(x, n); }

// Smallest i in [lo, hi] with value(i) > r, given value(hi) > r (inverse CDF over an
// inclusive prefix; Section 4.1.3 "WeightRandomVertex", step 2).
template <typename F>
__device__ __forceinline__ int32_t first_above_by(F value, int32_t lo, int32_t hi, uint64_t r) {
  int32_t n = hi - lo;
  while (n > 0) {
    const int32_t half = n >> 1;
    if (value(lo + half) <= r) {
      lo += half + 1;
      n -= half + 1;
    } else {
      n = half;
    }
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ int32_t first_above(const T* __restrict__ acc, int32_t lo, int32_t hi, uint64_t r) {
  return first_above_by([acc](int32_t i) { return static_cast<uint64_t>(acc[i]); }, lo, hi, r);
}

// Is key in the sorted row col[base .. base+len)?
__device__ __forceinline__ bool row_has(const int32_t* __restrict__ col, int32_t base, int32_t len, int32_t key) {
  int32_t lo = base, n = len;
  while (n > 1) {
    const int32_t half = n >> 1;
    if (col[lo + half] <= key) lo += half;
    n -= half;
  }
  return n == 1 && col[lo] == key;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// ---- edge hash set: open addressing with linear probing over 2^bits u64 slots ----
constexpr uint64_t kEmptySlot = ~0ull;

__device__ __forceinline__ uint64_t edge_key(int32_t a, int32_t b) {
  const uint32_t lo = (uint32_t)min(a, b), hi = (uint32_t)max(a, b);
  return (uint64_t)lo << 32 | hi;
}

// Fibonacci hashing: the top bits of key * 2^64 / phi.
__device__ __forceinline__ uint64_t edge_slot(uint64_t key, int bits) {
  return (key * 0x9E3779B97F4A7C15ull) >> (64 - bits);
}

// Settles a lookup of `key` whose home slot h held `first`: found, absent (an empty
// slot ends the probe sequence) or, rarely, more slots to walk.
__device__ __forceinline__ bool edge_hash_rest(const uint64_t* __restrict__ slots, int bits, uint64_t key, uint64_t h,
                                               uint64_t first) {
  if (first == key) return true;
  if (first == kEmptySlot) return false;
  const uint64_t mask = (1ull << bits) - 1;
  for (uint64_t i = 1; i <= mask; ++i) {
    h = (h + 1) & mask;
    const uint64_t x = slots[h];
    if (x == key) return true;
    if (x == kEmptySlot) return false;
  }
  return false;
}

// ---- edge filter: a blocked Bloom filter in front of the hash set ----
// Every edge sets 4 bits of one 64-bit word.  A pair whose 4 bits are not all set
// is certainly not an edge, so most non-edges are settled by one read of a table
// small enough to stay cached; the others and every edge go on to the hash set.  The
// word of a key is the top filter_bits bits of its Fibonacci hash (the high part of
// its home slot in the hash set, so the filter can be built from the set slot range by
// slot range); the 4 bit positions come from the splitmix64 finaliser (Steele, Lea and
// Flood, OOPSLA 2014) of the key.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t filter_mask(uint64_t z) {
  return (1ull << (z & 63)) | (1ull << ((z >> 6) & 63)) | (1ull << ((z >> 12) & 63)) | (1ull << ((z >> 18) & 63));
}

// Inclusive scan over the 64 lanes of a wave; `wrapped` is set on any 64-bit wrap.
__device__ __forceinline__ uint64_t wave_inclusive_scan(uint64_t x, bool& wrapped) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_up(x, off, 64);
    if (lane >= off) {
      const uint64_t z = x + y;
      wrapped |= z < x;
      x = z;
    }
  }
  return x;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ __forceinline__ uint64_t wave_sum_wrap(uint64_t x, bool& wrapped) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t z = x + __shfl_xor(x, off, 64);
    wrapped |= z < x;
    x = z;
  }
  return x;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x |= __shfl_xor(x, off, 64);
  return x;
}

// C(d, 3) and C(d, 4) for d < 2^31, exactly: the factorial denominators are
// divided out of the consecutive factors before multiplying, so only the final
// product can exceed 64 bits, which sets `over`.
__device__ __forceinline__ uint64_t choose3(uint64_t d, bool& over) {
  if (d < 3) return 0;
  uint64_t f0 = d, f1 = d - 1, f2 = d - 2;
  if ((f0 & 1) == 0) f0 >>= 1; else f1 >>= 1;
  if (f0 % 3 == 0) f0 /= 3; else if (f1 % 3 == 0) f1 /= 3; else f2 /= 3;
  const uint64_t p = f0 * f1;
  over |= __umul64hi(p, f2) != 0;
  return p * f2;
}

__device__ __forceinline__ uint64_t choose4(uint64_t d, bool& over) {
  if (d < 4) return 0;
  uint64_t f[4] = {d, d - 1, d - 2, d - 3};
  // one of four consecutive numbers is a multiple of 4, the one two away is even
  int i4 = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (f[i] % 4 == 0) i4 = i;
  f[i4] /= 4;
  f[i4 < 2 ? i4 + 2 : i4 - 2] /= 2;
  bool done = false;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (!done && f[i] % 3 == 0) {
      f[i] /= 3;
      done = true;
    }
  const uint64_t p = f[0] * f[1], q = f[2] * f[3];
  over |= __umul64hi(p, q) != 0;
  return p * q;
}

}  // namespace moss
