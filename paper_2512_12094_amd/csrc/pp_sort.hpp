// Key-sorted export of a store: the live strings in ascending order of their
// integer (Appendix E.2: qubit q is the base-4 digit of weight 4^q, with
// I, X, Y, Z = 0, 1, 2, 3; the same integer that picks a representative in
// Algorithms 2 and 3), so a merged set comes out one record per
// representative, sorted by key.
//
// Least-significant-digit radix sort of slot indices, 8 bits per pass, the
// digit read from the store through the index (no key arrays): per pass a
// histogram per tile of 4096 positions, one exclusive scan over the
// digit-major histogram, and a stable scatter.  The first pass reads the
// store's slots directly and drops the dead ones, so it also compacts.
// Ordering only: no arithmetic on coefficients.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pp_types.h"

constexpr int kSortBlock = 256;                       // = radix: thread t owns digit t
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;    // positions per tile
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kScanTile = 4096;                       // histogram entries per scan block

// Bit i of v moves to bit 2i (interleave by binary magic numbers).
__device__ __forceinline__ uint64_t sort_spread32(uint32_t v) {
  uint64_t r = v;
  r = (r | (r << 16)) & 0x0000FFFF0000FFFFull;
  r = (r | (r << 8)) & 0x00FF00FF00FF00FFull;
  r = (r | (r << 4)) & 0x0F0F0F0F0F0F0F0Full;
  r = (r | (r << 2)) & 0x3333333333333333ull;
  r = (r | (r << 1)) & 0x5555555555555555ull;
  return r;
}

// 64-bit word j of slot i's integer (qubits 32j .. 32j+31).  A letter's
// digit is 2z + (x xor z): I 00, X 01, Y 10, Z 11.
__device__ __forceinline__ uint64_t sort_int_word(const uint64_t* xs, const uint64_t* zs,
                                                  uint32_t cap, uint32_t i, int j) {
  const int w = j >> 1, sh = (j & 1) * 32;
  const uint64_t xw = xs[(size_t)w * cap + i], zw = zs[(size_t)w * cap + i];
  return (sort_spread32((uint32_t)(zw >> sh)) << 1) | sort_spread32((uint32_t)((xw ^ zw) >> sh));
}

struct SortPass {
  const uint64_t* x;       // store half: [W][cap]
  const uint64_t* z;
  const uint8_t* alive;    // first pass: liveness of slot i
  const uint32_t* src;     // later passes: slot at each position
  uint32_t* dst;           // slot at each output position
  uint32_t dst_cap;        // positions dst holds (a larger count is reported, not written)
  uint32_t* hist;          // [256][tiles], then exclusive offsets
  uint32_t cap;
  uint32_t n_in;           // positions read (store slots on the first pass)
  uint32_t tiles;
  int word;                // integer word j and bit shift inside it
  int shift;
  int first;
};

__device__ __forceinline__ bool sort_item(const SortPass& p, uint32_t i, uint32_t& slot,
                                          uint32_t& digit) {
  if (i >= p.n_in) return false;
  if (p.first) {
    if (!p.alive[i]) return false;
    slot = i;
  } else {
    slot = p.src[i];
  }
  digit = (uint32_t)(sort_int_word(p.x, p.z, p.cap, slot, p.word) >> p.shift) & 255u;
  return true;
}

__global__ __launch_bounds__(kSortBlock) void k_sort_hist(SortPass p) {
  __shared__ uint32_t cnt[kSortBlock];
  const int t = threadIdx.x;
  cnt[t] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * (uint32_t)kSortTile;
  for (int k = 0; k < kSortItems; ++k) {
    uint32_t slot, digit;
    if (sort_item(p, base + k * kSortBlock + t, slot, digit)) atomicAdd(&cnt[digit], 1u);
  }
  __syncthreads();
  p.hist[(size_t)t * p.tiles + blockIdx.x] = cnt[t];
}

// Exclusive scan of n entries in three launches: per-block totals, one
// block over the totals (which also writes the grand total), per-block
// rescan with the block's offset.
__device__ __forceinline__ uint32_t sort_block_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  // inclusive scan over kSortBlock threads, returns the exclusive prefix
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < kSortBlock; o <<= 1) {
    const uint32_t a = t >= o ? sh[t - o] : 0u;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const uint32_t incl = sh[t];
  total = sh[kSortBlock - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kSortBlock) void k_sort_scan_reduce(const uint32_t* a, uint32_t n,
                                                                 uint32_t* part) {
  __shared__ uint32_t sh[kSortBlock];
  const uint32_t base = blockIdx.x * (uint32_t)kScanTile;
  uint32_t s = 0;
  for (int k = threadIdx.x; k < kScanTile; k += kSortBlock)
    if (base + k < n) s += a[base + k];
  uint32_t total;
  (void)sort_block_scan(s, sh, total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(kSortBlock) void k_sort_scan_top(uint32_t* part, uint32_t n,
                                                              uint32_t* grand) {
  __shared__ uint32_t sh[kSortBlock];
  uint32_t carry = 0;
  for (uint32_t b = 0; b < n; b += kSortBlock) {
    const uint32_t i = b + threadIdx.x;
    const uint32_t v = i < n ? part[i] : 0u;
    uint32_t total;
    const uint32_t ex = sort_block_scan(v, sh, total);
    if (i < n) part[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *grand = carry;
}

__global__ __launch_bounds__(kSortBlock) void k_sort_scan_down(uint32_t* a, uint32_t n,
                                                               const uint32_t* part) {
  __shared__ uint32_t sh[kSortBlock];
  // thread t rescans the contiguous run [t*16, t*16 + 16) of the block's tile
  constexpr int kRun = kScanTile / kSortBlock;
  const uint32_t base = blockIdx.x * (uint32_t)kScanTile + threadIdx.x * kRun;
  uint32_t v[kRun], s = 0;
#pragma unroll
  for (int k = 0; k < kRun; ++k) {
    v[k] = base + k < n ? a[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = part[blockIdx.x] + sort_block_scan(s, sh, total);
#pragma unroll
  for (int k = 0; k < kRun; ++k) {
    if (base + k < n) a[base + k] = run;
    run += v[k];
  }
}

// Stable scatter of one tile: positions are taken 256 at a time in order;
// inside a wave, lanes with the same digit find each other with eight
// ballots, and earlier waves' counts come from LDS.
__global__ __launch_bounds__(kSortBlock) void k_sort_scatter(SortPass p) {
  __shared__ uint32_t base[kSortBlock];
  __shared__ uint32_t wcnt[kSortWaves][kSortBlock];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  base[t] = p.hist[(size_t)t * p.tiles + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kSortWaves; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const uint32_t tile = blockIdx.x * (uint32_t)kSortTile;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int k = 0; k < kSortItems; ++k) {
    uint32_t slot = 0, digit = 0;
    const bool valid = sort_item(p, tile + k * kSortBlock + t, slot, digit);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (digit >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = __popcll(peers & below);
    if (valid && lane == 63 - __clzll(peers)) wcnt[wave][digit] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[digit] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][digit];
      if (pos < p.dst_cap) p.dst[pos] = slot;
    }
    __syncthreads();
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      tot += wcnt[w][t];
      wcnt[w][t] = 0;
    }
    base[t] += tot;
    __syncthreads();
  }
}

// Rows in output order: x/z as W words per row, coefficients as FP64.
__global__ __launch_bounds__(kSortBlock) void k_sort_emit(const uint32_t* order, uint32_t n,
                                                          const uint64_t* xs, const uint64_t* zs,
                                                          const void* c, int f32, uint32_t cap,
                                                          int W, uint64_t* ox, uint64_t* oz,
                                                          double* oc) {
  const uint32_t r = blockIdx.x * kSortBlock + threadIdx.x;
  if (r >= n) return;
  const uint32_t i = order[r];
  for (int w = 0; w < W; ++w) {
    ox[(size_t)r * W + w] = xs[(size_t)w * cap + i];
    oz[(size_t)r * W + w] = zs[(size_t)w * cap + i];
  }
  oc[r] = f32 ? (double)static_cast<const float*>(c)[i] : static_cast<const double*>(c)[i];
}
