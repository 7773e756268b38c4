// Partitioned exact merge of large narrow-key record sets (Algorithm 1 step
// 2b; Algorithms 2 and 3 with the map of representatives replaced by a
// bucket partition and per-bucket LDS tables).
//
// Four one-instance launches, each gated on the instance's merge phase:
//
//   k_part_hist    tiles of kPartTileRec records: each live record's
//                  representative key, mixed once (h = mix64(key), a
//                  bijection) and stored for the later passes, its bucket
//                  (top pbits of h), LDS counts per bucket, one row of
//                  per-tile counts.
//   k_part_scan    column scan of the count matrix (per bucket, the tiles'
//                  exclusive offsets and the bucket total); the last block
//                  turns the totals into bucket bases and the list of
//                  aggregation items.
//   k_part_scatter every live record (h, coefficient) to its exact place in
//                  the bucket-contiguous staging array: kPartSub records at a
//                  time are counting-sorted by bucket in LDS and written out
//                  as runs.
//   k_part_agg     one block per bucket: every record of the bucket is added
//                  into an LDS table of kPartSlots mixed keys with exact carry-free
//                  sums (a coefficient's fixed-point value in 32-bit chunks,
//                  each added without carry into a 64-bit accumulator), and
//                  one term per key (unmix64(h)) is emitted.  A bucket with more than twice
//                  the average records (a few representatives holding many
//                  records) is cut into chunks summed by separate blocks into
//                  the global merge table, which the collect pass emits.  A
//                  bucket with more keys than the table takes is summed in
//                  2^k selector passes (the keys whose mix bits select pass q),
//                  each emitted on its own; a pass that still overflows adds
//                  its keys into the global table.
//
// Every key ends in exactly one place (the bucket's block, or the global
// table), sums are exact integers, so the result does not depend on the order
// of the records or on how the blocks are scheduled.
#pragma once
#include "pp_kernels.hpp"

namespace pp {

constexpr int kPHBlock = 512;    // histogram / scatter block
constexpr int kPCBlock = 1024;   // column scan block (16 waves)
constexpr int kPABlock = 1024;   // aggregation block (16 waves)
constexpr int kPASub = 2;        // records per thread per aggregation round

// Mixed key of "no record here" in the hashed array, and of an empty slot in
// the aggregation table: the mix of kEmpty64, the one key summed apart.
constexpr uint64_t kMixEmpty = mix64(kEmpty64);

__host__ __device__ __forceinline__ uint32_t part_bits(uint32_t M, uint32_t maxbits,
                                                       uint32_t shift) {
  const uint32_t need = (M >> shift) + ((M & ((1u << shift) - 1)) ? 1u : 0u);
  uint32_t bits = 0;
  while ((1u << bits) < need && bits < 31) ++bits;
  if (bits < (uint32_t)kPartMinBits) bits = kPartMinBits;
  if (bits > maxbits) bits = maxbits;
  return bits;
}

__device__ __forceinline__ uint32_t part_bucket(uint64_t h, uint32_t pbits) {
  return (uint32_t)(h >> (64 - pbits));
}
__device__ __forceinline__ uint32_t part_slot(uint64_t h) {
  return (uint32_t)(h >> 8) & (uint32_t)(kPartSlots - 1);
}
// selector of the passes over an overfull bucket (bits not used above)
__device__ __forceinline__ uint32_t part_sel(uint64_t h, uint32_t K) {
  return (uint32_t)(h >> 24) & (K - 1);
}

// Exclusive scan over a block of NB threads, one value each; *total = sum.
template <int NB>
__device__ __forceinline__ uint32_t bscan(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
  constexpr int NW = NB / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_tmp[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int w = 0; w < NW; ++w) { const uint32_t t = s_tmp[w]; s_tmp[w] = acc; acc += t; }
    s_tmp[NW] = acc;
  }
  __syncthreads();
  const uint32_t r = x - v + s_tmp[wid];
  *total = s_tmp[NW];
  __syncthreads();
  return r;
}

// Block sums of two counters for thread 0 (all threads call).
template <int NB>
__device__ __forceinline__ void bsum2(uint32_t a, uint32_t b, uint32_t* s_tmp, uint32_t* ta,
                                      uint32_t* tb) {
  constexpr int NW = NB / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += (uint32_t)__shfl_xor((int)a, o, 64);
    b += (uint32_t)__shfl_xor((int)b, o, 64);
  }
  if (lane == 0) { s_tmp[2 * wid] = a; s_tmp[2 * wid + 1] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t x = 0, y = 0;
    for (int w = 0; w < NW; ++w) { x += s_tmp[2 * w]; y += s_tmp[2 * w + 1]; }
    *ta = x;
    *tb = y;
  }
  __syncthreads();
}

__device__ __forceinline__ bool part_served(const InstBuf& b, const InstDyn& d, uint32_t phase) {
  return merge_served(b, d, true, phase) && use_part(b, d);
}

// Merge phases of the partitioned path (0 = not started; 1 = the collect
// pass's phase, shared with the one-pass merge).
enum : uint32_t { PH_SCAN = 10, PH_SCATTER = 11, PH_AGG = 12 };

// ---------------------------------------------------------------------------
// 1. histogram
// ---------------------------------------------------------------------------
template <int G>
__global__ __launch_bounds__(kPHBlock) void k_part_hist(Solo S) {
  extern __shared__ uint32_t s_h[];              // P counters
  __shared__ uint32_t s_flag;
  const InstBuf& b = S.b;
  InstDyn& d = *S.d;
  if (d.pc != S.k || !part_served(b, d, 0)) return;
  const uint32_t M = d.M;
  const uint32_t pbits = part_bits(M, b.pmaxbits, b.pshift), P = 1u << pbits;
  const uint32_t T = (M + kPartTileRec - 1) / kPartTileRec;
  const uint32_t workers = worker_count(T);
  if (blockIdx.x >= workers) return;
  const View v = view_of(b, d);
  bool range = false;
  constexpr int U = 4;
  for (uint32_t t = blockIdx.x; t < T; t += gridDim.x) {
    for (uint32_t q = threadIdx.x; q < P; q += kPHBlock) s_h[q] = 0;
    __syncthreads();
    const uint32_t lo = t * kPartTileRec;
    const uint32_t hi = M - lo < (uint32_t)kPartTileRec ? M : lo + kPartTileRec;
    for (uint32_t i0 = lo + threadIdx.x; i0 < hi; i0 += U * kPHBlock) {
      uint64_t x[U], z[U];
      uint8_t a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t i = i0 + u * kPHBlock;
        a[u] = i < hi ? v.al[i] : 0;
        x[u] = i < hi ? v.X[i] : 0;
        z[u] = i < hi ? v.Z[i] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t i = i0 + u * kPHBlock;
        if (i >= hi) continue;
        uint64_t h = kMixEmpty;
        if (a[u]) {
          const uint64_t key = narrow_key_t<G>(b, x[u], z[u]);
          if (key == kEmpty64) {                 // the one key equal to the empty marker
            fx_atomic_add(d.special_fx, fx_from_double(v.getc(i), &range));
            atomicOr(&d.special, 1u);
          } else {
            h = mix64(key);
            atomicAdd(&s_h[part_bucket(h, pbits)], 1u);
          }
        }
        b.phash[i] = h;
      }
    }
    __syncthreads();
    uint32_t* row = b.phist + (size_t)t * P;
    for (uint32_t q = threadIdx.x; q < P; q += kPHBlock) row[q] = s_h[q];
    __syncthreads();
  }
  if (range) atomicOr(&d.status, ST_RANGE);
  if (!last_block(S.sync, &s_flag, workers, false)) return;
  if (threadIdx.x == 0) {
    d.merged += d.live;
    d.pbits = pbits;
    d.pglobal = 0;
    d.plist_n = 0;
    d.pruns += 1;
    d.mphase = PH_SCAN;
  }
}

// ---------------------------------------------------------------------------
// 2. column scan + bucket bases + aggregation items
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPCBlock) void k_part_scan(Solo S) {
  constexpr int NW = kPCBlock / 64;
  __shared__ uint32_t s_part[NW][64];
  __shared__ uint32_t s_tmp[2 * NW + 2];
  __shared__ uint32_t s_flag;
  const InstBuf& b = S.b;
  InstDyn& d = *S.d;
  if (d.pc != S.k || !part_served(b, d, PH_SCAN)) return;
  const uint32_t M = d.M;
  const uint32_t pbits = d.pbits, P = 1u << pbits;
  const uint32_t T = (M + kPartTileRec - 1) / kPartTileRec;
  const uint32_t bands = P / 64;                 // P >= 64
  const uint32_t workers = bands < gridDim.x ? bands : gridDim.x;
  if (blockIdx.x >= workers) return;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t rows = (T + NW - 1) / NW;
  const uint32_t r0 = wid * rows, r1 = r0 + rows < T ? r0 + rows : T;
  for (uint32_t band = blockIdx.x; band < bands; band += gridDim.x) {
    const uint32_t col = band * 64 + lane;
    uint32_t sum = 0;
    for (uint32_t t = r0; t < r1; ++t) sum += b.phist[(size_t)t * P + col];
    s_part[wid][lane] = sum;
    __syncthreads();
    if (wid == 0) {
      uint32_t acc = 0;
      for (int w = 0; w < NW; ++w) { const uint32_t x = s_part[w][lane]; s_part[w][lane] = acc; acc += x; }
      b.ptot[col] = acc;
    }
    __syncthreads();
    uint32_t run = s_part[wid][lane];
    for (uint32_t t = r0; t < r1; ++t) {
      uint32_t* p = b.phist + (size_t)t * P + col;
      const uint32_t x = *p;
      *p = run;
      run += x;
    }
    __syncthreads();
  }
  if (!last_block(S.sync, &s_flag, workers, true)) return;
  // the last block: bucket bases and aggregation items
  constexpr int PER = (1 << kPartMaxBits) / kPCBlock;   // buckets per thread (<= 4)
  uint32_t cnt[PER], nch[PER];
  uint32_t mine = 0, total = 0, hot = 0;
  const uint32_t per = (P + kPCBlock - 1) / kPCBlock;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const uint32_t p = threadIdx.x * per + k;
    cnt[k] = ((uint32_t)k < per && p < P) ? ld_agent(&b.ptot[p]) : 0u;
    mine += cnt[k];
  }
  uint32_t off = bscan<kPCBlock>(mine, s_tmp, &total);
  // chunk length of a split bucket: twice the average
  const uint32_t avg = (total + P - 1) / P;
  const uint32_t chunk = 2 * (avg > 512u ? avg : 512u);
  uint32_t items = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const uint32_t p = threadIdx.x * per + k;
    if ((uint32_t)k >= per || p >= P) { nch[k] = 0; continue; }
    b.pbase[p] = off;
    off += cnt[k];
    nch[k] = cnt[k] == 0 ? 0u : (cnt[k] > chunk ? (cnt[k] + chunk - 1) / chunk : 1u);
    if (nch[k] > 1) ++hot;
    items += nch[k];
  }
  if (threadIdx.x == 0) b.pbase[P] = total;
  uint32_t nitems;
  uint32_t ioff = bscan<kPCBlock>(items, s_tmp, &nitems);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const uint32_t p = threadIdx.x * per + k;
    for (uint32_t j = 0; j < nch[k]; ++j) b.pwork[ioff++] = p | (j << 16);
  }
  uint32_t thot, tz;
  bsum2<kPCBlock>(hot, 0u, s_tmp, &thot, &tz);
  if (threadIdx.x == 0) {
    d.pnwork = nitems;
    d.pchunk = chunk;
    d.phot += thot;
    d.mphase = PH_SCATTER;
  }
}

// ---------------------------------------------------------------------------
// 3. scatter into the bucket-contiguous staging array
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPHBlock) void k_part_scatter(Solo S) {
  constexpr int R = kPartSub / kPHBlock;         // records per thread per sub-round
  constexpr int PT = (1 << kPartMaxBits) / kPHBlock;
  __shared__ ulonglong2 s_rec[kPartSub];
  extern __shared__ uint32_t s_dyn[];            // s_cnt[P], s_loc[P], s_cur[P]
  __shared__ uint32_t s_tmp[kPHBlock / 64 + 1];
  __shared__ uint32_t s_flag;
  const InstBuf& b = S.b;
  InstDyn& d = *S.d;
  if (d.pc != S.k || !part_served(b, d, PH_SCATTER)) return;
  const uint32_t M = d.M;
  const uint32_t pbits = d.pbits, P = 1u << pbits;
  uint32_t* s_cnt = s_dyn;
  uint32_t* s_loc = s_dyn + P;
  uint32_t* s_cur = s_dyn + 2 * P;
  const uint32_t T = (M + kPartTileRec - 1) / kPartTileRec;
  const uint32_t workers = worker_count(T);
  if (blockIdx.x >= workers) return;
  const View v = view_of(b, d);
  const uint32_t per = P / kPHBlock ? P / kPHBlock : 1u;   // buckets per thread in scans
  for (uint32_t t = blockIdx.x; t < T; t += gridDim.x) {
    for (uint32_t q = threadIdx.x; q < P; q += kPHBlock)
      s_cur[q] = b.pbase[q] + b.phist[(size_t)t * P + q];
    const uint32_t lo = t * kPartTileRec;
    const uint32_t hi = M - lo < (uint32_t)kPartTileRec ? M : lo + kPartTileRec;
    // the next sub-round's records are loaded while this one is sorted
    uint64_t nhk[R], ncb[R];
    auto load = [&](uint32_t r0) {
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const uint32_t i = r0 + k * kPHBlock + threadIdx.x;
        nhk[k] = i < hi ? b.phash[i] : kMixEmpty;
        ncb[k] = __double_as_longlong(i < hi ? v.getc(i) : 0.0);
      }
    };
    load(lo);
    for (uint32_t r0 = lo; r0 < hi; r0 += kPartSub) {
      for (uint32_t q = threadIdx.x; q < P; q += kPHBlock) s_cnt[q] = 0;
      uint64_t hk[R], cb[R];
#pragma unroll
      for (int k = 0; k < R; ++k) { hk[k] = nhk[k]; cb[k] = ncb[k]; }
      if (r0 + kPartSub < hi) load(r0 + kPartSub);
      __syncthreads();
      uint32_t at[R];                            // bucket << 16 | rank, or kNone32
#pragma unroll
      for (int k = 0; k < R; ++k) {
        at[k] = kNone32;
        if (hk[k] == kMixEmpty) continue;
        const uint32_t p = part_bucket(hk[k], pbits);
        at[k] = (p << 16) | atomicAdd(&s_cnt[p], 1u);
      }
      __syncthreads();
      // exclusive offsets of the buckets within this sub-round
      uint32_t loc[PT];
      uint32_t sum = 0;
#pragma unroll
      for (int k = 0; k < PT; ++k) {
        const uint32_t q = threadIdx.x * per + k;
        loc[k] = ((uint32_t)k < per && q < P) ? s_cnt[q] : 0u;
        sum += loc[k];
      }
      uint32_t nrec;
      uint32_t o = bscan<kPHBlock>(sum, s_tmp, &nrec);
#pragma unroll
      for (int k = 0; k < PT; ++k) {
        const uint32_t q = threadIdx.x * per + k;
        if ((uint32_t)k < per && q < P) s_loc[q] = o;
        o += loc[k];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < R; ++k) {
        if (at[k] == kNone32) continue;
        const uint32_t pos = s_loc[at[k] >> 16] + (at[k] & 0xffffu);
        s_rec[pos] = make_ulonglong2(hk[k], cb[k]);
      }
      __syncthreads();
      for (uint32_t j = threadIdx.x; j < nrec; j += kPHBlock) {
        const ulonglong2 e = s_rec[j];
        const uint32_t p = part_bucket(e.x, pbits);
        const uint32_t dst = s_cur[p] + (j - s_loc[p]);
        reinterpret_cast<ulonglong2*>(b.pstage)[dst] = e;
      }
      __syncthreads();
      for (uint32_t q = threadIdx.x; q < P; q += kPHBlock) s_cur[q] += s_cnt[q];
    }
    __syncthreads();
  }
  if (!last_block(S.sync, &s_flag, workers, false)) return;
  if (threadIdx.x == 0) d.mphase = PH_AGG;
}

// ---------------------------------------------------------------------------
// 4. aggregation per bucket
// ---------------------------------------------------------------------------
// A coefficient's fixed-point value c 2^kFxFrac (rounded as fx_from_double
// rounds) as three signed 64-bit addends for the 32-bit chunks q0, q0 + 1,
// q0 + 2: the 53-bit mantissa shifted by (shift mod 32) spans at most three
// chunks.  q0 <= 3, and a piece that would land in chunk 5 is always zero
// (|c| < 2^54), so it is added to chunk 4 as a zero.
struct Pieces {
  uint32_t q0;
  uint64_t a0, a1, a2;    // two's-complement addends (negated for c < 0)
};

__device__ __forceinline__ Pieces pieces_of(double c, bool* range) {
  Pieces r{0, 0, 0, 0};
  const uint64_t bits = __double_as_longlong(c);
  const int ex = (int)((bits >> 52) & 0x7FF);
  const uint64_t frac = bits & ((1ull << 52) - 1);
  if (ex == 0x7FF) { *range = true; return r; }
  const uint64_t mant = ex ? (frac | (1ull << 52)) : frac;
  const int sh = (ex ? ex - 1075 : -1074) + kFxFrac;   // value = mant * 2^sh units
  if (sh > kFxMaxShift) { *range = true; return r; }
  uint64_t lo;
  uint32_t hi = 0;
  if (sh < 0) {                                        // below one unit: rounded
    const int rs = -sh;
    lo = rs > 63 ? 0ull : ((mant + (1ull << (rs - 1))) >> rs);
  } else {
    const int b = sh & 31;
    r.q0 = (uint32_t)(sh >> 5);
    lo = mant << b;
    hi = b ? (uint32_t)(mant >> (64 - b)) : 0u;
  }
  const bool neg = (bits >> 63) != 0;
  const uint64_t p0 = lo & 0xffffffffull, p1 = lo >> 32, p2 = hi;
  r.a0 = neg ? 0ull - p0 : p0;
  r.a1 = neg ? 0ull - p1 : p1;
  r.a2 = neg ? 0ull - p2 : p2;
  return r;
}

// a * 2^(32 k) as a 192-bit two's-complement value (k < 5)
__device__ __forceinline__ Fx fx_chunk(int64_t a, int k) {
  const uint64_t s = a < 0 ? ~0ull : 0ull;
  uint64_t l[3] = {(uint64_t)a, s, s};
  const int words = k >> 1;
  if (k & 1) {
    l[2] = (l[2] << 32) | (l[1] >> 32);
    l[1] = (l[1] << 32) | (l[0] >> 32);
    l[0] = l[0] << 32;
  }
  Fx r{0, 0, 0};
  if (words == 0) r = Fx{l[0], l[1], l[2]};
  else if (words == 1) r = Fx{0, l[0], l[1]};
  else r = Fx{0, 0, l[0]};
  return r;
}

struct PartTable {
  uint64_t* key;                                  // [kPartSlots] mixed keys
  unsigned long long (*sum)[kPartSlots];          // [kPartChunks][kPartSlots]
  uint32_t* fill;
};

// Adds (mixed key h, pieces) to the LDS table; false when h is new and the
// table is full (a new key is refused once kPartFill keys are in; at most
// blockDim more can race past that check), or when kPartProbe probes did not
// reach h or an empty slot (a crowded table: the key is refused, whether or
// not it is further on, and the pass is redone another way).  `k` is the key
// already read from the home slot part_slot(h).
__device__ __forceinline__ void pa_put(const PartTable& tb, uint32_t s, const Pieces& pc) {
  const uint32_t q1 = pc.q0 + 1, q2 = pc.q0 + 2 < (uint32_t)kPartChunks ? pc.q0 + 2 : pc.q0 + 1;
  atomicAdd(&tb.sum[pc.q0][s], (unsigned long long)pc.a0);
  atomicAdd(&tb.sum[q1][s], (unsigned long long)pc.a1);
  atomicAdd(&tb.sum[q2][s], (unsigned long long)pc.a2);
}

__device__ __forceinline__ bool pa_add_from(const PartTable& tb, uint64_t h, uint64_t k,
                                            const Pieces& pc) {
  uint32_t s = part_slot(h);
  for (int probe = 0; probe < kPartProbe; ++probe) {
    if (k == kMixEmpty) {
      if (*(volatile uint32_t*)tb.fill >= (uint32_t)kPartFill) return false;
      k = atomicCAS((unsigned long long*)&tb.key[s], (unsigned long long)kMixEmpty,
                    (unsigned long long)h);
      if (k == kMixEmpty) {
        atomicAdd(tb.fill, 1u);
        k = h;
      }
    }
    if (k == h) {
      pa_put(tb, s, pc);
      return true;
    }
    s = (s + 1) & (uint32_t)(kPartSlots - 1);
    k = tb.key[s];
  }
  return false;
}

__device__ __forceinline__ bool pa_add(const PartTable& tb, uint64_t h, const Pieces& pc) {
  return pa_add_from(tb, h, tb.key[part_slot(h)], pc);
}

__device__ __forceinline__ Fx pa_value(const PartTable& tb, uint32_t s) {
  Fx v{0, 0, 0};
#pragma unroll
  for (int q = 0; q < kPartChunks; ++q) v = fx_add(v, fx_chunk((int64_t)tb.sum[q][s], q));
  return v;
}

__device__ __forceinline__ void pa_clear(const PartTable& tb) {
  for (int s = threadIdx.x; s < kPartSlots; s += kPABlock) {
    tb.key[s] = kMixEmpty;
#pragma unroll
    for (int q = 0; q < kPartChunks; ++q) tb.sum[q][s] = 0;
  }
  if (threadIdx.x == 0) *tb.fill = 0;
  __syncthreads();
}

// Global merge table: find-or-insert listing newly claimed slots, exact add.
__device__ __forceinline__ void mt_add_listed(const InstBuf& b, InstDyn& d, uint64_t key, Fx v) {
  const uint32_t bits = merge_bits(b, d);
  const uint64_t mask = (1ull << bits) - 1;
  uint64_t s = mix64(key) >> (64 - bits);
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    unsigned long long k = b.mkey[s];
    if (k == kEmpty64) {
      k = atomicCAS((unsigned long long*)&b.mkey[s], (unsigned long long)kEmpty64,
                    (unsigned long long)key);
      if (k == kEmpty64) {
        b.plist[atomicAdd(&d.plist_n, 1u)] = (uint32_t)s;
        k = key;
      }
    }
    if (k == key) {
      fx_atomic_add(&b.mfx[3 * s], v);
      return;
    }
    s = (s + 1) & mask;
  }
}

// Moves every key of the LDS table into the global merge table (as the key
// itself, unmix64(h)) and clears the table; returns this thread's keys.
__device__ __forceinline__ uint32_t pa_flush(const InstBuf& b, InstDyn& d, const PartTable& tb) {
  uint32_t n = 0;
  for (int s = threadIdx.x; s < kPartSlots; s += kPABlock) {
    const uint64_t h = tb.key[s];
    if (h == kMixEmpty) continue;
    mt_add_listed(b, d, unmix64(h), pa_value(tb, s));
    tb.key[s] = kMixEmpty;
#pragma unroll
    for (int q = 0; q < kPartChunks; ++q) tb.sum[q][s] = 0;
    ++n;
  }
  __syncthreads();
  if (threadIdx.x == 0) *tb.fill = 0;
  __syncthreads();
  return n;
}

__global__ __launch_bounds__(kPABlock) void k_part_agg(Solo S) {
  __shared__ uint64_t s_key[kPartSlots];
  __shared__ unsigned long long s_sum[kPartChunks][kPartSlots];
  __shared__ uint32_t s_fill, s_flag, s_base, s_stop;
  __shared__ uint32_t s_tmp[2 * (kPABlock / 64) + 2];
  const InstBuf& b = S.b;
  InstDyn& d = *S.d;
  if (d.pc != S.k || !part_served(b, d, PH_AGG)) return;
  const uint32_t nwork = d.pnwork;
  const uint32_t workers = worker_count(nwork);
  if (blockIdx.x >= workers) return;
  const PartTable tb{s_key, s_sum, &s_fill};
  const Op& mop = b.prog[d.pc];
  const NextGate ng(b, mop);
  const uint32_t chunk = d.pchunk;
  const ulonglong2* stage = reinterpret_cast<const ulonglong2*>(b.pstage);
  uint32_t my_live = 0, my_cnt = 0, my_glob = 0, my_over = 0;   // live/cnt/over: thread 0
  bool range = false;
  constexpr uint32_t kRound = kPASub * kPABlock;

  // One pass over records [lo, hi) of the staging array, adding those with
  // selector q of K; the next round's records are loaded while this round's
  // are added.  Global mode (`glob`): a round that finds the table full
  // flushes it into the global table and retries; returns false.  Otherwise
  // the rounds run without barriers; the first record the table refuses
  // stops the pass, which returns true (it is then redone another way) with
  // *est = the bucket's distinct keys estimated from what it saw (thread 0).
  auto pass = [&](uint32_t lo, uint32_t hi, uint32_t K, uint32_t q, bool glob,
                  uint32_t* est) -> bool {
    if (threadIdx.x == 0) s_stop = 0;
    pa_clear(tb);
    uint32_t proc = 0, refused = 0;
    bool over_any = false;
    uint64_t nh[kPASub], nc[kPASub];
    auto load = [&](uint32_t r0) {
#pragma unroll
      for (int k = 0; k < kPASub; ++k) {
        const uint32_t r = r0 + k * kPABlock + threadIdx.x;
        if (r < hi) {
          const ulonglong2 e = stage[r];
          nh[k] = e.x;
          nc[k] = e.y;
        } else {
          nh[k] = kMixEmpty;
          nc[k] = 0;
        }
      }
    };
    if (lo < hi) load(lo);
    for (uint32_t r0 = lo; r0 < hi; r0 += kRound) {
      // without global mode, the first refusal anywhere in the block stops
      // the pass (read without a barrier: a round or two may still run)
      if (!glob && *(volatile uint32_t*)&s_stop) break;
      uint64_t h[kPASub], cbv[kPASub];
#pragma unroll
      for (int k = 0; k < kPASub; ++k) { h[k] = nh[k]; cbv[k] = nc[k]; }
      if (r0 + kRound < hi) load(r0 + kRound);
      uint32_t fail = 0;
      // the home slots of all the round's records are read together; a
      // record whose key sits there (the usual case) adds at once
      uint64_t home[kPASub];
#pragma unroll
      for (int k = 0; k < kPASub; ++k) {
        if (h[k] != kMixEmpty && part_sel(h[k], K) != q) h[k] = kMixEmpty;
        home[k] = h[k] == kMixEmpty ? kMixEmpty : tb.key[part_slot(h[k])];
      }
#pragma unroll
      for (int k = 0; k < kPASub; ++k) {
        if (h[k] == kMixEmpty) continue;
        const Pieces pc = pieces_of(__longlong_as_double(cbv[k]), &range);
        ++proc;
        if (home[k] == h[k]) {
          pa_put(tb, part_slot(h[k]), pc);
        } else if (!pa_add_from(tb, h[k], home[k], pc)) {
          fail |= 1u << k;
          ++refused;
        }
      }
      if (!glob) {                                 // a refused record spoils the pass
        if (fail) {
          over_any = true;
          s_stop = 1;
        }
        continue;
      }
      while (__syncthreads_or(fail != 0)) {       // global mode: flush and retry
        my_glob += pa_flush(b, d, tb);
        uint32_t again = 0;
#pragma unroll
        for (int k = 0; k < kPASub; ++k)
          if ((fail >> k) & 1u) {
            if (!pa_add(tb, h[k], pieces_of(__longlong_as_double(cbv[k]), &range)))
              again |= 1u << k;
          }
        fail = again;
      }
    }
    if (!glob && __syncthreads_or(over_any)) {
      // distinct keys of the bucket, estimated from the records processed:
      // the keys the table holds plus every refused record, scaled up
      uint32_t tp, tr;
      bsum2<kPABlock>(proc, refused, s_tmp, &tp, &tr);
      if (threadIdx.x == 0) {
        const uint64_t seen = (uint64_t)s_fill + tr, n = hi - lo;
        *est = (uint32_t)std::min<uint64_t>((seen * n + (tp ? tp : 1) - 1) / (tp ? tp : 1),
                                            0xFFFFFFFFull);
      }
      return true;
    }
    __syncthreads();
    return false;
  };

  // Emits one term per key of the table (that the merge's truncation keeps).
  auto emit = [&]() {
    constexpr int PER = kPartSlots / kPABlock;
    uint32_t keep = 0, mine = 0, cnt = 0;
    double val[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint32_t s = k * kPABlock + threadIdx.x;
      val[k] = 0.0;
      const uint64_t h = s_key[s];
      if (h == kMixEmpty) continue;
      uint64_t x[kMaxW], z[kMaxW];
      narrow_decode(b, unmix64(h), x, z);
      val[k] = fx_to_double(pa_value(tb, s));
      if (merge_keeps(b, mop, x, z, val[k])) {
        keep |= 1u << k;
        ++mine;
      }
    }
    uint32_t tot;
    uint32_t off = bscan<kPABlock>(mine, s_tmp, &tot);
    if (threadIdx.x == 0) s_base = tot ? atomicAdd(&d.nuniq, tot) : 0u;
    __syncthreads();
    const uint32_t base = s_base;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (!((keep >> k) & 1u)) continue;
      const uint32_t s = k * kPABlock + threadIdx.x;
      const uint32_t pos = base + off++;
      if (pos >= b.cap) { atomicOr(&d.status, ST_OVERFLOW); continue; }
      uint64_t x[kMaxW], z[kMaxW];
      narrow_decode(b, unmix64(s_key[s]), x, z);
      emit_term(b, d, pos, x, z, val[k]);
      if (ng.anti(x, z, b.W)) ++cnt;
    }
    uint32_t tl, tc;
    bsum2<kPABlock>(mine, cnt, s_tmp, &tl, &tc);
    if (threadIdx.x == 0) {
      my_live += tl;
      my_cnt += tc;
    }
  };

  // Per item, a sequence of passes (one call site each for pass and emit,
  // which keeps the kernel's code small):
  //   split chunk:   one pass in global mode, flushed;
  //   bucket:        one pass; if the table overflowed, K selector passes,
  //                  each emitted, or (if it overflowed too) rerun in global
  //                  mode and flushed.
  for (uint32_t w = blockIdx.x; w < nwork; w += gridDim.x) {
    const uint32_t item = b.pwork[w];
    const uint32_t p = item & 0xffffu, j = item >> 16;
    const uint32_t blo = b.pbase[p], bn = b.ptot[p];
    const bool split = bn > chunk;
    const uint32_t lo = blo + (split ? j * chunk : 0u);
    const uint32_t hi = split ? (lo + chunk < blo + bn ? lo + chunk : blo + bn) : blo + bn;
    uint32_t K = 1, q = 0;
    bool glob = split;
    while (q < K) {
      uint32_t est = 0;
      const bool over = pass(lo, hi, K, q, glob, &est);
      if (glob) {
        my_glob += pa_flush(b, d, tb);
      } else if (!over) {
        emit();
      } else if (K == 1) {
        // more keys than the table takes: 2^k selector passes, each aimed
        // at three quarters of the table
        if (threadIdx.x == 0) {
          const uint64_t want = (4 * (uint64_t)est + 3 * kPartFill - 1) / (3 * kPartFill);
          uint32_t k2 = 2;
          while (k2 < want && k2 < (uint32_t)kPartMaxPasses) k2 <<= 1;
          s_flag = k2;
          ++my_over;
        }
        __syncthreads();
        K = s_flag;
        __syncthreads();
        continue;                                  // q = 0 of K
      } else {
        glob = true;                               // rerun this pass in global mode
        continue;
      }
      if (!split) glob = false;
      ++q;
    }
  }
  if (range) atomicOr(&d.status, ST_RANGE);
  // counts: one accumulator line per block group; the last block folds them
  uint32_t tg, tz;
  bsum2<kPABlock>(my_glob, 0u, s_tmp, &tg, &tz);
  const uint32_t nsh = acc_shards(workers);
  if (threadIdx.x == 0) {
    const uint64_t v = (uint64_t)my_live | ((uint64_t)my_cnt << 32);
    if (v) {
      unsigned long long* a = nsh == 1 ? (unsigned long long*)&d.acc
                                       : (unsigned long long*)&b.accs[(blockIdx.x % nsh) * kLineU64];
      consume(atomicAdd(a, (unsigned long long)v));
    }
    if (tg) {
      atomicAdd(&d.pglob, tg);
      consume(atomicOr(&d.pglobal, 1u));
    }
    if (my_over) consume(atomicAdd(&d.pover, my_over));
  }
  if (!last_block(S.sync, &s_flag, workers, true)) return;
  if (threadIdx.x == 0) {
    fold_acc(b, d, nsh);
    d.mphase = 1;                                // the collect pass emits the global keys
  }
}

}  // namespace pp
