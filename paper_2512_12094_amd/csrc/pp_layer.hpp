// Layer op: a commuting run of rotations applied bucket by bucket.
//
// Prop. 1 with the exact merge of identical strings and the truncation
// after every rotation (Algorithm 1 step 2a), for r <= kLayerMaxRot
// pairwise commuting rotations P_1..P_r of one sub-layer, in circuit order.
//
// Why buckets are closed.  Let a(Q) be the set of g with {P_g, Q} = 0.  For
// g in a(Q), P_g Q anticommutes with P_h exactly when Q does (the P's
// commute), so a is the same on the whole set Q <P_g : g in a(Q)>, which is
// everything the r rotations can make from Q.  Multiplying by such a P_g
// flips only bits inside the union of the x- and z-supports of {P_g : g in
// a}, so the key (a, x outside that x-union, z outside that z-union) is the
// same for every member.  A bucket of a hash of the key therefore holds, for
// each string in it, its partner under every rotation and every child the
// rotations can make: a block rotates its bucket in LDS with no other block.
//
// Within a bucket, rotation g runs over the strings live before it (their
// stamp equals g), each with its partner P_g Q found in the bucket's LDS
// hash table: both live -> the pair rotation (the lower index writes both),
// partner absent or dropped -> cos on Q and a child sin on P_g Q (a dropped
// partner's slot is reused), then the truncation of what changed, exactly as
// the one-rotation gate kernel does it, so the results are bitwise those of
// r gate launches.  Children of rotation g get indices past those it reads.
#pragma once
#include "pp_kernels.hpp"

namespace pp {

constexpr int kLBlock = 256;
constexpr int kLWaves = kLBlock / 64;

template <int WW> struct LayerCap;
template <> struct LayerCap<1> { static constexpr int n = 2048; };   // strings per bucket in LDS
template <> struct LayerCap<2> { static constexpr int n = 1024; };

// Bucket bits for a layer op over M entries: about 2^kLayerShift strings per
// bucket, more after failures (boost), at most lmaxbits.
__device__ __host__ __forceinline__ uint32_t layer_bits(uint32_t M, uint32_t boost,
                                                        uint32_t maxbits) {
  uint32_t lg = 0;
  while (lg < 32 && (1ull << lg) < (uint64_t)M) ++lg;
  int bits = (int)lg - kLayerShift + (int)boost;
  if (bits < 0) bits = 0;
  if (bits > (int)maxbits) bits = (int)maxbits;
  return (uint32_t)bits;
}

__device__ __forceinline__ uint64_t rot_word(const double* t, int k) {
  return (uint64_t)__double_as_longlong(t[k]);
}

// The bucket key's hash: anticommutation pattern and the bits no
// anticommuting rotation touches.
template <int WW>
__device__ __forceinline__ uint64_t layer_key(const uint64_t* x, const uint64_t* z, uint32_t r,
                                              const uint64_t (*px)[WW], const uint64_t (*pz)[WW]) {
  uint64_t a = 0, ux[WW], uz[WW];
#pragma unroll
  for (int w = 0; w < WW; ++w) ux[w] = uz[w] = 0;
  for (uint32_t g = 0; g < r; ++g) {
    uint32_t par = 0;
#pragma unroll
    for (int w = 0; w < WW; ++w) par += __popcll((x[w] & pz[g][w]) ^ (z[w] & px[g][w]));
    if (par & 1u) {
      a |= 1ull << g;
#pragma unroll
      for (int w = 0; w < WW; ++w) {
        ux[w] |= px[g][w];
        uz[w] |= pz[g][w];
      }
    }
  }
  uint64_t h = mix64(a ^ 0x2545f4914f6cdd1dull);
#pragma unroll
  for (int w = 0; w < WW; ++w) {
    h = mix64(h ^ (x[w] & ~ux[w]));
    h = mix64(h ^ (z[w] & ~uz[w]) ^ 0x9e3779b97f4a7c15ull);
  }
  return h;
}

// 1. Every live string of the current half to its bucket's staging slots.
template <int WW>
__global__ __launch_bounds__(kBlock) void k_layer_scatter(Solo S) {
  __shared__ uint64_t s_px[kLayerMaxRot][WW], s_pz[kLayerMaxRot][WW];
  const InstBuf& b = S.b;
  InstDyn& d = *S.d;
  if (d.pc != S.k) return;                 // an earlier op did not complete
  const Op& op = b.prog[S.k];
  const uint32_t r = op.nrot;
  for (uint32_t g = threadIdx.x; g < r; g += kBlock) {
#pragma unroll
    for (int w = 0; w < WW; ++w) {
      s_px[g][w] = rot_word(op.table, g * kLayerRec + w);
      s_pz[g][w] = rot_word(op.table, g * kLayerRec + kMaxW + w);
    }
  }
  __syncthreads();
  const uint32_t M = d.M;
  const uint32_t bits = layer_bits(M, d.lboost, b.lmaxbits);
  const uint32_t slots = b.lslots >> bits, L = b.lslots;
  const View v = view_of(b, d);
  bool over = op.fail_test != 0 && blockIdx.x == 0 && threadIdx.x == 0;
  const uint32_t Mrun = op.fail_test ? 0u : M;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < Mrun; i += gridDim.x * kBlock) {
    if (!v.al[i]) continue;
    uint64_t x[WW], z[WW];
#pragma unroll
    for (int w = 0; w < WW; ++w) {
      x[w] = v.X[(size_t)w * v.cap + i];
      z[w] = v.Z[(size_t)w * v.cap + i];
    }
    const double c = v.getc(i);
    const uint64_t h = layer_key<WW>(x, z, r, s_px, s_pz);
    const uint32_t bk = bits ? (uint32_t)(h >> (64 - bits)) : 0u;
    const uint32_t rank = atomicAdd(&b.lcount[bk], 1u);
    if (rank >= slots) { over = true; continue; }
    const size_t pos = (size_t)bk * slots + rank;
#pragma unroll
    for (int w = 0; w < WW; ++w) {
      b.lstx[(size_t)w * L + pos] = x[w];
      b.lstz[(size_t)w * L + pos] = z[w];
    }
    b.lstc[pos] = c;
  }
  if (over) atomicOr(&d.lfail, 1u);
}

template <int WW>
__device__ __forceinline__ uint32_t lds_hash(const uint64_t* x, const uint64_t* z) {
  uint64_t h = x[0] * 0x9e3779b97f4a7c15ull ^ z[0] * 0xc2b2ae3d27d4eb4full;
  if (WW > 1) h = (h ^ (h >> 29)) * 0xbf58476d1ce4e5b9ull ^ x[WW - 1] * 0x94d049bb133111ebull ^
                  z[WW - 1] * 0xff51afd7ed558ccdull;
  return (uint32_t)((h ^ (h >> 31)) >> 32);
}

// Liveness stamps: a string kept through rotation g gets g + 1, a string
// revived by rotation g (its slot reused for a child) gets kRevived + g + 1.
// Rotation g reads the strings live before it: stamp g or kRevived + g, or
// g + 1 when its pair's leader already kept it (a revival by rotation g,
// kRevived + g + 1, is not live before it).
constexpr uint8_t kRevived = 128;
__device__ __forceinline__ bool live_before(uint8_t st, uint32_t g) {
  return st == g || st == g + 1 || st == kRevived + g;
}
__device__ __forceinline__ bool live_after(uint8_t st, uint32_t g) {
  return st == g + 1 || st == kRevived + g + 1;
}

// 2. One block per bucket (grid-stride over buckets): the r rotations in
// LDS, then the survivors to the other half.  The last block folds the
// sums and advances the program (or reports the failure).
template <int WW>
__global__ __launch_bounds__(kLBlock) void k_layer_apply(Solo S) {
  constexpr int CAP = LayerCap<WW>::n, HS = 2 * CAP;
  constexpr int NS = 7;                    // sums, see below
  __shared__ uint64_t s_x[WW][CAP], s_z[WW][CAP];
  __shared__ double s_c[CAP];
  __shared__ uint8_t s_st[CAP];            // liveness stamp
  __shared__ uint16_t s_hash[HS];          // index + 1, 0 = empty
  __shared__ uint64_t s_px[kLayerMaxRot][WW], s_pz[kLayerMaxRot][WW];
  __shared__ double s_cs[kLayerMaxRot], s_sn[kLayerMaxRot];
  __shared__ uint32_t s_inc[3], s_n0, s_fail, s_flag, s_tmp[kLWaves + 1], s_base;
  __shared__ uint64_t s_red[kLWaves][NS];
  const InstBuf& b = S.b;
  InstDyn& d = *S.d;
  if (d.pc != S.k) return;                 // uniform: pc changes only in the last block
  const Op& op = b.prog[S.k];
  const uint32_t r = op.nrot;
  const double eps = op.eps;
  const int wmax = op.wmax;
  const bool full = op.full_check != 0, gtab = op.gtab != 0;
  const bool has_next = op.next_gate != kNone32;
  uint64_t nxm[WW], nzm[WW];
#pragma unroll
  for (int w = 0; w < WW; ++w) { nxm[w] = op.nx[w]; nzm[w] = op.nz[w]; }
  for (uint32_t g = threadIdx.x; g < r; g += kLBlock) {
#pragma unroll
    for (int w = 0; w < WW; ++w) {
      s_px[g][w] = rot_word(op.table, g * kLayerRec + w);
      s_pz[g][w] = rot_word(op.table, g * kLayerRec + kMaxW + w);
    }
    s_cs[g] = op.table[g * kLayerRec + 2 * kMaxW];
    s_sn[g] = op.table[g * kLayerRec + 2 * kMaxW + 1];
  }
  const uint32_t M = d.M;
  const uint32_t bits = layer_bits(M, d.lboost, b.lmaxbits);
  const uint32_t P = 1u << bits, slots = b.lslots >> bits, L = b.lslots;
  const bool failed = ld_agent(&d.lfail) != 0;   // the scatter launch has ended
  const uint32_t ho = d.half ^ 1u;
  const uint32_t gen1 = d.gen + 1;
  const bool f32 = b.f32 != 0;
  const uint32_t cap = b.cap;
  // sums: [0] live before each rotation, [1] anticommuting with it,
  // [2] survivors, [3] survivors anticommuting with the next gate,
  // [4] children, [5] strings held at the end, [6] strings entering
  uint64_t sum[NS] = {0, 0, 0, 0, 0, 0, 0};
  bool bad = false;
  auto heavy = [&](const uint64_t* x, const uint64_t* z) {
    if (wmax < 0) return false;
    int w8 = 0;
#pragma unroll
    for (int w = 0; w < WW; ++w) w8 += __popcll(x[w] | z[w]);
    return w8 > wmax;
  };
  // index of the string (x, z) in the bucket, or -1
  auto find = [&](const uint64_t* x, const uint64_t* z) -> int {
    uint32_t sl = lds_hash<WW>(x, z) & (HS - 1);
    for (int probe = 0; probe < HS; ++probe) {
      const uint32_t e = *reinterpret_cast<volatile uint16_t*>(&s_hash[sl]);
      if (e == 0) return -1;
      const int j = (int)e - 1;
      bool eq = true;
#pragma unroll
      for (int w = 0; w < WW; ++w) eq = eq && s_x[w][j] == x[w] && s_z[w][j] == z[w];
      if (eq) return j;
      sl = (sl + 1) & (HS - 1);
    }
    return -1;
  };
  // publishes index j (its string already written) under (x, z)
  auto insert = [&](const uint64_t* x, const uint64_t* z, int j) {
    uint32_t sl = lds_hash<WW>(x, z) & (HS - 1);
    for (int probe = 0; probe < HS; ++probe) {
      const uintptr_t a = reinterpret_cast<uintptr_t>(&s_hash[sl]);
      uint32_t* wp = reinterpret_cast<uint32_t*>(a & ~uintptr_t(3));
      const uint32_t shift = (a & 2) ? 16u : 0u;
      uint32_t old = *reinterpret_cast<volatile uint32_t*>(wp);
      for (;;) {
        if ((old >> shift) & 0xFFFFu) break;                      // slot taken
        const uint32_t got = atomicCAS(wp, old, old | ((uint32_t)(j + 1) << shift));
        if (got == old) return;
        old = got;
      }
      sl = (sl + 1) & (HS - 1);
    }
  };

  for (uint32_t bk = blockIdx.x; bk < P; bk += gridDim.x) {
    __syncthreads();                       // the previous bucket's LDS is free
    if (threadIdx.x == 0) {
      const uint32_t cnt = b.lcount[bk];
      b.lcount[bk] = 0;                    // zero for the next layer op
      s_n0 = cnt < slots ? cnt : slots;
      s_fail = s_n0 > (uint32_t)CAP ? 1u : 0u;
      s_inc[0] = s_inc[1] = s_inc[2] = 0;
    }
    for (int t = threadIdx.x; t < HS / 2; t += kLBlock) reinterpret_cast<uint32_t*>(s_hash)[t] = 0;
    __syncthreads();
    if (failed || s_fail) { bad = bad || s_fail; continue; }   // uniform
    const uint32_t n0 = s_n0;
    const size_t base = (size_t)bk * slots;
    sum[6] += threadIdx.x == 0 ? n0 : 0u;
    for (uint32_t j = threadIdx.x; j < n0; j += kLBlock) {
      uint64_t x[WW], z[WW];
#pragma unroll
      for (int w = 0; w < WW; ++w) {
        x[w] = b.lstx[(size_t)w * L + base + j];
        z[w] = b.lstz[(size_t)w * L + base + j];
        s_x[w][j] = x[w];
        s_z[w][j] = z[w];
      }
      s_c[j] = b.lstc[base + j];
      s_st[j] = 0;
      __threadfence_block();
      insert(x, z, (int)j);
    }
    __syncthreads();
    uint32_t ng = n0;                      // strings before rotation g
    for (uint32_t g = 0; g < r; ++g) {
      if (threadIdx.x == 0) s_inc[(g + 1) % 3] = 0;
      uint64_t px[WW], pz[WW];
#pragma unroll
      for (int w = 0; w < WW; ++w) { px[w] = s_px[g][w]; pz[w] = s_pz[g][w]; }
      const double cs = s_cs[g], sn = s_sn[g];
      const bool chk = g == 0 && full;
      const uint8_t kept = (uint8_t)(g + 1), back = (uint8_t)(kRevived + g + 1);
      for (uint32_t j = threadIdx.x; j < ng; j += kLBlock) {
        if (!live_before(s_st[j], g)) continue;
        ++sum[0];
        uint64_t qx[WW], qz[WW];
#pragma unroll
        for (int w = 0; w < WW; ++w) { qx[w] = s_x[w][j]; qz[w] = s_z[w][j]; }
        if (!anticommutes(qx, qz, px, pz, WW)) {      // unchanged
          const double cq = s_c[j];
          if (!chk || (fabs(cq) >= eps && !heavy(qx, qz))) s_st[j] = kept;
          continue;
        }
        ++sum[1];
        uint64_t rx[WW], rz[WW];
#pragma unroll
        for (int w = 0; w < WW; ++w) { rx[w] = qx[w] ^ px[w]; rz[w] = qz[w] ^ pz[w]; }
        const int p = find(rx, rz);
        const bool plive = p >= 0 && (uint32_t)p < ng && live_before(s_st[p], g);
        if (plive && (uint32_t)p < j) continue;       // the partner's thread leads
        const int sig = product_sign(px, pz, qx, qz, rx, rz, WW);   // i P Q = sig R
        const double cq = s_c[j];
        if (plive) {                       // Q and R = PQ live: a rotation of the pair
          double nq, nr;
          rotate_pair(f32, cs, sn, sig, cq, s_c[p], &nq, &nr);
          s_c[j] = nq;
          s_c[p] = nr;
          if (fabs(nq) >= eps && !(chk && heavy(qx, qz))) s_st[j] = kept;
          if (fabs(nr) >= eps && !(chk && heavy(rx, rz))) s_st[p] = kept;
        } else {
          double nq, child;
          rotate_single(f32, cs, sn, sig, cq, &nq, &child);
          s_c[j] = nq;
          if (fabs(nq) >= eps && !(chk && heavy(qx, qz))) s_st[j] = kept;
          if (fabs(child) >= eps && !heavy(rx, rz)) {
            ++sum[4];
            if (p >= 0) {                  // a dropped string comes back in its slot
              s_c[p] = child;
              s_st[p] = back;
            } else {
              const uint32_t k = ng + atomicAdd(&s_inc[g % 3], 1u);
              if (k >= (uint32_t)CAP) {
                s_fail = 1;
              } else {
#pragma unroll
                for (int w = 0; w < WW; ++w) { s_x[w][k] = rx[w]; s_z[w][k] = rz[w]; }
                s_c[k] = child;
                s_st[k] = back;
                __threadfence_block();
                insert(rx, rz, (int)k);
              }
            }
          }
        }
      }
      __syncthreads();
      const uint32_t add = s_inc[g % 3];
      ng = ng + add < (uint32_t)CAP ? ng + add : (uint32_t)CAP;
    }
    sum[5] += threadIdx.x == 0 ? ng : 0u;
    if (s_fail) { bad = true; continue; }  // uniform: read after the last barrier
    // survivors to the other half: one atomic per block and bucket
    uint32_t mine = 0;
    for (uint32_t j = threadIdx.x; j < ng; j += kLBlock) mine += live_after(s_st[j], r - 1) ? 1u : 0u;
    uint32_t total;
    uint32_t off = block_scan(mine, s_tmp, &total);
    if (threadIdx.x == 0) s_base = total ? atomicAdd(&d.nuniq, total) : 0u;
    __syncthreads();
    const uint32_t ob = s_base;
    sum[2] += mine;
    for (uint32_t j = threadIdx.x; j < ng; j += kLBlock) {
      if (!live_after(s_st[j], r - 1)) continue;
      const uint32_t pos = ob + off++;
      uint64_t x[kMaxW] = {}, z[kMaxW] = {};
#pragma unroll
      for (int w = 0; w < WW; ++w) { x[w] = s_x[w][j]; z[w] = s_z[w][j]; }
      if (has_next && anticommutes(x, z, nxm, nzm, WW)) ++sum[3];
      if (pos >= cap) { atomicOr(&d.status, ST_OVERFLOW); continue; }
#pragma unroll
      for (int w = 0; w < WW; ++w) {
        b.x[ho][(size_t)w * cap + pos] = x[w];
        b.z[ho][(size_t)w * cap + pos] = z[w];
      }
      if (f32)
        static_cast<float*>(b.c[ho])[pos] = (float)s_c[j];
      else
        static_cast<double*>(b.c[ho])[pos] = s_c[j];
      b.alive[ho][0][pos] = 1;
      if (gtab) gt_insert(b.gtab, b.hg_bits, gen1, pos, hash_key(x, z, WW, 0));
    }
  }
  // block sums -> this block's shard line, entries 1..NS
  {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      uint64_t t = sum[k];
      for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
      if (lane == 0) s_red[wid][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < NS) {
      uint64_t t = 0;
      for (int q = 0; q < kLWaves; ++q) t += s_red[q][threadIdx.x];
      if (t)
        atomicAdd((unsigned long long*)&b.accs[(blockIdx.x % kAccShards) * kLineU64 + 1 + threadIdx.x],
                  (unsigned long long)t);
    }
    if (threadIdx.x == 0 && bad) atomicOr(&d.lfail, 1u);
  }
  if (!last_block(S.sync, &s_flag, gridDim.x, true)) return;
  if (threadIdx.x != 0) return;
  uint64_t t[NS];
  for (int k = 0; k < NS; ++k) t[k] = 0;
  for (int sh = 0; sh < kAccShards; ++sh)
    for (int k = 0; k < NS; ++k)
      t[k] += atomicExch((unsigned long long*)&b.accs[sh * kLineU64 + 1 + k], 0ull);
  const uint32_t out = ld_agent(&d.nuniq);
  d.nuniq = 0;
  if (ld_agent(&d.status) & ST_OVERFLOW) {  // the survivors did not fit: grow, run again
    d.lneed = out;
    d.lfail = 0;
    d.failed_pc = d.pc;
    return;
  }
  if (ld_agent(&d.lfail)) {                 // a bucket did not fit: the host decides
    d.lfail = 0;
    d.status |= ST_LAYER;
    d.failed_pc = d.pc;
    return;
  }
  d.propagated += t[0];
  d.merged += t[0] + t[1];
  d.anti_total += t[1];
  d.key_reads += t[6];                      // each key read once
  d.coef_rw += t[6];                        // each coefficient read and written once
  d.appended += t[4];
  d.M = out;
  d.Mnext = out;
  d.live = out;
  d.count = (uint32_t)t[3];
  const uint64_t held = t[5] > out ? t[5] : out;
  if (held > d.peak) d.peak = held < 0xFFFFFFFFull ? (uint32_t)held : 0xFFFFFFFFu;
  d.half = ho;
  d.parity = 0;
  if (gtab) d.gen = gen1;
  d.count_for = op.next_gate;
  d.pc += 1 + op.skip;
}

}  // namespace pp
