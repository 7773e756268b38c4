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
// The same holds for any union of such sets, so within a bucket each wave
// takes the strings of whole sets (by the key's hash): a wave rotates its
// strings with no other wave and no barrier, and runs only the rotations one
// of its strings anticommutes with (a is shared by a set's members).
//
// A wave's rotation g runs over its strings live before it, each with its
// partner P_g Q found in the wave's LDS hash table: both live -> the pair
// rotation (the lower index writes both), partner absent or dropped -> cos
// on Q and a child sin on P_g Q (a dropped partner's slot is reused), then
// the truncation of what changed, exactly as the one-rotation gate kernel
// does it, so the results are bitwise those of r gate launches.  Children
// of rotation g get indices past those it reads.
#pragma once
#include "pp_kernels.hpp"

namespace pp {

constexpr uint32_t kAlive = 0xFFu;   // died field of a live string (see live_before)

template <int WW> struct LayerCap;
template <> struct LayerCap<1> { static constexpr int n = 2048; };   // strings per bucket in LDS
template <> struct LayerCap<2> { static constexpr int n = 1024; };

// Bucket bits for a layer op over M entries: about 2^shift strings per
// bucket, more after failures (boost), at most maxbits.
__device__ __host__ __forceinline__ uint32_t layer_bits(uint32_t M, int32_t boost,
                                                        uint32_t maxbits, uint32_t shift) {
  uint32_t lg = 0;
  while (lg < 32 && (1ull << lg) < (uint64_t)M) ++lg;
  int bits = (int)lg - (int)shift + boost;   // boost: from earlier failures
  if (bits < 0) bits = 0;
  if (bits > (int)maxbits) bits = (int)maxbits;
  return (uint32_t)bits;
}

__device__ __forceinline__ uint64_t rot_word(const double* t, int k) {
  return (uint64_t)__double_as_longlong(t[k]);
}

// The bucket key's hash (anticommutation pattern and the bits no
// anticommuting rotation touches); *pat = the pattern.
template <int WW>
__device__ __forceinline__ uint64_t layer_key(const uint64_t* x, const uint64_t* z, uint32_t r,
                                              const uint64_t (*px)[WW], const uint64_t (*pz)[WW],
                                              uint64_t* pat) {
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
  *pat = a;
  return h;
}

constexpr int kLTile = 4;                  // strings per thread per scatter round
constexpr int kLAggMax = 2048;             // buckets counted in LDS before the global add

// 1. Every live string of the current half to its bucket's staging slots,
// with its pattern and key hash.  A round of kBlock * kLTile strings counts
// its strings per bucket in LDS and reserves each bucket's slots with one
// global add (buckets up to kLAggMax; beyond, one global add per string).
template <int WW>
__global__ __launch_bounds__(kBlock) void k_layer_scatter(Solo S) {
  __shared__ uint64_t s_px[kLayerMaxRot][WW], s_pz[kLayerMaxRot][WW];
  __shared__ uint32_t s_cnt[kLAggMax];
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
  const uint32_t M = op.fail_test ? 0u : d.M;
  const uint32_t bits = layer_bits(d.M, d.lboost, b.lmaxbits, b.lshift);
  const uint32_t P = 1u << bits, slots = b.lslots >> bits, L = b.lslots;
  const bool agg = P <= (uint32_t)kLAggMax;
  const View v = view_of(b, d);
  bool over = op.fail_test != 0 && blockIdx.x == 0 && threadIdx.x == 0;
  const uint32_t round = kBlock * kLTile;
  const uint32_t rounds = (M + round - 1) / round;
  for (uint32_t t = blockIdx.x; t < rounds; t += gridDim.x) {
    if (agg) {
      __syncthreads();
      for (uint32_t k = threadIdx.x; k < P; k += kBlock) s_cnt[k] = 0;
    }
    __syncthreads();                       // rotations loaded, counts zero
    uint64_t x[kLTile][WW], z[kLTile][WW], a[kLTile];
    double c[kLTile];
    uint32_t bk[kLTile], rank[kLTile], h32[kLTile];
    bool has[kLTile];
#pragma unroll
    for (int k = 0; k < kLTile; ++k) {
      const uint32_t i = t * round + k * kBlock + threadIdx.x;
      has[k] = i < M && v.al[i];
      if (!has[k]) continue;
#pragma unroll
      for (int w = 0; w < WW; ++w) {
        x[k][w] = v.X[(size_t)w * v.cap + i];
        z[k][w] = v.Z[(size_t)w * v.cap + i];
      }
      c[k] = v.getc(i);
      const uint64_t h = layer_key<WW>(x[k], z[k], r, s_px, s_pz, &a[k]);
      h32[k] = (uint32_t)h;
      bk[k] = bits ? (uint32_t)(h >> (64 - bits)) : 0u;
      rank[k] = agg ? atomicAdd(&s_cnt[bk[k]], 1u) : atomicAdd(&b.lcount[bk[k]], 1u);
    }
    if (agg) {
      __syncthreads();
      for (uint32_t k = threadIdx.x; k < P; k += kBlock) {
        const uint32_t n = s_cnt[k];
        s_cnt[k] = n ? atomicAdd(&b.lcount[k], n) : 0u;   // this round's first slot
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kLTile; ++k) {
      if (!has[k]) continue;
      const uint32_t rk = agg ? s_cnt[bk[k]] + rank[k] : rank[k];
      if (rk >= slots) { over = true; continue; }
      const size_t pos = (size_t)bk[k] * slots + rk;
#pragma unroll
      for (int w = 0; w < WW; ++w) {
        b.lstx[(size_t)w * L + pos] = x[k][w];
        b.lstz[(size_t)w * L + pos] = z[k][w];
      }
      b.lstc[pos] = c[k];
      b.lsta[pos] = a[k];
      b.lsth[pos] = h32[k];
    }
  }
  if (over) atomicOr(&d.lfail, 1u);        // a bucket's staging slots overflowed
}

template <int WW>
__device__ __forceinline__ uint32_t lds_hash(const uint64_t* x, const uint64_t* z) {
  uint64_t h = x[0] * 0x9e3779b97f4a7c15ull ^ z[0] * 0xc2b2ae3d27d4eb4full;
  if (WW > 1) h = (h ^ (h >> 29)) * 0xbf58476d1ce4e5b9ull ^ x[WW - 1] * 0x94d049bb133111ebull ^
                  z[WW - 1] * 0xff51afd7ed558ccdull;
  return (uint32_t)((h ^ (h >> 31)) >> 32);
}


// Exclusive scan of one value per thread over a block of NW waves; *total
// = block sum.  s_tmp needs NW + 1 entries.  Contains __syncthreads.
template <int NW>
__device__ __forceinline__ uint32_t block_scan_n(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
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

__device__ __forceinline__ uint16_t lds_load16(const uint16_t* p) {
  return *reinterpret_cast<const volatile uint16_t*>(p);
}

// local index of the string (x, z) in a wave's LDS table (its strings at
// base + local index), or -1
template <int WW, int CAP>
__device__ __forceinline__ int lds_find(const uint16_t* tab, int HS, const uint64_t (*sx)[CAP],
                                        const uint64_t (*sz)[CAP], uint32_t base,
                                        const uint64_t* x, const uint64_t* z) {
  uint32_t sl = lds_hash<WW>(x, z) & (HS - 1);
  for (int probe = 0; probe < HS; ++probe) {
    const uint32_t e = lds_load16(&tab[sl]);
    if (e == 0) return -1;
    const int j = (int)e - 1;
    bool eq = true;
#pragma unroll
    for (int w = 0; w < WW; ++w) eq = eq && sx[w][base + j] == x[w] && sz[w][base + j] == z[w];
    if (eq) return j;
    sl = (sl + 1) & (HS - 1);
  }
  return -1;
}

// publishes index j (its string already written) under (x, z)
template <int WW>
__device__ __forceinline__ void lds_insert(uint16_t* tab, int HS, const uint64_t* x,
                                           const uint64_t* z, int j) {
  uint32_t sl = lds_hash<WW>(x, z) & (HS - 1);
  for (int probe = 0; probe < HS; ++probe) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(&tab[sl]);
    uint32_t* wp = reinterpret_cast<uint32_t*>(a & ~uintptr_t(3));
    const uint32_t shift = (a & 2) ? 16u : 0u;
    uint32_t old = *reinterpret_cast<volatile uint32_t*>(wp);
    for (;;) {
      if ((old >> shift) & 0xFFFFu) break;                        // slot taken
      const uint32_t got = atomicCAS(wp, old, old | ((uint32_t)(j + 1) << shift));
      if (got == old) return;
      old = got;
    }
    sl = (sl + 1) & (HS - 1);
  }
}

template <int WW>
__device__ __forceinline__ bool layer_heavy(const uint64_t* x, const uint64_t* z, int wmax) {
  if (wmax < 0) return false;
  int n = 0;
#pragma unroll
  for (int w = 0; w < WW; ++w) n += __popcll(x[w] | z[w]);
  return n > wmax;
}

// The bucket's survivors (every LDS slot whose string lives; unused slots
// read as dropped) to the other half of the store (one atomic per block and
// bucket), with gate-table entries when the op asks for them.
template <int WW, int NB, int CAP>
__device__ __forceinline__ void emit_survivors(const InstBuf& b, InstDyn& d, const Op& op,
                                               const uint64_t (*sx)[CAP], const uint64_t (*sz)[CAP],
                                               const double* sc, const uint16_t* life,
                                               uint32_t* s_tmp,
                                               uint32_t* s_base, uint32_t* out, uint32_t* next) {
  constexpr int NW = NB / 64;
  auto alive = [&](uint32_t j) { return (life[j] & 0xFFu) == kAlive; };   // unused slots: died 0
  uint32_t mine = 0;
  for (uint32_t j = threadIdx.x; j < (uint32_t)CAP; j += NB) mine += alive(j) ? 1u : 0u;
  uint32_t total;
  uint32_t off = block_scan_n<NW>(mine, s_tmp, &total);
  if (threadIdx.x == 0) *s_base = total ? atomicAdd(&d.nuniq, total) : 0u;
  __syncthreads();
  const uint32_t ob = *s_base, cap = b.cap, ho = d.half ^ 1u;
  const bool has_next = op.next_gate != kNone32, gtab = op.gtab != 0;
  *out += mine;
  for (uint32_t j = threadIdx.x; j < (uint32_t)CAP; j += NB) {
    if (!alive(j)) continue;
    const uint32_t pos = ob + off++;
    uint64_t x[kMaxW] = {}, z[kMaxW] = {};
#pragma unroll
    for (int w = 0; w < WW; ++w) { x[w] = sx[w][j]; z[w] = sz[w][j]; }
    uint64_t nx[kMaxW] = {}, nz[kMaxW] = {};
#pragma unroll
    for (int w = 0; w < WW; ++w) { nx[w] = op.nx[w]; nz[w] = op.nz[w]; }
    if (has_next && anticommutes(x, z, nx, nz, WW)) ++*next;
    if (pos >= cap) { atomicOr(&d.status, ST_OVERFLOW); continue; }
#pragma unroll
    for (int w = 0; w < WW; ++w) {
      b.x[ho][(size_t)w * cap + pos] = x[w];
      b.z[ho][(size_t)w * cap + pos] = z[w];
    }
    if (b.f32)
      static_cast<float*>(b.c[ho])[pos] = (float)sc[j];
    else
      static_cast<double*>(b.c[ho])[pos] = sc[j];
    b.alive[ho][0][pos] = 1;
    if (gtab) gt_insert(b.gtab, b.hg_bits, d.gen + 1, pos, hash_key(x, z, WW, 0));
  }
}

// Last block, one thread: folds the sums; on success the op's counts, the
// other half becomes current and pc passes the op's fallback copies.
__device__ __forceinline__ void layer_finish(const InstBuf& b, InstDyn& d, const Op& op, int ns) {
  uint64_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int sh = 0; sh < kAccShards; ++sh)
    for (int k = 0; k < ns; ++k)
      t[k] += atomicExch((unsigned long long*)&b.accs[sh * kLineU64 + 1 + k], 0ull);
  const uint32_t out = ld_agent(&d.nuniq);
  d.nuniq = 0;
  if (ld_agent(&d.status) & ST_OVERFLOW) {  // the survivors did not fit: grow, run again
    d.lneed = out;
    d.lfail = 0;
    d.failed_pc = d.pc;
    return;
  }
  const uint32_t why = ld_agent(&d.lfail);
  if (why) {                                // a bucket did not fit: the host decides
    d.lfail = 0;
    d.lwhy = why;                           // 1 staging slots, 2 LDS
    d.lfails += 1;
    d.status |= ST_LAYER;
    d.failed_pc = d.pc;
    return;
  }
  d.lops += 1;
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
  d.half ^= 1u;
  d.parity = 0;
  if (op.gtab) d.gen += 1;
  d.count_for = op.next_gate;
  d.pc += 1 + op.skip;
}

// Liveness of a bucket's string: born (the rotation before which it first
// exists: 0, or g + 1 for a child of rotation g) and died (the rotation
// after which it was dropped, kAlive while it lives), packed in 16 bits so
// that one store changes both.  A string is live before rotation g iff
// born <= g <= died.  Rotation g writes `died = g` for strings it drops and
// (g + 1, kAlive) for a dropped string it makes again; a string's own thread
// never reads these mid-rotation values as "live before" wrongly: died = g
// still reads live before g, and born = g + 1 reads not live.
__device__ __forceinline__ bool live_before(uint32_t life, uint32_t g) {
  return (life >> 8) <= g && (life & 0xFFu) >= g;
}
__device__ __forceinline__ uint16_t life_of(uint32_t born, uint32_t died) {
  return (uint16_t)((born << 8) | died);
}

// 2. One block per bucket (grid-stride over buckets): the bucket's strings
// into LDS (one hash table), then the rotations some of them anticommute
// with (and the first one if the op re-checks every string there), each
// over all the bucket's strings with a block barrier after it; then the
// survivors go to the other half.  The last block folds the sums and
// advances the program (or reports the failure).  Live counts before each
// rotation follow from the strings entering and the births and drops of
// the rotations before it.
template <int WW, int NB>
__global__ __launch_bounds__(NB) void k_layer_apply(Solo S) {
  constexpr int kLWaves = NB / 64;
  constexpr int CAP = LayerCap<WW>::n, HS = 2 * CAP;
  constexpr int NS = 7;                    // sums, see below
  __shared__ uint64_t s_x[WW][CAP], s_z[WW][CAP];
  __shared__ double s_c[CAP];
  __shared__ uint16_t s_life[CAP];
  __shared__ uint16_t s_hash[HS];          // index + 1, 0 = empty
  __shared__ uint64_t s_px[kLayerMaxRot][WW], s_pz[kLayerMaxRot][WW];
  __shared__ double s_cs[kLayerMaxRot], s_sn[kLayerMaxRot];
  __shared__ unsigned long long s_pat;     // rotations some string anticommutes with
  __shared__ uint32_t s_inc[3], s_n0, s_fail, s_flag, s_tmp[kLWaves + 1], s_base;
  __shared__ uint64_t s_red[kLWaves][NS];
  const InstBuf& b = S.b;
  InstDyn& d = *S.d;
  if (d.pc != S.k) return;                 // uniform: pc changes only in the last block
  const Op& op = b.prog[S.k];
  const uint32_t r = op.nrot;
  for (uint32_t g = threadIdx.x; g < r; g += NB) {
#pragma unroll
    for (int w = 0; w < WW; ++w) {
      s_px[g][w] = rot_word(op.table, g * kLayerRec + w);
      s_pz[g][w] = rot_word(op.table, g * kLayerRec + kMaxW + w);
    }
    s_cs[g] = op.table[g * kLayerRec + 2 * kMaxW];
    s_sn[g] = op.table[g * kLayerRec + 2 * kMaxW + 1];
  }
  const uint32_t M = d.M;
  const uint32_t bits = layer_bits(M, d.lboost, b.lmaxbits, b.lshift);
  const uint32_t P = 1u << bits, slots = b.lslots >> bits;
  const bool failed = ld_agent(&d.lfail) != 0;   // the scatter launch has ended
  const double eps = op.eps;
  const int wmax = op.wmax;
  const bool full = op.full_check != 0;
  const bool f32 = b.f32 != 0;
  // per-thread sums: live before each rotation (as r * entering + weighted
  // births - drops), anticommuting, survivors, survivors anticommuting with
  // the next gate, children, strings held at the end, strings entering
  int64_t s_lw = 0;
  uint32_t s_an = 0, s_out = 0, s_nx = 0, s_ch = 0, s_held = 0, s_in = 0;
  bool bad = false;

  for (uint32_t bk = blockIdx.x; bk < P; bk += gridDim.x) {
    __syncthreads();                       // the previous bucket's LDS is free
    if (threadIdx.x == 0) {
      const uint32_t cnt = b.lcount[bk];
      b.lcount[bk] = 0;                    // zero for the next layer op
      s_n0 = cnt < slots ? cnt : slots;
      s_fail = s_n0 > (uint32_t)CAP ? 1u : 0u;
      s_inc[0] = s_inc[1] = s_inc[2] = 0;
      s_pat = 0;
    }
    for (int t = threadIdx.x; t < HS / 2; t += NB) reinterpret_cast<uint32_t*>(s_hash)[t] = 0;
    for (int t = threadIdx.x; t < CAP; t += NB) s_life[t] = life_of(0xFF, 0);   // unused: never live
    __syncthreads();
    if (failed || s_fail) { bad = bad || s_fail; continue; }   // uniform
    const uint32_t n0 = s_n0;
    {
      const size_t base = (size_t)bk * slots, L = b.lslots;
      if (threadIdx.x == 0) s_in += n0;
      s_lw += threadIdx.x == 0 ? (int64_t)r * n0 : 0;
      uint64_t pat = 0;
      for (uint32_t j = threadIdx.x; j < n0; j += NB) {
        uint64_t x[WW], z[WW];
#pragma unroll
        for (int q = 0; q < WW; ++q) {
          x[q] = b.lstx[(size_t)q * L + base + j];
          z[q] = b.lstz[(size_t)q * L + base + j];
          s_x[q][j] = x[q];
          s_z[q][j] = z[q];
        }
        s_c[j] = b.lstc[base + j];
        pat |= b.lsta[base + j];
        s_life[j] = life_of(0, kAlive);
        __threadfence_block();
        lds_insert<WW>(s_hash, HS, x, z, (int)j);
      }
      for (int o = 32; o > 0; o >>= 1) pat |= __shfl_xor(pat, o, 64);
      if ((threadIdx.x & 63) == 0 && pat) atomicOr(&s_pat, (unsigned long long)pat);
    }
    __syncthreads();
    uint64_t todo = s_pat | (full ? 1ull : 0ull);
    uint32_t ng = n0, q = 0;               // strings before the rotation; rotations run
    while (todo) {
      const uint32_t g = (uint32_t)__builtin_ctzll(todo);
      todo &= todo - 1;
      if (threadIdx.x == 0) s_inc[(q + 1) % 3] = 0;
      const bool chk = g == 0 && full;
      const int wt = (int)(r - 1 - g);     // rotations after g (live-count weight)
      int born_here = 0, died_here = 0;
      uint64_t px[WW], pz[WW];             // the rotation, in registers
#pragma unroll
      for (int w = 0; w < WW; ++w) { px[w] = s_px[g][w]; pz[w] = s_pz[g][w]; }
      const double cs = s_cs[g], sn = s_sn[g];
      for (uint32_t j = threadIdx.x; j < ng; j += NB) {
        // key, stamp and coefficient in one round trip (a coefficient read
        // here is used only by a string that leads its pair or has none,
        // and no other thread writes those)
        uint64_t qx[WW], qz[WW];
#pragma unroll
        for (int w = 0; w < WW; ++w) { qx[w] = s_x[w][j]; qz[w] = s_z[w][j]; }
        const uint32_t life = s_life[j];
        const double cq = s_c[j];
        uint32_t par = 0;
#pragma unroll
        for (int w = 0; w < WW; ++w) par += __popcll((qx[w] & pz[w]) ^ (qz[w] & px[w]));
        const bool anti = par & 1u;
        if (!anti && !chk) continue;       // untouched (and live or not, unchanged)
        if (!live_before(life, g)) continue;
        if (!anti) {                       // the sub-layer's first rotation checks all
          if (!(fabs(cq) >= eps && !layer_heavy<WW>(qx, qz, wmax))) {
            s_life[j] = life_of(life >> 8, g);
            ++died_here;
          }
          continue;
        }
        ++s_an;
        uint64_t rx[WW], rz[WW];
#pragma unroll
        for (int w = 0; w < WW; ++w) { rx[w] = qx[w] ^ px[w]; rz[w] = qz[w] ^ pz[w]; }
        const int pk = lds_find<WW>(s_hash, HS, s_x, s_z, 0, rx, rz);
        const uint32_t p = (uint32_t)pk;
        uint32_t plife = 0;
        double cp = 0.0;
        if (pk >= 0) { plife = s_life[p]; cp = s_c[p]; }
        const bool plive = pk >= 0 && p < ng && live_before(plife, g);
        if (plive && p < j) continue;      // the partner's thread leads
        const int sig = product_sign(px, pz, qx, qz, rx, rz, WW);   // i P Q = sig R
        if (plive) {                       // Q and R = PQ live: a rotation of the pair
          double nq, nr;
          rotate_pair(f32, cs, sn, sig, cq, cp, &nq, &nr);
          s_c[j] = nq;
          s_c[p] = nr;
          if (!(fabs(nq) >= eps && !(chk && layer_heavy<WW>(qx, qz, wmax)))) {
            s_life[j] = life_of(life >> 8, g);
            ++died_here;
          }
          if (!(fabs(nr) >= eps && !(chk && layer_heavy<WW>(rx, rz, wmax)))) {
            s_life[p] = life_of(plife >> 8, g);
            ++died_here;
          }
        } else {
          double nq, child;
          rotate_single(f32, cs, sn, sig, cq, &nq, &child);
          s_c[j] = nq;
          if (!(fabs(nq) >= eps && !(chk && layer_heavy<WW>(qx, qz, wmax)))) {
            s_life[j] = life_of(life >> 8, g);
            ++died_here;
          }
          if (fabs(child) >= eps && !layer_heavy<WW>(rx, rz, wmax)) {
            ++s_ch;
            if (pk >= 0) {                 // a dropped string comes back in its slot
              s_c[p] = child;
              s_life[p] = life_of(g + 1, kAlive);
              ++born_here;
            } else {
              const uint32_t k = ng + atomicAdd(&s_inc[q % 3], 1u);
              if (k >= (uint32_t)CAP) {
                s_fail = 1;
              } else {
#pragma unroll
                for (int w = 0; w < WW; ++w) { s_x[w][k] = rx[w]; s_z[w][k] = rz[w]; }
                s_c[k] = child;
                s_life[k] = life_of(g + 1, kAlive);
                ++born_here;
                __threadfence_block();
                lds_insert<WW>(s_hash, HS, rx, rz, (int)k);
              }
            }
          }
        }
      }
      s_lw += (int64_t)wt * (born_here - died_here);
      __syncthreads();
      const uint32_t add = s_inc[q % 3];
      ng = ng + add < (uint32_t)CAP ? ng + add : (uint32_t)CAP;
      ++q;
    }
    if (threadIdx.x == 0) s_held += ng;
    if (s_fail) { bad = true; continue; }  // uniform: read after the last barrier
    emit_survivors<WW, NB>(b, d, op, s_x, s_z, s_c, s_life, s_tmp, &s_base, &s_out, &s_nx);
  }
  // block sums -> this block's shard line, entries 1..NS
  {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t v[NS] = {(uint64_t)s_lw, s_an, s_out, s_nx, s_ch, s_held, s_in};
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      uint64_t t = v[k];
      for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
      if (lane == 0) s_red[wid][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < NS) {
      uint64_t t = 0;
      for (int w = 0; w < kLWaves; ++w) t += s_red[w][threadIdx.x];
      if (t)
        atomicAdd((unsigned long long*)&b.accs[(blockIdx.x % kAccShards) * kLineU64 + 1 + threadIdx.x],
                  (unsigned long long)t);
    }
    if (threadIdx.x == 0 && bad) atomicOr(&d.lfail, 2u);   // a bucket overflowed the LDS
  }
  if (!last_block(S.sync, &s_flag, gridDim.x, true)) return;
  if (threadIdx.x == 0) layer_finish(b, d, op, NS);
}

}  // namespace pp
