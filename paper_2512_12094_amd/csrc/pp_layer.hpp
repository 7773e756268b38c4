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

// strings per thread per scatter round: one gives the most rounds (blocks)
// and the shortest chain per block (measured faster than 2, 4 or 8)
constexpr int kLTile = 1;
constexpr int kLAggMax = 2048;             // buckets counted in LDS before the global add

// 1. Every live string of the current half to its bucket's staging slots,
// with its pattern and key hash.  A round of kBlock * kLTile strings counts
// its strings per bucket in LDS and reserves each bucket's slots with one
// global add (buckets up to kLAggMax; beyond, one global add per string).
template <int WW>
struct ScatterSh {
  uint64_t px[kLayerMaxRot][WW], pz[kLayerMaxRot][WW];
  uint32_t cnt[kLAggMax];
};

// The op's rotation strings into LDS (the caller synchronises before use).
template <int WW, int NT>
__device__ __forceinline__ void load_rot_strings(const Op& op, uint64_t (*px)[WW],
                                                 uint64_t (*pz)[WW]) {
  for (uint32_t g = threadIdx.x; g < op.nrot; g += NT) {
#pragma unroll
    for (int w = 0; w < WW; ++w) {
      px[g][w] = rot_word(op.table, g * kLayerRec + w);
      pz[g][w] = rot_word(op.table, g * kLayerRec + kMaxW + w);
    }
  }
}

// Round t (kBlock * kLTile entries from t * kBlock * kLTile) of one
// instance's scatter; M = the entries scattered (0 for a forced failure),
// bits = the op's bucket bits.  Returns true if a bucket's staging slots
// overflowed.  Every thread of the block calls it (barriers inside).
template <int WW>
__device__ __forceinline__ bool scatter_round(const InstBuf& b, const InstDyn& d, const Op& op,
                                              uint32_t M, uint32_t bits, uint32_t t,
                                              ScatterSh<WW>& sh) {
  const uint32_t r = op.nrot;
  const uint32_t P = 1u << bits, slots = b.lslots >> bits, L = b.lslots;
  const bool agg = P <= (uint32_t)kLAggMax;
  const View v = view_of(b, d);
  const uint32_t round = kBlock * kLTile;
  bool over = false;
  if (agg) {
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < P; k += kBlock) sh.cnt[k] = 0;
  }
  __syncthreads();                         // rotations loaded, counts zero
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
    const uint64_t h = layer_key<WW>(x[k], z[k], r, sh.px, sh.pz, &a[k]);
    h32[k] = (uint32_t)h;
    bk[k] = bits ? (uint32_t)(h >> (64 - bits)) : 0u;
    rank[k] = agg ? atomicAdd(&sh.cnt[bk[k]], 1u) : atomicAdd(&b.lcount[bk[k]], 1u);
  }
  if (agg) {
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < P; k += kBlock) {
      const uint32_t n = sh.cnt[k];
      sh.cnt[k] = n ? atomicAdd(&b.lcount[k], n) : 0u;   // this round's first slot
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kLTile; ++k) {
    if (!has[k]) continue;
    const uint32_t rk = agg ? sh.cnt[bk[k]] + rank[k] : rank[k];
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
  return over;
}

template <int WW>
__global__ __launch_bounds__(kBlock) void k_layer_scatter(Solo S) {
  __shared__ ScatterSh<WW> sh;
  const InstBuf& b = S.b;
  InstDyn& d = *S.d;
  if (d.pc != S.k) return;                 // an earlier op did not complete
  const Op& op = b.prog[S.k];
  load_rot_strings<WW, kBlock>(op, sh.px, sh.pz);
  const uint32_t M = op.fail_test ? 0u : d.M;
  const uint32_t bits = layer_bits(d.M, d.lboost, b.lmaxbits, b.lshift);
  bool over = op.fail_test != 0 && blockIdx.x == 0 && threadIdx.x == 0;
  const uint32_t rounds = (M + kBlock * kLTile - 1) / (kBlock * kLTile);
  for (uint32_t t = blockIdx.x; t < rounds; t += gridDim.x)
    over = scatter_round<WW>(b, d, op, M, bits, t, sh) || over;
  if (over) atomicOr(&d.lfail, 1u);        // a bucket's staging slots overflowed
}

// An instance of a batch takes the layer op when it stands at one with
// staging, its key width matches the kernel's and nothing stopped it.
template <int WW>
__device__ __forceinline__ bool layer_served(const InstBuf& b, const InstDyn& d) {
  const Op* op = cur_op(b, d);
  return op && op->type == OP_LAYER && b.W == WW && b.lcount && !b.nolayer &&
         !(d.status & ST_OVERFLOW);
}

// Batched form, step 1: every instance that stands at a layer op scatters;
// rounds of all instances are dealt out to the blocks.  Block 0 records in
// each instance whether this step serves it (d.lserved, read by step 2).
template <int WW>
__global__ __launch_bounds__(kBlock) void k_layer_scatter_multi(Ctx C) {
  __shared__ uint32_t s_pref[kMaxInst];
  __shared__ uint32_t s_tmp[kWaves + 1];
  __shared__ ScatterSh<WW> sh;
  const int ninst = *C.ninst;
  const uint32_t round = kBlock * kLTile;
  const uint32_t total = plan_tiles(ninst, [&](int i) -> uint32_t {
    const InstBuf& b = *C.bufs[i];
    const InstDyn& d = *C.dyns[i];
    if (!layer_served<WW>(b, d)) return 0u;
    const uint32_t M = b.prog[d.pc].fail_test ? 0u : d.M;
    return M ? (M + round - 1) / round : 1u;   // a forced failure takes one empty round
  }, s_pref, s_tmp);
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < ninst; i += kBlock)
      if (C.bufs[i]->W == WW) C.dyns[i]->lserved = layer_served<WW>(*C.bufs[i], *C.dyns[i]) ? 1u : 0u;
  int cur = -1;
  for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_inst(s_pref, ninst, t);
    const InstBuf& b = *C.bufs[i];
    InstDyn& d = *C.dyns[i];
    const Op& op = b.prog[d.pc];
    if (i != cur) {
      __syncthreads();                     // the last round's rotations are read
      load_rot_strings<WW, kBlock>(op, sh.px, sh.pz);
      cur = i;
    }
    const uint32_t M = op.fail_test ? 0u : d.M;
    const uint32_t bits = layer_bits(d.M, d.lboost, b.lmaxbits, b.lshift);
    const bool over = scatter_round<WW>(b, d, op, M, bits, t - s_pref[i], sh) ||
                      (op.fail_test != 0 && t == s_pref[i] && threadIdx.x == 0);
    if (over) atomicOr(&d.lfail, 1u);      // a bucket's staging slots overflowed
  }
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
__device__ __forceinline__ void layer_finish(const InstBuf& b, InstDyn& d, const Op& op, int ns,
                                             bool batched) {
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
  if (why) {                                // a bucket did not fit
    d.lfail = 0;
    d.lwhy = why;                           // 1 staging slots, 2 LDS
    d.lfails += 1;
    if (batched) {                          // the batched form runs the gate copies
      d.lfb += 1;
      d.pc += 1;
      return;
    }
    d.status |= ST_LAYER;                   // the one-instance path: the host decides
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

// 2. One block per bucket: the bucket's strings into LDS (one hash table),
// then the rotations some of them anticommute with (and the first one if
// the op re-checks every string there), each over all the bucket's strings
// with a block barrier after it; then the survivors go to the other half.
// Live counts before each rotation follow from the strings entering and the
// births and drops of the rotations before it.
template <int WW, int NB>
struct ApplySh {
  static constexpr int CAP = LayerCap<WW>::n, HS = 2 * CAP, NW = NB / 64, NS = 7;
  uint64_t x[WW][CAP], z[WW][CAP];
  double c[CAP];
  uint16_t life[CAP];
  uint16_t hash[HS];                       // index + 1, 0 = empty
  uint64_t px[kLayerMaxRot][WW], pz[kLayerMaxRot][WW];
  double cs[kLayerMaxRot], sn[kLayerMaxRot];
  unsigned long long pat;                  // rotations some string anticommutes with
  uint32_t inc[3], n0, fail, flag, tmp[NW + 1], base;
  uint64_t red[NW][NS];
};

// Per-thread sums of one instance: live before each rotation (as r *
// entering + weighted births - drops), anticommuting, survivors, survivors
// anticommuting with the next gate, children, strings held at the end,
// strings entering; bad: a bucket did not fit the LDS.
struct LayerSums {
  int64_t lw = 0;
  uint32_t an = 0, out = 0, nx = 0, ch = 0, held = 0, in = 0;
  bool bad = false;
};

template <int WW, int NB>
__device__ __forceinline__ void load_rotations(const Op& op, ApplySh<WW, NB>& sh) {
  load_rot_strings<WW, NB>(op, sh.px, sh.pz);
  for (uint32_t g = threadIdx.x; g < op.nrot; g += NB) {
    sh.cs[g] = op.table[g * kLayerRec + 2 * kMaxW];
    sh.sn[g] = op.table[g * kLayerRec + 2 * kMaxW + 1];
  }
}

// Bucket bk of one instance (bits: the op's bucket bits).  Every thread of
// the block calls it; it starts with a barrier (the LDS of the previous
// bucket, and the rotations, are then free and loaded).
template <int WW, int NB>
__device__ __forceinline__ void apply_bucket(const InstBuf& b, InstDyn& d, const Op& op,
                                             uint32_t bits, uint32_t bk, ApplySh<WW, NB>& sh,
                                             LayerSums& sum) {
  constexpr int CAP = ApplySh<WW, NB>::CAP, HS = ApplySh<WW, NB>::HS;
  const uint32_t r = op.nrot;
  const uint32_t slots = b.lslots >> bits;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t cnt = b.lcount[bk];
    b.lcount[bk] = 0;                      // zero for the next layer op
    sh.n0 = cnt < slots ? cnt : slots;
    sh.fail = sh.n0 > (uint32_t)CAP ? 1u : 0u;
    sh.inc[0] = sh.inc[1] = sh.inc[2] = 0;
    sh.pat = 0;
  }
  for (int t = threadIdx.x; t < HS / 2; t += NB) reinterpret_cast<uint32_t*>(sh.hash)[t] = 0;
  for (int t = threadIdx.x; t < CAP; t += NB) sh.life[t] = life_of(0xFF, 0);   // unused: never live
  __syncthreads();
  if (sh.fail) { sum.bad = true; return; }   // uniform
  const uint32_t n0 = sh.n0;
  {
    const size_t base = (size_t)bk * slots, L = b.lslots;
    if (threadIdx.x == 0) sum.in += n0;
    sum.lw += threadIdx.x == 0 ? (int64_t)r * n0 : 0;
    uint64_t pat = 0;
    for (uint32_t j = threadIdx.x; j < n0; j += NB) {
      uint64_t x[WW], z[WW];
#pragma unroll
      for (int q = 0; q < WW; ++q) {
        x[q] = b.lstx[(size_t)q * L + base + j];
        z[q] = b.lstz[(size_t)q * L + base + j];
        sh.x[q][j] = x[q];
        sh.z[q][j] = z[q];
      }
      sh.c[j] = b.lstc[base + j];
      pat |= b.lsta[base + j];
      sh.life[j] = life_of(0, kAlive);
      __threadfence_block();
      lds_insert<WW>(sh.hash, HS, x, z, (int)j);
    }
    for (int o = 32; o > 0; o >>= 1) pat |= __shfl_xor(pat, o, 64);
    if ((threadIdx.x & 63) == 0 && pat) atomicOr(&sh.pat, (unsigned long long)pat);
  }
  __syncthreads();
  const double eps = op.eps;
  const int wmax = op.wmax;
  const bool full = op.full_check != 0;
  const bool f32 = b.f32 != 0;
  uint64_t todo = sh.pat | (full ? 1ull : 0ull);
  uint32_t ng = n0, q = 0;                 // strings before the rotation; rotations run
  while (todo) {
    const uint32_t g = (uint32_t)__builtin_ctzll(todo);
    todo &= todo - 1;
    if (threadIdx.x == 0) sh.inc[(q + 1) % 3] = 0;
    const bool chk = g == 0 && full;
    const int wt = (int)(r - 1 - g);       // rotations after g (live-count weight)
    int born_here = 0, died_here = 0;
    uint64_t px[WW], pz[WW];               // the rotation, in registers
#pragma unroll
    for (int w = 0; w < WW; ++w) { px[w] = sh.px[g][w]; pz[w] = sh.pz[g][w]; }
    const double cs = sh.cs[g], sn = sh.sn[g];
    for (uint32_t j = threadIdx.x; j < ng; j += NB) {
      // key, stamp and coefficient in one round trip (a coefficient read
      // here is used only by a string that leads its pair or has none, and
      // no other thread writes those)
      uint64_t qx[WW], qz[WW];
#pragma unroll
      for (int w = 0; w < WW; ++w) { qx[w] = sh.x[w][j]; qz[w] = sh.z[w][j]; }
      const uint32_t life = sh.life[j];
      const double cq = sh.c[j];
      uint32_t par = 0;
#pragma unroll
      for (int w = 0; w < WW; ++w) par += __popcll((qx[w] & pz[w]) ^ (qz[w] & px[w]));
      const bool anti = par & 1u;
      if (!anti && !chk) continue;         // untouched (and live or not, unchanged)
      if (!live_before(life, g)) continue;
      if (!anti) {                         // the sub-layer's first rotation checks all
        if (!(fabs(cq) >= eps && !layer_heavy<WW>(qx, qz, wmax))) {
          sh.life[j] = life_of(life >> 8, g);
          ++died_here;
        }
        continue;
      }
      ++sum.an;
      uint64_t rx[WW], rz[WW];
#pragma unroll
      for (int w = 0; w < WW; ++w) { rx[w] = qx[w] ^ px[w]; rz[w] = qz[w] ^ pz[w]; }
      const int pk = lds_find<WW>(sh.hash, HS, sh.x, sh.z, 0, rx, rz);
      const uint32_t p = (uint32_t)pk;
      uint32_t plife = 0;
      double cp = 0.0;
      if (pk >= 0) { plife = sh.life[p]; cp = sh.c[p]; }
      const bool plive = pk >= 0 && p < ng && live_before(plife, g);
      if (plive && p < j) continue;        // the partner's thread leads
      const int sig = product_sign(px, pz, qx, qz, rx, rz, WW);   // i P Q = sig R
      if (plive) {                         // Q and R = PQ live: a rotation of the pair
        double nq, nr;
        rotate_pair(f32, cs, sn, sig, cq, cp, &nq, &nr);
        sh.c[j] = nq;
        sh.c[p] = nr;
        if (!(fabs(nq) >= eps && !(chk && layer_heavy<WW>(qx, qz, wmax)))) {
          sh.life[j] = life_of(life >> 8, g);
          ++died_here;
        }
        if (!(fabs(nr) >= eps && !(chk && layer_heavy<WW>(rx, rz, wmax)))) {
          sh.life[p] = life_of(plife >> 8, g);
          ++died_here;
        }
      } else {
        double nq, child;
        rotate_single(f32, cs, sn, sig, cq, &nq, &child);
        sh.c[j] = nq;
        if (!(fabs(nq) >= eps && !(chk && layer_heavy<WW>(qx, qz, wmax)))) {
          sh.life[j] = life_of(life >> 8, g);
          ++died_here;
        }
        if (fabs(child) >= eps && !layer_heavy<WW>(rx, rz, wmax)) {
          ++sum.ch;
          if (pk >= 0) {                   // a dropped string comes back in its slot
            sh.c[p] = child;
            sh.life[p] = life_of(g + 1, kAlive);
            ++born_here;
          } else {
            const uint32_t k = ng + atomicAdd(&sh.inc[q % 3], 1u);
            if (k >= (uint32_t)CAP) {
              sh.fail = 1;
            } else {
#pragma unroll
              for (int w = 0; w < WW; ++w) { sh.x[w][k] = rx[w]; sh.z[w][k] = rz[w]; }
              sh.c[k] = child;
              sh.life[k] = life_of(g + 1, kAlive);
              ++born_here;
              __threadfence_block();
              lds_insert<WW>(sh.hash, HS, rx, rz, (int)k);
            }
          }
        }
      }
    }
    sum.lw += (int64_t)wt * (born_here - died_here);
    __syncthreads();
    const uint32_t add = sh.inc[q % 3];
    ng = ng + add < (uint32_t)CAP ? ng + add : (uint32_t)CAP;
    ++q;
  }
  if (threadIdx.x == 0) sum.held += ng;
  if (sh.fail) { sum.bad = true; return; }  // uniform: read after the last barrier
  emit_survivors<WW, NB>(b, d, op, sh.x, sh.z, sh.c, sh.life, sh.tmp, &sh.base, &sum.out, &sum.nx);
}

// The block's sums of one instance to its shard line (entries 1..NS) and
// its LDS overflow flag; resets the sums.  Every thread calls it.
template <int WW, int NB>
__device__ __forceinline__ void flush_sums(const InstBuf& b, InstDyn& d, ApplySh<WW, NB>& sh,
                                           LayerSums& sum) {
  constexpr int NS = ApplySh<WW, NB>::NS, NW = ApplySh<WW, NB>::NW;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t v[NS] = {(uint64_t)sum.lw, sum.an, sum.out, sum.nx, sum.ch, sum.held, sum.in};
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    uint64_t t = v[k];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) sh.red[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < NS) {
    uint64_t t = 0;
    for (int w = 0; w < NW; ++w) t += sh.red[w][threadIdx.x];
    if (t)
      atomicAdd((unsigned long long*)&b.accs[(blockIdx.x % kAccShards) * kLineU64 + 1 + threadIdx.x],
                (unsigned long long)t);
  }
  if (threadIdx.x == 0 && sum.bad) atomicOr(&d.lfail, 2u);   // a bucket overflowed the LDS
  sum = LayerSums();
}

template <int WW, int NB>
__global__ __launch_bounds__(NB) void k_layer_apply(Solo S) {
  __shared__ ApplySh<WW, NB> sh;
  const InstBuf& b = S.b;
  InstDyn& d = *S.d;
  if (d.pc != S.k) return;                 // uniform: pc changes only in the last block
  const Op& op = b.prog[S.k];
  load_rotations<WW, NB>(op, sh);
  const uint32_t bits = layer_bits(d.M, d.lboost, b.lmaxbits, b.lshift);
  // the scatter's failure (bit 0, set before this launch); bit 1 comes from
  // blocks of this launch and must not steer a block's control flow
  const bool failed = (ld_agent(&d.lfail) & 1u) != 0;
  LayerSums sum;
  for (uint32_t bk = blockIdx.x; bk < (1u << bits); bk += gridDim.x) {
    if (failed) {                          // only zero the counts (uniform)
      if (threadIdx.x == 0) b.lcount[bk] = 0;
      continue;
    }
    apply_bucket<WW, NB>(b, d, op, bits, bk, sh, sum);
  }
  flush_sums<WW, NB>(b, d, sh, sum);
  if (!last_block(S.sync, &sh.flag, gridDim.x, true)) return;
  if (threadIdx.x == 0) layer_finish(b, d, op, ApplySh<WW, NB>::NS, false);
}

// Block scan for NB-thread blocks over instances (as plan_tiles).
template <int NB, class F>
__device__ __forceinline__ uint32_t plan_tiles_n(int ninst, F tiles, uint32_t* s_pref,
                                                 uint32_t* s_tmp) {
  constexpr int kPer = (kMaxInst + NB - 1) / NB;
  uint32_t loc[kPer];
  uint32_t sum = 0;
  const int base = threadIdx.x * kPer;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = base + k;
    loc[k] = (i < ninst) ? tiles(i) : 0u;
    sum += loc[k];
  }
  uint32_t total;
  uint32_t off = block_scan_n<NB / 64>(sum, s_tmp, &total);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = base + k;
    if (i < ninst) s_pref[i] = off;
    off += loc[k];
  }
  __syncthreads();
  return total;
}

// Batched form, step 2: the buckets of every instance whose layer op step 1
// took, dealt out to the blocks; the last block finishes those instances
// (a bucket that did not fit sends the instance to the op's gate copies).
template <int WW, int NB>
__global__ __launch_bounds__(NB) void k_layer_apply_multi(Ctx C) {
  __shared__ uint32_t s_pref[kMaxInst];
  extern __shared__ __align__(16) uint64_t s_layer_dyn[];   // sizeof(ApplySh<WW, NB>) bytes
  ApplySh<WW, NB>& sh = *reinterpret_cast<ApplySh<WW, NB>*>(s_layer_dyn);
  const int ninst = *C.ninst;
  auto served = [&](int i) {
    return C.bufs[i]->W == WW && ld_agent(&C.dyns[i]->lserved) != 0;
  };
  const uint32_t total = plan_tiles_n<NB>(ninst, [&](int i) -> uint32_t {
    if (!served(i)) return 0u;
    const InstBuf& b = *C.bufs[i];
    const InstDyn& d = *C.dyns[i];
    return 1u << layer_bits(d.M, d.lboost, b.lmaxbits, b.lshift);
  }, s_pref, sh.tmp);
  LayerSums sum;
  int cur = -1;
  for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_inst(s_pref, ninst, t);
    const InstBuf& b = *C.bufs[i];
    InstDyn& d = *C.dyns[i];
    const Op& op = b.prog[d.pc];
    if (i != cur) {
      if (cur >= 0) flush_sums<WW, NB>(*C.bufs[cur], *C.dyns[cur], sh, sum);
      __syncthreads();                     // the last bucket's rotations are read
      load_rotations<WW, NB>(op, sh);
      cur = i;
    }
    const uint32_t bits = layer_bits(d.M, d.lboost, b.lmaxbits, b.lshift);
    const uint32_t bk = t - s_pref[i];
    if (ld_agent(&d.lfail) & 1u) {         // the scatter failed: only zero the counts
      if (threadIdx.x == 0) b.lcount[bk] = 0;
      continue;
    }
    apply_bucket<WW, NB>(b, d, op, bits, bk, sh, sum);
  }
  if (cur >= 0) flush_sums<WW, NB>(*C.bufs[cur], *C.dyns[cur], sh, sum);
  if (!last_block(C.sync, &sh.flag, gridDim.x, true)) return;
  for (int i = threadIdx.x; i < ninst; i += NB) {
    if (!served(i)) continue;
    const InstBuf& b = *C.bufs[i];
    InstDyn& d = *C.dyns[i];
    d.lserved = 0;
    layer_finish(b, d, b.prog[d.pc], ApplySh<WW, NB>::NS, true);
  }
}

}  // namespace pp
