// gfx950 kernels of the symmetry-merging Pauli propagation library.
//
// Every kernel serves a list of instances (one for the single-handle calls,
// up to kMaxInst for the batched form).  A kernel is launched with a fixed
// grid; each block first plans the work of the instances whose current
// operation (program[pc]) belongs to this kernel, as a prefix sum of tiles
// in LDS, then walks the tiles grid-stride.  The last block to finish
// (threadfence + done counter) advances the program counters.  Term counts
// therefore stay on the device and launches never depend on them, so the
// per-step sequence of launches can be captured into a HIP graph.
//
// Paper: Teng, Chang, Rudolph, Holmes, arXiv:2512.12094.
#pragma once
#include <hip/hip_runtime.h>

#include "pp_fixed.h"
#include "pp_types.h"

namespace pp {

constexpr int kBlock = 256;
constexpr int kItems = 4;
constexpr int kTile = kBlock * kItems;
constexpr int kWaves = kBlock / 64;

// Loops over the W words of a string run to the compile-time kMaxW with a
// guard, so per-string arrays of kMaxW words are indexed by constants and
// stay in registers (a runtime trip count would put them in scratch).
#define PP_FOR_W(w, lo, n, lim) _Pragma("unroll") for (int w = (lo); w < (lim); ++w) if (w < (n))

struct Ctx {
  const InstBuf* const* bufs;
  InstDyn* const* dyns;
  const int* ninst;     // device-resident instance count (graph-stable)
  uint32_t* sync;       // done counter, reset by the last block
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// splitmix64 finalizer (Steele, Lea, Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014): a bijective 64-bit mixer.
__host__ __device__ __forceinline__ constexpr uint64_t mix64(uint64_t v) {
  v ^= v >> 30;
  v *= 0xbf58476d1ce4e5b9ull;
  v ^= v >> 27;
  v *= 0x94d049bb133111ebull;
  v ^= v >> 31;
  return v;
}

// Inverse of mix64: each xor-shift undone by folding the shifted copies back
// in, each odd multiplier by its inverse modulo 2^64 (Newton iteration).
__host__ __device__ constexpr uint64_t inv_mod64(uint64_t a) {
  uint64_t x = a;
  for (int i = 0; i < 6; ++i) x *= 2 - a * x;
  return x;
}
__host__ __device__ __forceinline__ constexpr uint64_t unmix64(uint64_t v) {
  v ^= (v >> 31) ^ (v >> 62);
  v *= inv_mod64(0x94d049bb133111ebull);
  v ^= (v >> 27) ^ (v >> 54);
  v *= inv_mod64(0xbf58476d1ce4e5b9ull);
  v ^= (v >> 30) ^ (v >> 60);
  return v;
}
static_assert(unmix64(mix64(0x0123456789abcdefull)) == 0x0123456789abcdefull, "unmix64");

__device__ __forceinline__ uint64_t hash_key(const uint64_t* x, const uint64_t* z, int W,
                                    uint64_t seed) {
  uint64_t h = mix64(seed ^ 0x9e3779b97f4a7c15ull);
  PP_FOR_W(w, 0, W, kMaxW) {
    h = mix64(h ^ x[w]);
    h = mix64(h ^ z[w] ^ 0x632be59bd9b4e019ull);
  }
  return h;
}

// Symplectic product: P and Q anticommute iff the number of qubits where
// x_Q z_P + z_Q x_P = 1 is odd.
__device__ __forceinline__ bool anticommutes(const uint64_t* qx, const uint64_t* qz,
                                    const uint64_t* px, const uint64_t* pz, int W) {
  uint32_t par = 0;
  PP_FOR_W(w, 0, W, kMaxW) par += __popcll((qx[w] & pz[w]) ^ (qz[w] & px[w]));
  return par & 1u;
}

__device__ __forceinline__ int weight(const uint64_t* x, const uint64_t* z, int W) {
  int s = 0;
  PP_FOR_W(w, 0, W, kMaxW) s += __popcll(x[w] | z[w]);
  return s;
}

// With P = i^{|px&pz|} X^px Z^pz (Y = iXZ per qubit), P Q = i^phi R with
// phi = |px&pz| + |qx&qz| + 2|pz&qx| - |rx&rz| (mod 4) and R = P xor Q.
// For anticommuting P, Q the phi is odd and iPQ = i^{1+phi} R = sigma R with
// sigma = +1 for phi = 3 and -1 for phi = 1.
__device__ __forceinline__ int product_sign(const uint64_t* px, const uint64_t* pz,
                                   const uint64_t* qx, const uint64_t* qz,
                                   const uint64_t* rx, const uint64_t* rz, int W) {
  int phi = 0;
  PP_FOR_W(w, 0, W, kMaxW)
    phi += __popcll(px[w] & pz[w]) + __popcll(qx[w] & qz[w]) +
           2 * __popcll(pz[w] & qx[w]) - __popcll(rx[w] & rz[w]);
  return ((phi & 3) == 3) ? 1 : -1;
}

// int(a) < int(b) in the paper's base-4 order (qubit q = digit of weight
// 4^q, digit = (x xor z) + 2 z: I0 X1 Y2 Z3), one word.
__device__ __forceinline__ bool int_less1(uint64_t xa, uint64_t za, uint64_t xb, uint64_t zb) {
  const uint64_t d = (xa ^ xb) | (za ^ zb);
  if (d == 0) return false;
  const int t = 63 - __clzll(d);
  const uint32_t ca = (uint32_t)(((xa ^ za) >> t) & 1) | (uint32_t)(((za >> t) & 1) << 1);
  const uint32_t cb = (uint32_t)(((xb ^ zb) >> t) & 1) | (uint32_t)(((zb >> t) & 1) << 1);
  return ca < cb;
}

// rotate right by j within n bits (0 <= j < n): bit (q + j) mod n -> bit q,
// i.e. T^j (qubit q of T^j s is qubit q + j of s).
__device__ __forceinline__ uint64_t rotr_n(uint64_t v, int j, int n, uint64_t mask) {
  if (j == 0) return v;
  return ((v >> j) | (v << (n - j))) & mask;
}

// Algorithm 2 representative for n <= 64: the translation with the smallest
// base-4 integer.  That translation puts a longest cyclic run of identities
// on the most significant qubits (any other one has a non-identity digit
// among those top digits), so only the translations that align a longest
// run with the top are compared; a string without identities compares all.
__device__ __forceinline__ void canon_translation(uint64_t x, uint64_t z, int n,
                                         uint64_t* rx, uint64_t* rz) {
  const uint64_t mask = (n == 64) ? ~0ull : ((1ull << n) - 1);
  const uint64_t idm = ~(x | z) & mask;
  if (idm == mask) { *rx = 0; *rz = 0; return; }
  uint64_t bx = x, bz = z;
  if (idm == 0) {
    for (int j = 1; j < n; ++j) {
      const uint64_t tx = rotr_n(x, j, n, mask), tz = rotr_n(z, j, n, mask);
      if (int_less1(tx, tz, bx, bz)) { bx = tx; bz = tz; }
    }
  } else {
    // S_len bit a <=> qubits a .. a+len-1 (cyclic) are all identities.
    // (loops unrolled over the 7 levels so that pw stays in registers)
    uint64_t pw[7];
    pw[0] = idm;
    int nb = 1;
#pragma unroll
    for (int k = 1; k < 7; ++k) {
      pw[k] = 0;
      if ((1 << k) <= n) {
        pw[k] = pw[k - 1] & rotr_n(pw[k - 1], 1 << (k - 1), n, mask);
        nb = k + 1;
      }
    }
    uint64_t cur = mask;
    int len = 0;
#pragma unroll
    for (int b = 6; b >= 0; --b) {
      if (b >= nb || len + (1 << b) > n - 1) continue;
      const uint64_t cand = cur & rotr_n(pw[b], len, n, mask);
      if (cand) { cur = cand; len += 1 << b; }
    }
    // cur: starts of the longest runs; translation j = (a + len) mod n puts
    // the run starting at qubit a onto qubits n-len .. n-1.
    bool first = true;
    while (cur) {
      const int a = __ffsll((unsigned long long)cur) - 1;
      cur &= cur - 1;
      int j = a + len;
      if (j >= n) j -= n;
      const uint64_t tx = rotr_n(x, j, n, mask), tz = rotr_n(z, j, n, mask);
      if (first || int_less1(tx, tz, bx, bz)) { bx = tx; bz = tz; first = false; }
    }
  }
  *rx = bx;
  *rz = bz;
}

// The same representative for n <= 32 in 32-bit words: a rotation within
// n = 32 bits is one funnel shift (v_alignbit_b32), and every step of the
// search above is a 32-bit operation instead of a 64-bit pair.
__device__ __forceinline__ uint32_t rotr32(uint32_t v, int j, int n, uint32_t mask) {
  if (n == 32) return __builtin_amdgcn_alignbit(v, v, (uint32_t)j);
  if (j == 0) return v;
  return ((v >> j) | (v << (n - j))) & mask;
}

__device__ __forceinline__ bool int_less32(uint32_t xa, uint32_t za, uint32_t xb, uint32_t zb) {
  const uint32_t d = (xa ^ xb) | (za ^ zb);
  if (d == 0) return false;
  const int t = 31 - __clz(d);
  const uint32_t ca = (((xa ^ za) >> t) & 1u) | (((za >> t) & 1u) << 1);
  const uint32_t cb = (((xb ^ zb) >> t) & 1u) | (((zb >> t) & 1u) << 1);
  return ca < cb;
}

__device__ __forceinline__ void canon_translation32(uint32_t x, uint32_t z, int n, uint32_t* rx,
                                                    uint32_t* rz) {
  const uint32_t mask = (n == 32) ? ~0u : ((1u << n) - 1);
  const uint32_t idm = ~(x | z) & mask;
  uint32_t bx = x, bz = z;
  if (__builtin_expect(idm == 0, 0)) {      // no identity: compare all n translations
    for (int j = 1; j < n; ++j) {
      const uint32_t tx = rotr32(x, j, n, mask), tz = rotr32(z, j, n, mask);
      if (int_less32(tx, tz, bx, bz)) { bx = tx; bz = tz; }
    }
    *rx = bx;
    *rz = bz;
    return;
  }
  // pw[k] bit a: qubits a .. a + 2^k - 1 (cyclic) are all identities
  uint32_t pw[6];
  pw[0] = idm;
#pragma unroll
  for (int k = 1; k < 6; ++k)
    pw[k] = (1 << k) <= n ? pw[k - 1] & rotr32(pw[k - 1], 1 << (k - 1), n, mask) : 0u;
  // longest run length and its starts, by selects (no divergent branch):
  // the all-identity string has a run of n starting everywhere, which puts
  // it on itself below
  uint32_t cur = mask;
  int len = 0;
#pragma unroll
  for (int b = 5; b >= 0; --b) {
    if ((1 << b) > n) continue;               // uniform: n is the same for every lane
    const uint32_t cand = cur & rotr32(pw[b], len < n ? len : 0, n, mask);
    const bool take = cand != 0 && len + (1 << b) <= n;
    cur = take ? cand : cur;
    len = take ? len + (1 << b) : len;
  }
  // translation j = (a + len) mod n puts the run starting at a on the top
  // qubits; the first start unconditionally, the others in a loop (rare)
  int j0 = __ffs(cur) - 1 + len;
  if (j0 >= n) j0 -= n;
  bx = rotr32(x, j0, n, mask);
  bz = rotr32(z, j0, n, mask);
  cur &= cur - 1;
  if (__builtin_expect(cur != 0, 0) && len < n) {
    while (cur) {
      const int a = __ffs(cur) - 1;
      cur &= cur - 1;
      int j = a + len;
      if (j >= n) j -= n;
      const uint32_t tx = rotr32(x, j, n, mask), tz = rotr32(z, j, n, mask);
      if (int_less32(tx, tz, bx, bz)) { bx = tx; bz = tz; }
    }
  }
  *rx = bx;
  *rz = bz;
}

// Dihedral group D_n: the smaller of the translation representatives of the
// string and of its reflection (qubit q -> n-1-q), i.e. the minimum over all
// 2n translations and reflected translations.
__device__ __forceinline__ void canon_dihedral(uint64_t x, uint64_t z, int n, uint64_t* rx,
                                               uint64_t* rz) {
  uint64_t ax, az, bx, bz;
  canon_translation(x, z, n, &ax, &az);
  const uint64_t xr = __brevll(x) >> (64 - n), zr = __brevll(z) >> (64 - n);
  canon_translation(xr, zr, n, &bx, &bz);
  if (int_less1(bx, bz, ax, az)) {
    ax = bx;
    az = bz;
  }
  *rx = ax;
  *rz = az;
}

// Translations of an lx x ly torus (qubit q = x + lx*y, n = lx*ly <= 64):
// the minimum over all shifts.  Shifting by b rows is a rotation of the
// whole mask by b*lx bits; shifting every row by a columns moves the bits
// with x >= a down by a and wraps the others, with masks replicated over the
// rows.
__device__ __forceinline__ void canon_torus(uint64_t x, uint64_t z, int n, int lx, uint64_t* rx,
                                            uint64_t* rz) {
  const int ly = n / lx;
  const uint64_t mask = (n == 64) ? ~0ull : ((1ull << n) - 1);
  uint64_t rep = 0;                        // bit 0 of every row
  for (int y = 0; y < ly; ++y) rep |= 1ull << (lx * y);
  uint64_t bx = x, bz = z;
  for (int b = 0; b < ly; ++b) {
    const uint64_t yx = rotr_n(x, b * lx, n, mask), yz = rotr_n(z, b * lx, n, mask);
    for (int a = 0; a < lx; ++a) {
      uint64_t tx = yx, tz = yz;
      if (a) {
        const uint64_t low = (((1ull << (lx - a)) - 1) * rep) & mask;   // columns < lx - a
        const uint64_t high = mask & ~low;
        tx = ((yx >> a) & low) | ((yx << (lx - a)) & high);
        tz = ((yz >> a) & low) | ((yz << (lx - a)) & high);
      }
      if (int_less1(tx, tz, bx, bz)) {
        bx = tx;
        bz = tz;
      }
    }
  }
  *rx = bx;
  *rz = bz;
}

// Any finite group of qubit permutations given by its element list (n <= 64):
// the minimum over the listed images, image g taking qubit gperm[g*n + q] of
// the string to qubit q.
__device__ __forceinline__ void canon_explicit(uint64_t x, uint64_t z, int n,
                                               const uint8_t* gperm, uint32_t gsize,
                                               uint64_t* rx, uint64_t* rz) {
  uint64_t bx = x, bz = z;
  for (uint32_t g = 0; g < gsize; ++g) {
    const uint8_t* p = gperm + (size_t)g * n;
    uint64_t tx = 0, tz = 0;
    for (int q = 0; q < n; ++q) {
      const int src = p[q];
      tx |= ((x >> src) & 1ull) << q;
      tz |= ((z >> src) & 1ull) << q;
    }
    if (int_less1(tx, tz, bx, bz)) {
      bx = tx;
      bz = tz;
    }
  }
  *rx = bx;
  *rz = bz;
}

// Algorithm 3: counts of X, Y, Z letters.
__device__ __forceinline__ void perm_counts(const uint64_t* x, const uint64_t* z, int W,
                                   uint32_t* nx, uint32_t* ny, uint32_t* nz) {
  uint32_t a = 0, b = 0, c = 0;
  PP_FOR_W(w, 0, W, kMaxW) {
    a += __popcll(x[w] & ~z[w]);
    b += __popcll(x[w] & z[w]);
    c += __popcll(z[w] & ~x[w]);
  }
  *nx = a; *ny = b; *nz = c;
}

// Z^{nZ} Y^{nY} X^{nX} from qubit 0: z bits [0, nZ+nY), x bits [nZ, nZ+nY+nX).
__device__ __forceinline__ void perm_rep(uint32_t nx, uint32_t ny, uint32_t nz, int W,
                                uint64_t* rx, uint64_t* rz) {
  const uint32_t zlo = 0, zhi = nz + ny, xlo = nz, xhi = nz + ny + nx;
  PP_FOR_W(w, 0, W, kMaxW) {
    const uint32_t lo = 64u * w, hi = lo + 64u;
    auto range = [&](uint32_t a, uint32_t b) -> uint64_t {  // bits [a,b) of this word
      const uint32_t s = a > lo ? a : lo, e = b < hi ? b : hi;
      if (s >= e) return 0ull;
      const uint32_t len = e - s;
      const uint64_t m = (len == 64) ? ~0ull : ((1ull << len) - 1);
      return m << (s - lo);
    };
    rx[w] = range(xlo, xhi);
    rz[w] = range(zlo, zhi);
  }
}

// Narrow merge key of a one-word string for a group known at compile time
// (0 none, 1 Z_n, 3 D_n, 4 torus, 5 explicit; n <= 32): the representative
// packed as x | z << 32.
template <int G>
__device__ __forceinline__ uint64_t narrow_key_t(const InstBuf& b, uint64_t x, uint64_t z) {
  if constexpr (G == 1) {
    uint32_t ax, az;
    canon_translation32((uint32_t)x, (uint32_t)z, b.n, &ax, &az);
    return (uint64_t)ax | ((uint64_t)az << 32);
  } else if constexpr (G == 3) {
    uint32_t ax, az, bx, bz;
    canon_translation32((uint32_t)x, (uint32_t)z, b.n, &ax, &az);
    const uint32_t xr = __brev((uint32_t)x) >> (32 - b.n), zr = __brev((uint32_t)z) >> (32 - b.n);
    canon_translation32(xr, zr, b.n, &bx, &bz);
    if (int_less32(bx, bz, ax, az)) { ax = bx; az = bz; }
    return (uint64_t)ax | ((uint64_t)az << 32);
  } else if constexpr (G == 4) {
    uint64_t rx, rz;
    canon_torus(x, z, b.n, b.lx, &rx, &rz);
    return rx | (rz << 32);
  } else if constexpr (G == 5) {
    uint64_t rx, rz;
    canon_explicit(x, z, b.n, b.gperm, b.gsize, &rx, &rz);
    return rx | (rz << 32);
  } else {
    return x | (z << 32);
  }
}

// Narrow merge key: the representative itself, packed into 64 bits.
__device__ __forceinline__ uint64_t narrow_key(const InstBuf& b, const uint64_t* x,
                                      const uint64_t* z) {
  if (b.group == 2) {
    uint32_t nx, ny, nz;
    perm_counts(x, z, b.W, &nx, &ny, &nz);
    return (uint64_t)nx | ((uint64_t)ny << 8) | ((uint64_t)nz << 16);
  }
  uint64_t rx = x[0], rz = z[0];
  if (b.group == 1) {                       // n <= 32 here
    uint32_t ax, az;
    canon_translation32((uint32_t)x[0], (uint32_t)z[0], b.n, &ax, &az);
    return (uint64_t)ax | ((uint64_t)az << 32);
  }
  if (b.group == 3) {
    uint32_t ax, az, bx, bz;
    canon_translation32((uint32_t)x[0], (uint32_t)z[0], b.n, &ax, &az);
    const uint32_t xr = __brev((uint32_t)x[0]) >> (32 - b.n), zr = __brev((uint32_t)z[0]) >> (32 - b.n);
    canon_translation32(xr, zr, b.n, &bx, &bz);
    if (int_less32(bx, bz, ax, az)) { ax = bx; az = bz; }
    return (uint64_t)ax | ((uint64_t)az << 32);
  }
  if (b.group == 4) canon_torus(x[0], z[0], b.n, b.lx, &rx, &rz);
  if (b.group == 5) canon_explicit(x[0], z[0], b.n, b.gperm, b.gsize, &rx, &rz);
  return rx | (rz << 32);   // n <= 32
}

__device__ __forceinline__ void narrow_decode(const InstBuf& b, uint64_t key, uint64_t* rx,
                                     uint64_t* rz) {
  if (b.group == 2) {
    perm_rep((uint32_t)(key & 0xff), (uint32_t)((key >> 8) & 0xff),
             (uint32_t)((key >> 16) & 0xff), b.W, rx, rz);
    return;
  }
  rx[0] = key & 0xffffffffull;
  rz[0] = key >> 32;
  PP_FOR_W(w, 1, b.W, kMaxW) { rx[w] = 0; rz[w] = 0; }
}

// Representative as a string (wide path: Z_n with n <= 64, or identity).
__device__ __forceinline__ void rep_string(const InstBuf& b, const uint64_t* x, const uint64_t* z,
                                  uint64_t* rx, uint64_t* rz) {
  if (b.group == 1 || b.group == 3 || b.group == 4 || b.group == 5) {
    if (b.group == 1)
      canon_translation(x[0], z[0], b.n, rx, rz);
    else if (b.group == 3)
      canon_dihedral(x[0], z[0], b.n, rx, rz);
    else if (b.group == 4)
      canon_torus(x[0], z[0], b.n, b.lx, rx, rz);
    else
      canon_explicit(x[0], z[0], b.n, b.gperm, b.gsize, rx, rz);
    PP_FOR_W(w, 1, b.W, kMaxW) { rx[w] = 0; rz[w] = 0; }
  } else if (b.group == 2) {
    uint32_t nx, ny, nz;
    perm_counts(x, z, b.W, &nx, &ny, &nz);
    perm_rep(nx, ny, nz, b.W, rx, rz);
  } else {
    PP_FOR_W(w, 0, b.W, kMaxW) { rx[w] = x[w]; rz[w] = z[w]; }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Exclusive block scan of one value per thread; *total = block sum.
// s_tmp needs kWaves + 1 entries.  Contains __syncthreads.
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
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
    for (int w = 0; w < kWaves; ++w) { const uint32_t t = s_tmp[w]; s_tmp[w] = acc; acc += t; }
    s_tmp[kWaves] = acc;
  }
  __syncthreads();
  const uint32_t r = x - v + s_tmp[wid];
  *total = s_tmp[kWaves];
  __syncthreads();
  return r;
}


// Makes the wave wait for a returned value (an atomic's result) before it
// issues anything after this point; emits no instruction of its own.
__device__ __forceinline__ void consume(uint64_t v) { asm volatile("" : : "v"(v)); }

__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Launches of up to kTreeMin working blocks count on one line (one atomic
// round trip less on the critical path); larger ones use the shards.
constexpr uint32_t kTreeMin = 256;
__device__ __forceinline__ uint32_t acc_shards(uint32_t workers) {
  return workers > kTreeMin ? (uint32_t)kAccShards : 1u;
}

// Last block, one thread: moves the shard totals into d.acc and clears the
// shards (with one shard the blocks added to d.acc itself).
__device__ __forceinline__ void fold_acc(const InstBuf& b, InstDyn& d, uint32_t nsh) {
  if (nsh == 1) {
    d.acc = ld_agent(&d.acc);
    return;
  }
  uint64_t v = 0;
  for (uint32_t s = 0; s < nsh; ++s)
    v += atomicExch((unsigned long long*)&b.accs[s * kLineU64], 0ull);
  d.acc += v;
}

// Thread 0: adds the statistic v of kind k to this block's shard line; the
// result is not waited for (no kernel reads the statistics back).
__device__ __forceinline__ void add_stat(const InstBuf& b, int k, uint64_t v) {
  if (v) atomicAdd((unsigned long long*)&b.stats[(k * kAccShards + blockIdx.x % kAccShards) * kLineU64],
                   (unsigned long long)v);
}

// live = low half, anticommuting count = high half; clears the accumulator.
__device__ __forceinline__ void take_acc(InstDyn& d) {
  const uint64_t v = d.acc;
  d.live = (uint32_t)v;
  d.count = (uint32_t)(v >> 32);
  d.acc = 0;
}

// Block-wide "am I the last working block of this launch" over the
// `workers` blocks that had tiles.  Beyond kTreeMin workers the done
// counter is a two-level tree:
// block b counts in shard b % kSyncShards, the block completing a shard
// counts in the root, and the block completing the root is the last one.
// Within a launch, blocks hand results to the last block only through
// device-scope atomics that thread 0 issued and waited on (their returned
// values are consumed) before it counts itself, and every level's count is
// issued only after the level below returned, so no fence is needed.
// `fence` adds one for a last block that reads plain stores of other blocks
// (the multi-instance runner keeps it).
__device__ __forceinline__ bool last_block(uint32_t* sync, uint32_t* s_flag, uint32_t workers,
                                  bool fence = false) {
  if (workers <= 1) return true;       // block 0 did all the work itself
  __syncthreads();
  if (threadIdx.x == 0 && workers <= kTreeMin) {   // one level
    if (fence) __threadfence();
    const uint32_t t = atomicAdd(sync, 1u);
    *s_flag = (t == workers - 1) ? 1u : 0u;
    if (*s_flag) atomicExch(sync, 0u);
  } else if (threadIdx.x == 0) {
    if (fence) __threadfence();
    const uint32_t sh = blockIdx.x % kSyncShards;
    const uint32_t members = (workers - sh + kSyncShards - 1) / kSyncShards;
    const uint32_t roots = workers < (uint32_t)kSyncShards ? workers : kSyncShards;
    uint32_t* cs = sync + (1 + sh) * kLineU32;
    uint32_t last = 0;
    if (atomicAdd(cs, 1u) == members - 1) {
      atomicExch(cs, 0u);
      if (atomicAdd(sync, 1u) == roots - 1) {
        atomicExch(sync, 0u);
        last = 1;
      }
    }
    *s_flag = last;
  }
  __syncthreads();
  const bool r = *s_flag != 0;
  if (r && fence) __threadfence();
  return r;
}

// last_block for thread 0 alone (the block's other threads have left), with
// no fence: for kinds whose last block reads only the accumulators.
__device__ __forceinline__ bool last_block_one(uint32_t* sync, uint32_t workers) {
  if (workers <= 1) return true;
  if (workers <= kTreeMin) {
    const uint32_t t = atomicAdd(sync, 1u);
    if (t != workers - 1) return false;
    atomicExch(sync, 0u);
    return true;
  }
  const uint32_t sh = blockIdx.x % kSyncShards;
  const uint32_t members = (workers - sh + kSyncShards - 1) / kSyncShards;
  const uint32_t roots = workers < (uint32_t)kSyncShards ? workers : kSyncShards;
  uint32_t* cs = sync + (1 + sh) * kLineU32;
  if (atomicAdd(cs, 1u) != members - 1) return false;
  atomicExch(cs, 0u);
  if (atomicAdd(sync, 1u) != roots - 1) return false;
  atomicExch(sync, 0u);
  return true;
}

// Thread 0 of each working block of a launch of at most kTreeMin blocks over
// a store below 2^26 entries: counts the block done and adds its live and
// anticommuting counts (each below 2^26) in the same 64-bit atomic, so the
// last block learns the launch's totals from the atomic's result, with no
// separate accumulator round trip.  Returns true in the last block, with
// the totals as live | count << 32 in *acc.
constexpr uint32_t kPackedCap = 1u << 26;
__device__ __forceinline__ bool last_block_packed(uint32_t* sync, uint32_t workers, uint32_t live,
                                                  uint32_t cnt, bool fence, uint64_t* acc) {
  const uint64_t mask = (1ull << 26) - 1;
  const uint64_t v = (1ull << 52) | ((uint64_t)cnt << 26) | live;
  uint64_t tot = v;
  if (workers > 1) {
    if (fence) __threadfence();
    unsigned long long* w = (unsigned long long*)(sync + kPackedLine * kLineU32);
    const uint64_t old = atomicAdd(w, (unsigned long long)v);
    if ((old >> 52) != workers - 1) return false;
    atomicExch(w, 0ull);                 // every other block has added its share
    tot = old + v;
    if (fence) __threadfence();
  }
  *acc = (tot & mask) | (((tot >> 26) & mask) << 32);
  return true;
}

// Blocks beyond the tile count leave at once; block 0 always stays so that
// the program counters advance even when no instance has work.
__device__ __forceinline__ uint32_t worker_count(uint32_t total) {
  return total < gridDim.x ? (total ? total : 1u) : gridDim.x;
}

// Prefix of tiles over instances: s_pref[i] = first tile of instance i.
// tiles(i) returns the tile count of instance i (0 when not served).
template <class F>
__device__ __forceinline__ uint32_t plan_tiles(int ninst, F tiles, uint32_t* s_pref, uint32_t* s_tmp) {
  constexpr int kPer = kMaxInst / kBlock;
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
  uint32_t off = block_scan(sum, s_tmp, &total);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = base + k;
    if (i < ninst) s_pref[i] = off;
    off += loc[k];
  }
  __syncthreads();
  return total;
}

__device__ __forceinline__ int find_inst(const uint32_t* s_pref, int ninst, uint32_t t) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_pref[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int IT>
__device__ __forceinline__ uint32_t ceil_tiles(uint32_t n) { return (n + kBlock * IT - 1) / (kBlock * IT); }

__device__ __forceinline__ const Op* cur_op(const InstBuf& b, const InstDyn& d) {
  return d.pc < b.prog_len ? &b.prog[d.pc] : nullptr;
}

// Past the current op; where LAYER ops are off (the batched form), past
// every LAYER op too: the GATE(S) copies of its rotations follow it.
__device__ __forceinline__ void next_op(const InstBuf& b, InstDyn& d) {
  uint32_t pc = d.pc + 1;
  while (b.nolayer && pc < b.prog_len && b.prog[pc].type == OP_LAYER) ++pc;
  d.pc = pc;
}

// ---------------------------------------------------------------------------
// gate table
// ---------------------------------------------------------------------------
// Finds the live entry with key (rx, rz) among entries [0, Mstart), else -1.
// Entries appended by the running gate (index >= Mstart) are skipped: no
// gate ever looks up a string that the same gate appends, except the
// appending thread itself, which knows it is absent.
// The candidate's liveness, key words and coefficient are loaded together
// (a slot of the current generation always holds an index below cap), so a
// probe costs one dependent round trip after the slot itself; *c receives
// the found entry's coefficient.
// Probing from slot s, `done` probes already made.
template <class V>
__device__ __forceinline__ int64_t gt_lookup_from(const InstBuf& b, uint32_t gen, uint32_t Mstart,
                                                  const V& view, const uint64_t* rx,
                                                  const uint64_t* rz, uint64_t s, uint64_t done,
                                                  double* c) {
  const int W = b.W;
  const uint32_t cap = b.cap;
  const uint64_t mask = (1ull << b.hg_bits) - 1;
  for (uint64_t probe = done; probe <= mask; ++probe) {
    const uint64_t v = b.gtab[s];
    if ((uint32_t)(v >> 32) != gen) return -1;
    const uint32_t idx = (uint32_t)v;
    const uint8_t a = view.al[idx];
    uint64_t kx[kMaxW], kz[kMaxW];
    PP_FOR_W(w, 0, W, kMaxW) {
      kx[w] = view.X[(size_t)w * cap + idx];
      kz[w] = view.Z[(size_t)w * cap + idx];
    }
    const double cj = view.getc(idx);
    if (idx < Mstart && a) {
      bool eq = true;
      PP_FOR_W(w, 0, W, kMaxW) eq = eq && kx[w] == rx[w] && kz[w] == rz[w];
      if (eq) {
        *c = cj;
        return idx;
      }
    }
    s = (s + 1) & mask;
  }
  return -1;
}

template <class V>
__device__ __forceinline__ int64_t gt_lookup(const InstBuf& b, uint32_t gen, uint32_t Mstart,
                                             const V& view, const uint64_t* rx,
                                             const uint64_t* rz, double* c) {
  return gt_lookup_from(b, gen, Mstart, view, rx, rz, hash_key(rx, rz, b.W, 0) >> (64 - b.hg_bits),
                        0, c);
}

// gt_lookup for N keys at once: the first probe of every key is issued
// together (slot loads, then the candidates' liveness, keys and
// coefficients), so N lookups cost the round trips of one; a key whose first
// slot holds another live key continues with gt_lookup from the next slot.
// want[m] false skips key m (idx[m] = -1).
template <int N, class V>
__device__ __forceinline__ void gt_lookup_n(const InstBuf& b, uint32_t gen, uint32_t Mstart,
                                            const V& view, const bool* want,
                                            const uint64_t (*rx)[kMaxW],
                                            const uint64_t (*rz)[kMaxW], int64_t* idx, double* c) {
  const int W = b.W;
  const uint32_t cap = b.cap;
  const uint64_t mask = (1ull << b.hg_bits) - 1;
  uint64_t s[N], v[N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    s[m] = hash_key(rx[m], rz[m], W, 0) >> (64 - b.hg_bits);
    v[m] = want[m] ? b.gtab[s[m]] : 0ull;
  }
  uint8_t a[N];
  uint64_t kx[N][kMaxW], kz[N][kMaxW];
  double cj[N];
  bool hit[N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    hit[m] = want[m] && (uint32_t)(v[m] >> 32) == gen;
    const uint32_t k = hit[m] ? (uint32_t)v[m] : 0u;   // slot of this generation: k < cap
    a[m] = view.al[k];
    PP_FOR_W(w, 0, W, kMaxW) {
      kx[m][w] = view.X[(size_t)w * cap + k];
      kz[m][w] = view.Z[(size_t)w * cap + k];
    }
    cj[m] = view.getc(k);
  }
#pragma unroll
  for (int m = 0; m < N; ++m) {
    idx[m] = -1;
    if (!hit[m]) continue;                   // skipped, or an empty slot: absent
    const uint32_t k = (uint32_t)v[m];
    bool eq = k < Mstart && a[m];
    PP_FOR_W(w, 0, W, kMaxW) eq = eq && kx[m][w] == rx[m][w] && kz[m][w] == rz[m][w];
    if (eq) {
      idx[m] = k;
      c[m] = cj[m];
    } else {
      idx[m] = gt_lookup_from(b, gen, Mstart, view, rx[m], rz[m], (s[m] + 1) & mask, 1, &c[m]);
    }
  }
}

// Inserts index `idx` (insert-only: the caller guarantees that no live entry
// with this key exists and that no thread compares keys of this generation
// in the same launch, so no key is read here).
__device__ __forceinline__ void gt_insert(uint64_t* gtab, uint32_t bits, uint32_t gen, uint32_t idx,
                                 uint64_t h) {
  const uint64_t mask = (1ull << bits) - 1;
  uint64_t s = h >> (64 - bits);
  const uint64_t nv = ((uint64_t)gen << 32) | idx;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    unsigned long long v = gtab[s];
    while ((uint32_t)(v >> 32) != gen) {
      const unsigned long long old =
          atomicCAS((unsigned long long*)&gtab[s], v, (unsigned long long)nv);
      if (old == v) return;
      v = old;
    }
    s = (s + 1) & mask;
  }
}

// ---------------------------------------------------------------------------
// exact sums: 192-bit two's-complement fixed point, kFxFrac fraction bits
// ---------------------------------------------------------------------------
// acc += v with one integer atomic per non-zero limb; the carries returned
// by the lower limbs are added into the next limb, so the final value is the
// exact sum of all contributions whatever their order.
__device__ __forceinline__ void fx_atomic_add(uint64_t* acc, Fx v) {
  unsigned long long* a = (unsigned long long*)acc;
  uint64_t c0 = 0;
  if (v.l0) {
    const uint64_t o0 = atomicAdd(&a[0], (unsigned long long)v.l0);
    c0 = (o0 + v.l0 < o0) ? 1u : 0u;
  }
  const uint64_t t1 = v.l1 + c0;
  uint64_t c1 = (t1 < c0) ? 1u : 0u;
  if (t1) {
    const uint64_t o1 = atomicAdd(&a[1], (unsigned long long)t1);
    c1 += (o1 + t1 < o1) ? 1u : 0u;
  }
  const uint64_t t2 = v.l2 + c1;
  if (t2) atomicAdd(&a[2], (unsigned long long)t2);
}

// As fx_atomic_add, but every limb's atomic returns and the last value is
// consumed, so the whole addition has completed when this returns.
__device__ __forceinline__ void fx_atomic_add_wait(uint64_t* acc, Fx v) {
  unsigned long long* a = (unsigned long long*)acc;
  const uint64_t o0 = atomicAdd(&a[0], (unsigned long long)v.l0);
  const uint64_t c0 = (o0 + v.l0 < o0) ? 1u : 0u;
  const uint64_t t1 = v.l1 + c0;
  uint64_t c1 = (t1 < c0) ? 1u : 0u;
  const uint64_t o1 = atomicAdd(&a[1], (unsigned long long)t1);
  c1 += (o1 + t1 < o1) ? 1u : 0u;
  consume(atomicAdd(&a[2], (unsigned long long)(v.l2 + c1)));
}

__device__ __forceinline__ Fx wave_sum_fx(Fx v) {
  for (int o = 32; o > 0; o >>= 1) {
    Fx w;
    w.l0 = __shfl_xor(v.l0, o, 64);
    w.l1 = __shfl_xor(v.l1, o, 64);
    w.l2 = __shfl_xor(v.l2, o, 64);
    v = fx_add(v, w);
  }
  return v;
}

// ---------------------------------------------------------------------------
// merge table
// ---------------------------------------------------------------------------
// Slots of the merge table used by a merge of the current d.M records:
// at least twice the records (load factor <= 1/2).
__device__ __forceinline__ uint32_t merge_bits(const InstBuf& b, const InstDyn& d) {
  const uint64_t need = 2ull * d.M;
  const uint32_t bits = need > 1 ? 64u - (uint32_t)__clzll((long long)(need - 1)) : 0u;
  return bits < 10u ? (10u < b.hm_bits ? 10u : b.hm_bits) : (bits < b.hm_bits ? bits : b.hm_bits);
}

// Find-or-insert of a 64-bit key; returns the slot.
__device__ __forceinline__ uint64_t mt_slot(uint64_t* mkey, uint32_t bits, uint64_t key) {
  const uint64_t mask = (1ull << bits) - 1;
  uint64_t s = mix64(key) >> (64 - bits);
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    unsigned long long k = mkey[s];
    if (k == kEmpty64) {
      k = atomicCAS((unsigned long long*)&mkey[s], (unsigned long long)kEmpty64,
                    (unsigned long long)key);
      if (k == kEmpty64) return s;
    }
    if (k == key) return s;
    s = (s + 1) & mask;
  }
  return kEmpty64;   // unreachable: the table is at most half full
}

__device__ __forceinline__ void mt_add(const InstBuf& b, InstDyn& d, uint64_t key, Fx v) {
  if (key == kEmpty64) {        // the one key equal to the empty marker
    fx_atomic_add(d.special_fx, v);
    atomicOr(&d.special, 1u);
    return;
  }
  const uint64_t s = mt_slot(b.mkey, merge_bits(b, d), key);
  if (s != kEmpty64) fx_atomic_add(&b.mfx[3 * s], v);
}

// Adds (key, v) of every active lane, first combining lanes of one wave
// that share a key (large orbits, e.g. S_n, collapse many records onto few
// representatives).  Must be called by all lanes of the wave.
__device__ __forceinline__ void wave_merge_add(const InstBuf& b, InstDyn& d, bool act,
                                      uint64_t key, Fx v) {
  const int lane = threadIdx.x & 63;
  for (int it = 0; it < 4; ++it) {
    const unsigned long long am = __ballot(act);
    if (am == 0) return;
    const int leader = __ffsll((unsigned long long)am) - 1;
    const uint64_t lk = __shfl(key, leader, 64);
    const bool m = act && key == lk;
    const unsigned long long mm = __ballot(m);
    if (__popcll(mm) == 1) break;
    const Fx zero{0, 0, 0};
    const Fx s = wave_sum_fx(m ? v : zero);
    if (lane == leader) mt_add(b, d, lk, s);
    if (m) act = false;
  }
  if (act) mt_add(b, d, key, v);
}

// ---------------------------------------------------------------------------
// views
// ---------------------------------------------------------------------------
struct View {
  uint64_t* X;
  uint64_t* Z;
  void* C;          // double[] or, when f32, float[]
  uint8_t* al;      // alive, current parity
  uint8_t* aln;     // alive, other parity
  uint32_t cap;
  int W;
  bool f32;
  // coefficient i as FP64 (exact for either storage)
  __device__ __forceinline__ double getc(uint32_t i) const {
    return f32 ? (double)static_cast<const float*>(C)[i] : static_cast<const double*>(C)[i];
  }
  // stores c, rounded to FP32 when the storage is FP32
  __device__ __forceinline__ void setc(uint32_t i, double c) const {
    if (f32)
      static_cast<float*>(C)[i] = (float)c;
    else
      static_cast<double*>(C)[i] = c;
  }
};

__device__ __forceinline__ View view_of(const InstBuf& b, const InstDyn& d) {
  View v;
  const uint32_t h = d.half, p = d.parity;
  v.X = b.x[h];
  v.Z = b.z[h];
  v.C = b.c[h];
  v.al = b.alive[h][p];
  v.aln = b.alive[h][p ^ 1];
  v.cap = b.cap;
  v.W = b.W;
  v.f32 = b.f32 != 0;
  return v;
}

// The rotation of a pair on span{Q, R} (R = PQ, i P Q = sig R, i P R = -sig Q):
//   c_Q' = cos c_Q - sig sin c_R,   c_R' = cos c_R + sig sin c_Q.
// In FP32 mode cos and sin are rounded to FP32 once and the products and
// sums are FP32 operations; results are returned widened to FP64 (exact).
__device__ __forceinline__ void rotate_pair(bool f32, double cs, double sn, int sig, double cq, double cr,
                                   double* nq, double* nr) {
  if (f32) {
    const float c = (float)cs, s = (float)sn, q = (float)cq, r = (float)cr;
    const float aq = c * q, bq = s * r, ar = c * r, br = s * q;
    *nq = (double)(sig > 0 ? aq - bq : aq + bq);
    *nr = (double)(sig > 0 ? ar + br : ar - br);
  } else {
    const double aq = cs * cq, bq = sn * cr, ar = cs * cr, br = sn * cq;
    *nq = sig > 0 ? aq - bq : aq + bq;
    *nr = sig > 0 ? ar + br : ar - br;
  }
}

// Partner absent: c_Q' = cos c_Q and the new string R gets sig sin c_Q.
__device__ __forceinline__ void rotate_single(bool f32, double cs, double sn, int sig, double cq,
                                     double* nq, double* child) {
  if (f32) {
    const float c = (float)cs, s = (float)sn, q = (float)cq;
    const float t = s * q;
    *nq = (double)(c * q);
    *child = (double)(sig > 0 ? t : -t);
  } else {
    const double t = sn * cq;
    *nq = cs * cq;
    *child = sig > 0 ? t : -t;
  }
}

__device__ __forceinline__ void load_key(const View& v, uint32_t i, uint64_t* x, uint64_t* z) {
  PP_FOR_W(w, 0, v.W, kMaxW) {
    x[w] = v.X[(size_t)w * v.cap + i];
    z[w] = v.Z[(size_t)w * v.cap + i];
  }
}

// ---------------------------------------------------------------------------
// GATE: one Pauli rotation (Prop. 1) + exact merge + truncation
// ---------------------------------------------------------------------------
// What a gate launch needs of its op, read once into registers.
struct GateArgs {
  uint64_t px[kMaxFuse][kMaxW], pz[kMaxFuse][kMaxW];   // rotations 1..nrot
  uint64_t nx[kMaxW], nz[kMaxW];                       // the next gate's rotation
  double cs[kMaxFuse], sn[kMaxFuse], eps;
  int wmax;
  uint32_t type, nrot;
  bool full, has_next;
};

__device__ __forceinline__ GateArgs gate_args(const Op& op) {
  GateArgs g;
#pragma unroll
  for (int w = 0; w < kMaxW; ++w) {
    g.px[0][w] = op.px[w];
    g.pz[0][w] = op.pz[w];
#pragma unroll
    for (int r = 1; r < kMaxFuse; ++r) {
      g.px[r][w] = op.qx[r - 1][w];
      g.pz[r][w] = op.qz[r - 1][w];
    }
    g.nx[w] = op.nx[w];
    g.nz[w] = op.nz[w];
  }
  g.cs[0] = op.cs;
  g.sn[0] = op.sn;
#pragma unroll
  for (int r = 1; r < kMaxFuse; ++r) {
    g.cs[r] = op.qcs[r - 1];
    g.sn[r] = op.qsn[r - 1];
  }
  g.eps = op.eps;
  g.wmax = op.wmax;
  g.type = op.type;
  g.nrot = op.type == OP_GATES ? op.nrot : 1u;
  g.full = op.full_check != 0;
  g.has_next = op.next_gate != kNone32;
  return g;
}

// Appends of a launch of r rotations over `live` terms, `count` of them
// anticommuting with the first: the first appends at most `count`, each
// later one at most the terms live before it, and the live terms at most
// double per rotation: count + (2^(r-1) - 1)(live + count).
__device__ __host__ __forceinline__ uint64_t gate_append_bound(uint32_t nrot, uint64_t live,
                                                               uint64_t count) {
  return count + (((uint64_t)1 << (nrot - 1)) - 1) * (live + count);
}

// 0 = not served, 1 = run, 2 = would overflow, from the op type and the
// instance's status, count tag, entries, live and anticommuting counts
__device__ __forceinline__ int gate_state_of(uint32_t type, uint32_t nrot, uint32_t pc,
                                             uint32_t status, uint32_t count_for, uint32_t M,
                                             uint32_t live, uint32_t count, uint32_t cap) {
  const uint64_t bound = gate_append_bound(type == OP_GATES ? nrot : 1u, live, count);
  const bool gate = type == OP_GATE || type == OP_GATES;
  const int fits = (count_for != pc || (uint64_t)M + bound > cap) ? 2 : 1;
  return ((status & ST_OVERFLOW) || !gate) ? 0 : fits;
}

// 0 = not served, 1 = run, 2 = would overflow (multi-instance form)
__device__ __forceinline__ int gate_state(const InstBuf& b, const InstDyn& d) {
  const Op* op = cur_op(b, d);
  if (!op) return 0;
  return gate_state_of(op->type, op->nrot, d.pc, d.status, d.count_for, d.M, d.live, d.count,
                       b.cap);
}

struct Smem {
  uint32_t tmp[kWaves + 1];
  uint32_t red[kWaves][8];   // block_sums: per-wave partial sums
  uint32_t base;
  uint32_t flag;
  uint64_t wfx[kWaves][3];
  // counts and expectation partial sum of this block's tiles of one
  // instance, kept by thread 0 and added to the instance once (flush);
  // pstat: a multi-rotation op's statistics (STAT_*)
  uint32_t plive, pcnt, pstat[kStatKinds];
  uint64_t pfx[3];
};

__device__ __forceinline__ void pend_reset(Smem& sm) {
  sm.plive = sm.pcnt = 0;
#pragma unroll
  for (int k = 0; k < kStatKinds; ++k) sm.pstat[k] = 0;
  sm.pfx[0] = sm.pfx[1] = sm.pfx[2] = 0;
}

// Block totals of N per-thread counters, for thread 0: each wave sums with
// lane exchanges, one barrier, then thread 0 adds the waves' sums (one
// barrier where N separate block reductions take 3N).  `trail` adds a
// barrier after the read, for callers with no barrier before their next
// call.
template <int N, bool trail = true>
__device__ __forceinline__ void block_sums(const uint32_t (&v)[N], Smem& sm, uint32_t (&out)[N]) {
  static_assert(N <= 8, "block_sums: at most 8 counters");
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    uint32_t x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += (uint32_t)__shfl_xor((int)x, o, 64);
    if (lane == 0) sm.red[wid][k] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      uint32_t t = 0;
      for (int w = 0; w < kWaves; ++w) t += sm.red[w][k];
      out[k] = t;
    }
  }
  if (trail) __syncthreads();
}

// Thread 0: adds the pending statistics and expectation sum to the instance
// and, unless the counts travel with the done count (`packed`), the pending
// live / anticommuting counts; resets them.
__device__ __forceinline__ void flush(const InstBuf& b, InstDyn& d, Smem& sm, uint32_t nsh,
                                      bool packed = false) {
#pragma unroll
  for (int k = 0; k < kStatKinds; ++k) add_stat(b, k, sm.pstat[k]);
  const uint64_t v = (uint64_t)sm.plive | ((uint64_t)sm.pcnt << 32);
  if (!packed && v) {
    unsigned long long* a = nsh == 1 ? (unsigned long long*)&d.acc
                                     : (unsigned long long*)&b.accs[(blockIdx.x % nsh) * kLineU64];
    consume(atomicAdd(a, (unsigned long long)v));
  }
  if (sm.pfx[0] | sm.pfx[1] | sm.pfx[2]) fx_atomic_add_wait(d.expect_fx, Fx{sm.pfx[0], sm.pfx[1], sm.pfx[2]});
  pend_reset(sm);
}

template <int IT>
__device__ __forceinline__ void gate_tile(const InstBuf& b, InstDyn& d, const GateArgs& g,
                                          const View& v, uint32_t M, uint32_t gen, uint32_t tile,
                                          Smem& sm) {
  uint32_t* s_tmp = sm.tmp;
  uint32_t* s_base = &sm.base;
  const int W = v.W;
  const double cs = g.cs[0], sn = g.sn[0], eps = g.eps;
  const int wmax = g.wmax;
  const bool full = g.full;
  const uint64_t* px = g.px[0];
  const uint64_t* pz = g.pz[0];
  const uint64_t* nxm = g.nx;
  const uint64_t* nzm = g.nz;
  const bool has_next = g.has_next;
  uint32_t my_live = 0, my_cnt = 0;
  uint64_t chx[IT][kMaxW], chz[IT][kMaxW];
  double chc[IT];
  bool chv[IT];

  auto tally = [&](const uint64_t* x, const uint64_t* z) {
    ++my_live;
    if (has_next && anticommutes(x, z, nxm, nzm, W)) ++my_cnt;
  };
  auto heavy = [&](const uint64_t* x, const uint64_t* z) {
    return wmax >= 0 && weight(x, z, W) > wmax;
  };

#pragma unroll
  for (int k = 0; k < IT; ++k) {
    chv[k] = false;
    const uint32_t i = tile * (kBlock * IT) + k * kBlock + threadIdx.x;
    if (i >= M) continue;
    // liveness, key and coefficient of entry i are loaded together (i < M <= cap)
    const uint8_t alive_i = v.al[i];
    uint64_t qx[kMaxW], qz[kMaxW];
    load_key(v, i, qx, qz);
    const double ci = v.getc(i);
    if (!alive_i) { v.aln[i] = 0; continue; }
    if (!anticommutes(qx, qz, px, pz, W)) {        // [P, Q] = 0: unchanged
      bool keep = true;
      if (full) keep = fabs(ci) >= eps && !heavy(qx, qz);
      v.aln[i] = keep ? 1 : 0;
      if (keep) tally(qx, qz);
      continue;
    }
    uint64_t rx[kMaxW], rz[kMaxW];
    PP_FOR_W(w, 0, W, kMaxW) { rx[w] = qx[w] ^ px[w]; rz[w] = qz[w] ^ pz[w]; }
    const int sig = product_sign(px, pz, qx, qz, rx, rz, W);   // i P Q = sig R
    double cj = 0.0;
    const int64_t j = gt_lookup(b, gen, M, v, rx, rz, &cj);
    if (j >= 0) {
      if ((uint32_t)j < i) continue;                 // the partner's thread leads
      // Both Q and R = PQ live: the gate acts on span{Q, R} as a rotation.
      // i P R = -sig Q.
      double nq, nr;
      rotate_pair(v.f32, cs, sn, sig, ci, cj, &nq, &nr);
      v.setc(i, nq);
      v.setc((uint32_t)j, nr);
      const bool kq = fabs(nq) >= eps && !(full && heavy(qx, qz));
      const bool kr = fabs(nr) >= eps && !(full && heavy(rx, rz));
      v.aln[i] = kq ? 1 : 0;
      v.aln[j] = kr ? 1 : 0;
      if (kq) tally(qx, qz);
      if (kr) tally(rx, rz);
    } else {
      double nq, child;
      rotate_single(v.f32, cs, sn, sig, ci, &nq, &child);
      v.setc(i, nq);
      const bool kq = fabs(nq) >= eps && !(full && heavy(qx, qz));
      v.aln[i] = kq ? 1 : 0;
      if (kq) tally(qx, qz);
      if (fabs(child) >= eps && !heavy(rx, rz)) {
        chv[k] = true;
        PP_FOR_W(w, 0, W, kMaxW) { chx[k][w] = rx[w]; chz[k][w] = rz[w]; }
        chc[k] = child;
        tally(rx, rz);
      }
    }
  }
  // append the new strings: one atomic per tile
  uint32_t mine = 0;
#pragma unroll
  for (int k = 0; k < IT; ++k) mine += chv[k] ? 1u : 0u;
  uint32_t total;
  uint32_t off = block_scan(mine, s_tmp, &total);
  if (threadIdx.x == 0) *s_base = total ? atomicAdd(&d.Mnext, total) : 0u;
  __syncthreads();
  const uint32_t base = *s_base;
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    if (!chv[k]) continue;
    const uint32_t pos = base + off++;
    if (pos >= v.cap) { atomicOr(&d.status, ST_OVERFLOW); continue; }   // guard
    PP_FOR_W(w, 0, W, kMaxW) {
      v.X[(size_t)w * v.cap + pos] = chx[k][w];
      v.Z[(size_t)w * v.cap + pos] = chz[k][w];
    }
    v.setc(pos, chc[k]);
    v.aln[pos] = 1;
    gt_insert(b.gtab, b.hg_bits, gen, pos, hash_key(chx[k], chz[k], W, 0));
  }
  // (the tile's append scan has its barriers before the next tile's sums)
  const uint32_t v2[2] = {my_live, my_cnt};
  uint32_t t2[2];
  block_sums<2, false>(v2, sm, t2);
  if (threadIdx.x == 0) {
    sm.plive += t2[0];
    sm.pcnt += t2[1];
  }
}

// K mutually commuting rotations P_1..P_K of a sub-layer in one pass
// (OP_GATES).  For a live Q, the strings Q * P^s (s a subset of the rotations
// that anticommute with Q; P^s their product) only mix among themselves
// under the K gates, and since the P_g commute every member shares Q's
// anticommutation with each P_g.  So the group's lowest-index live member
// applies gate 1, its exact merge and its truncation, then gate 2 and so on,
// to the whole group in registers: the same arithmetic in the same order as
// K one-gate passes, with one lookup round and one launch.  Member m (a bit
// mask over the rotations) exists when its bits are all anticommuting ones;
// gate g pairs members m and m | 2^g.  The host fuses only rotations whose
// strings are independent (no product of a nonempty subset is the
// identity), so the 2^K members are distinct.  New strings are appended
// after each row of the tile.
template <int IT, int K>
__device__ __forceinline__ void gates_tile(const InstBuf& b, InstDyn& d, const GateArgs& ga,
                                           const View& v, uint32_t M, uint32_t gen, uint32_t tile,
                                           Smem& sm) {
  constexpr int NM = 1 << K;
  uint32_t* s_tmp = sm.tmp;
  uint32_t* s_base = &sm.base;
  const int W = v.W;
  const double eps = ga.eps;
  const int wmax = ga.wmax;
  const bool full = ga.full;
  const uint64_t* nxm = ga.nx;
  const uint64_t* nzm = ga.nz;
  const bool has_next = ga.has_next;
  // my_lv / my_an: live terms after each rotation but the last, and those of
  // them anticommuting with the next rotation (summed over the rotations)
  uint32_t my_live = 0, my_cnt = 0, my_rw = 0, my_lv = 0, my_an = 0;

  auto heavy = [&](const uint64_t* x, const uint64_t* z) {
    return wmax >= 0 && weight(x, z, W) > wmax;
  };
  auto tally = [&](const uint64_t* x, const uint64_t* z) {
    ++my_live;
    if (has_next && anticommutes(x, z, nxm, nzm, W)) ++my_cnt;
  };

#pragma unroll
  for (int k = 0; k < IT; ++k) {
    uint64_t mx[NM][kMaxW], mz[NM][kMaxW];
    double c[NM];
    bool ex[NM], was[NM], pres[NM];
    int64_t idx[NM];
    bool an[K];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      ex[m] = was[m] = pres[m] = false;
      idx[m] = -1;
      c[m] = 0.0;
    }
#pragma unroll
    for (int g = 0; g < K; ++g) an[g] = false;
    const uint32_t i = tile * (kBlock * IT) + k * kBlock + threadIdx.x;
    bool lead = false;
    if (i < M) {
      const uint8_t alive_i = v.al[i];
      load_key(v, i, mx[0], mz[0]);
      c[0] = v.getc(i);
      if (!alive_i) {
        v.aln[i] = 0;
      } else {
        bool any = false;
#pragma unroll
        for (int g = 0; g < K; ++g) {
          an[g] = anticommutes(mx[0], mz[0], ga.px[g], ga.pz[g], W);
          any = any || an[g];
        }
        if (!any) {                        // untouched by every rotation
          bool keep = true;
          if (full) keep = fabs(c[0]) >= eps && !heavy(mx[0], mz[0]);
          v.aln[i] = keep ? 1 : 0;
          if (keep) {
            my_lv += K - 1;
            tally(mx[0], mz[0]);
          }
        } else {
#pragma unroll
          for (int m = 1; m < NM; ++m) {
            bool e = true;
#pragma unroll
            for (int g = 0; g < K; ++g)
              if ((m >> g) & 1) e = e && an[g];
            ex[m] = e;
            const int g0 = 31 - __clz(m);          // highest rotation in m
            const int rest = m & ~(1 << g0);       // m = rest | 2^g0, rest < m
            PP_FOR_W(w, 0, W, kMaxW) {
              mx[m][w] = mx[rest][w] ^ ga.px[g0][w];
              mz[m][w] = mz[rest][w] ^ ga.pz[g0][w];
            }
          }
          ex[0] = true;
          gt_lookup_n<NM - 1>(b, gen, M, v, &ex[1], &mx[1], &mz[1], &idx[1], &c[1]);
          idx[0] = i;
          was[0] = true;
          lead = true;
#pragma unroll
          for (int m = 1; m < NM; ++m) {
            was[m] = idx[m] >= 0;
            if (was[m] && (uint32_t)idx[m] < i) lead = false;   // a lower member leads
          }
        }
      }
    }
    if (lead) {
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        pres[m] = was[m];
        if (was[m]) ++my_rw;
      }
#pragma unroll
      for (int g = 0; g < K; ++g) {
        const bool chk = g == 0 && full;   // the sub-layer's first gate re-checks all
        if (!an[g]) {
          if (chk)
#pragma unroll
            for (int m = 0; m < NM; ++m)
              if (pres[m]) pres[m] = fabs(c[m]) >= eps && !heavy(mx[m], mz[m]);
        } else {
          const int step = 1 << g;
#pragma unroll
          for (int A = 0; A < NM; ++A) {
            if ((A & step) || !ex[A] || !ex[A + step]) continue;
            const int B = A + step;
            // i P_g A = sig B, and i P_g B = -sig A
            const int sig = product_sign(ga.px[g], ga.pz[g], mx[A], mz[A], mx[B], mz[B], W);
            if (pres[A] && pres[B]) {
              double nA, nB;
              rotate_pair(v.f32, ga.cs[g], ga.sn[g], sig, c[A], c[B], &nA, &nB);
              c[A] = nA;
              c[B] = nB;
              pres[A] = fabs(nA) >= eps && !(chk && heavy(mx[A], mz[A]));
              pres[B] = fabs(nB) >= eps && !(chk && heavy(mx[B], mz[B]));
            } else if (pres[A] || pres[B]) {
              const int S = pres[A] ? A : B, T = pres[A] ? B : A;   // source, new string
              double nS, child;
              rotate_single(v.f32, ga.cs[g], ga.sn[g], pres[A] ? sig : -sig, c[S], &nS, &child);
              c[S] = nS;
              pres[S] = fabs(nS) >= eps && !(chk && heavy(mx[S], mz[S]));
              if (fabs(child) >= eps && !heavy(mx[T], mz[T])) {
                c[T] = child;
                pres[T] = true;
              }
            }
          }
        }
        if (g < K - 1)
#pragma unroll
          for (int m = 0; m < NM; ++m)
            if (pres[m]) {
              ++my_lv;
              if (an[g + 1 < K ? g + 1 : 0]) ++my_an;
            }
      }
      // members that were live keep their slot; tally the survivors
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        if (was[m]) {
          v.setc((uint32_t)idx[m], c[m]);
          v.aln[idx[m]] = pres[m] ? 1 : 0;
        }
        if (pres[m]) tally(mx[m], mz[m]);
      }
    }
    // append the new members of this row: one atomic per block and row
    uint32_t mine = 0;
#pragma unroll
    for (int m = 1; m < NM; ++m) mine += (lead && pres[m] && !was[m]) ? 1u : 0u;
    uint32_t total;
    uint32_t off = block_scan(mine, s_tmp, &total);
    if (total) {
      if (threadIdx.x == 0) *s_base = atomicAdd(&d.Mnext, total);
      __syncthreads();
      const uint32_t base = *s_base;
#pragma unroll
      for (int m = 1; m < NM; ++m) {
        if (!(lead && pres[m] && !was[m])) continue;
        const uint32_t pos = base + off++;
        if (pos >= v.cap) { atomicOr(&d.status, ST_OVERFLOW); continue; }   // guard
        PP_FOR_W(w, 0, W, kMaxW) {
          v.X[(size_t)w * v.cap + pos] = mx[m][w];
          v.Z[(size_t)w * v.cap + pos] = mz[m][w];
        }
        v.setc(pos, c[m]);
        v.aln[pos] = 1;
        gt_insert(b.gtab, b.hg_bits, gen, pos, hash_key(mx[m], mz[m], W, 0));
      }
    }
  }
  // (every tile runs an append scan, whose barriers precede the next sums)
  const uint32_t v5[5] = {my_live, my_cnt, my_lv, my_an, my_rw};
  uint32_t t5[5];
  block_sums<5, false>(v5, sm, t5);
  if (threadIdx.x == 0) {
    sm.plive += t5[0];
    sm.pcnt += t5[1];
    sm.pstat[STAT_LIVE] += t5[2];
    sm.pstat[STAT_ANTI] += t5[3];
    sm.pstat[STAT_RW] += t5[4];
  }
}

// The same K-rotation op with one lane per group member: the 2^K lanes of a
// lane group hold the members Q * P^s of one term Q's group (lane index =
// s), so the lookups, signs, rotations and checks of a group run side by
// side and a rotation pairs lane s with lane s ^ 2^g through a lane
// exchange.  Every lane computes exactly the value the one-thread form
// computes for its member (the pair rotation from either side gives the same
// operations on the same operands), so the two forms agree bitwise.  A
// block covers kBlock / 2^K terms per row; IT rows are loaded before any
// append, and the new strings of all rows are appended with one atomic.
template <int IT, int K>
__device__ __forceinline__ void gates_lane_tile(const InstBuf& b, InstDyn& d, const GateArgs& ga,
                                                const View& v, uint32_t M, uint32_t gen,
                                                uint32_t tile, Smem& sm) {
  constexpr int G = 1 << K;
  constexpr uint32_t kRow = kBlock / G;      // terms per row of the tile
  uint32_t* s_tmp = sm.tmp;
  uint32_t* s_base = &sm.base;
  const int W = v.W;
  const double eps = ga.eps;
  const int wmax = ga.wmax;
  const bool full = ga.full;
  const int m = (int)(threadIdx.x & (G - 1));  // this lane's member
  uint32_t my_live = 0, my_cnt = 0, my_rw = 0, my_lv = 0, my_an = 0;
  uint64_t chx[IT][kMaxW], chz[IT][kMaxW];
  double chc[IT];
  bool chv[IT];

  auto heavy = [&](const uint64_t* x, const uint64_t* z) {
    return wmax >= 0 && weight(x, z, W) > wmax;
  };
  auto tally = [&](const uint64_t* x, const uint64_t* z) {
    ++my_live;
    if (ga.has_next && anticommutes(x, z, ga.nx, ga.nz, W)) ++my_cnt;
  };

#pragma unroll
  for (int k = 0; k < IT; ++k) {
    chv[k] = false;
    const uint32_t i = (tile * IT + k) * kRow + (threadIdx.x >> K);
    const bool valid = i < M;
    uint64_t qx[kMaxW], qz[kMaxW], mx[kMaxW], mz[kMaxW];
    PP_FOR_W(w, 0, W, kMaxW) { qx[w] = qz[w] = 0; }
    double cq = 0.0;
    uint8_t alive = 0;
    if (valid) {
      alive = v.al[i];
      load_key(v, i, qx, qz);
      cq = v.getc(i);
    }
    bool an[K], any = false, ex = alive != 0;
#pragma unroll
    for (int g = 0; g < K; ++g) {
      an[g] = anticommutes(qx, qz, ga.px[g], ga.pz[g], W);
      any = any || an[g];
      if ((m >> g) & 1) ex = ex && an[g];
    }
    ex = ex && any;
    PP_FOR_W(w, 0, W, kMaxW) { mx[w] = qx[w]; mz[w] = qz[w]; }
#pragma unroll
    for (int g = 0; g < K; ++g)
      if ((m >> g) & 1) PP_FOR_W(w, 0, W, kMaxW) { mx[w] ^= ga.px[g][w]; mz[w] ^= ga.pz[g][w]; }
    if (m == 0 && valid) {
      if (!alive) {
        v.aln[i] = 0;
      } else if (!any) {                     // untouched by every rotation
        bool keep = true;
        if (full) keep = fabs(cq) >= eps && !heavy(qx, qz);
        v.aln[i] = keep ? 1 : 0;
        if (keep) {
          my_lv += K - 1;
          tally(qx, qz);
        }
      }
    }
    int64_t idx = -1;
    double c = 0.0;
    if (ex) {
      if (m == 0) {
        idx = i;
        c = cq;
      } else {
        idx = gt_lookup(b, gen, M, v, mx, mz, &c);
      }
    }
    const bool was = idx >= 0;
    // the group's lowest live index leads it
    uint32_t low = was ? (uint32_t)idx : 0xFFFFFFFFu;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) low = min(low, (uint32_t)__shfl_xor((int)low, o, 64));
    const bool lead = ex && low == i;
    bool pres = lead && was;
    if (pres) ++my_rw;
#pragma unroll
    for (int g = 0; g < K; ++g) {
      const bool chk = g == 0 && full;      // the sub-layer's first gate re-checks all
      const double cp = __shfl_xor(c, 1 << g, 64);
      const bool pp = __shfl_xor((int)pres, 1 << g, 64) != 0;
      if (lead) {
        if (!an[g]) {
          if (chk && pres) pres = fabs(c) >= eps && !heavy(mx, mz);
        } else {
          uint64_t rx[kMaxW], rz[kMaxW];
          PP_FOR_W(w, 0, W, kMaxW) { rx[w] = mx[w] ^ ga.px[g][w]; rz[w] = mz[w] ^ ga.pz[g][w]; }
          const int sig = product_sign(ga.px[g], ga.pz[g], mx, mz, rx, rz, W);  // i P_g me = sig partner
          if (pres && pp) {
            double n0, n1;
            rotate_pair(v.f32, ga.cs[g], ga.sn[g], sig, c, cp, &n0, &n1);
            c = n0;
            pres = fabs(n0) >= eps && !(chk && heavy(mx, mz));
          } else if (pres) {
            double n0, child;
            rotate_single(v.f32, ga.cs[g], ga.sn[g], sig, c, &n0, &child);
            c = n0;
            pres = fabs(n0) >= eps && !(chk && heavy(mx, mz));
          } else if (pp) {                    // the partner's new string is me
            double n0, child;
            rotate_single(v.f32, ga.cs[g], ga.sn[g], -sig, cp, &n0, &child);
            if (fabs(child) >= eps && !heavy(mx, mz)) {
              c = child;
              pres = true;
            }
          }
        }
        if (g < K - 1 && pres) {
          ++my_lv;
          if (an[g + 1 < K ? g + 1 : 0]) ++my_an;
        }
      }
    }
    if (lead) {
      if (was) {
        v.setc((uint32_t)idx, c);
        v.aln[idx] = pres ? 1 : 0;
      } else if (pres) {
        chv[k] = true;
        PP_FOR_W(w, 0, W, kMaxW) { chx[k][w] = mx[w]; chz[k][w] = mz[w]; }
        chc[k] = c;
      }
      if (pres) tally(mx, mz);
    }
  }
  // append the new strings of all rows: one atomic per tile
  uint32_t mine = 0;
#pragma unroll
  for (int k = 0; k < IT; ++k) mine += chv[k] ? 1u : 0u;
  uint32_t total;
  uint32_t off = block_scan(mine, s_tmp, &total);
  if (total) {
    if (threadIdx.x == 0) *s_base = atomicAdd(&d.Mnext, total);
    __syncthreads();
    const uint32_t base = *s_base;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      if (!chv[k]) continue;
      const uint32_t pos = base + off++;
      if (pos >= v.cap) { atomicOr(&d.status, ST_OVERFLOW); continue; }   // guard
      PP_FOR_W(w, 0, W, kMaxW) {
        v.X[(size_t)w * v.cap + pos] = chx[k][w];
        v.Z[(size_t)w * v.cap + pos] = chz[k][w];
      }
      v.setc(pos, chc[k]);
      v.aln[pos] = 1;
      gt_insert(b.gtab, b.hg_bits, gen, pos, hash_key(chx[k], chz[k], W, 0));
    }
  }
  // (every tile runs an append scan, whose barriers precede the next sums)
  const uint32_t v5[5] = {my_live, my_cnt, my_lv, my_an, my_rw};
  uint32_t t5[5];
  block_sums<5, false>(v5, sm, t5);
  if (threadIdx.x == 0) {
    sm.plive += t5[0];
    sm.pcnt += t5[1];
    sm.pstat[STAT_LIVE] += t5[2];
    sm.pstat[STAT_ANTI] += t5[3];
    sm.pstat[STAT_RW] += t5[4];
  }
}

// ---------------------------------------------------------------------------
// Kernel kinds.  Each kind provides
//   state(b, d)   0: instance not served by this kernel now, 1: run,
//                 2: would overflow (gate only: mark and skip);
//   elems(b, d)   number of elements the tiles cover;
//   tile<IT>()    the work of one tile of kBlock * IT elements;
//   finish()      run by every thread of the last block, per served
//                 instance: fold the accumulators, advance pc.
// run_multi serves a list of instances (batched form); run_solo serves one
// instance whose current op index is a launch argument, so a captured
// sequence of solo launches replays a fixed list of operations.
// ---------------------------------------------------------------------------
// Launch argument of the one-instance kernels.  The instance's buffer
// descriptor travels by value (kernel-argument loads, no dependent global
// load before the program can be read).
struct Solo {
  InstBuf b;
  InstDyn* d;
  uint32_t* sync;
  uint32_t k;          // index of the op this launch executes
};

// next gate's Pauli string, for the anticommutation count that bounds the
// next gate's appends
struct NextGate {
  bool has;
  uint64_t x[kMaxW], z[kMaxW];
  __device__ NextGate(const InstBuf& b, const Op& op) {
    has = op.next_gate != kNone32;
    PP_FOR_W(w, 0, b.W, kMaxW) { x[w] = op.nx[w]; z[w] = op.nz[w]; }
  }
  __device__ __forceinline__ bool anti(const uint64_t* qx, const uint64_t* qz, int W) const {
    return has && anticommutes(qx, qz, x, z, W);
  }
};

__device__ __forceinline__ void add_counts(InstDyn&, uint32_t live, uint32_t cnt, Smem& sm) {
  const uint32_t v2[2] = {live, cnt};
  uint32_t t2[2];
  block_sums<2>(v2, sm, t2);
  if (threadIdx.x == 0) {
    sm.plive += t2[0];
    sm.pcnt += t2[1];
  }
}

// Mode 0 runs any gate op (the multi-instance kernel, whose instances may
// stand at any); the one-instance kernels are built per rotation count
// (Mode = 1, 2 or 3), so each keeps only the registers it needs.
__device__ __forceinline__ uint32_t rotations_of(const Op& op) {
  return op.type == OP_GATES ? op.nrot : 1u;
}

template <int Mode, int IT>
__device__ __forceinline__ void gate_tile_any(const InstBuf& b, InstDyn& d, const GateArgs& g,
                                              const View& v, uint32_t M, uint32_t gen, uint32_t t,
                                              Smem& sm) {
  if (Mode == 1 || (Mode == 0 && g.nrot == 1))
    gate_tile<IT>(b, d, g, v, M, gen, t, sm);
  else if (Mode == 2 || (Mode == 0 && g.nrot == 2))
    gates_tile<IT, 2>(b, d, g, v, M, gen, t, sm);
  else
    gates_tile<IT, 3>(b, d, g, v, M, gen, t, sm);
}

template <int Mode>
struct GateKindT {
  __device__ __forceinline__ static bool needs_fence(const InstBuf&, const InstDyn&) { return false; }
  __device__ __forceinline__ static int state(const InstBuf& b, const InstDyn& d) {
    const int st = gate_state(b, d);
    if (Mode && st && rotations_of(b.prog[d.pc]) != (uint32_t)Mode) return 0;
    return st;
  }
  __device__ __forceinline__ static uint32_t elems(const InstBuf&, const InstDyn& d) { return d.M; }
  template <int IT>
  __device__ __forceinline__ static void tile(const InstBuf& b, InstDyn& d, uint32_t t, Smem& sm) {
    const GateArgs g = gate_args(b.prog[d.pc]);
    const View v = view_of(b, d);
    gate_tile_any<Mode, IT>(b, d, g, v, d.M, d.gen, t, sm);
  }
  __device__ __forceinline__ static void finish(const InstBuf& b, InstDyn& d, uint32_t, Smem&) {
    const Op& op = b.prog[d.pc];
    d.propagated += d.live;
    d.merged += (uint64_t)d.live + d.count;
    d.anti_total += d.count;
    d.key_reads += d.live;
    // a multi-rotation op's later rotations and rewritten coefficients
    // went to the statistics lines
    if (rotations_of(op) == 1) d.coef_rw += d.count;
    d.appended += ld_agent(&d.Mnext) - d.M;
    d.M = ld_agent(&d.Mnext);
    d.Mnext = d.M;
    if (d.M > d.peak) d.peak = d.M;
    d.parity ^= 1u;
    take_acc(d);
    d.count_for = op.next_gate;
    next_op(b, d);
  }
};

// MERGE, narrow keys: one pass, representative -> hash table -> exact sums
__device__ __forceinline__ bool merge_served(const InstBuf& b, const InstDyn& d, bool narrow,
                                    uint32_t phase) {
  if (d.status & ST_OVERFLOW) return false;
  const Op* op = cur_op(b, d);
  if (!op || op->type != OP_MERGE) return false;
  if (b.group == 0 && !op->force_full) return false;   // plain PP: compaction
  return (b.narrow != 0) == narrow && d.mphase == phase;
}

// The partitioned merge (pp_merge.hpp) takes large narrow-key merges (not S_n).
__device__ __forceinline__ bool use_part(const InstBuf& b, const InstDyn& d) {
  return b.pstage != nullptr && !b.nopart && b.narrow && b.group != 2 && d.M >= kPartMin;
}


struct MergeNarrowKind {
  __device__ __forceinline__ static bool needs_fence(const InstBuf&, const InstDyn&) { return false; }
  __device__ __forceinline__ static int state(const InstBuf& b, const InstDyn& d) {
    return (merge_served(b, d, true, 0) && !use_part(b, d)) ? 1 : 0;
  }
  __device__ __forceinline__ static uint32_t elems(const InstBuf&, const InstDyn& d) { return d.M; }
  template <int IT>
  __device__ __forceinline__ static void tile(const InstBuf& b, InstDyn& d, uint32_t t, Smem&) {
    const View v = view_of(b, d);
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const uint32_t i = t * (kBlock * IT) + k * kBlock + threadIdx.x;
      const bool act = i < d.M && v.al[i];
      uint64_t key = 0;
      Fx c{0, 0, 0};
      bool range = false;
      if (act) {
        uint64_t qx[kMaxW], qz[kMaxW];
        load_key(v, i, qx, qz);
        key = narrow_key(b, qx, qz);
        c = fx_from_double(v.getc(i), &range);
      }
      if (range) atomicOr(&d.status, ST_RANGE);
      wave_merge_add(b, d, act, key, c);
    }
  }
  __device__ __forceinline__ static void finish(const InstBuf&, InstDyn& d, uint32_t, Smem&) {
    d.merged += d.live;
    d.mphase = 1;
  }
};

// MERGE, wide keys: (1) representative + 64-bit hash slot, (2) the first
// record of each slot owns it; every record compares its representative with
// the owner's (a mismatch is a hash collision: the merge restarts with
// another seed) and adds its coefficient.
struct MergeWide1Kind {
  __device__ __forceinline__ static bool needs_fence(const InstBuf&, const InstDyn&) { return false; }
  __device__ __forceinline__ static int state(const InstBuf& b, const InstDyn& d) {
    return merge_served(b, d, false, 0) ? 1 : 0;
  }
  __device__ __forceinline__ static uint32_t elems(const InstBuf&, const InstDyn& d) { return d.M; }
  template <int IT>
  __device__ __forceinline__ static void tile(const InstBuf& b, InstDyn& d, uint32_t t, Smem&) {
    const View v = view_of(b, d);
    const int W = b.W;
    const uint64_t seed = d.seed;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const uint32_t i = t * (kBlock * IT) + k * kBlock + threadIdx.x;
      if (i >= d.M) continue;
      if (!v.al[i]) { b.wslot[i] = kNone32; continue; }
      uint64_t qx[kMaxW], qz[kMaxW], rx[kMaxW], rz[kMaxW];
      load_key(v, i, qx, qz);
      rep_string(b, qx, qz, rx, rz);
      PP_FOR_W(w, 0, W, kMaxW) {
        b.wrep[(size_t)w * b.cap + i] = rx[w];
        b.wrep[(size_t)(W + w) * b.cap + i] = rz[w];
      }
      uint64_t h = hash_key(rx, rz, W, seed);
      if (h == kEmpty64) h -= 1;
      b.wslot[i] = (uint32_t)mt_slot(b.mkey, merge_bits(b, d), h);
    }
  }
  __device__ __forceinline__ static void finish(const InstBuf&, InstDyn& d, uint32_t, Smem&) {
    d.merged += d.live;
    d.mphase = 1;
  }
};

struct MergeWide2Kind {
  __device__ __forceinline__ static bool needs_fence(const InstBuf&, const InstDyn&) { return false; }
  __device__ __forceinline__ static int state(const InstBuf& b, const InstDyn& d) {
    return merge_served(b, d, false, 1) ? 1 : 0;
  }
  __device__ __forceinline__ static uint32_t elems(const InstBuf&, const InstDyn& d) { return d.M; }
  template <int IT>
  __device__ __forceinline__ static void tile(const InstBuf& b, InstDyn& d, uint32_t t, Smem&) {
    const View v = view_of(b, d);
    const int W = b.W;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const uint32_t i = t * (kBlock * IT) + k * kBlock + threadIdx.x;
      if (i >= d.M) continue;
      const uint32_t s = b.wslot[i];
      if (s == kNone32) continue;
      const uint32_t o = atomicCAS(&b.mown[s], kNone32, i);
      const uint32_t owner = (o == kNone32) ? i : o;
      bool same = true;
      if (owner != i)
        PP_FOR_W(w, 0, 2 * W, 2 * kMaxW)
          same = same && b.wrep[(size_t)w * b.cap + i] == b.wrep[(size_t)w * b.cap + owner];
      if (same) {
        bool range = false;
        fx_atomic_add(&b.mfx[3 * (size_t)s], fx_from_double(v.getc(i), &range));
        if (range) atomicOr(&d.status, ST_RANGE);
      } else {
        atomicOr(&d.status, ST_COLLISION);
      }
    }
  }
  __device__ __forceinline__ static void finish(const InstBuf&, InstDyn& d, uint32_t, Smem&) {
    d.mphase = 2;
  }
};

// A merge that carries its sub-layer's truncation emits a term only if the
// coefficient as stored (FP32-rounded in FP32 mode) is at least eps and the
// weight at most wmax, exactly what a truncation pass after the merge keeps.
__device__ __forceinline__ bool merge_keeps(const InstBuf& b, const Op& op, const uint64_t* x,
                                            const uint64_t* z, double c) {
  if (!op.trunc) return true;
  const double cs = b.f32 ? (double)(float)c : c;
  return fabs(cs) >= op.eps && !(op.wmax >= 0 && weight(x, z, b.W) > op.wmax);
}

// Writes one output term at the cursor position `pos` of the other half.
__device__ __forceinline__ void emit_term(const InstBuf& b, const InstDyn& d, uint32_t pos,
                                 const uint64_t* x, const uint64_t* z, double c) {
  const uint32_t h = d.half ^ 1u;
  const int W = b.W;
  PP_FOR_W(w, 0, W, kMaxW) {
    b.x[h][(size_t)w * b.cap + pos] = x[w];
    b.z[h][(size_t)w * b.cap + pos] = z[w];
  }
  if (b.f32)
    static_cast<float*>(b.c[h])[pos] = (float)c;
  else
    static_cast<double*>(b.c[h])[pos] = c;
  b.alive[h][0][pos] = 1;
  b.alive[h][1][pos] = 1;
  gt_insert(b.gtab, b.hg_bits, d.gen + 1, pos, hash_key(x, z, W, 0));
}

// After a merge or compaction: the other half becomes current.
__device__ __forceinline__ void finish_rebuild(const InstBuf& b, InstDyn& d) {
  const Op& op = b.prog[d.pc];
  d.merge_in += d.live;
  d.merge_out += d.nuniq;
  d.M = d.nuniq;
  d.Mnext = d.M;
  d.half ^= 1u;
  d.parity = 0;
  d.gen += 1;
  take_acc(d);
  d.count_for = op.next_gate;
  d.nuniq = 0;
  d.mphase = 0;
  d.pglobal = 0;
  d.plist_n = 0;
  next_op(b, d);
}

// Collect: every occupied merge slot becomes one representative of the new
// half; slots are cleared for the next merge.
struct CollectKind {
  __device__ __forceinline__ static bool needs_fence(const InstBuf&, const InstDyn&) { return false; }
  __device__ __forceinline__ static int state(const InstBuf& b, const InstDyn& d) {
    return (merge_served(b, d, true, 1) || merge_served(b, d, false, 2)) ? 1 : 0;
  }
  // after a partitioned merge only the listed slots (keys of split or
  // overfull buckets) are occupied
  __device__ __forceinline__ static bool listed(const InstBuf& b, const InstDyn& d) {
    return b.narrow && use_part(b, d);
  }
  __device__ __forceinline__ static uint32_t elems(const InstBuf& b, const InstDyn& d) {
    if (listed(b, d)) return d.pglobal ? d.plist_n : 0u;
    return 1u << merge_bits(b, d);
  }
  template <int IT>
  __device__ __forceinline__ static void tile(const InstBuf& b, InstDyn& d, uint32_t t, Smem& sm) {
    const bool collided = (d.status & ST_COLLISION) != 0;
    const bool lst = listed(b, d);
    const uint32_t nslots = lst ? d.plist_n : 1u << merge_bits(b, d);
    const int W = b.W;
    const Op& mop = b.prog[d.pc];
    const NextGate ng(b, mop);
    uint64_t ox[IT][kMaxW], oz[IT][kMaxW];
    double oc[IT];
    bool ov[IT];
    uint32_t mine = 0, my_cnt = 0;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      ov[k] = false;
      const uint32_t e = t * (kBlock * IT) + k * kBlock + threadIdx.x;
      if (e >= nslots) continue;
      const uint32_t s = lst ? b.plist[e] : e;
      const uint64_t key = b.mkey[s];
      if (key == kEmpty64) continue;
      if (!collided) {
        if (b.narrow) {
          narrow_decode(b, key, ox[k], oz[k]);
        } else {
          const uint32_t o = b.mown[s];
          PP_FOR_W(w, 0, W, kMaxW) {
            ox[k][w] = b.wrep[(size_t)w * b.cap + o];
            oz[k][w] = b.wrep[(size_t)(W + w) * b.cap + o];
          }
        }
        const Fx f{b.mfx[3 * (size_t)s], b.mfx[3 * (size_t)s + 1], b.mfx[3 * (size_t)s + 2]};
        oc[k] = fx_to_double(f);
        ov[k] = merge_keeps(b, mop, ox[k], oz[k], oc[k]);
        if (ov[k]) {
          ++mine;
          if (ng.anti(ox[k], oz[k], W)) ++my_cnt;
        }
      }
      b.mkey[s] = kEmpty64;
      b.mfx[3 * (size_t)s] = 0;
      b.mfx[3 * (size_t)s + 1] = 0;
      b.mfx[3 * (size_t)s + 2] = 0;
      if (!b.narrow) b.mown[s] = kNone32;
    }
    uint32_t tot;
    uint32_t off = block_scan(mine, sm.tmp, &tot);
    if (threadIdx.x == 0) sm.base = tot ? atomicAdd(&d.nuniq, tot) : 0u;
    __syncthreads();
    const uint32_t base = sm.base;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      if (!ov[k]) continue;
      const uint32_t pos = base + off++;
      if (pos >= b.cap) { atomicOr(&d.status, ST_OVERFLOW); continue; }
      emit_term(b, d, pos, ox[k], oz[k], oc[k]);
    }
    add_counts(d, mine, my_cnt, sm);
  }
  __device__ __forceinline__ static void finish(const InstBuf& b, InstDyn& d, uint32_t, Smem&) {
    if (d.status & ST_COLLISION) {     // retry this merge with another seed
      d.status &= ~ST_COLLISION;
      d.special = 0;
      d.special_fx[0] = d.special_fx[1] = d.special_fx[2] = 0;
      d.seed += 1;
      d.mphase = 0;
      d.nuniq = 0;
      d.acc = 0;
      return;
    }
    d.nuniq = ld_agent(&d.nuniq);
    if (d.special) {                   // narrow key equal to the empty marker
      uint64_t x[kMaxW], z[kMaxW];
      narrow_decode(b, kEmpty64, x, z);
      const uint32_t pos = d.nuniq;
      const Fx f{d.special_fx[0], d.special_fx[1], d.special_fx[2]};
      const double c = fx_to_double(f);
      if (!merge_keeps(b, b.prog[d.pc], x, z, c)) {
        // truncated with the merge
      } else if (pos < b.cap) {
        emit_term(b, d, pos, x, z, c);
        d.nuniq = pos + 1;
        const NextGate ng(b, b.prog[d.pc]);
        d.acc += 1ull + (ng.anti(x, z, b.W) ? (1ull << 32) : 0ull);
      } else {
        d.status |= ST_OVERFLOW;
      }
      d.special = 0;
      d.special_fx[0] = d.special_fx[1] = d.special_fx[2] = 0;
    }
    finish_rebuild(b, d);
  }
};

// MERGE for plain PP: the set is already free of duplicates, so the merge
// only drops dead entries (compaction into the other half).
__device__ __forceinline__ bool compact_served(const InstBuf& b, const InstDyn& d) {
  if (d.status & ST_OVERFLOW) return false;
  const Op* op = cur_op(b, d);
  return op && op->type == OP_MERGE && b.group == 0 && !op->force_full;
}

struct CompactKind {
  __device__ __forceinline__ static bool needs_fence(const InstBuf&, const InstDyn&) { return false; }
  __device__ __forceinline__ static int state(const InstBuf& b, const InstDyn& d) {
    return compact_served(b, d) ? 1 : 0;
  }
  __device__ __forceinline__ static uint32_t elems(const InstBuf&, const InstDyn& d) { return d.M; }
  template <int IT>
  __device__ __forceinline__ static void tile(const InstBuf& b, InstDyn& d, uint32_t t, Smem& sm) {
    const View v = view_of(b, d);
    const int W = b.W;
    const Op& mop = b.prog[d.pc];
    const NextGate ng(b, mop);
    bool ov[IT];
    uint32_t mine = 0, my_cnt = 0;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const uint32_t i = t * (kBlock * IT) + k * kBlock + threadIdx.x;
      ov[k] = i < d.M && v.al[i];
      if (ov[k] && mop.trunc) {            // the merge's truncation
        uint64_t x[kMaxW], z[kMaxW];
        load_key(v, i, x, z);
        ov[k] = merge_keeps(b, mop, x, z, v.getc(i));
      }
      mine += ov[k] ? 1u : 0u;
    }
    uint32_t tot;
    uint32_t off = block_scan(mine, sm.tmp, &tot);
    if (threadIdx.x == 0) sm.base = tot ? atomicAdd(&d.nuniq, tot) : 0u;
    __syncthreads();
    const uint32_t base = sm.base;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      if (!ov[k]) continue;
      const uint32_t i = t * (kBlock * IT) + k * kBlock + threadIdx.x;
      const uint32_t pos = base + off++;
      if (pos >= b.cap) { atomicOr(&d.status, ST_OVERFLOW); continue; }
      uint64_t x[kMaxW], z[kMaxW];
      load_key(v, i, x, z);
      emit_term(b, d, pos, x, z, v.getc(i));
      if (ng.anti(x, z, W)) ++my_cnt;
    }
    add_counts(d, mine, my_cnt, sm);
  }
  __device__ __forceinline__ static void finish(const InstBuf& b, InstDyn& d, uint32_t, Smem&) {
    d.merged += d.live;
    d.nuniq = ld_agent(&d.nuniq);
    finish_rebuild(b, d);
  }
};

// DAMP / TRUNC / COUNT / EXPECT: one streaming pass over the live terms
__device__ __forceinline__ bool scan_served(const InstBuf& b, const InstDyn& d) {
  if (d.status & ST_OVERFLOW) return false;
  const Op* op = cur_op(b, d);
  if (!op) return false;
  return op->type == OP_DAMP || op->type == OP_TRUNC || op->type == OP_COUNT ||
         op->type == OP_EXPECT;
}

struct ScanKind {
  __device__ __forceinline__ static bool needs_fence(const InstBuf&, const InstDyn&) { return false; }
  __device__ __forceinline__ static int state(const InstBuf& b, const InstDyn& d) {
    return scan_served(b, d) ? 1 : 0;
  }
  __device__ __forceinline__ static uint32_t elems(const InstBuf&, const InstDyn& d) { return d.M; }
  template <int IT>
  __device__ __forceinline__ static void tile(const InstBuf& b, InstDyn& d, uint32_t t, Smem& sm) {
    const View v = view_of(b, d);
    const int W = b.W, n = b.n;
    const Op& op = b.prog[d.pc];
    const uint32_t type = op.type;
    const NextGate ng(b, op);
    uint32_t my_live = 0, my_cnt = 0;
    Fx acc{0, 0, 0};
    bool range = false;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const uint32_t i = t * (kBlock * IT) + k * kBlock + threadIdx.x;
      if (i >= d.M || !v.al[i]) continue;
      uint64_t x[kMaxW], z[kMaxW];
      load_key(v, i, x, z);
      double c = v.getc(i);
      if (type == OP_DAMP) {
        const double f = op.table[weight(x, z, W)];
        c = v.f32 ? (double)((float)c * (float)f) : c * f;
        v.setc(i, c);
      } else if (type == OP_TRUNC) {
        const bool keep = fabs(c) >= op.eps && !(op.wmax >= 0 && weight(x, z, W) > op.wmax);
        if (!keep) { v.al[i] = 0; continue; }
      } else if (type == OP_EXPECT) {
        uint32_t nx, ny, nz;
        perm_counts(x, z, W, &nx, &ny, &nz);
        const double term =
            c * op.table[nx] * op.table[(n + 1) + ny] * op.table[2 * (n + 1) + nz];
        acc = fx_add(acc, fx_from_double(term, &range));
      }
      ++my_live;
      if (ng.anti(x, z, W)) ++my_cnt;
    }
    if (type == OP_EXPECT) {          // exact sum: integer limbs, any order
      if (range) atomicOr(&d.status, ST_RANGE);
      const Fx w = wave_sum_fx(acc);
      const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
      if (lane == 0) { sm.wfx[wid][0] = w.l0; sm.wfx[wid][1] = w.l1; sm.wfx[wid][2] = w.l2; }
      __syncthreads();
      if (threadIdx.x == 0) {
        Fx s{sm.pfx[0], sm.pfx[1], sm.pfx[2]};
        for (int q = 0; q < kWaves; ++q) s = fx_add(s, Fx{sm.wfx[q][0], sm.wfx[q][1], sm.wfx[q][2]});
        sm.pfx[0] = s.l0;
        sm.pfx[1] = s.l1;
        sm.pfx[2] = s.l2;
      }
      __syncthreads();
    }
    add_counts(d, my_live, my_cnt, sm);
  }
  __device__ __forceinline__ static void finish(const InstBuf& b, InstDyn& d, uint32_t, Smem&) {
    const Op& op = b.prog[d.pc];
    if (op.type == OP_EXPECT) {
      const Fx f{ld_agent(&d.expect_fx[0]), ld_agent(&d.expect_fx[1]),
                 ld_agent(&d.expect_fx[2])};
      d.expect = fx_to_double(f);
      d.expect_fx[0] = d.expect_fx[1] = d.expect_fx[2] = 0;
    }
    take_acc(d);
    d.count_for = op.next_gate;
    next_op(b, d);
  }
};

// ---------------------------------------------------------------------------
// runners
// ---------------------------------------------------------------------------
template <class K, int IT>
__device__ __forceinline__ void run_multi(const Ctx& C, Smem& sm, uint32_t* s_pref) {
  const int ninst = *C.ninst;
  const uint32_t total = plan_tiles(ninst, [&](int i) -> uint32_t {
    const InstBuf& b = *C.bufs[i];
    const InstDyn& d = *C.dyns[i];
    return K::state(b, d) == 1 ? ceil_tiles<IT>(K::elems(b, d)) : 0u;
  }, s_pref, sm.tmp);
  const uint32_t workers = worker_count(total);
  if (blockIdx.x >= workers) return;
  const uint32_t nsh = acc_shards(workers);
  if (threadIdx.x == 0) pend_reset(sm);
  int cur = -1;                            // instance of the pending counts
  for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_inst(s_pref, ninst, t);
    if (i != cur) {
      if (cur >= 0 && threadIdx.x == 0) flush(*C.bufs[cur], *C.dyns[cur], sm, nsh);
      cur = i;
    }
    K::template tile<IT>(*C.bufs[i], *C.dyns[i], t - s_pref[i], sm);
  }
  if (cur >= 0 && threadIdx.x == 0) flush(*C.bufs[cur], *C.dyns[cur], sm, nsh);
  if (!last_block(C.sync, &sm.flag, workers, true)) return;
  // one thread per instance: each finish touches only its own instance
  for (int i = threadIdx.x; i < ninst; i += kBlock) {
    const InstBuf& b = *C.bufs[i];
    InstDyn& d = *C.dyns[i];
    const int st = K::state(b, d);
    if (st == 2) {
      d.status |= ST_OVERFLOW;
      d.failed_pc = d.pc;
      continue;
    }
    if (st != 1) continue;
    fold_acc(b, d, nsh);
    K::finish(b, d, ceil_tiles<IT>(K::elems(b, d)), sm);
  }
}

template <class K, int IT>
__device__ __forceinline__ void run_solo(const Solo& S, Smem& sm) {
  const InstBuf& b = S.b;
  InstDyn& d = *S.d;
  if (d.pc != S.k) return;                 // an earlier op did not complete
  const int st = K::state(b, d);
  if (st == 2) {
    if (blockIdx.x == 0 && threadIdx.x == 0) { d.status |= ST_OVERFLOW; d.failed_pc = d.pc; }
    return;
  }
  if (st != 1) return;
  const uint32_t tiles = ceil_tiles<IT>(K::elems(b, d));
  const uint32_t workers = worker_count(tiles);
  if (blockIdx.x >= workers) return;
  const uint32_t nsh = acc_shards(workers);
  const bool packed = workers <= kTreeMin && b.cap < kPackedCap;
  const bool fence = K::needs_fence(b, d);
  if (threadIdx.x == 0) pend_reset(sm);
  for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) K::template tile<IT>(b, d, t, sm);
  if (packed) {
    if (fence) __syncthreads();            // the block's stores precede its count
    if (threadIdx.x != 0) return;
    const uint32_t live = sm.plive, cnt = sm.pcnt;
    flush(b, d, sm, nsh, true);
    uint64_t acc;
    if (!last_block_packed(S.sync, workers, live, cnt, fence, &acc)) return;
    d.acc += acc;                          // onto what earlier launches of the op left
    K::finish(b, d, tiles, sm);
    return;
  }
  if (threadIdx.x == 0) flush(b, d, sm, nsh);
  if (!last_block(S.sync, &sm.flag, workers, fence)) return;
  if (threadIdx.x == 0) {
    fold_acc(b, d, nsh);
    K::finish(b, d, tiles, sm);
  }
}

// One-instance gate launch of a Mode-rotation op.  Everything that decides
// whether and how the launch works (the op, which the launch argument names,
// and the instance's state) is read up front, so the op's loads do not wait
// for the program counter; the term loads then wait for one round trip.
template <int Mode, int IT, bool Lane = false>
__device__ __forceinline__ void run_gate_solo(const Solo& S, Smem& sm) {
  const InstBuf& b = S.b;
  InstDyn& d = *S.d;
  const GateArgs g = gate_args(b.prog[S.k]);    // S.k < prog_len
  const uint32_t pc = d.pc, status = d.status, count_for = d.count_for, M = d.M;
  const uint32_t live = d.live, count = d.count, gen = d.gen;
  const View v = view_of(b, d);
  // one decision from all of them (no branch before every load is issued:
  // the op's fields are waited on here, together with the state);
  // pc != S.k: an earlier op did not complete
  uint64_t all = __double_as_longlong(g.cs[0]) ^ __double_as_longlong(g.sn[0]) ^
                 __double_as_longlong(g.cs[1]) ^ __double_as_longlong(g.sn[1]) ^
                 __double_as_longlong(g.eps) ^ (uint64_t)g.wmax;
#pragma unroll
  for (int w = 0; w < kMaxW; ++w)
    all ^= g.px[0][w] ^ g.pz[0][w] ^ g.px[1][w] ^ g.pz[1][w] ^ g.nx[w] ^ g.nz[w];
  consume(all);
  int st = gate_state_of(g.type, g.nrot, pc, status, count_for, M, live, count, b.cap);
  st = (pc == S.k && g.nrot == (uint32_t)Mode) ? st : 0;
  if (st == 2) {
    if (blockIdx.x == 0 && threadIdx.x == 0) { d.status |= ST_OVERFLOW; d.failed_pc = pc; }
    return;
  }
  if (st != 1) return;
  // lane form: kBlock / 2^Mode terms per row
  const uint32_t tiles = Lane ? (uint32_t)(((uint64_t)M * (1u << Mode) + kBlock * IT - 1) / (kBlock * IT))
                              : ceil_tiles<IT>(M);
  const uint32_t workers = worker_count(tiles);
  if (blockIdx.x >= workers) return;
  const uint32_t nsh = acc_shards(workers);
  const bool packed = workers <= kTreeMin && b.cap < kPackedCap;
  if (threadIdx.x == 0) pend_reset(sm);
  for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    if constexpr (Lane)
      gates_lane_tile<IT, (Mode > 1 ? Mode : 2)>(b, d, g, v, M, gen, t, sm);
    else
      gate_tile_any<Mode, IT>(b, d, g, v, M, gen, t, sm);
  }
  if (threadIdx.x != 0) return;            // thread 0 holds the block's counts
  if (packed) {
    const uint32_t live = sm.plive, cnt = sm.pcnt;
    flush(b, d, sm, nsh, true);
    uint64_t acc;
    if (!last_block_packed(S.sync, workers, live, cnt, false, &acc)) return;
    d.acc += acc;                          // onto what earlier launches of the op left
    GateKindT<Mode>::finish(b, d, tiles, sm);
    return;
  }
  flush(b, d, sm, nsh);
  if (!last_block_one(S.sync, workers)) return;
  fold_acc(b, d, nsh);
  GateKindT<Mode>::finish(b, d, tiles, sm);
}

#define PP_KERNEL_PAIR(name, Kind)                                                    \
  template <int IT>                                                                  \
  __global__ __launch_bounds__(kBlock) void name(Ctx C) {                             \
    __shared__ uint32_t s_pref[kMaxInst];                                            \
    __shared__ Smem sm;                                                              \
    run_multi<Kind, IT>(C, sm, s_pref);                                              \
  }                                                                                  \
  template <int IT>                                                                  \
  __global__ __launch_bounds__(kBlock) void name##_solo(Solo S) {                     \
    __shared__ Smem sm;                                                              \
    run_solo<Kind, IT>(S, sm);                                                       \
  }

using GateKind = GateKindT<0>;
template <int IT>
__global__ __launch_bounds__(kBlock) void k_gate(Ctx C) {
  __shared__ uint32_t s_pref[kMaxInst];
  __shared__ Smem sm;
  run_multi<GateKind, IT>(C, sm, s_pref);
}
template <int IT>
__global__ __launch_bounds__(kBlock) void k_gate_solo(Solo S) {
  __shared__ Smem sm;
  run_gate_solo<1, IT>(S, sm);
}
template <int IT>
__global__ __launch_bounds__(kBlock) void k_gate2_solo(Solo S) {
  __shared__ Smem sm;
  run_gate_solo<2, IT>(S, sm);
}
template <int IT>
__global__ __launch_bounds__(kBlock) void k_gate3_solo(Solo S) {
  __shared__ Smem sm;
  run_gate_solo<3, IT>(S, sm);
}
// lane forms of the multi-rotation ops (smaller sets)
template <int IT>
__global__ __launch_bounds__(kBlock) void k_gate2_lane_solo(Solo S) {
  __shared__ Smem sm;
  run_gate_solo<2, IT, true>(S, sm);
}
template <int IT>
__global__ __launch_bounds__(kBlock) void k_gate3_lane_solo(Solo S) {
  __shared__ Smem sm;
  run_gate_solo<3, IT, true>(S, sm);
}
PP_KERNEL_PAIR(k_merge_narrow, MergeNarrowKind)
PP_KERNEL_PAIR(k_merge_wide1, MergeWide1Kind)
PP_KERNEL_PAIR(k_merge_wide2, MergeWide2Kind)
PP_KERNEL_PAIR(k_merge_collect, CollectKind)
PP_KERNEL_PAIR(k_compact, CompactKind)
PP_KERNEL_PAIR(k_scan_op, ScanKind)

// ---------------------------------------------------------------------------
// Initial state of a new store's tables, in one launch (grid-stride): gate
// table slots free (generation 0), merge keys empty, merge sums, count
// accumulators and (wide keys) slot owners cleared, the four alive arrays
// zero (written as 64-bit words; the allocations are 8-byte aligned).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_init_store(InstBuf nb, uint64_t ng, uint64_t nm,
                                                       uint32_t wide) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const uint64_t first = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  for (uint64_t i = first; i < ng; i += stride) nb.gtab[i] = 0;
  for (uint64_t i = first; i < nm; i += stride) {
    nb.mkey[i] = kEmpty64;
    nb.mfx[3 * i] = nb.mfx[3 * i + 1] = nb.mfx[3 * i + 2] = 0;
    if (wide) nb.mown[i] = kNone32;
  }
  for (uint64_t i = first; i < kAccBytes / sizeof(uint64_t); i += stride) nb.accs[i] = 0;
  const uint64_t words = nb.cap / 8;
  for (uint64_t i = first; i < words; i += stride)
#pragma unroll
    for (int a = 0; a < 4; ++a) reinterpret_cast<uint64_t*>(nb.alive[a >> 1][a & 1])[i] = 0;
  for (uint64_t i = 8 * words + first; i < nb.cap; i += stride)
#pragma unroll
    for (int a = 0; a < 4; ++a) nb.alive[a >> 1][a & 1][i] = 0;
}

// ---------------------------------------------------------------------------
// Host-driven growth / compaction of one instance into a new store.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_grow(InstBuf src, InstBuf dst, InstDyn* dp,
                                                 uint32_t* sync) {
  __shared__ uint32_t s_tmp[kWaves + 1];
  __shared__ uint32_t s_flag, s_base_v;
  uint32_t* s_base = &s_base_v;
  InstDyn& d = *dp;
  const View v = view_of(src, d);
  const uint32_t M = d.M;
  const int W = src.W;
  const uint32_t tiles = (M + kTile - 1) / kTile;
  const uint32_t workers = worker_count(tiles);
  if (blockIdx.x >= workers) return;
  for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    bool ov[kItems];
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const uint32_t i = tile * kTile + k * kBlock + threadIdx.x;
      ov[k] = i < M && v.al[i];
      mine += ov[k] ? 1u : 0u;
    }
    uint32_t tot;
    uint32_t off = block_scan(mine, s_tmp, &tot);
    if (threadIdx.x == 0) *s_base = tot ? atomicAdd(&d.nuniq, tot) : 0u;
    __syncthreads();
    const uint32_t base = *s_base;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      if (!ov[k]) continue;
      const uint32_t i = tile * kTile + k * kBlock + threadIdx.x;
      const uint32_t pos = base + off++;
      if (pos >= dst.cap) { atomicOr(&d.status, ST_OVERFLOW); continue; }
      uint64_t x[kMaxW], z[kMaxW];
      load_key(v, i, x, z);
      PP_FOR_W(w, 0, W, kMaxW) {
        dst.x[0][(size_t)w * dst.cap + pos] = x[w];
        dst.z[0][(size_t)w * dst.cap + pos] = z[w];
      }
      if (v.f32)
        static_cast<float*>(dst.c[0])[pos] = static_cast<const float*>(v.C)[i];
      else
        static_cast<double*>(dst.c[0])[pos] = static_cast<const double*>(v.C)[i];
      dst.alive[0][0][pos] = 1;
      dst.alive[0][1][pos] = 1;
      gt_insert(dst.gtab, dst.hg_bits, 1u, pos, hash_key(x, z, W, 0));
    }
  }
  if (!last_block(sync, &s_flag, workers)) return;
  if (threadIdx.x == 0) {
    d.M = ld_agent(&d.nuniq);
    d.Mnext = d.M;
    d.nuniq = 0;
    d.half = 0;
    d.parity = 0;
    d.gen = 1;
  }
}

__global__ void k_set_pc(InstDyn* d, uint32_t pc) { d->pc = pc; }

// Copies the per-instance dynamic state into one contiguous buffer (host
// polling of a batch with one transfer).
__global__ void k_gather_dyn(InstDyn* const* dyns, const int* ninst, InstDyn* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < *ninst) out[i] = *dyns[i];
}

}  // namespace pp
