// Exact sums for the symmetry merge: a coefficient becomes a 192-bit
// two's-complement fixed-point integer with kFxFrac fraction bits (three
// little-endian 64-bit limbs).  Integer addition is associative, so an orbit
// sum accumulated in any order is the same exact value, rounded to FP64 once
// by fx_to_double.  Host and device share these functions.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pp_types.h"

namespace pp {

struct Fx {
  uint64_t l0, l1, l2;
};

__host__ __device__ __forceinline__ Fx fx_neg(Fx v) {
  Fx r;
  r.l0 = ~v.l0 + 1;
  const uint64_t c0 = (r.l0 == 0) ? 1u : 0u;
  r.l1 = ~v.l1 + c0;
  const uint64_t c1 = (c0 && r.l1 == 0) ? 1u : 0u;
  r.l2 = ~v.l2 + c1;
  return r;
}

__host__ __device__ __forceinline__ Fx fx_add(Fx a, Fx b) {
  Fx r;
  r.l0 = a.l0 + b.l0;
  const uint64_t c0 = r.l0 < a.l0 ? 1u : 0u;
  r.l1 = a.l1 + b.l1;
  uint64_t c1 = r.l1 < a.l1 ? 1u : 0u;
  r.l1 += c0;
  c1 += (r.l1 < c0) ? 1u : 0u;
  r.l2 = a.l2 + b.l2 + c1;
  return r;
}

// c * 2^kFxFrac as an integer: exact for |c| >= 2^(52 - kFxFrac), rounded
// to the nearest multiple of 2^-kFxFrac below that; |c| >= 2^54 (or a NaN/Inf)
// raises *range.
__host__ __device__ __forceinline__ Fx fx_from_double(double c, bool* range) {
  Fx r{0, 0, 0};
  const uint64_t bits = __builtin_bit_cast(uint64_t, c);
  const bool neg = (bits >> 63) != 0;
  const int ex = (int)((bits >> 52) & 0x7FF);
  const uint64_t frac = bits & ((1ull << 52) - 1);
  if (ex == 0 && frac == 0) return r;
  if (ex == 0x7FF) { *range = true; return r; }
  const uint64_t mant = ex ? (frac | (1ull << 52)) : frac;
  const int e2 = ex ? ex - 1075 : -1074;
  const int sh = e2 + kFxFrac;
  if (sh > kFxMaxShift) { *range = true; return r; }
  if (sh >= 0) {
    const int q = sh >> 6, b = sh & 63;
    const uint64_t lo = mant << b, hi = b ? (mant >> (64 - b)) : 0ull;
    if (q == 0) { r.l0 = lo; r.l1 = hi; } else { r.l1 = lo; r.l2 = hi; }
  } else {
    const int rs = -sh;
    r.l0 = rs > 63 ? 0ull : ((mant + (1ull << (rs - 1))) >> rs);
  }
  return neg ? fx_neg(r) : r;
}

// Rounds the 192-bit value to the nearest double (ties to even).
__host__ __device__ __forceinline__ double fx_to_double(Fx v) {
  const bool neg = (int64_t)v.l2 < 0;
  if (neg) v = fx_neg(v);
  int p;
  if (v.l2) p = 128 + 63 - __builtin_clzll(v.l2);
  else if (v.l1) p = 64 + 63 - __builtin_clzll(v.l1);
  else if (v.l0) p = 63 - __builtin_clzll(v.l0);
  else return 0.0;
  double d;
  if (p <= 63) {
    d = ldexp((double)v.l0, -kFxFrac);                 // uint64 -> double rounds once
  } else {
    const int sh = p - 63;                             // 1 .. 127
    const int q = sh >> 6, b = sh & 63;
    const uint64_t L[3] = {v.l0, v.l1, v.l2};
    uint64_t t = L[q] >> b;
    if (b && q + 1 < 3) t |= L[q + 1] << (64 - b);
    bool sticky = b ? (L[q] & ((1ull << b) - 1)) != 0 : false;
    for (int k = 0; k < q; ++k) sticky = sticky || L[k] != 0;
    if (sticky) t |= 1ull;                             // below the rounding bit
    d = ldexp((double)t, sh - kFxFrac);
  }
  return neg ? -d : d;
}

}  // namespace pp
