// Reference oracle for symmetry-merging Pauli propagation
// (Teng, Chang, Rudolph, Holmes, "Leveraging Symmetry Merging in Pauli
// Propagation", arXiv:2512.12094).
//
// TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously-correct
// host implementation that the tests, the smoke check and the benchmark's
// CPU-baseline leg use to check the HIP library.  The product path never
// links, loads or calls it, and it shares no code with the HIP sources.
//
// Everything is FP64 with exact integer Pauli algebra, kept in std::map
// containers, one term at a time, in the order the paper states the steps:
//
//   * Pauli strings: symplectic (x, z) bit masks, one bit per qubit
//     (Appendix E.2, "symplectic representation"); letters are looked up
//     qubit by qubit.
//   * Products of Pauli strings are taken letter by letter from the
//     single-qubit multiplication table of the Pauli matrices.
//   * Gate rule (Prop. 1, proof part (2)): a rotation commutes with Q or
//     splits Q into a cosine and a sine branch.  Angle convention: the gate
//     is exp(-i theta/2 P), for which the Heisenberg image of an
//     anticommuting Q is cos(theta) Q + sin(theta) (iPQ).
//   * Identical strings produced by a gate are merged (standard PP, Sec. I)
//     and the result is truncated by coefficient and weight.
//   * Symmetry merge (Algorithm 1 step 1 / step 2b; Algorithms 2 and 3):
//     every string is replaced by its lowest-integer orbit representative
//     (Definition "lowest integer representation", Appendix E.2) and the
//     coefficients of one orbit are added (each distinct string once).
//   * Expectation (Algorithm 1 step 3) in a symmetric product state.
//
// parity pinned: see tests/test_oracle_pins.py (matrix products, Burnside
// counts, dense 2^n evolution, Theorem 1, density-matrix noise).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

namespace {

constexpr int kMaxWords = 2;   // up to 128 qubits

struct Pauli {
  std::array<uint64_t, kMaxWords> x{};
  std::array<uint64_t, kMaxWords> z{};
};

// Any strict total order works as a container order; the paper's integer
// order is only used where a representative is chosen (int_less below).
bool operator<(const Pauli& a, const Pauli& b) {
  return std::tie(a.x, a.z) < std::tie(b.x, b.z);
}
bool operator==(const Pauli& a, const Pauli& b) {
  return a.x == b.x && a.z == b.z;
}

enum Letter { I = 0, X = 1, Y = 2, Z = 3 };

int get_letter(const Pauli& p, int q) {
  const int xb = (p.x[q / 64] >> (q % 64)) & 1;
  const int zb = (p.z[q / 64] >> (q % 64)) & 1;
  if (!xb && !zb) return I;
  if (xb && !zb) return X;
  if (xb && zb) return Y;
  return Z;
}

void set_letter(Pauli& p, int q, int l) {
  const uint64_t bit = uint64_t(1) << (q % 64);
  p.x[q / 64] &= ~bit;
  p.z[q / 64] &= ~bit;
  if (l == X || l == Y) p.x[q / 64] |= bit;
  if (l == Y || l == Z) p.z[q / 64] |= bit;
}

int weight(const Pauli& p, int n) {
  int w = 0;
  for (int q = 0; q < n; ++q) w += get_letter(p, q) != I;
  return w;
}

// Single-qubit products of Pauli matrices: sigma_a sigma_b = i^k sigma_c.
// (XY = iZ, YZ = iX, ZX = iY, and the reversed orders carry -i = i^3.)
struct Prod { int c; int k; };
const Prod kProd[4][4] = {
    //        I          X          Y          Z
    /* I */ {{I, 0}, {X, 0}, {Y, 0}, {Z, 0}},
    /* X */ {{X, 0}, {I, 0}, {Z, 1}, {Y, 3}},
    /* Y */ {{Y, 0}, {Z, 3}, {I, 0}, {X, 1}},
    /* Z */ {{Z, 0}, {Y, 1}, {X, 3}, {I, 0}},
};

// P * Q = i^k R ; returns k in {0,1,2,3} and writes R.
int multiply(const Pauli& P, const Pauli& Q, int n, Pauli* R) {
  Pauli r;
  int k = 0;
  for (int q = 0; q < n; ++q) {
    const Prod pr = kProd[get_letter(P, q)][get_letter(Q, q)];
    set_letter(r, q, pr.c);
    k = (k + pr.k) % 4;
  }
  *R = r;
  return k;
}

// Lowest-integer representation (Appendix E.2): I->00, X->01, Y->10,
// Z->11, qubit q is the base-4 digit of weight 4^q.  Compare the integers
// digit by digit from the most significant qubit down.
bool int_less(const Pauli& a, const Pauli& b, int n) {
  for (int q = n - 1; q >= 0; --q) {
    const int da = get_letter(a, q), db = get_letter(b, q);
    if (da != db) return da < db;
  }
  return false;
}

// Translation T^j: qubit q of the result carries qubit (q + j) mod n of s
// (T shifts the string to the left, T.(IXI) = XII).
Pauli translate(const Pauli& s, int j, int n) {
  Pauli t;
  for (int q = 0; q < n; ++q) set_letter(t, q, get_letter(s, (q + j) % n));
  return t;
}

enum Group { kNone = 0, kTranslation = 1, kPermutation = 2, kDihedral = 3, kTorus = 4,
             kExplicit = 5 };

// A qubit permutation g as a list: qubit q of g.s carries qubit perm[q] of s.
Pauli permute(const Pauli& s, const uint8_t* perm, int n) {
  Pauli t;
  for (int q = 0; q < n; ++q) set_letter(t, q, get_letter(s, perm[q]));
  return t;
}

// Any finite group of qubit permutations given by its element list: the
// representative is the argmin of int(g s) over the listed elements.
Pauli canon_explicit(const Pauli& s, int n, const std::vector<uint8_t>& perms) {
  Pauli best = s;
  for (size_t g = 0; g * n < perms.size(); ++g) {
    const Pauli t = permute(s, &perms[g * n], n);
    if (int_less(t, best, n)) best = t;
  }
  return best;
}

// 2D translation on an lx x ly torus, qubit q = x + lx*y: qubit (x, y) of
// the result carries qubit ((x+a) mod lx, (y+b) mod ly) of s.
Pauli translate2d(const Pauli& s, int a, int b, int lx, int ly) {
  Pauli t;
  for (int y = 0; y < ly; ++y)
    for (int x = 0; x < lx; ++x)
      set_letter(t, x + lx * y, get_letter(s, (x + a) % lx + lx * ((y + b) % ly)));
  return t;
}

// Reflection of the ring: qubit q of the result carries qubit n-1-q of s.
Pauli reflect(const Pauli& s, int n) {
  Pauli t;
  for (int q = 0; q < n; ++q) set_letter(t, q, get_letter(s, n - 1 - q));
  return t;
}

// Algorithm 2: the representative is the argmin of int(T^j s), j = 0..n-1.
Pauli canon_translation(const Pauli& s, int n) {
  Pauli best = s;
  for (int j = 1; j < n; ++j) {
    const Pauli t = translate(s, j, n);
    if (int_less(t, best, n)) best = t;
  }
  return best;
}

// Algorithm 3: count (n_X, n_Y, n_Z); the representative is
// Z^{nZ} Y^{nY} X^{nX} I^{rest}, written from qubit 0 upward.
Pauli canon_permutation(const Pauli& s, int n) {
  int nx = 0, ny = 0, nz = 0;
  for (int q = 0; q < n; ++q) {
    const int l = get_letter(s, q);
    nx += l == X;
    ny += l == Y;
    nz += l == Z;
  }
  Pauli r;
  int q = 0;
  for (int i = 0; i < nz; ++i) set_letter(r, q++, Z);
  for (int i = 0; i < ny; ++i) set_letter(r, q++, Y);
  for (int i = 0; i < nx; ++i) set_letter(r, q++, X);
  return r;
}

// Dihedral group D_n (translations and the reflection of the ring), the
// first wider group the paper's outlook names: the representative is the
// argmin of int(g s) over all 2n elements g = T^j and T^j R.
Pauli canon_dihedral(const Pauli& s, int n) {
  const Pauli r = reflect(s, n);
  Pauli best = s;
  for (int j = 0; j < n; ++j) {
    const Pauli a = translate(s, j, n), b = translate(r, j, n);
    if (int_less(a, best, n)) best = a;
    if (int_less(b, best, n)) best = b;
  }
  return best;
}

// Translations of the torus Z_lx x Z_ly (a 2D lattice of the kind the
// paper's Fig. 3 merges over): the representative is the argmin of
// int(T_(a,b) s) over all lx*ly translations.
Pauli canon_torus(const Pauli& s, int n, int lx) {
  const int ly = n / lx;
  Pauli best = s;
  for (int b = 0; b < ly; ++b)
    for (int a = 0; a < lx; ++a) {
      const Pauli t = translate2d(s, a, b, lx, ly);
      if (int_less(t, best, n)) best = t;
    }
  return best;
}

Pauli canon(const Pauli& s, int n, int group, int lx = 0) {
  if (group == kTranslation) return canon_translation(s, n);
  if (group == kPermutation) return canon_permutation(s, n);
  if (group == kDihedral) return canon_dihedral(s, n);
  if (group == kTorus) return canon_torus(s, n, lx);
  return s;
}

// Correctly rounded sum of doubles (Shewchuk, "Adaptive Precision
// Floating-Point Arithmetic and Fast Robust Geometric Predicates", 1997):
// keep the running sum as non-overlapping partials, each new addend folded
// in with exact two-sums; finally add the partials from the largest down,
// correcting a result that lands halfway between two doubles.
double exact_sum(const std::vector<double>& xs) {
  std::vector<double> partials;
  for (double x : xs) {
    size_t k = 0;
    for (double y : partials) {
      if (std::fabs(x) < std::fabs(y)) std::swap(x, y);
      const double hi = x + y;
      const double lo = y - (hi - x);
      if (lo != 0.0) partials[k++] = lo;
      x = hi;
    }
    partials.resize(k);
    partials.push_back(x);
  }
  if (partials.empty()) return 0.0;
  size_t n = partials.size();
  double hi = partials[--n], lo = 0.0;
  while (n > 0) {
    const double x = hi, y = partials[--n];
    hi = x + y;
    const double yr = hi - x;
    lo = y - yr;
    if (lo != 0.0) break;
  }
  if (n > 0 && ((lo < 0.0 && partials[n - 1] < 0.0) || (lo > 0.0 && partials[n - 1] > 0.0))) {
    const double y = lo * 2.0;
    const double x = hi + y;
    if (y == x - hi) hi = x;
  }
  return hi;
}

struct Oracle {
  int n = 0;
  int group = kNone;
  int lx = 0;                // torus width (group kTorus)
  std::vector<uint8_t> perms;  // group kExplicit: elements x n
  std::map<Pauli, double> terms;
  uint64_t propagated = 0;   // sum over gates of the terms tested
  uint64_t merged = 0;       // sum over merge points of the records entering
};

Pauli load(const uint64_t* x, const uint64_t* z, int n) {
  Pauli p;
  const int W = (n + 63) / 64;
  for (int w = 0; w < W; ++w) {
    p.x[w] = x[w];
    p.z[w] = z[w];
  }
  return p;
}

void truncate_map(std::map<Pauli, double>& m, int n, double eps, int wmax) {
  for (auto it = m.begin(); it != m.end();) {
    const bool small = std::fabs(it->second) < eps;
    const bool heavy = wmax >= 0 && weight(it->first, n) > wmax;
    if (small || heavy)
      it = m.erase(it);
    else
      ++it;
  }
}

}  // namespace

extern "C" {

void* orc_create(int n, int group) {
  if (n < 1 || n > 64 * kMaxWords || group == kTorus) return nullptr;
  auto* o = new Oracle;
  o->n = n;
  o->group = group;
  return o;
}

// A handle merging under the group whose m elements are the rows of perms
// (m x n, row g: qubit q of g.s carries qubit perms[g*n + q] of s).
void* orc_create_group(int n, const uint8_t* perms, size_t m) {
  if (n < 1 || n > 64 * kMaxWords || m == 0) return nullptr;
  auto* o = new Oracle;
  o->n = n;
  o->group = kExplicit;
  o->perms.assign(perms, perms + m * n);
  return o;
}

void orc_canon_group(int n, const uint8_t* perms, size_t m, const uint64_t* x,
                     const uint64_t* z, uint64_t* rx, uint64_t* rz) {
  const std::vector<uint8_t> p(perms, perms + m * n);
  const Pauli r = canon_explicit(load(x, z, n), n, p);
  for (int w = 0; w < (n + 63) / 64; ++w) {
    rx[w] = r.x[w];
    rz[w] = r.z[w];
  }
}

// A handle merging under the translations of an lx x ly torus.
void* orc_create_torus(int lx, int ly) {
  if (lx < 1 || ly < 1 || lx * ly > 64 * kMaxWords) return nullptr;
  auto* o = new Oracle;
  o->n = lx * ly;
  o->group = kTorus;
  o->lx = lx;
  return o;
}

void orc_destroy(void* h) { delete static_cast<Oracle*>(h); }

// Adds c to the coefficient of the string (x, z): O = sum_s Tr[O s] s.
void orc_add_term(void* h, const uint64_t* x, const uint64_t* z, double c) {
  auto* o = static_cast<Oracle*>(h);
  o->terms[load(x, z, o->n)] += c;
}

// Algorithm 1 step 1 and step 2b (Algorithms 2 and 3): replace every string
// by its orbit representative and add the coefficients of each orbit.  The
// algorithms leave the order of the additions open; the orbit sum is taken
// exactly and rounded once (exact_sum), so it does not depend on that order.
void orc_merge(void* h) {
  auto* o = static_cast<Oracle*>(h);
  o->merged += o->terms.size();
  std::map<Pauli, std::vector<double>> addends;
  for (const auto& [s, c] : o->terms)
    addends[o->group == kExplicit ? canon_explicit(s, o->n, o->perms)
                                  : canon(s, o->n, o->group, o->lx)].push_back(c);
  std::map<Pauli, double> merged;
  for (const auto& [r, v] : addends) merged[r] = exact_sum(v);
  o->terms.swap(merged);
}

// One Pauli rotation exp(-i theta/2 P) in the Heisenberg picture, then the
// exact merge of identical strings and the truncation (drop |c| < eps or
// weight > wmax; eps = 0 and wmax < 0 switch them off).
void orc_apply_gate(void* h, const uint64_t* px, const uint64_t* pz,
                    double theta, double eps, int wmax) {
  auto* o = static_cast<Oracle*>(h);
  const Pauli P = load(px, pz, o->n);
  const double cs = std::cos(theta), sn = std::sin(theta);
  std::map<Pauli, double> out;
  size_t records = 0;
  for (const auto& [Q, c] : o->terms) {
    Pauli R;
    const int k = multiply(P, Q, o->n, &R);   // P Q = i^k R
    if (k % 2 == 0) {                          // [P, Q] = 0: Q is unchanged
      out[Q] += c;
      records += 1;
    } else {                                   // {P, Q} = 0
      // i P Q = i^(k+1) R, and k+1 is even: the sign is real.
      const double sign = ((k + 1) % 4 == 0) ? 1.0 : -1.0;
      out[Q] += cs * c;
      out[R] += sign * (sn * c);
      records += 2;
    }
  }
  o->propagated += o->terms.size();
  o->merged += records;
  truncate_map(out, o->n, eps, wmax);
  o->terms.swap(out);
}

// Depolarising noise on every qubit in the Heisenberg picture: each
// non-identity letter of a string damps its coefficient by (1 - p).
void orc_damp(void* h, double p) {
  auto* o = static_cast<Oracle*>(h);
  for (auto& [s, c] : o->terms) c *= std::pow(1.0 - p, double(weight(s, o->n)));
}

void orc_truncate(void* h, double eps, int wmax) {
  auto* o = static_cast<Oracle*>(h);
  truncate_map(o->terms, o->n, eps, wmax);
}

// Tr[rho O] for rho = (psi psi^dag)^{(x)n}, <psi|X|psi> = bx etc.
double orc_expectation(void* h, double bx, double by, double bz) {
  auto* o = static_cast<Oracle*>(h);
  double sum = 0.0, comp = 0.0;   // Neumaier summation
  for (const auto& [s, c] : o->terms) {
    double v = c;
    for (int q = 0; q < o->n; ++q) {
      const int l = get_letter(s, q);
      if (l == X) v *= bx;
      if (l == Y) v *= by;
      if (l == Z) v *= bz;
    }
    const double t = sum + v;
    if (std::fabs(sum) >= std::fabs(v))
      comp += (sum - t) + v;
    else
      comp += (v - t) + sum;
    sum = t;
  }
  return sum + comp;
}

size_t orc_size(void* h) { return static_cast<Oracle*>(h)->terms.size(); }

// Rows of W = ceil(n/64) words each, in ascending order of the strings'
// integers (Appendix E.2: the same base-4 integer that picks the
// representative), so the set comes out key-sorted.
void orc_export(void* h, uint64_t* x, uint64_t* z, double* c) {
  auto* o = static_cast<Oracle*>(h);
  const int W = (o->n + 63) / 64;
  std::vector<const std::pair<const Pauli, double>*> rows;
  rows.reserve(o->terms.size());
  for (const auto& t : o->terms) rows.push_back(&t);
  const int n = o->n;
  std::sort(rows.begin(), rows.end(),
            [n](const auto* a, const auto* b) { return int_less(a->first, b->first, n); });
  for (size_t r = 0; r < rows.size(); ++r) {
    for (int w = 0; w < W; ++w) {
      x[r * W + w] = rows[r]->first.x[w];
      z[r * W + w] = rows[r]->first.z[w];
    }
    c[r] = rows[r]->second;
  }
}

void orc_counters(void* h, uint64_t* propagated, uint64_t* merged) {
  auto* o = static_cast<Oracle*>(h);
  *propagated = o->propagated;
  *merged = o->merged;
}

// Single-string helpers for the tests.
void orc_canon_torus(int lx, int ly, const uint64_t* x, const uint64_t* z, uint64_t* rx,
                     uint64_t* rz) {
  const int n = lx * ly;
  const Pauli r = canon(load(x, z, n), n, kTorus, lx);
  for (int w = 0; w < (n + 63) / 64; ++w) {
    rx[w] = r.x[w];
    rz[w] = r.z[w];
  }
}

void orc_canon(int n, int group, const uint64_t* x, const uint64_t* z,
               uint64_t* rx, uint64_t* rz) {
  const Pauli r = canon(load(x, z, n), n, group);
  for (int w = 0; w < (n + 63) / 64; ++w) {
    rx[w] = r.x[w];
    rz[w] = r.z[w];
  }
}

int orc_multiply(int n, const uint64_t* ax, const uint64_t* az,
                 const uint64_t* bx, const uint64_t* bz, uint64_t* rx,
                 uint64_t* rz) {
  Pauli r;
  const int k = multiply(load(ax, az, n), load(bx, bz, n), n, &r);
  for (int w = 0; w < (n + 63) / 64; ++w) {
    rx[w] = r.x[w];
    rz[w] = r.z[w];
  }
  return k;
}

// Algorithm 1 step 1 on a stream of raw rows (x, z, c): every row is one
// addend of its orbit's sum (repeated rows included, not added together
// first); per representative the exact sum of its addends, rounded once.
// Writes the representatives in container order to ox/oz (m rows of W
// words, caller-allocated) and oc; returns how many.
size_t orc_merge_records(int n, int group, const uint64_t* x, const uint64_t* z,
                         const double* c, size_t m, uint64_t* ox, uint64_t* oz, double* oc) {
  const int W = (n + 63) / 64;
  std::map<Pauli, std::vector<double>> addends;
  for (size_t r = 0; r < m; ++r)
    addends[canon(load(x + r * W, z + r * W, n), n, group)].push_back(c[r]);
  size_t k = 0;
  for (const auto& [rep, v] : addends) {
    for (int w = 0; w < W; ++w) {
      ox[k * W + w] = rep.x[w];
      oz[k * W + w] = rep.z[w];
    }
    oc[k] = exact_sum(v);
    ++k;
  }
  return k;
}

double orc_exact_sum(const double* v, size_t n) {
  return exact_sum(std::vector<double>(v, v + n));
}

int orc_int_less(int n, const uint64_t* ax, const uint64_t* az,
                 const uint64_t* bx, const uint64_t* bz) {
  return int_less(load(ax, az, n), load(bx, bz, n), n) ? 1 : 0;
}

}  // extern "C"
