// Host side of the C ABI declared in include/pp.h.
//
// A handle holds one instance: its term store (two halves plus tables, see
// pp_types.h), a device copy of its buffer descriptor and dynamic state,
// and a scratch program.  Every call turns into a short program of device
// operations (pp_types.h: OpType) that the kernels of pp_kernels.hpp
// execute; the host only re-launches after growing the store.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pp.h"
#include "pp_kernels.hpp"
#include "pp_merge.hpp"
#include "pp_layer.hpp"
#include "pp_sort.hpp"
#include "pp_types.h"

using namespace pp;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

struct Tuning {
  int gate_items = 1;     // terms per thread in the gate kernel
  int stream_items = 1;   // terms per thread in merge / compaction / scan kernels
  int max_blocks = 2048;  // persistent grid cap
  int graph_steps = 32;   // batched steps per captured graph
  int gates_per_step = 4; // gate launches per batched step
  int part_shift = kPartShift;    // log2 records per bucket of the partitioned merge
  int part_agg_blocks = 0;        // aggregation blocks (0: one per item, up to 3P/2)
  int layer_shift = kLayerShift;  // log2 strings per bucket of the layer op
  int layer_block = 512;          // threads per bucket block of the layer op (256 or 512)
};
Tuning g_tune;
int g_fuse = kMaxFuse;    // pp_set_gate_fusion: rotations per gate launch (<= 1: off)
int g_lanes = 0;          // pp_set_gate_fusion: lane-per-member form for smaller sets
int g_layer = 1;          // pp_set_layer_ops: 0 off, 1 on, 2 on but every op falls back
int g_prof_default = 0;   // pp_profile(NULL, every): new handles start timed

#define HIP_TRY(expr)                                                            \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(PP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

uint32_t ceil_log2(uint64_t v) {
  uint32_t b = 0;
  while ((1ull << b) < v) ++b;
  return b;
}

}  // namespace

struct pp_program {
  int n = 0;
  bool has_layer = false;     // some op is a layer op
  std::vector<Op> ops;        // host copy (table pointers already device)
  Op* d_ops = nullptr;
  double* d_tab = nullptr;
  size_t n_gates = 0;
};

// solo_program: sub-layers per chunk (the host reads the device state once
// per chunk), chunks launched ahead of the oldest unchecked one, and the
// pinned state slots / events they cycle through (>= the chunks in flight).
constexpr int kChunkSubs = 1;
constexpr size_t kSoloInflight = 2;
constexpr int kSoloSlots = 4;
static_assert(kSoloSlots >= (int)kSoloInflight, "a chunk in flight would reuse a live slot");

struct pp_state {
  int n = 0, W = 1, group = 0;
  hipStream_t stream = nullptr;
  pp_allocator alloc{};
  bool use_alloc = false;
  size_t max_terms = 0;
  InstBuf buf{};                       // host mirror of the descriptor
  std::vector<void*> store;            // allocations of the current store
  InstBuf* d_buf = nullptr;
  InstDyn* d_dyn = nullptr;
  const InstBuf** d_bufp = nullptr;    // 1-entry pointer arrays for Ctx
  InstDyn** d_dynp = nullptr;
  int* d_ninst = nullptr;
  uint32_t* d_sync = nullptr;
  uint64_t* d_stats = nullptr;        // kStatBytes of statistics lines
  Op* d_ops = nullptr;
  size_t ops_cap = 0;
  double* d_tab = nullptr;
  size_t tab_cap = 0;
  InstDyn* h_dyn = nullptr;            // pinned
  double* h_na = nullptr;              // pinned: result and flag of pp_expectation_noalloc
  // transaction of a pp_apply_layer / pp_merge_canonicalize call: the store
  // at the call's start (kept, not freed, if the store grows meanwhile) and
  // a device copy of what the call may change in it
  bool txn = false;
  InstBuf txn_buf{};
  std::vector<std::vector<void*>> retired;   // stores replaced during the call
  void* txn_backup = nullptr;
  uint32_t txn_m = 0, txn_half = 0, txn_parity = 0;
  bool shrunk = false;                 // a finished batched instance's store was compacted
  bool layer_used = false;             // layer ops ran: stores carry their staging
  bool layer_off = false;              // layer ops failed too often: their fallbacks run
  int layer_fallbacks = 0;             // layer ops that fell back (this handle)
  size_t fb_lo = 0, fb_hi = 0;         // fallback ops [fb_lo, fb_hi) that launch_range runs
  bool layer_tried[2 * kLayerMaxBoost + 1] = {};   // bucket boosts a failing layer op tried
  size_t layer_fail_pc = ~size_t(0);   // the layer op they were tried for
  int layer_retries = 0;               // runs of that op with other bucket counts
  const pp_program* batch_prog = nullptr;
  const std::vector<Op>* run_ops_list = nullptr;   // ops of a pp_apply_* call in flight
  int fail_code = PP_OK;               // why a batched instance stopped
  InstDyn* solo_slots = nullptr;       // pinned status slots of solo_program
  hipEvent_t solo_ev[kSoloSlots] = {};
  // pinned staging ring for program uploads of calls that do not sync
  struct Stage {
    char* h = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
  } ring[4];
  unsigned ring_pos = 0;
  // per-kernel timing with events on this stream (pp_profile): every
  // prof_every-th run of back-to-back launches of one kind is bracketed by
  // two events, and the interval is shared by the run's launches (0 = off)
  int prof_every = 0;
  uint32_t m_hint = 0;     // term count last read back (picks tile sizes)
  double m_growth = 2.0;   // records a merge took over the set size before it (last seen)
  uint64_t m_prev_in = 0;  // merge_in and set size at the last read-back
  uint32_t m_prev = 0;
  int lx = 0;              // torus width (PP_GROUP_TORUS)
  std::vector<uint8_t> gperm;   // PP_GROUP_EXPLICIT: element list (host copy)
  uint8_t* d_gperm = nullptr;   // and its device copy
  uint64_t prof_seen[PP_KERNEL_KINDS] = {};
  struct Pend {
    int k;
    uint32_t len;
    hipEvent_t a, b;
  };
  std::vector<Pend> pend;
  std::vector<hipEvent_t> pool;
  uint64_t prof_n[PP_KERNEL_KINDS] = {};
  double prof_ms[PP_KERNEL_KINDS] = {};
};

namespace {

void* dev_alloc(pp_state* s, size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  if (s->use_alloc) return s->alloc.alloc(bytes, s->stream, s->alloc.ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dev_free(pp_state* s, void* p) {
  if (!p) return;
  if (s->use_alloc)
    s->alloc.free(p, s->stream, s->alloc.ctx);
  else
    (void)hipFree(p);
}

hipEvent_t prof_event(pp_state* s) {
  hipEvent_t e = nullptr;
  if (!s->pool.empty()) {
    e = s->pool.back();
    s->pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  return e;
}

// Records an event before a sampled run of launches (or returns nullptr).
hipEvent_t prof_begin(pp_state* s, int kind) {
  if (s->prof_every <= 0) return nullptr;
  if (s->prof_seen[kind]++ % (uint64_t)s->prof_every != 0) return nullptr;
  hipEvent_t a = prof_event(s);
  if (a) (void)hipEventRecord(a, s->stream);
  return a;
}

void prof_end(pp_state* s, int kind, hipEvent_t a, uint32_t len = 1) {
  if (!a) return;
  hipEvent_t b = prof_event(s);
  if (!b) return;
  (void)hipEventRecord(b, s->stream);
  s->pend.push_back({kind, len, a, b});
}

// Folds the finished intervals in (unfinished ones stay pending).
void prof_resolve(pp_state* s) {
  size_t keep = 0;
  for (size_t i = 0; i < s->pend.size(); ++i) {
    const auto p = s->pend[i];
    if (hipEventQuery(p.b) != hipSuccess) {
      s->pend[keep++] = p;
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      s->prof_n[p.k] += p.len;
      s->prof_ms[p.k] += ms;
    }
    s->pool.push_back(p.a);
    s->pool.push_back(p.b);
  }
  s->pend.resize(keep);
}

Ctx single_ctx(pp_state* s) {
  Ctx c;
  c.bufs = s->d_bufp;
  c.dyns = s->d_dynp;
  c.ninst = s->d_ninst;
  c.sync = s->d_sync;
  return c;
}

int upload_buf(pp_state* s) {
  HIP_TRY(hipMemcpyAsync(s->d_buf, &s->buf, sizeof(InstBuf), hipMemcpyHostToDevice, s->stream));
  return PP_OK;
}

void prof_resolve(pp_state* s);

int read_dyn(pp_state* s) {
  HIP_TRY(hipMemcpyAsync(s->h_dyn, s->d_dyn, sizeof(InstDyn), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->m_hint = s->h_dyn->M;
  prof_resolve(s);
  return PP_OK;
}

// The work counters: the instance's own plus its statistics lines (the
// later rotations of multi-rotation ops).
int read_counters(pp_state* s, uint64_t out[8]) {
  int rc = read_dyn(s);
  if (rc) return rc;
  std::vector<uint64_t> st(kStatBytes / sizeof(uint64_t));
  HIP_TRY(hipMemcpyAsync(st.data(), s->d_stats, kStatBytes, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  uint64_t sum[kStatKinds] = {0, 0, 0};
  for (int k = 0; k < kStatKinds; ++k)
    for (int h = 0; h < kAccShards; ++h) sum[k] += st[(size_t)(k * kAccShards + h) * kLineU64];
  const InstDyn& d = *s->h_dyn;
  out[0] = d.propagated + sum[STAT_LIVE];
  out[1] = d.merged + sum[STAT_LIVE] + sum[STAT_ANTI];
  out[2] = d.anti_total + sum[STAT_ANTI];
  out[3] = d.appended;
  out[4] = d.merge_in;
  out[5] = d.merge_out;
  out[6] = d.key_reads;
  out[7] = d.coef_rw + sum[STAT_RW];
  return PP_OK;
}

// Allocates a store of capacity `cap` (both halves and all tables).
// With `dry` set, nothing is allocated or launched: *dry receives the bytes
// the store would take.
// Bucket bits a layer op may use over `slots` staging slots: every bucket
// keeps at least kLayerMinSlots of them.
uint32_t layer_max_bits(uint32_t slots) {
  uint32_t bits = 0;
  while (bits < (uint32_t)kLayerMaxBits && (slots >> (bits + 1)) >= (uint32_t)kLayerMinSlots) ++bits;
  return bits;
}

int alloc_store(pp_state* s, uint32_t cap, InstBuf* b, std::vector<void*>* allocs,
                size_t* dry = nullptr) {
  const int W = s->W;
  InstBuf nb = s->buf;
  nb.cap = cap;
  nb.hg_bits = std::max<uint32_t>(10, ceil_log2(2ull * cap));
  nb.hm_bits = nb.hg_bits;
  if (s->group == PP_GROUP_PERMUTATION) {
    // a permutation merge has at most binom(n+3, 3) representatives
    const uint64_t reps = (uint64_t)(s->n + 3) * (s->n + 2) * (s->n + 1) / 6;
    nb.hm_bits = std::min(nb.hm_bits, std::max<uint32_t>(10, ceil_log2(2 * reps)));
  }
  const size_t ng = size_t(1) << nb.hg_bits, nm = size_t(1) << nb.hm_bits;
  std::vector<void*> got;
  auto take = [&](size_t bytes) -> void* {
    if (dry) {
      *dry += (std::max<size_t>(bytes, 256) + 255) / 256 * 256;
      return reinterpret_cast<void*>(uintptr_t(256));
    }
    void* p = dev_alloc(s, bytes);
    if (p) got.push_back(p);
    return p;
  };
  bool ok = true;
  for (int h = 0; h < 2; ++h) {
    ok = ok && (nb.x[h] = (uint64_t*)take(sizeof(uint64_t) * W * cap));
    ok = ok && (nb.z[h] = (uint64_t*)take(sizeof(uint64_t) * W * cap));
    ok = ok && (nb.c[h] = take((nb.f32 ? sizeof(float) : sizeof(double)) * cap));
    for (int p = 0; p < 2; ++p) ok = ok && (nb.alive[h][p] = (uint8_t*)take(cap));
  }
  ok = ok && (nb.gtab = (uint64_t*)take(sizeof(uint64_t) * ng));
  ok = ok && (nb.mkey = (uint64_t*)take(sizeof(uint64_t) * nm));
  ok = ok && (nb.mfx = (uint64_t*)take(3 * sizeof(uint64_t) * nm));
  ok = ok && (nb.accs = (uint64_t*)take(kAccBytes));
  // staging of the partitioned merge (narrow keys, not S_n, large stores)
  nb.phash = nullptr;
  nb.pstage = nullptr;
  nb.phist = nullptr;
  nb.ptot = nullptr;
  nb.pbase = nullptr;
  nb.pwork = nullptr;
  nb.plist = nullptr;
  nb.pmaxbits = 0;
  if (nb.narrow && s->group != PP_GROUP_PERMUTATION && cap >= kPartMin) {
    nb.pshift = (uint32_t)g_tune.part_shift;
    nb.pmaxbits = part_bits(cap, kPartMaxBits, nb.pshift);
    const size_t P = size_t(1) << nb.pmaxbits;
    const size_t tiles = (cap + kPartTileRec - 1) / kPartTileRec;
    ok = ok && (nb.phash = (uint64_t*)take(sizeof(uint64_t) * cap));
    ok = ok && (nb.pstage = (uint64_t*)take(2 * sizeof(uint64_t) * cap));
    ok = ok && (nb.phist = (uint32_t*)take(sizeof(uint32_t) * tiles * P));
    ok = ok && (nb.ptot = (uint32_t*)take(sizeof(uint32_t) * P));
    ok = ok && (nb.pbase = (uint32_t*)take(sizeof(uint32_t) * (P + 1)));
    ok = ok && (nb.pwork = (uint32_t*)take(sizeof(uint32_t) * 2 * P));
    ok = ok && (nb.plist = (uint32_t*)take(sizeof(uint32_t) * nm));
  }
  // staging of the layer op (once a layer op has run on this handle)
  nb.lstx = nb.lstz = nullptr;
  nb.lstc = nullptr;
  nb.lsta = nullptr;
  nb.lsth = nullptr;
  nb.lcount = nullptr;
  nb.lslots = 0;
  nb.lmaxbits = 0;
  if (s->layer_used) {
    nb.lslots = 1u << ceil_log2(cap);
    nb.lmaxbits = layer_max_bits(nb.lslots);
    ok = ok && (nb.lstx = (uint64_t*)take(sizeof(uint64_t) * W * nb.lslots));
    ok = ok && (nb.lstz = (uint64_t*)take(sizeof(uint64_t) * W * nb.lslots));
    ok = ok && (nb.lstc = (double*)take(sizeof(double) * nb.lslots));
    ok = ok && (nb.lsta = (uint64_t*)take(sizeof(uint64_t) * nb.lslots));
    ok = ok && (nb.lsth = (uint32_t*)take(sizeof(uint32_t) * nb.lslots));
    ok = ok && (nb.lcount = (uint32_t*)take(sizeof(uint32_t) << nb.lmaxbits));
  }
  const bool wide = !nb.narrow;
  nb.mown = nullptr;
  nb.wrep = nullptr;
  nb.wslot = nullptr;
  if (wide) {
    ok = ok && (nb.mown = (uint32_t*)take(sizeof(uint32_t) * nm));
    ok = ok && (nb.wrep = (uint64_t*)take(sizeof(uint64_t) * 2 * W * cap));
    ok = ok && (nb.wslot = (uint32_t*)take(sizeof(uint32_t) * cap));
  }
  if (!ok) {
    for (void* p : got) dev_free(s, p);
    return fail(PP_ENOMEM, "allocation of a term store of capacity " + std::to_string(cap) +
                               " failed");
  }
  if (dry) return PP_OK;
  // the tables' initial state in one launch (instead of a fill per array)
  const uint64_t init_elems = std::max<uint64_t>({ng, nm, cap / 8});
  const int init_grid = (int)std::min<uint64_t>(
      std::max<uint64_t>(1, (init_elems + 4 * kBlock - 1) / (4 * kBlock)), 2048);
  hipLaunchKernelGGL(k_init_store, dim3(init_grid), dim3(kBlock), 0, s->stream, nb, (uint64_t)ng,
                     (uint64_t)nm, wide ? 1u : 0u);
  HIP_TRY(hipGetLastError());
  if (nb.lcount)
    HIP_TRY(hipMemsetAsync(nb.lcount, 0, sizeof(uint32_t) << nb.lmaxbits, s->stream));
  *b = nb;
  *allocs = std::move(got);
  return PP_OK;
}

void free_store(pp_state* s, std::vector<void*>& allocs) {
  for (void* p : allocs) dev_free(s, p);
  allocs.clear();
}

int launch_blocks(uint64_t elements, int items = 4) {
  const uint64_t tile = (uint64_t)kBlock * items;
  const uint64_t tiles = (elements + tile - 1) / tile;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(tiles, (uint64_t)g_tune.max_blocks));
}

using KernelFn = void (*)(Ctx);

#define PP_PICK(kern, it) \
  ((it) == 1 ? &kern<1> : (it) == 2 ? &kern<2> : (it) == 8 ? &kern<8> : &kern<4>)

// Kernel of a kind with the tuned items per thread.
KernelFn kernel_of(int kind) {
  const int gi = g_tune.gate_items, si = g_tune.stream_items;
  switch (kind) {
    case PP_K_GATE: return PP_PICK(k_gate, gi);
    case PP_K_MERGE_NARROW: return PP_PICK(k_merge_narrow, si);
    case PP_K_MERGE_WIDE1: return PP_PICK(k_merge_wide1, si);
    case PP_K_MERGE_WIDE2: return PP_PICK(k_merge_wide2, si);
    case PP_K_MERGE_COLLECT: return PP_PICK(k_merge_collect, si);
    case PP_K_COMPACT: return PP_PICK(k_compact, si);
    default: return PP_PICK(k_scan_op, si);
  }
}

using SoloFn = void (*)(Solo);

// Launches over large sets take at least kBigItems items per thread: a tile
// reserves its appended strings with one atomic on the instance's cursor,
// and those atomics serialise, so fewer, larger tiles run faster there.
constexpr uint32_t kBigSet = 1u << 19;
constexpr int kBigItems = 4;

int gate_items(bool big) { return big ? std::max(g_tune.gate_items, kBigItems) : g_tune.gate_items; }
int stream_items(bool big) {
  return big ? std::max(g_tune.stream_items, kBigItems) : g_tune.stream_items;
}

// Rows per tile of the lane form of an r-rotation op over a set last seen
// with `hint` terms: the fewest that keep the launch within kTreeMin
// blocks (one append atomic and one done count per block), or 0 when the
// set is too large for the lane form.
int lane_items(uint32_t hint, uint32_t nrot) {
  if (!g_lanes || nrot < 2) return 0;
  const uint64_t lanes = (uint64_t)std::max<uint32_t>(hint, 1) << nrot;
  for (int it = 1; it <= 8; it *= 2)
    if ((lanes + (uint64_t)kBlock * it - 1) / ((uint64_t)kBlock * it) <= kTreeMin) return it;
  return 0;
}

// The histogram pass canonicalises, so it is built per group.
SoloFn part_hist_of(int group) {
  switch (group) {
    case PP_GROUP_TRANSLATION: return &k_part_hist<1>;
    case PP_GROUP_DIHEDRAL: return &k_part_hist<3>;
    case PP_GROUP_TORUS: return &k_part_hist<4>;
    case PP_GROUP_EXPLICIT: return &k_part_hist<5>;
    default: return &k_part_hist<0>;
  }
}

SoloFn solo_of(int kind, bool big, uint32_t nrot = 1, int lane_it = 0, int group = 0) {
  const int gi = gate_items(big), si = stream_items(big);
  switch (kind) {
    case PP_K_GATE:
      if (lane_it)
        return nrot == 3 ? PP_PICK(k_gate3_lane_solo, lane_it) : PP_PICK(k_gate2_lane_solo, lane_it);
      return nrot == 3 ? PP_PICK(k_gate3_solo, gi)
             : nrot == 2 ? PP_PICK(k_gate2_solo, gi)
                         : PP_PICK(k_gate_solo, gi);
    case PP_K_MERGE_NARROW: return PP_PICK(k_merge_narrow_solo, si);
    case PP_K_MERGE_WIDE1: return PP_PICK(k_merge_wide1_solo, si);
    case PP_K_MERGE_WIDE2: return PP_PICK(k_merge_wide2_solo, si);
    case PP_K_MERGE_COLLECT: return PP_PICK(k_merge_collect_solo, si);
    case PP_K_COMPACT: return PP_PICK(k_compact_solo, si);
    case PP_K_PART_HIST: return part_hist_of(group);
    case PP_K_PART_SCAN: return &k_part_scan;
    case PP_K_PART_SCATTER: return &k_part_scatter;
    case PP_K_PART_AGG: return &k_part_agg;
    default: return PP_PICK(k_scan_op_solo, si);
  }
}

SoloFn layer_of(int kind, int W) {
  if (kind == PP_K_LAYER_SCATTER) return W == 1 ? &k_layer_scatter<1> : &k_layer_scatter<2>;
  if (g_tune.layer_block == 256) return W == 1 ? &k_layer_apply<1, 256> : &k_layer_apply<2, 256>;
  return W == 1 ? &k_layer_apply<1, 512> : &k_layer_apply<2, 512>;
}

// The layer op's staging, allocated when a handle first runs one (and
// then with every store it grows into).
int ensure_layer(pp_state* s) {
  if (s->buf.lcount) return PP_OK;
  s->layer_used = true;
  InstBuf& nb = s->buf;
  const int W = s->W;
  nb.lslots = 1u << ceil_log2(nb.cap);
  nb.lmaxbits = layer_max_bits(nb.lslots);
  std::vector<void*> got;
  auto take = [&](size_t bytes) -> void* {
    void* p = dev_alloc(s, bytes);
    if (p) got.push_back(p);
    return p;
  };
  bool ok = (nb.lstx = (uint64_t*)take(sizeof(uint64_t) * W * nb.lslots)) != nullptr;
  ok = ok && (nb.lstz = (uint64_t*)take(sizeof(uint64_t) * W * nb.lslots));
  ok = ok && (nb.lstc = (double*)take(sizeof(double) * nb.lslots));
  ok = ok && (nb.lsta = (uint64_t*)take(sizeof(uint64_t) * nb.lslots));
  ok = ok && (nb.lsth = (uint32_t*)take(sizeof(uint32_t) * nb.lslots));
  ok = ok && (nb.lcount = (uint32_t*)take(sizeof(uint32_t) << nb.lmaxbits));
  if (!ok) {
    for (void* p : got) dev_free(s, p);
    nb.lstx = nb.lstz = nullptr;
    nb.lstc = nullptr;
    nb.lsta = nullptr;
    nb.lsth = nullptr;
    nb.lcount = nullptr;
    nb.lslots = nb.lmaxbits = 0;
    return fail(PP_ENOMEM, "allocation of the layer staging failed");
  }
  HIP_TRY(hipMemsetAsync(nb.lcount, 0, sizeof(uint32_t) << nb.lmaxbits, s->stream));
  for (void* p : got) s->store.push_back(p);
  return upload_buf(s);
}

int items_of(int kind, bool big = false) {
  return kind == PP_K_GATE ? gate_items(big) : stream_items(big);
}

// Grows (or just compacts) the store so that the op that stopped fits:
// live + count entries for a gate, 2^(r-1) (live + count) for an op of r
// rotations (each later rotation may append one string per term live
// before it).
int grow(pp_state* s) {
  const InstDyn& d = *s->h_dyn;
  const std::vector<Op>* ops = s->batch_prog ? &s->batch_prog->ops : s->run_ops_list;
  const uint32_t nrot =
      ops && d.pc < ops->size() && (*ops)[d.pc].type == OP_GATES ? (*ops)[d.pc].nrot : 1u;
  // after compaction M = live: live + appends <= 2^(nrot-1) (live + count);
  // a layer op whose survivors did not fit says how many there were
  const bool layer = ops && d.pc < ops->size() && (*ops)[d.pc].type == OP_LAYER;
  const uint64_t need = layer ? std::max<uint64_t>((uint64_t)d.lneed, (uint64_t)d.live + d.count)
                              : (uint64_t)d.live + gate_append_bound(nrot, d.live, d.count);
  // same capacity (a compaction) when the live terms leave enough room;
  // the headroom shrinks from 4x to 1.5x for very large sets
  const uint64_t head = need < (1ull << 24) ? 4 * need : need < (1ull << 27) ? 2 * need
                                                                            : need * 3 / 2;
  uint64_t cap = std::max<uint64_t>({(uint64_t)s->buf.cap, head, 4096});
  if (cap > 0xFFFFFFF0ull) cap = 0xFFFFFFF0ull;
  if (s->max_terms && cap > s->max_terms) cap = s->max_terms;
  if (cap < need + 1)
    return fail(PP_ECAPACITY, "term store would need " + std::to_string(need + 1) +
                                  " entries, limit " + std::to_string(s->max_terms));
  InstBuf nb;
  std::vector<void*> allocs;
  int rc = alloc_store(s, (uint32_t)cap, &nb, &allocs);
  if (rc) return rc;
  nb.prog = s->buf.prog;
  nb.prog_len = s->buf.prog_len;
  hipEvent_t ev = prof_begin(s, PP_K_GROW);
  hipLaunchKernelGGL(k_grow, dim3(launch_blocks(d.M)), dim3(kBlock), 0, s->stream, s->buf, nb,
                     s->d_dyn, s->d_sync);
  prof_end(s, PP_K_GROW, ev);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (s->txn)
    s->retired.push_back(std::move(s->store));   // the call may still roll back to it
  else
    free_store(s, s->store);
  s->store = std::move(allocs);
  s->buf = nb;
  int r = upload_buf(s);
  if (r) return r;
  return read_dyn(s);
}

int ensure_ops(pp_state* s, size_t nops, size_t ntab) {
  if (nops > s->ops_cap) {
    dev_free(s, s->d_ops);
    s->ops_cap = std::max<size_t>(nops, 2 * s->ops_cap);
    s->d_ops = (Op*)dev_alloc(s, sizeof(Op) * s->ops_cap);
    if (!s->d_ops) return fail(PP_ENOMEM, "program buffer");
  }
  if (ntab > s->tab_cap) {
    dev_free(s, s->d_tab);
    s->tab_cap = std::max<size_t>(ntab, 2 * s->tab_cap);
    s->d_tab = (double*)dev_alloc(s, sizeof(double) * s->tab_cap);
    if (!s->d_tab) return fail(PP_ENOMEM, "table buffer");
  }
  return PP_OK;
}

bool is_part_kind(int kind) {
  return kind == PP_K_PART_HIST || kind == PP_K_PART_SCAN || kind == PP_K_PART_SCATTER ||
         kind == PP_K_PART_AGG;
}

// Grids of the partitioned merge's kernels, sized for the store's capacity
// (the device takes its sizes from the live record count and idles the
// surplus blocks): tiles of kPartTileRec records, one column band of 64
// buckets per scan block, one aggregation item per block up to 3P/2.
int part_grid(const InstBuf& b, int kind) {
  const uint64_t P = uint64_t(1) << std::max<uint32_t>(b.pmaxbits, kPartMinBits);
  const uint64_t tiles = (b.cap + kPartTileRec - 1) / kPartTileRec;
  uint64_t g = kind == PP_K_PART_SCAN ? P / 64 : kind == PP_K_PART_AGG ? 3 * P / 2 : tiles;
  if (kind == PP_K_PART_AGG && g_tune.part_agg_blocks)   // blocks walk the items grid-stride
    g = std::min<uint64_t>(g, (uint64_t)g_tune.part_agg_blocks);
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(g, 4096));
}

// Dynamic LDS of the partitioned merge's kernels: the histogram's P
// counters, the scatter's three arrays of P (P = 2^pmaxbits, the most the
// device may pick for this store).
size_t part_lds(const InstBuf& b, int kind) {
  static std::once_flag once;
  std::call_once(once, [] {   // the most any store may ask for
    const int most = 3 * (1 << kPartMaxBits) * (int)sizeof(uint32_t);
    (void)hipFuncSetAttribute((const void*)&k_part_scatter,
                              hipFuncAttributeMaxDynamicSharedMemorySize, most);
    for (const void* f : {(const void*)&k_part_hist<0>, (const void*)&k_part_hist<1>,
                          (const void*)&k_part_hist<3>, (const void*)&k_part_hist<4>,
                          (const void*)&k_part_hist<5>})
      (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, most / 3);
  });
  const size_t P = size_t(1) << std::max<uint32_t>(b.pmaxbits, kPartMinBits);
  if (kind == PP_K_PART_HIST) return P * sizeof(uint32_t);
  if (kind == PP_K_PART_SCATTER) return 3 * P * sizeof(uint32_t);
  return 0;
}

// Launches the kernels that execute ops[from..] assuming none overflows.
// Kernel kinds that execute one op of this handle.
void kinds_of(const pp_state* s, const Op& op, std::vector<int>* out) {
  switch (op.type) {
    case OP_GATE:
    case OP_GATES:
      out->push_back(PP_K_GATE);
      break;
    case OP_LAYER:
      out->push_back(PP_K_LAYER_SCATTER);
      out->push_back(PP_K_LAYER_APPLY);
      break;
    case OP_MERGE:
      if (s->group == PP_GROUP_NONE && !op.force_full) {
        out->push_back(PP_K_COMPACT);
      } else if (s->buf.narrow) {
        out->push_back(PP_K_MERGE_NARROW);
        if (s->buf.pstage && !s->buf.nopart) {   // large merges: partitioned
          out->push_back(PP_K_PART_HIST);
          out->push_back(PP_K_PART_SCAN);
          out->push_back(PP_K_PART_SCATTER);
          out->push_back(PP_K_PART_AGG);
        }
        out->push_back(PP_K_MERGE_COLLECT);
      } else {
        out->push_back(PP_K_MERGE_WIDE1);
        out->push_back(PP_K_MERGE_WIDE2);
        out->push_back(PP_K_MERGE_COLLECT);
      }
      break;
    default:
      out->push_back(PP_K_SCAN);
      break;
  }
}

// Launches the single-instance kernels of ops [from, to) (op index k is a
// launch argument: a launch whose op is not the current one does nothing,
// so everything after an overflow is skipped on the device).  With
// profiling on, each run of back-to-back launches of one kind is timed as a
// whole, so the events do not sit between the launches they time.
int launch_range(pp_state* s, const Op* ops, size_t from, size_t to) {
  std::vector<int> kinds;
  s->buf.lshift = (uint32_t)g_tune.layer_shift;   // layer ops launched from here on
  const bool big = s->m_hint >= kBigSet;   // last term count seen on the host
  // a set last seen well below the partitioned merge's threshold merges
  // unpartitioned (correct at any size): the partitioned kernels are not
  // launched.  The records a merge takes are estimated from the last set
  // size and the growth of the last sub-layer seen (at least 2x).
  const double grow_f = std::max(2.0, std::min(1.5 * s->m_growth, 1e9));
  const bool small = (double)s->m_hint * grow_f < (double)kPartMin;
  int run_kind = -1;
  uint32_t run_len = 0;
  hipEvent_t run_ev = nullptr;
  for (size_t k = from; k < to; ++k) {
    // a layer op's fallback copies run only after it failed (or with layer
    // ops off for this handle, in place of it)
    if (ops[k].type == OP_LAYER && s->buf.nolayer) continue;
    if (ops[k].fallback && !s->buf.nolayer && !(k >= s->fb_lo && k < s->fb_hi)) continue;
    kinds.clear();
    kinds_of(s, ops[k], &kinds);
    for (int kind : kinds) {
      if (small && is_part_kind(kind)) continue;
      const bool layer = kind == PP_K_LAYER_SCATTER || kind == PP_K_LAYER_APPLY;
      if (layer) {
        int rc = ensure_layer(s);
        if (rc) return rc;
      }
      if (kind != run_kind) {
        if (run_kind >= 0) prof_end(s, run_kind, run_ev, run_len);
        run_kind = kind;
        run_len = 0;
        run_ev = prof_begin(s, kind);
      }
      const uint64_t elems = kind == PP_K_MERGE_COLLECT ? (1ull << s->buf.hm_bits) : s->buf.cap;
      const uint32_t nrot = ops[k].type == OP_GATES ? ops[k].nrot : 1u;
      const int lane_it = kind == PP_K_GATE && !big ? lane_items(s->m_hint, nrot) : 0;
      int grid = is_part_kind(kind) ? part_grid(s->buf, kind)
                 : lane_it            ? launch_blocks(elems << nrot, lane_it)
                                      : launch_blocks(elems, items_of(kind, big));
      if (kind == PP_K_LAYER_APPLY) {       // about two blocks per bucket of the last size seen
        const uint32_t bits = layer_bits(std::max<uint32_t>(s->m_hint, 1), s->h_dyn->lboost,
                                         s->buf.lmaxbits, s->buf.lshift);
        grid = (int)std::min<uint32_t>(1u << bits, 8192u);   // one bucket per block
      }
      const int block = kind == PP_K_PART_SCAN ? kPCBlock
                        : kind == PP_K_PART_AGG ? kPABlock
                        : kind == PP_K_LAYER_APPLY ? g_tune.layer_block
                        : is_part_kind(kind)    ? kPHBlock
                                                : kBlock;
      Solo S;
      S.b = s->buf;
      if (small) S.b.nopart = 1;
      S.d = s->d_dyn;
      S.sync = s->d_sync;
      S.k = (uint32_t)k;
      if (layer)
        hipLaunchKernelGGL(layer_of(kind, s->W), dim3(grid), dim3(block), 0, s->stream, S);
      else
        hipLaunchKernelGGL(solo_of(kind, big, nrot, lane_it, s->group), dim3(grid), dim3(block),
                           part_lds(s->buf, kind), s->stream, S);
      ++run_len;
    }
  }
  if (run_kind >= 0) prof_end(s, run_kind, run_ev, run_len);
  HIP_TRY(hipGetLastError());
  return PP_OK;
}

int launch_ops(pp_state* s, const std::vector<Op>& ops, size_t from) {
  return launch_range(s, ops.data(), from, ops.size());
}

// Uploads `ops` (and `tab`), runs them to completion, growing the store
// when a gate does not fit.  Synchronises unless `nosync` and no op can
// overflow.
using TabRefs = std::vector<std::pair<size_t, size_t>>;   // (op index, table offset)

int run_ops(pp_state* s, std::vector<Op> ops, const std::vector<double>& tab,
            const TabRefs& refs, bool nosync) {
  if (ops.empty()) return PP_OK;
  int rc = ensure_ops(s, ops.size(), tab.size());
  if (rc) return rc;
  for (const auto& r : refs) ops[r.first].table = s->d_tab + r.second;
  s->buf.prog = s->d_ops;
  s->buf.prog_len = (uint32_t)ops.size();
  s->buf.nopart = 0;
  s->batch_prog = nullptr;
  s->run_ops_list = &ops;
  struct Reset {
    pp_state* s;
    ~Reset() { s->run_ops_list = nullptr; }
  } reset{s};
  {
    // ops, tables and the buffer descriptor go through pinned staging
    auto& st = s->ring[s->ring_pos++ % 4];
    const size_t ob = sizeof(Op) * ops.size(), tb = sizeof(double) * tab.size();
    const size_t bb = sizeof(InstBuf);
    if (st.used) HIP_TRY(hipEventSynchronize(st.ev));
    if (!st.ev) HIP_TRY(hipEventCreateWithFlags(&st.ev, hipEventDisableTiming));
    if (st.cap < ob + tb + bb) {
      if (st.h) HIP_TRY(hipHostFree(st.h));
      st.h = nullptr;
      st.cap = std::max<size_t>(ob + tb + bb, 4096);
      HIP_TRY(hipHostMalloc((void**)&st.h, st.cap, hipHostMallocDefault));
    }
    std::memcpy(st.h, &s->buf, bb);
    std::memcpy(st.h + bb, ops.data(), ob);
    if (tb) std::memcpy(st.h + bb + ob, tab.data(), tb);
    HIP_TRY(hipMemcpyAsync(s->d_buf, st.h, bb, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->d_ops, st.h + bb, ob, hipMemcpyHostToDevice, s->stream));
    if (tb)
      HIP_TRY(hipMemcpyAsync(s->d_tab, st.h + bb + ob, tb, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipEventRecord(st.ev, s->stream));
    st.used = true;
  }
  // pc = 0
  hipLaunchKernelGGL(k_set_pc, dim3(1), dim3(1), 0, s->stream, s->d_dyn, 0u);
  if ((rc = launch_ops(s, ops, 0))) return rc;
  bool can_overflow = false;
  for (const auto& op : ops) can_overflow |= op.type == OP_GATE || op.type == OP_GATES || op.type == OP_MERGE;
  if (nosync && !can_overflow) return PP_OK;
  for (int guard = 0; guard < 1000; ++guard) {
    if ((rc = read_dyn(s))) return rc;
    const InstDyn& d = *s->h_dyn;
    if (d.status & ST_RANGE)
      return fail(PP_EINVAL, "a coefficient is not finite or exceeds 2^54 in magnitude");
    if (d.pc >= ops.size()) return PP_OK;
    if (d.status & ST_OVERFLOW) {
      const uint32_t at = d.pc;
      if ((rc = grow(s))) {
        // the store holds the result of ops [0, at); let later calls run
        const std::string msg = g_err;
        s->h_dyn->status &= ~ST_OVERFLOW;
        (void)hipMemcpyAsync(&s->d_dyn->status, &s->h_dyn->status, sizeof(uint32_t),
                             hipMemcpyHostToDevice, s->stream);
        (void)hipStreamSynchronize(s->stream);
        g_err = msg + " (" + std::to_string(at) + " of " + std::to_string(ops.size()) +
                " operations applied)";
        return rc;
      }
      s->h_dyn->status &= ~ST_OVERFLOW;
      HIP_TRY(hipMemcpyAsync(&s->d_dyn->status, &s->h_dyn->status, sizeof(uint32_t),
                             hipMemcpyHostToDevice, s->stream));
    }
    if ((rc = launch_ops(s, ops, s->h_dyn->pc))) return rc;
  }
  return fail(PP_EDEVICE, "program did not complete");
}

Op make_op(uint32_t type) {
  Op op;
  std::memset(&op, 0, sizeof(op));
  op.type = type;
  op.nrot = type == OP_GATE ? 1u : 0u;
  op.next_gate = kNone32;
  op.wmax = -1;
  return op;
}

// next_gate of every op: the first GATE(S) op after it (after a LAYER op's
// own fallback copies for the LAYER op; LAYER ops themselves count no
// anticommuting terms ahead, so they are not in the chain).
void set_next_gates(std::vector<Op>& ops) {
  std::vector<uint32_t> first(ops.size() + 1, kNone32);
  for (size_t k = ops.size(); k-- > 0;)
    first[k] = (ops[k].type == OP_GATE || ops[k].type == OP_GATES) ? (uint32_t)k : first[k + 1];
  for (size_t k = 0; k < ops.size(); ++k) {
    const size_t after = ops[k].type == OP_LAYER ? k + 1 + ops[k].skip : k + 1;
    const uint32_t next = first[std::min(after, ops.size())];
    ops[k].next_gate = next;
    for (int w = 0; w < kMaxW; ++w) {
      ops[k].nx[w] = next == kNone32 ? 0 : ops[next].px[w];
      ops[k].nz[w] = next == kNone32 ? 0 : ops[next].pz[w];
    }
  }
}

void fuse_gates(std::vector<Op>& ops, size_t from, int W);

// Gate ops ops[from..] of one sub-layer: when they are kLayerMinRot to
// kLayerMaxRot pairwise commuting rotations, a LAYER op carrying them (its
// rotation table appended to `tab`) is put in front of them and they become
// its fallback copies.
void add_layer_op(std::vector<Op>& ops, size_t from, size_t to_gate_end, int W,
                  std::vector<double>& tab, TabRefs& refs, bool merge_follows) {
  if (!g_layer) return;
  const size_t r = to_gate_end - from;
  if (r < (size_t)kLayerMinRot || r > (size_t)kLayerMaxRot) return;
  for (size_t a = from; a < to_gate_end; ++a) {
    if (ops[a].type != OP_GATE) return;
    for (size_t c = a + 1; c < to_gate_end; ++c) {
      int odd = 0;
      for (int w = 0; w < W; ++w)
        odd += __builtin_popcountll((ops[a].px[w] & ops[c].pz[w]) ^ (ops[a].pz[w] & ops[c].px[w]));
      if (odd & 1) return;
    }
  }
  Op layer = make_op(OP_LAYER);
  layer.nrot = (uint32_t)r;
  layer.eps = ops[from].eps;
  layer.wmax = ops[from].wmax;
  layer.full_check = ops[from].full_check;
  layer.gtab = merge_follows ? 0u : 1u;
  layer.fail_test = g_layer == 2 ? 1u : 0u;
  for (int w = 0; w < kMaxW; ++w) {       // the first rotation (for the op's own record)
    layer.px[w] = ops[from].px[w];
    layer.pz[w] = ops[from].pz[w];
  }
  refs.push_back({from, tab.size()});
  for (size_t a = from; a < to_gate_end; ++a) {
    double rec[kLayerRec] = {};
    for (int w = 0; w < kMaxW; ++w) {
      std::memcpy(&rec[w], &ops[a].px[w], sizeof(double));
      std::memcpy(&rec[kMaxW + w], &ops[a].pz[w], sizeof(double));
    }
    rec[2 * kMaxW] = ops[a].cs;
    rec[2 * kMaxW + 1] = ops[a].sn;
    tab.insert(tab.end(), rec, rec + kLayerRec);
  }
  fuse_gates(ops, from, W);
  for (size_t a = from; a < ops.size(); ++a) ops[a].fallback = 1;
  layer.skip = (uint32_t)(ops.size() - from);
  ops.insert(ops.begin() + from, layer);
}

// Gate ops ops[from..] (consecutive gates of one sub-layer) are grouped into
// multi-rotation ops of up to g_fuse rotations: a gate joins the group
// before it when it commutes with every member, has the same truncation
// parameters, and its string is independent of theirs over GF(2) (no
// product of a nonempty subset of the group's strings is the identity), so
// the 2^r strings Q * P^s of a group are distinct.  Only the first gate of
// a sub-layer carries the full re-check, and it always starts a group.
void fuse_gates(std::vector<Op>& ops, size_t from, int W) {
  if (g_fuse < 2) return;
  std::vector<Op> out;
  size_t k = from;
  while (k < ops.size()) {
    Op f = ops[k];
    ++k;
    if (f.type != OP_GATE) {
      out.push_back(f);
      continue;
    }
    // span of the group's strings (x words then z words), 2^r entries
    std::vector<std::array<uint64_t, 2 * kMaxW>> span(1);
    span[0].fill(0);
    auto key_of = [&](const Op& o) {
      std::array<uint64_t, 2 * kMaxW> v;
      v.fill(0);
      for (int w = 0; w < W; ++w) {
        v[w] = o.px[w];
        v[kMaxW + w] = o.pz[w];
      }
      return v;
    };
    auto extend = [&](const std::array<uint64_t, 2 * kMaxW>& p) {
      const size_t n = span.size();
      for (size_t j = 0; j < n; ++j) {
        auto q = span[j];
        for (int w = 0; w < 2 * kMaxW; ++w) q[w] ^= p[w];
        span.push_back(q);
      }
    };
    extend(key_of(f));
    std::vector<const Op*> members{&ops[k - 1]};
    uint32_t nrot = 1;
    while (nrot < (uint32_t)g_fuse && k < ops.size()) {
      const Op& b = ops[k];
      bool ok = b.type == OP_GATE && !b.full_check && b.eps == f.eps && b.wmax == f.wmax;
      for (const Op* m : members) {
        int odd = 0;
        for (int w = 0; w < W; ++w)
          odd += __builtin_popcountll((m->px[w] & b.pz[w]) ^ (m->pz[w] & b.px[w]));
        ok = ok && !(odd & 1);
      }
      const auto kb = key_of(b);
      for (const auto& q : span) ok = ok && q != kb;
      if (!ok) break;
      extend(kb);
      members.push_back(&b);
      for (int w = 0; w < kMaxW; ++w) {
        f.qx[nrot - 1][w] = b.px[w];
        f.qz[nrot - 1][w] = b.pz[w];
      }
      f.qcs[nrot - 1] = b.cs;
      f.qsn[nrot - 1] = b.sn;
      ++nrot;
      ++k;
    }
    if (nrot > 1) {
      f.type = OP_GATES;
      f.nrot = nrot;
    }
    out.push_back(f);
  }
  ops.resize(from);
  ops.insert(ops.end(), out.begin(), out.end());
}

bool valid_group_n(int group, int n) {
  if (group == PP_GROUP_TRANSLATION || group == PP_GROUP_DIHEDRAL) return n >= 2 && n <= 64;
  if (group == PP_GROUP_NONE || group == PP_GROUP_PERMUTATION) return n >= 1 && n <= 128;
  return false;
}

bool row_in_range(const uint64_t* x, const uint64_t* z, int n, int W) {
  for (int w = 0; w < W; ++w) {
    const int bits = std::min(64, n - 64 * w);
    const uint64_t m = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
    if ((x[w] & ~m) || (z[w] & ~m)) return false;
  }
  return true;
}

// Gate multiset closed under the group (Eq. (action): every group element
// maps the layer onto itself).
int check_symmetric(const pp_state* s, const uint64_t* gx, const uint64_t* gz,
                    const double* theta, size_t K) {
  const int n = s->n, W = s->W;
  using Key = std::tuple<uint64_t, uint64_t, uint64_t, uint64_t, double>;
  auto key = [&](const uint64_t* x, const uint64_t* z, double t) {
    return Key(x[0], W > 1 ? x[1] : 0, z[0], W > 1 ? z[1] : 0, t);
  };
  if (s->group == PP_GROUP_TRANSLATION || s->group == PP_GROUP_DIHEDRAL) {
    std::map<Key, long> mult;
    for (size_t k = 0; k < K; ++k) mult[key(gx + k * W, gz + k * W, theta[k])] += 1;
    const uint64_t mask = n == 64 ? ~0ull : ((1ull << n) - 1);
    auto reflect = [&](uint64_t v) {     // qubit q -> n-1-q
      uint64_t r = 0;
      for (int q = 0; q < n; ++q)
        if ((v >> q) & 1) r |= 1ull << (n - 1 - q);
      return r;
    };
    for (const auto& [k, m] : mult) {
      const uint64_t x = std::get<0>(k), z = std::get<2>(k);
      const uint64_t tx = ((x >> 1) | (x << (n - 1))) & mask;   // T shifts left
      const uint64_t tz = ((z >> 1) | (z << (n - 1))) & mask;
      const uint64_t t1[1] = {tx}, t2[1] = {tz};
      auto it = mult.find(key(t1, t2, std::get<4>(k)));
      if (it == mult.end() || it->second != m)
        return fail(PP_ENOTSYM, "gate layer is not closed under translations");
      if (s->group == PP_GROUP_DIHEDRAL) {
        const uint64_t r1[1] = {reflect(x)}, r2[1] = {reflect(z)};
        auto jt = mult.find(key(r1, r2, std::get<4>(k)));
        if (jt == mult.end() || jt->second != m)
          return fail(PP_ENOTSYM, "gate layer is not closed under the reflection");
      }
    }
  } else if (s->group == PP_GROUP_TORUS) {
    // closed under the two generators: x + 1 within each row, y + 1
    std::map<Key, long> mult;
    for (size_t k = 0; k < K; ++k) mult[key(gx + k * W, gz + k * W, theta[k])] += 1;
    const int lx = s->lx, ly = n / lx;
    auto shift = [&](uint64_t v, int a, int b) {   // qubit (x,y) <- (x+a, y+b)
      uint64_t r = 0;
      for (int y = 0; y < ly; ++y)
        for (int x = 0; x < lx; ++x)
          if ((v >> ((x + a) % lx + lx * ((y + b) % ly))) & 1) r |= 1ull << (x + lx * y);
      return r;
    };
    for (const auto& [k, m] : mult) {
      const uint64_t x = std::get<0>(k), z = std::get<2>(k);
      for (int g = 0; g < 2; ++g) {
        const uint64_t t1[1] = {shift(x, g == 0, g == 1)}, t2[1] = {shift(z, g == 0, g == 1)};
        auto it = mult.find(key(t1, t2, std::get<4>(k)));
        if (it == mult.end() || it->second != m)
          return fail(PP_ENOTSYM, "gate layer is not closed under the torus translations");
      }
    }
  } else if (s->group == PP_GROUP_EXPLICIT) {
    std::map<Key, long> mult;
    for (size_t k = 0; k < K; ++k) mult[key(gx + k * W, gz + k * W, theta[k])] += 1;
    const size_t m = s->gperm.size() / n;
    for (const auto& [k, mu] : mult) {
      const uint64_t x = std::get<0>(k), z = std::get<2>(k);
      for (size_t g = 0; g < m; ++g) {
        const uint8_t* p = &s->gperm[g * n];
        uint64_t tx = 0, tz = 0;
        for (int q = 0; q < n; ++q) {
          tx |= ((x >> p[q]) & 1ull) << q;
          tz |= ((z >> p[q]) & 1ull) << q;
        }
        const uint64_t t1[1] = {tx}, t2[1] = {tz};
        auto it = mult.find(key(t1, t2, std::get<4>(k)));
        if (it == mult.end() || it->second != mu)
          return fail(PP_ENOTSYM, "gate layer is not closed under the group");
      }
    }
  } else if (s->group == PP_GROUP_PERMUTATION) {
    std::map<std::tuple<int, int, int, double>, long> cls;
    std::map<Key, long> mult;
    for (size_t k = 0; k < K; ++k) {
      const uint64_t* x = gx + k * W;
      const uint64_t* z = gz + k * W;
      int a = 0, b = 0, c = 0;
      for (int w = 0; w < W; ++w) {
        a += __builtin_popcountll(x[w] & ~z[w]);
        b += __builtin_popcountll(x[w] & z[w]);
        c += __builtin_popcountll(z[w] & ~x[w]);
      }
      cls[{a, b, c, theta[k]}] += 1;
      if (++mult[key(x, z, theta[k])] > 1)
        return fail(PP_ENOTSYM, "repeated gate in a permutation-symmetric layer");
    }
    for (const auto& [c, m] : cls) {
      // number of distinct strings with (nX, nY, nZ) letters: multinomial
      const int a = std::get<0>(c), b = std::get<1>(c), cc = std::get<2>(c);
      double lg = std::lgamma(n + 1.0) - std::lgamma(a + 1.0) - std::lgamma(b + 1.0) -
                  std::lgamma(cc + 1.0) - std::lgamma(n - a - b - cc + 1.0);
      const double cnt = std::exp(lg);
      if (std::fabs(cnt - (double)m) > 0.5)
        return fail(PP_ENOTSYM, "gate layer is not closed under permutations");
    }
  }
  return PP_OK;
}

}  // namespace

extern "C" {

const char* pp_last_error(void) { return g_err.c_str(); }

int pp_set_tuning(int gate_items, int stream_items, int max_blocks, int graph_steps,
                  int gates_per_step) {
  auto ok_items = [](int v) { return v == 0 || v == 1 || v == 2 || v == 4 || v == 8; };
  if (!ok_items(gate_items) || !ok_items(stream_items))
    return fail(PP_EINVAL, "items per thread must be 0 (keep), 1, 2, 4 or 8");
  if (max_blocks < 0 || graph_steps < 0 || gates_per_step < 0 || gates_per_step > 64)
    return fail(PP_EINVAL, "tuning value out of range");
  if (gate_items) g_tune.gate_items = gate_items;
  if (stream_items) g_tune.stream_items = stream_items;
  if (max_blocks) g_tune.max_blocks = max_blocks;
  if (graph_steps) g_tune.graph_steps = graph_steps;
  if (gates_per_step) g_tune.gates_per_step = gates_per_step;
  return PP_OK;
}

int pp_set_merge_tuning(int bucket_log2, int agg_blocks) {
  if (bucket_log2 != 0 && (bucket_log2 < 10 || bucket_log2 > 18))
    return fail(PP_EINVAL, "bucket_log2 must be 0 (keep) or 10..18");
  if (agg_blocks < 0 || agg_blocks > 4096)
    return fail(PP_EINVAL, "agg_blocks must be 0 (one per item) .. 4096");
  if (bucket_log2) g_tune.part_shift = bucket_log2;
  g_tune.part_agg_blocks = agg_blocks;
  return PP_OK;
}

int pp_set_layer_tuning(int bucket_log2, int block) {
  if (bucket_log2 != 0 && (bucket_log2 < 4 || bucket_log2 > 11))
    return fail(PP_EINVAL, "bucket_log2 must be 0 (keep) or 4..11");
  if (block != 0 && block != 256 && block != 512)
    return fail(PP_EINVAL, "block must be 0 (keep), 256 or 512");
  if (bucket_log2) g_tune.layer_shift = bucket_log2;
  if (block) g_tune.layer_block = block;
  return PP_OK;
}

int pp_get_layer_tuning(int out[2]) {
  if (!out) return fail(PP_EINVAL, "NULL argument");
  out[0] = g_tune.layer_shift;
  out[1] = g_tune.layer_block;
  return PP_OK;
}

int pp_get_merge_tuning(int out[2]) {
  if (!out) return fail(PP_EINVAL, "NULL argument");
  out[0] = g_tune.part_shift;
  out[1] = g_tune.part_agg_blocks;
  return PP_OK;
}

int pp_set_gate_fusion(int max_rotations, int lanes) {
  if (max_rotations < 0 || max_rotations > kMaxFuse)
    return fail(PP_EINVAL, "max_rotations must be 0.." + std::to_string(kMaxFuse));
  if (lanes != 0 && lanes != 1) return fail(PP_EINVAL, "lanes must be 0 or 1");
  g_fuse = max_rotations;
  g_lanes = lanes;
  return PP_OK;
}

int pp_set_layer_ops(int mode) {
  if (mode < 0 || mode > 2) return fail(PP_EINVAL, "mode must be 0, 1 or 2");
  g_layer = mode;
  return PP_OK;
}

int pp_get_tuning(int out[5]) {
  if (!out) return fail(PP_EINVAL, "NULL argument");
  out[0] = g_tune.gate_items;
  out[1] = g_tune.stream_items;
  out[2] = g_tune.max_blocks;
  out[3] = g_tune.graph_steps;
  out[4] = g_tune.gates_per_step;
  return PP_OK;
}

void pp_destroy(pp_state* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  free_store(s, s->store);
  dev_free(s, s->d_ops);
  dev_free(s, s->d_tab);
  dev_free(s, s->d_buf);
  dev_free(s, s->d_dyn);
  dev_free(s, s->d_bufp);
  dev_free(s, s->d_dynp);
  dev_free(s, s->d_ninst);
  dev_free(s, s->d_sync);
  dev_free(s, s->d_stats);
  dev_free(s, s->d_gperm);
  if (s->h_dyn) (void)hipHostFree(s->h_dyn);
  if (s->h_na) (void)hipHostFree(s->h_na);
  for (auto& st : s->ring) {
    if (st.h) (void)hipHostFree(st.h);
    if (st.ev) (void)hipEventDestroy(st.ev);
  }
  prof_resolve(s);
  for (hipEvent_t e : s->pool) (void)hipEventDestroy(e);
  if (s->solo_slots) (void)hipHostFree(s->solo_slots);
  for (auto e : s->solo_ev)
    if (e) (void)hipEventDestroy(e);
  delete s;
}

namespace {

// pp_create and pp_create_torus (lx = torus width, 0 for the other groups).
int create_handle(pp_state** out, int n_qubits, int group, int lx, int dtype,
                  const uint64_t* obs_x, const uint64_t* obs_z, const double* obs_coef,
                  size_t n_obs, void* hip_stream, const pp_allocator* alloc,
                  const std::vector<uint8_t>* gperm = nullptr) {
  if (!out) return fail(PP_EINVAL, "out is NULL");
  *out = nullptr;
  if (dtype != PP_F64 && dtype != PP_F32_COMPENSATED)
    return fail(PP_EINVAL, "dtype must be PP_F64 or PP_F32_COMPENSATED");
  if (n_obs && (!obs_x || !obs_z || !obs_coef)) return fail(PP_EINVAL, "observable is NULL");
  if (n_obs > 0x3FFFFFFFull) return fail(PP_EINVAL, "too many observable rows");
  const int W = (n_qubits + 63) / 64;
  for (size_t r = 0; r < n_obs; ++r)
    if (!row_in_range(obs_x + r * W, obs_z + r * W, n_qubits, W))
      return fail(PP_EINVAL, "observable row " + std::to_string(r) + " has bits >= n_qubits");
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(PP_EINVAL, "incomplete allocator");

  std::unique_ptr<pp_state> s(new pp_state);
  s->n = n_qubits;
  s->W = W;
  s->group = group;
  s->stream = (hipStream_t)hip_stream;
  s->prof_every = g_prof_default;
  if (alloc) {
    s->alloc = *alloc;
    s->use_alloc = true;
  }
  std::memset(&s->buf, 0, sizeof(InstBuf));
  s->buf.n = n_qubits;
  s->buf.W = W;
  s->buf.group = group;
  s->buf.narrow = (group == PP_GROUP_PERMUTATION || n_qubits <= 32) ? 1u : 0u;
  s->buf.f32 = dtype == PP_F32_COMPENSATED ? 1u : 0u;
  s->buf.lx = lx;
  s->lx = lx;

  HIP_TRY(hipHostMalloc((void**)&s->h_dyn, sizeof(InstDyn), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void**)&s->h_na, 2 * sizeof(double), hipHostMallocDefault));
  s->d_buf = (InstBuf*)dev_alloc(s.get(), sizeof(InstBuf));
  s->d_dyn = (InstDyn*)dev_alloc(s.get(), sizeof(InstDyn));
  s->d_bufp = (const InstBuf**)dev_alloc(s.get(), sizeof(void*));
  s->d_dynp = (InstDyn**)dev_alloc(s.get(), sizeof(void*));
  s->d_ninst = (int*)dev_alloc(s.get(), sizeof(int));
  s->d_sync = (uint32_t*)dev_alloc(s.get(), kSyncBytes);
  s->d_stats = (uint64_t*)dev_alloc(s.get(), kStatBytes);
  s->buf.stats = s->d_stats;
  if (!s->d_buf || !s->d_dyn || !s->d_bufp || !s->d_dynp || !s->d_ninst || !s->d_sync ||
      !s->d_stats) {
    pp_destroy(s.release());
    return fail(PP_ENOMEM, "handle allocation failed");
  }
  const int one = 1;
  int rc;
  auto bail = [&](int code) {
    pp_destroy(s.release());
    return code;
  };
  if (gperm) {                            // the group's element list, on the device
    s->gperm = *gperm;
    s->d_gperm = (uint8_t*)dev_alloc(s.get(), s->gperm.size());
    if (!s->d_gperm) return bail(fail(PP_ENOMEM, "group element list allocation failed"));
    if (hipMemcpyAsync(s->d_gperm, s->gperm.data(), s->gperm.size(), hipMemcpyHostToDevice,
                       s->stream))
      return bail(fail(PP_EDEVICE, "group element list upload failed"));
    s->buf.gperm = s->d_gperm;
    s->buf.gsize = (uint32_t)(s->gperm.size() / n_qubits);
  }
  if (hipMemcpyAsync(s->d_bufp, &s->d_buf, sizeof(void*), hipMemcpyHostToDevice, s->stream) ||
      hipMemcpyAsync(s->d_dynp, &s->d_dyn, sizeof(void*), hipMemcpyHostToDevice, s->stream) ||
      hipMemcpyAsync(s->d_ninst, &one, sizeof(int), hipMemcpyHostToDevice, s->stream) ||
      hipMemsetAsync(s->d_sync, 0, kSyncBytes, s->stream) ||
      hipMemsetAsync(s->d_stats, 0, kStatBytes, s->stream))
    return bail(fail(PP_EDEVICE, "handle initialisation failed"));

  const uint32_t cap = (uint32_t)std::max<uint64_t>(4096, 2 * n_obs);
  if ((rc = alloc_store(s.get(), cap, &s->buf, &s->store))) return bail(rc);

  // rows -> word-major planes of half 0, all alive
  std::vector<uint64_t> xs((size_t)W * cap, 0), zs((size_t)W * cap, 0);
  for (size_t r = 0; r < n_obs; ++r)
    for (int w = 0; w < W; ++w) {
      xs[(size_t)w * cap + r] = obs_x[r * W + w];
      zs[(size_t)w * cap + r] = obs_z[r * W + w];
    }
  std::vector<uint8_t> ones(std::max<size_t>(n_obs, 1), 1);
  // FP32 storage: each observable coefficient is rounded once
  std::vector<float> cf(s->buf.f32 ? n_obs : 0);
  for (size_t r = 0; r < cf.size(); ++r) cf[r] = (float)obs_coef[r];
  const void* csrc = s->buf.f32 ? (const void*)cf.data() : (const void*)obs_coef;
  const size_t csize = (s->buf.f32 ? sizeof(float) : sizeof(double)) * n_obs;
  if (hipMemcpyAsync(s->buf.x[0], xs.data(), sizeof(uint64_t) * xs.size(), hipMemcpyHostToDevice,
                     s->stream) ||
      hipMemcpyAsync(s->buf.z[0], zs.data(), sizeof(uint64_t) * zs.size(), hipMemcpyHostToDevice,
                     s->stream) ||
      (n_obs && hipMemcpyAsync(s->buf.c[0], csrc, csize, hipMemcpyHostToDevice, s->stream)) ||
      (n_obs && hipMemcpyAsync(s->buf.alive[0][0], ones.data(), n_obs, hipMemcpyHostToDevice,
                               s->stream)))
    return bail(fail(PP_EDEVICE, "observable upload failed"));
  InstDyn& d = *s->h_dyn;
  std::memset(&d, 0, sizeof(InstDyn));
  d.M = d.Mnext = (uint32_t)n_obs;
  d.peak = (uint32_t)n_obs;
  d.gen = 1;
  d.count_for = kNone32;
  d.live = (uint32_t)n_obs;
  d.seed = 1;
  d.failed_pc = kNone32;
  s->m_hint = (uint32_t)n_obs;
  if (hipMemcpyAsync(s->d_dyn, &d, sizeof(InstDyn), hipMemcpyHostToDevice, s->stream))
    return bail(fail(PP_EDEVICE, "state upload failed"));
  // Algorithm 1, step 1: merge the rows by representative (duplicates too)
  std::vector<Op> ops(1, make_op(OP_MERGE));
  ops[0].force_full = 1;
  if ((rc = run_ops(s.get(), ops, {}, {}, false))) return bail(rc);
  *out = s.release();
  return PP_OK;
}

}  // namespace

int pp_create(pp_state** out, int n_qubits, int group, int dtype, const uint64_t* obs_x,
              const uint64_t* obs_z, const double* obs_coef, size_t n_obs, void* hip_stream,
              const pp_allocator* alloc) {
  if (!valid_group_n(group, n_qubits))
    return fail(PP_EINVAL, "unsupported (group, n_qubits) = (" + std::to_string(group) + ", " +
                               std::to_string(n_qubits) + ")");
  return create_handle(out, n_qubits, group, 0, dtype, obs_x, obs_z, obs_coef, n_obs, hip_stream,
                       alloc);
}

int pp_create_group(pp_state** out, int n_qubits, const uint8_t* perms, size_t n_elems,
                    int dtype, const uint64_t* obs_x, const uint64_t* obs_z,
                    const double* obs_coef, size_t n_obs, void* hip_stream,
                    const pp_allocator* alloc) {
  const int n = n_qubits;
  if (n < 2 || n > 64) return fail(PP_EINVAL, "explicit groups need 2 <= n_qubits <= 64");
  if (!perms || n_elems < 1 || n_elems > 1024)
    return fail(PP_EINVAL, "the element list needs 1..1024 rows");
  std::set<std::vector<uint8_t>> rows;
  for (size_t g = 0; g < n_elems; ++g) {
    std::vector<uint8_t> r(perms + g * n, perms + (g + 1) * n);
    std::vector<uint8_t> seen(n, 0);
    for (uint8_t q : r) {
      if (q >= n || seen[q]) return fail(PP_EINVAL, "row " + std::to_string(g) + " is not a permutation");
      seen[q] = 1;
    }
    if (!rows.insert(r).second) return fail(PP_EINVAL, "repeated group element");
  }
  std::vector<uint8_t> id(n);
  for (int q = 0; q < n; ++q) id[q] = (uint8_t)q;
  if (!rows.count(id)) return fail(PP_EINVAL, "the identity is not in the element list");
  std::vector<uint8_t> c(n);
  for (const auto& a : rows)                // (a.(b.s))[q] = s[b[a[q]]]
    for (const auto& b : rows) {
      for (int q = 0; q < n; ++q) c[q] = b[a[q]];
      if (!rows.count(c)) return fail(PP_EINVAL, "the element list is not closed under composition");
    }
  const std::vector<uint8_t> flat(perms, perms + n_elems * n);
  return create_handle(out, n, PP_GROUP_EXPLICIT, 0, dtype, obs_x, obs_z, obs_coef, n_obs,
                       hip_stream, alloc, &flat);
}

int pp_create_torus(pp_state** out, int lx, int ly, int dtype, const uint64_t* obs_x,
                    const uint64_t* obs_z, const double* obs_coef, size_t n_obs,
                    void* hip_stream, const pp_allocator* alloc) {
  if (lx < 1 || ly < 1 || lx * ly < 2 || lx * ly > 64)
    return fail(PP_EINVAL, "unsupported torus " + std::to_string(lx) + " x " + std::to_string(ly));
  return create_handle(out, lx * ly, PP_GROUP_TORUS, lx, dtype, obs_x, obs_z, obs_coef, n_obs,
                       hip_stream, alloc);
}

int pp_work_counters(pp_state* s, uint64_t out[8]) {
  if (!s || !out) return fail(PP_EINVAL, "NULL argument");
  return read_counters(s, out);
}

int pp_store_bytes(int n_qubits, int group, int dtype, size_t cap, size_t* out) {
  if (!out) return fail(PP_EINVAL, "NULL argument");
  if (!valid_group_n(group, n_qubits) && group != PP_GROUP_EXPLICIT)
    return fail(PP_EINVAL, "unsupported (group, n_qubits)");
  if (cap == 0 || cap > 0xFFFFFFF0ull) return fail(PP_EINVAL, "cap out of range");
  pp_state st;
  st.n = n_qubits;
  st.W = (n_qubits + 63) / 64;
  st.group = group;
  std::memset(&st.buf, 0, sizeof(InstBuf));
  st.buf.n = n_qubits;
  st.buf.W = st.W;
  st.buf.group = group;
  st.buf.narrow = (group == PP_GROUP_PERMUTATION || n_qubits <= 32) ? 1u : 0u;
  st.buf.f32 = dtype == PP_F32_COMPENSATED ? 1u : 0u;
  InstBuf b;
  std::vector<void*> none;
  size_t bytes = 0;
  int rc = alloc_store(&st, (uint32_t)cap, &b, &none, &bytes);
  if (rc) return rc;
  *out = bytes;
  return PP_OK;
}

int pp_layer_stats(pp_state* s, uint64_t out[4]) {
  if (!s || !out) return fail(PP_EINVAL, "NULL argument");
  int rc = read_dyn(s);
  if (rc) return rc;
  out[0] = s->h_dyn->lops;
  out[1] = s->h_dyn->lfails;
  out[2] = (uint64_t)s->layer_fallbacks + s->h_dyn->lfb;
  out[3] = s->layer_off ? 1u : 0u;
  return PP_OK;
}

int pp_peak_terms(pp_state* s, size_t* out) {
  if (!s || !out) return fail(PP_EINVAL, "NULL argument");
  int rc = read_dyn(s);
  if (rc) return rc;
  *out = s->h_dyn->peak;
  return PP_OK;
}

int pp_merge_stats(pp_state* s, uint64_t out[4]) {
  if (!s || !out) return fail(PP_EINVAL, "NULL argument");
  int rc = read_dyn(s);
  if (rc) return rc;
  const InstDyn& d = *s->h_dyn;
  out[0] = d.pruns;
  out[1] = d.phot;
  out[2] = d.pover;
  out[3] = d.pglob;
  return PP_OK;
}

int pp_profile(pp_state* s, int every) {
  if (every < 0) return fail(PP_EINVAL, "every must be >= 0");
  if (!s) {
    g_prof_default = every;
    return PP_OK;
  }
  int rc = read_dyn(s);
  if (rc) return rc;
  s->prof_every = every;
  for (int k = 0; k < PP_KERNEL_KINDS; ++k) {
    s->prof_n[k] = 0;
    s->prof_ms[k] = 0.0;
    s->prof_seen[k] = 0;
  }
  return PP_OK;
}

int pp_profile_read(pp_state* s, uint64_t launches[PP_KERNEL_KINDS],
                    double milliseconds[PP_KERNEL_KINDS]) {
  if (!s || !launches || !milliseconds) return fail(PP_EINVAL, "NULL argument");
  int rc = read_dyn(s);
  if (rc) return rc;
  for (int k = 0; k < PP_KERNEL_KINDS; ++k) {
    launches[k] = s->prof_n[k];
    milliseconds[k] = s->prof_ms[k];
  }
  return PP_OK;
}

int pp_set_max_terms(pp_state* s, size_t max_terms) {
  if (!s) return fail(PP_EINVAL, "state is NULL");
  s->max_terms = max_terms;
  return PP_OK;
}

// Transactions.  A gate rotates coefficients in place and flips the alive
// parity; it never changes a key below the entry count M (children go past
// M), and a merge writes only the other half.  So the state of a call's
// start is restored from: the instance's dynamic state, the statistics
// lines, and the first M coefficients and current-parity alive flags of the
// current half; plus the store itself when the call grew it (the old one is
// kept until the call ends).  The copies are stream-ordered (no
// synchronisation); M, half and parity come from the host mirror, which
// every call that can change them refreshes.
size_t txn_bytes(const pp_state* s, uint32_t M) {
  const size_t cs = s->buf.f32 ? sizeof(float) : sizeof(double);
  return sizeof(InstDyn) + kStatBytes + (size_t)M * (cs + 1) + 64;
}

int txn_begin(pp_state* s) {
  const InstDyn& h = *s->h_dyn;
  const uint32_t M = h.M;
  void* b = dev_alloc(s, txn_bytes(s, M));
  if (!b) return fail(PP_ENOMEM, "transaction backup allocation failed");
  char* p = static_cast<char*>(b);
  const size_t cs = s->buf.f32 ? sizeof(float) : sizeof(double);
  HIP_TRY(hipMemcpyAsync(p, s->d_dyn, sizeof(InstDyn), hipMemcpyDeviceToDevice, s->stream));
  p += sizeof(InstDyn);
  HIP_TRY(hipMemcpyAsync(p, s->d_stats, kStatBytes, hipMemcpyDeviceToDevice, s->stream));
  p += kStatBytes;
  if (M) {
    HIP_TRY(hipMemcpyAsync(p, s->buf.c[h.half], (size_t)M * cs, hipMemcpyDeviceToDevice,
                           s->stream));
    p += (size_t)M * cs;
    HIP_TRY(hipMemcpyAsync(p, s->buf.alive[h.half][h.parity], M, hipMemcpyDeviceToDevice,
                           s->stream));
  }
  s->txn = true;
  s->txn_buf = s->buf;
  s->txn_backup = b;
  s->txn_m = M;
  s->txn_half = h.half;
  s->txn_parity = h.parity;
  return PP_OK;
}

void txn_end(pp_state* s) {
  dev_free(s, s->txn_backup);
  s->txn_backup = nullptr;
  for (auto& st : s->retired) free_store(s, st);
  s->retired.clear();
  s->txn = false;
}

// Restores the state of the call's start; returns `rc` (the call's error).
int txn_rollback(pp_state* s, int rc) {
  const std::string msg = g_err;
  if (s->buf.x[0] != s->txn_buf.x[0] && !s->retired.empty()) {
    free_store(s, s->store);                     // the grown store
    s->store = std::move(s->retired.front());
    s->retired.erase(s->retired.begin());
  }
  s->buf = s->txn_buf;
  char* p = static_cast<char*>(s->txn_backup);
  const size_t cs = s->buf.f32 ? sizeof(float) : sizeof(double);
  const uint32_t M = s->txn_m;
  bool ok = hipMemcpyAsync(s->d_buf, &s->buf, sizeof(InstBuf), hipMemcpyHostToDevice,
                           s->stream) == hipSuccess;
  ok = ok && hipMemcpyAsync(s->d_dyn, p, sizeof(InstDyn), hipMemcpyDeviceToDevice,
                            s->stream) == hipSuccess;
  p += sizeof(InstDyn);
  ok = ok && hipMemcpyAsync(s->d_stats, p, kStatBytes, hipMemcpyDeviceToDevice,
                            s->stream) == hipSuccess;
  p += kStatBytes;
  if (M) {
    ok = ok && hipMemcpyAsync(s->buf.c[s->txn_half], p, (size_t)M * cs,
                              hipMemcpyDeviceToDevice, s->stream) == hipSuccess;
    p += (size_t)M * cs;
    ok = ok && hipMemcpyAsync(s->buf.alive[s->txn_half][s->txn_parity], p, M,
                              hipMemcpyDeviceToDevice, s->stream) == hipSuccess;
  }
  ok = ok && hipStreamSynchronize(s->stream) == hipSuccess;
  txn_end(s);
  if (ok) (void)read_dyn(s);
  g_err = ok ? msg + " (the handle is as before the call)"
             : msg + " (restoring the handle's state also failed)";
  return ok ? rc : PP_EDEVICE;
}

// Runs ops as one transaction: on any error the handle is restored.
int run_ops_txn(pp_state* s, const std::vector<Op>& ops) {
  int rc = txn_begin(s);
  if (rc) return rc;
  rc = run_ops(s, ops, {}, {}, false);
  if (rc) return txn_rollback(s, rc);
  txn_end(s);
  return PP_OK;
}

int pp_apply_layer(pp_state* s, const uint64_t* gate_x, const uint64_t* gate_z,
                   const double* theta, size_t n_gates, int merge_every, double inner_eps,
                   int inner_max_weight) {
  if (!s) return fail(PP_EINVAL, "state is NULL");
  if (merge_every != 1) return fail(PP_EINVAL, "merge_every must be 1");
  if (!(inner_eps >= 0.0)) return fail(PP_EINVAL, "inner_eps must be >= 0");
  if (n_gates == 0) return PP_OK;
  if (!gate_x || !gate_z || !theta) return fail(PP_EINVAL, "gate arrays are NULL");
  const int W = s->W;
  for (size_t k = 0; k < n_gates; ++k) {
    if (!row_in_range(gate_x + k * W, gate_z + k * W, s->n, W))
      return fail(PP_EINVAL, "gate " + std::to_string(k) + " has bits >= n_qubits");
    if (!std::isfinite(theta[k])) return fail(PP_EINVAL, "non-finite angle");
  }
  int rc = check_symmetric(s, gate_x, gate_z, theta, n_gates);
  if (rc) return rc;
  std::vector<Op> ops;
  ops.reserve(n_gates + 1);
  ops.push_back(make_op(OP_COUNT));
  for (size_t k = 0; k < n_gates; ++k) {
    Op op = make_op(OP_GATE);
    for (int w = 0; w < W; ++w) {
      op.px[w] = gate_x[k * W + w];
      op.pz[w] = gate_z[k * W + w];
    }
    op.cs = std::cos(theta[k]);
    op.sn = std::sin(theta[k]);
    op.eps = inner_eps;
    op.wmax = inner_max_weight < 0 ? -1 : inner_max_weight;
    op.full_check = k == 0;
    ops.push_back(op);
  }
  fuse_gates(ops, 1, W);
  set_next_gates(ops);
  return run_ops_txn(s, ops);
}

int pp_merge_canonicalize(pp_state* s) {
  if (!s) return fail(PP_EINVAL, "state is NULL");
  std::vector<Op> ops(1, make_op(OP_MERGE));
  return run_ops_txn(s, ops);
}

int pp_truncate(pp_state* s, double eps, int max_weight, double depol_p) {
  if (!s) return fail(PP_EINVAL, "state is NULL");
  if (!(eps >= 0.0)) return fail(PP_EINVAL, "eps must be >= 0");
  if (!(depol_p >= 0.0 && depol_p <= 1.0)) return fail(PP_EINVAL, "depol_p must be in [0, 1]");
  std::vector<Op> ops;
  std::vector<double> tab;
  TabRefs refs;
  if (depol_p > 0.0) {
    refs.push_back({ops.size(), tab.size()});
    for (int w = 0; w <= s->n; ++w) tab.push_back(std::pow(1.0 - depol_p, (double)w));
    ops.push_back(make_op(OP_DAMP));
  }
  if (eps > 0.0 || max_weight >= 0) {
    Op op = make_op(OP_TRUNC);
    op.eps = eps;
    op.wmax = max_weight < 0 ? -1 : max_weight;
    ops.push_back(op);
  }
  return run_ops(s, ops, tab, refs, true);
}

int pp_expectation(pp_state* s, const double bloch_xyz[3], double* out) {
  if (!s || !bloch_xyz || !out) return fail(PP_EINVAL, "NULL argument");
  std::vector<double> tab;
  for (int a = 0; a < 3; ++a) {
    double p = 1.0;
    for (int k = 0; k <= s->n; ++k) {
      tab.push_back(p);
      p *= bloch_xyz[a];
    }
  }
  std::vector<Op> ops(1, make_op(OP_EXPECT));
  int rc = run_ops(s, ops, tab, {{0, 0}}, false);
  if (rc) return rc;
  *out = s->h_dyn->expect;
  return PP_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free expectation.  Its working memory (the powers table, one
// exact partial sum per tile of kNaTile entries, the done counter, the
// result) is the file-scope device array `scratch`, of a fixed size; every
// GPU holds its own copy.  Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (na_scratch_ptr).
// ---------------------------------------------------------------------------
namespace {

constexpr int kNaTile = 2048;                  // entries per tile (256 threads x 8)
constexpr uint32_t kNaMaxTiles = 65536;        // entries at most 2^27
constexpr int kNaTab = 3 * (64 * kMaxW + 1);   // bx^k, by^k, bz^k for k = 0..n

struct NaScratch {
  double tab[kNaTab];
  double result;
  uint32_t range;                              // a term out of the fixed-point range
  uint32_t done;                               // blocks done
  uint64_t part[kNaMaxTiles][3];               // exact partial sum of each tile
};

static __device__ __align__(256) unsigned char scratch[sizeof(NaScratch)];

// Powers table (the same products, in the same order, as pp_expectation's
// host table), and the counters cleared by a kernel rather than a memset.
__global__ void k_na_init(NaScratch* sc, double bx, double by, double bz, int n) {
  const int a = threadIdx.x;
  if (a < 3) {
    const double b = a == 0 ? bx : a == 1 ? by : bz;
    double p = 1.0;
    for (int k = 0; k <= n; ++k) {
      sc->tab[a * (n + 1) + k] = p;
      p *= b;
    }
  }
  if (a == 0) {
    sc->range = 0;
    sc->done = 0;
    sc->result = 0.0;
  }
}

// One exact partial sum per tile of live terms (the expectation's terms as
// the scan kernel forms them), then the last block adds the partials and
// rounds once.
__global__ __launch_bounds__(kBlock) void k_na_expect(InstBuf b, const InstDyn* dp, NaScratch* sc,
                                                      uint32_t tiles) {
  __shared__ uint64_t s_w[kWaves][3];
  __shared__ uint32_t s_last;
  const InstDyn& d = *dp;
  const View v = view_of(b, d);
  const uint32_t M = d.M;
  const int W = b.W, n = b.n;
  bool range = false;
  for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    Fx acc{0, 0, 0};
    for (int k = 0; k < kNaTile / kBlock; ++k) {
      const uint32_t i = t * kNaTile + k * kBlock + threadIdx.x;
      if (i >= M || !v.al[i]) continue;
      uint64_t x[kMaxW], z[kMaxW];
      load_key(v, i, x, z);
      uint32_t nx, ny, nz;
      perm_counts(x, z, W, &nx, &ny, &nz);
      const double term = v.getc(i) * sc->tab[nx] * sc->tab[(n + 1) + ny] * sc->tab[2 * (n + 1) + nz];
      acc = fx_add(acc, fx_from_double(term, &range));
    }
    const Fx w = wave_sum_fx(acc);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { s_w[wid][0] = w.l0; s_w[wid][1] = w.l1; s_w[wid][2] = w.l2; }
    __syncthreads();
    if (threadIdx.x == 0) {
      Fx s{0, 0, 0};
      for (int q = 0; q < kWaves; ++q) s = fx_add(s, Fx{s_w[q][0], s_w[q][1], s_w[q][2]});
      sc->part[t][0] = s.l0;
      sc->part[t][1] = s.l1;
      sc->part[t][2] = s.l2;
    }
    __syncthreads();
  }
  if (range) atomicOr(&sc->range, 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(&sc->done, 1u) == gridDim.x - 1 ? 1u : 0u;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  Fx acc{0, 0, 0};
  for (uint32_t t = threadIdx.x; t < tiles; t += kBlock)
    acc = fx_add(acc, Fx{ld_agent(&sc->part[t][0]), ld_agent(&sc->part[t][1]),
                         ld_agent(&sc->part[t][2])});
  const Fx w = wave_sum_fx(acc);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { s_w[wid][0] = w.l0; s_w[wid][1] = w.l1; s_w[wid][2] = w.l2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    Fx s{0, 0, 0};
    for (int q = 0; q < kWaves; ++q) s = fx_add(s, Fx{s_w[q][0], s_w[q][1], s_w[q][2]});
    sc->result = fx_to_double(s);
    sc->done = 0;
  }
}

std::mutex g_na_mu;
void* g_na_ptr[256] = {};                      // scratch's address, per device

// The device address of `scratch` on the current device (looked up once per
// device, with that device current).
int na_scratch_ptr(NaScratch** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 256) return fail(PP_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_na_ptr[dev] = p;
  }
  *out = static_cast<NaScratch*>(g_na_ptr[dev]);
  return PP_OK;
}

}  // namespace

int pp_expectation_noalloc(pp_state* s, const double bloch_xyz[3], double* out) {
  if (!s || !bloch_xyz || !out) return fail(PP_EINVAL, "NULL argument");
  NaScratch* sc = nullptr;
  int rc = na_scratch_ptr(&sc);
  if (rc) return rc;
  if ((rc = read_dyn(s))) return rc;            // the entry count, into pinned memory
  const uint32_t M = s->h_dyn->M;
  const uint64_t tiles = ((uint64_t)M + kNaTile - 1) / kNaTile;
  if (tiles > kNaMaxTiles)
    return fail(PP_EINVAL, "pp_expectation_noalloc takes stores of at most " +
                               std::to_string((uint64_t)kNaMaxTiles * kNaTile) +
                               " entries (this one holds " + std::to_string(M) + ")");
  hipLaunchKernelGGL(k_na_init, dim3(1), dim3(64), 0, s->stream, sc, bloch_xyz[0], bloch_xyz[1],
                     bloch_xyz[2], s->n);
  const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(tiles, 2048));
  hipLaunchKernelGGL(k_na_expect, dim3(grid), dim3(kBlock), 0, s->stream, s->buf,
                     (const InstDyn*)s->d_dyn, sc, (uint32_t)tiles);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(s->h_na, &sc->result, 2 * sizeof(double), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  uint32_t range = 0;
  std::memcpy(&range, s->h_na + 1, sizeof(range));
  if (range) return fail(PP_EINVAL, "a coefficient is not finite or exceeds 2^54 in magnitude");
  *out = s->h_na[0];
  return PP_OK;
}

int pp_num_terms(pp_state* s, size_t* out) {
  if (!s || !out) return fail(PP_EINVAL, "NULL argument");
  int rc = read_dyn(s);
  if (rc) return rc;
  *out = s->h_dyn->live;
  return PP_OK;
}

int pp_counters(pp_state* s, uint64_t out[2]) {
  if (!s || !out) return fail(PP_EINVAL, "NULL argument");
  uint64_t all[8];
  int rc = read_counters(s, all);
  if (rc) return rc;
  out[0] = all[0];
  out[1] = all[1];
  return PP_OK;
}

int pp_export_terms(pp_state* s, uint64_t* x, uint64_t* z, double* coef, size_t cap,
                    size_t* n_out) {
  if (!s || !n_out) return fail(PP_EINVAL, "NULL argument");
  int rc = read_dyn(s);
  if (rc) return rc;
  const InstDyn d = *s->h_dyn;
  if (cap < d.live) return fail(PP_EINVAL, "export capacity " + std::to_string(cap) + " < " +
                                               std::to_string(d.live) + " live terms");
  if (d.live && (!x || !z || !coef)) return fail(PP_EINVAL, "export arrays are NULL");
  *n_out = 0;
  const int W = s->W, n = s->n;
  const uint32_t M = d.M, C = s->buf.cap, N = (uint32_t)d.live;
  if (N == 0) return PP_OK;
  // Workspace: two orders, the histogram of the first pass (the largest),
  // the scan's block totals and grand total, and the rows.
  const uint32_t tiles0 = (M + kSortTile - 1) / kSortTile;
  const size_t nhist = (size_t)kSortBlock * tiles0;
  const uint32_t nscan = (uint32_t)((nhist + kScanTile - 1) / kScanTile);
  const size_t rows = (size_t)N * W * sizeof(uint64_t);
  struct Ws {
    pp_state* s;
    std::vector<void*> p;
    ~Ws() { for (void* q : p) dev_free(s, q); }
    void* get(size_t bytes) {
      void* q = dev_alloc(s, bytes);
      if (q) p.push_back(q);
      return q;
    }
  } ws{s, {}};
  auto* ord0 = static_cast<uint32_t*>(ws.get(sizeof(uint32_t) * N));
  auto* ord1 = static_cast<uint32_t*>(ws.get(sizeof(uint32_t) * N));
  auto* hist = static_cast<uint32_t*>(ws.get(sizeof(uint32_t) * nhist));
  auto* part = static_cast<uint32_t*>(ws.get(sizeof(uint32_t) * (nscan + 1)));
  auto* ox = static_cast<uint64_t*>(ws.get(rows));
  auto* oz = static_cast<uint64_t*>(ws.get(rows));
  auto* oc = static_cast<double*>(ws.get(sizeof(double) * N));
  if (!ord0 || !ord1 || !hist || !part || !ox || !oz || !oc)
    return fail(PP_ENOMEM, "export workspace");
  SortPass p{};
  p.x = s->buf.x[d.half];
  p.z = s->buf.z[d.half];
  p.alive = s->buf.alive[d.half][d.parity];
  p.cap = C;
  uint32_t* out = ord0;
  bool first = true;
  uint32_t total = 0;
  for (int j = 0; 32 * j < n; ++j) {
    const int bits = 2 * std::min(32, n - 32 * j);
    for (int sh = 0; sh < bits; sh += 8) {
      p.first = first;
      p.n_in = first ? M : N;
      p.tiles = (p.n_in + kSortTile - 1) / kSortTile;
      p.word = j;
      p.shift = sh;
      p.src = first ? nullptr : out;
      p.dst = first ? ord0 : (out == ord0 ? ord1 : ord0);
      p.dst_cap = N;
      p.hist = hist;
      const uint32_t nh = kSortBlock * p.tiles;
      const uint32_t nb = (nh + kScanTile - 1) / kScanTile;
      hipLaunchKernelGGL(k_sort_hist, dim3(p.tiles), dim3(kSortBlock), 0, s->stream, p);
      hipLaunchKernelGGL(k_sort_scan_reduce, dim3(nb), dim3(kSortBlock), 0, s->stream, hist, nh,
                         part);
      hipLaunchKernelGGL(k_sort_scan_top, dim3(1), dim3(kSortBlock), 0, s->stream, part, nb,
                         part + nscan);
      hipLaunchKernelGGL(k_sort_scan_down, dim3(nb), dim3(kSortBlock), 0, s->stream, hist, nh,
                         part);
      hipLaunchKernelGGL(k_sort_scatter, dim3(p.tiles), dim3(kSortBlock), 0, s->stream, p);
      HIP_TRY(hipGetLastError());
      if (first) {
        HIP_TRY(hipMemcpyAsync(&total, part + nscan, sizeof(uint32_t), hipMemcpyDeviceToHost,
                               s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        if (total != N)
          return fail(PP_EDEVICE, "live count mismatch: " + std::to_string(total) +
                                      " flagged, " + std::to_string(N) + " counted");
      }
      out = p.dst;
      first = false;
    }
  }
  hipLaunchKernelGGL(k_sort_emit, dim3((N + kSortBlock - 1) / kSortBlock), dim3(kSortBlock), 0,
                     s->stream, out, N, p.x, p.z, s->buf.c[d.half], (int)s->buf.f32, C, W, ox,
                     oz, oc);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(x, ox, rows, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(z, oz, rows, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(coef, oc, sizeof(double) * N, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  *n_out = N;
  return PP_OK;
}

// ---------------------------------------------------------------------------
// programs and the batched form
// ---------------------------------------------------------------------------
int pp_program_create(pp_program** out, int n_qubits, size_t n_sub, const size_t* sub_start,
                      const uint64_t* gate_x, const uint64_t* gate_z, const double* theta,
                      const double* eps, const int* max_weight, const double* depol_p,
                      const double bloch_xyz[3], const int* merge_after) {
  if (!out) return fail(PP_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_qubits < 1 || n_qubits > 128) return fail(PP_EINVAL, "n_qubits out of range");
  if (!sub_start || !eps || !max_weight || !depol_p || !bloch_xyz)
    return fail(PP_EINVAL, "NULL argument");
  const int W = (n_qubits + 63) / 64;
  const size_t K = sub_start[n_sub];
  if (sub_start[0] != 0) return fail(PP_EINVAL, "sub_start[0] must be 0");
  for (size_t j = 0; j < n_sub; ++j)
    if (sub_start[j + 1] < sub_start[j]) return fail(PP_EINVAL, "sub_start not monotone");
  if (K && (!gate_x || !gate_z || !theta)) return fail(PP_EINVAL, "gate arrays are NULL");
  for (size_t k = 0; k < K; ++k)
    if (!row_in_range(gate_x + k * W, gate_z + k * W, n_qubits, W))
      return fail(PP_EINVAL, "gate " + std::to_string(k) + " has bits >= n_qubits");
  std::unique_ptr<pp_program> p(new pp_program);
  p->n = n_qubits;
  p->n_gates = K;
  std::vector<double> tab;
  TabRefs refs;
  std::vector<Op>& ops = p->ops;
  ops.push_back(make_op(OP_COUNT));
  for (size_t j = 0; j < n_sub; ++j) {
    if (!(eps[j] >= 0.0) || !(depol_p[j] >= 0.0 && depol_p[j] <= 1.0))
      return fail(PP_EINVAL, "bad sub-layer parameters");
    if (depol_p[j] > 0.0) {
      refs.push_back({ops.size(), tab.size()});
      for (int w = 0; w <= n_qubits; ++w) tab.push_back(std::pow(1.0 - depol_p[j], (double)w));
      ops.push_back(make_op(OP_DAMP));
    }
    const size_t first_gate = ops.size();
    const bool merge_follows = !merge_after || merge_after[j];
    for (size_t k = sub_start[j]; k < sub_start[j + 1]; ++k) {
      Op op = make_op(OP_GATE);
      for (int w = 0; w < W; ++w) {
        op.px[w] = gate_x[k * W + w];
        op.pz[w] = gate_z[k * W + w];
      }
      op.cs = std::cos(theta[k]);
      op.sn = std::sin(theta[k]);
      op.eps = eps[j];
      op.wmax = max_weight[j] < 0 ? -1 : max_weight[j];
      op.full_check = k == sub_start[j];
      ops.push_back(op);
    }
    const size_t before = ops.size();
    add_layer_op(ops, first_gate, ops.size(), W, tab, refs, merge_follows);
    if (ops.size() == before) fuse_gates(ops, first_gate, W);
    const bool trunc = eps[j] > 0.0 || max_weight[j] >= 0;
    if (!merge_after || merge_after[j]) {
      Op merge = make_op(OP_MERGE);
      if (trunc) {                          // the truncation rides with the merge
        merge.trunc = 1;
        merge.eps = eps[j];
        merge.wmax = max_weight[j] < 0 ? -1 : max_weight[j];
      }
      ops.push_back(merge);
    } else if (trunc) {                     // merge deferred: truncation alone
      Op op = make_op(OP_TRUNC);
      op.eps = eps[j];
      op.wmax = max_weight[j] < 0 ? -1 : max_weight[j];
      ops.push_back(op);
    }
  }
  {
    refs.push_back({ops.size(), tab.size()});
    ops.push_back(make_op(OP_EXPECT));
    for (int a = 0; a < 3; ++a) {
      double v = 1.0;
      for (int k = 0; k <= n_qubits; ++k) {
        tab.push_back(v);
        v *= bloch_xyz[a];
      }
    }
  }
  set_next_gates(ops);
  for (const auto& op : ops) p->has_layer = p->has_layer || op.type == OP_LAYER;
  if (hipMalloc((void**)&p->d_ops, sizeof(Op) * ops.size()) != hipSuccess ||
      hipMalloc((void**)&p->d_tab, sizeof(double) * std::max<size_t>(tab.size(), 1)) !=
          hipSuccess) {
    pp_program_destroy(p.release());
    return fail(PP_ENOMEM, "program allocation failed");
  }
  for (const auto& r : refs) ops[r.first].table = p->d_tab + r.second;
  if (hipMemcpy(p->d_tab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice) ||
      hipMemcpy(p->d_ops, ops.data(), sizeof(Op) * ops.size(), hipMemcpyHostToDevice)) {
    pp_program_destroy(p.release());
    return fail(PP_EDEVICE, "program upload failed");
  }
  *out = p.release();
  return PP_OK;
}

int pp_program_info(const pp_program* p, uint64_t out[4]) {
  if (!p || !out) return fail(PP_EINVAL, "NULL argument");
  uint64_t gates = 0, layers = 0;  // apply ops the one-instance path runs
  for (const auto& op : p->ops) {
    gates += (op.type == OP_GATE || op.type == OP_GATES) && !op.fallback;
    layers += op.type == OP_LAYER;
  }
  out[0] = p->ops.size();
  out[1] = gates + layers;
  out[2] = p->n_gates;
  out[3] = layers;
  return PP_OK;
}

void pp_program_destroy(pp_program* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  if (p->d_ops) (void)hipFree(p->d_ops);
  if (p->d_tab) (void)hipFree(p->d_tab);
  delete p;
}

}  // extern "C"

namespace {

// One batched context per stream: device pointer arrays, a done counter and
// the captured graph of `graph_steps` steps.
struct BatchCtx {
  hipStream_t stream = nullptr;
  const InstBuf** d_bufp = nullptr;
  InstDyn** d_dynp = nullptr;
  int* d_ninst = nullptr;
  uint32_t* d_sync = nullptr;
  InstDyn* d_gather = nullptr;
  InstDyn* h_gather = nullptr;
  int* h_ninst = nullptr;
  const InstBuf** h_bufp = nullptr;
  InstDyn** h_dynp = nullptr;
  hipGraphExec_t exec = nullptr;
  int exec_steps = 0, exec_blocks = 0, exec_sig = 0;
  int layer_w = 0;   // bit w-1: some instance runs layer ops with w key words
};

std::mutex g_batch_mu;
std::map<hipStream_t, BatchCtx*> g_batches;

int batch_ctx(hipStream_t stream, BatchCtx** out) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  auto it = g_batches.find(stream);
  if (it != g_batches.end()) {
    *out = it->second;
    return PP_OK;
  }
  auto* b = new BatchCtx;
  b->stream = stream;
  if (hipMalloc((void**)&b->d_bufp, sizeof(void*) * kMaxInst) ||
      hipMalloc((void**)&b->d_dynp, sizeof(void*) * kMaxInst) ||
      hipMalloc((void**)&b->d_ninst, sizeof(int)) || hipMalloc((void**)&b->d_sync, kSyncBytes) ||
      hipMalloc((void**)&b->d_gather, sizeof(InstDyn) * kMaxInst) ||
      hipHostMalloc((void**)&b->h_gather, sizeof(InstDyn) * kMaxInst, hipHostMallocDefault) ||
      hipHostMalloc((void**)&b->h_ninst, sizeof(int), hipHostMallocDefault) ||
      hipHostMalloc((void**)&b->h_bufp, sizeof(void*) * kMaxInst, hipHostMallocDefault) ||
      hipHostMalloc((void**)&b->h_dynp, sizeof(void*) * kMaxInst, hipHostMallocDefault) ||
      hipMemset(b->d_sync, 0, kSyncBytes)) {
    return fail(PP_ENOMEM, "batch context allocation failed");
  }
  g_batches[stream] = b;
  *out = b;
  return PP_OK;
}

// One batched step: every instance inside a layer advances up to
// gates_per_step gates, then merges, compactions and the streaming ops run
// for the instances that reached them (two scans: truncation, then the
// next layer's damping).
// Dynamic LDS of the batched layer apply (above the 64 KB default).
template <int WW>
void allow_layer_lds() {
  static std::once_flag once;
  std::call_once(once, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_layer_apply_multi<WW, 512>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(ApplySh<WW, 512>));
  });
}

void launch_step(BatchCtx* b, int blocks) {
  Ctx C;
  C.bufs = b->d_bufp;
  C.dyns = b->d_dynp;
  C.ninst = b->d_ninst;
  C.sync = b->d_sync;
  const dim3 g(blocks), t(kBlock);
  // layer ops first: an instance at one finishes it within the step
  if (b->layer_w & 1) {
    allow_layer_lds<1>();
    hipLaunchKernelGGL(k_layer_scatter_multi<1>, g, t, 0, b->stream, C);
    hipLaunchKernelGGL((k_layer_apply_multi<1, 512>), g, dim3(512), sizeof(ApplySh<1, 512>),
                       b->stream, C);
  }
  if (b->layer_w & 2) {
    allow_layer_lds<2>();
    hipLaunchKernelGGL(k_layer_scatter_multi<2>, g, t, 0, b->stream, C);
    hipLaunchKernelGGL((k_layer_apply_multi<2, 512>), g, dim3(512), sizeof(ApplySh<2, 512>),
                       b->stream, C);
  }
  for (int k = 0; k < std::max(1, g_tune.gates_per_step); ++k)
    hipLaunchKernelGGL(kernel_of(PP_K_GATE), g, t, 0, b->stream, C);
  for (int kind : {PP_K_MERGE_NARROW, PP_K_MERGE_WIDE1, PP_K_MERGE_WIDE2, PP_K_MERGE_COLLECT,
                   PP_K_COMPACT, PP_K_SCAN, PP_K_SCAN})
    hipLaunchKernelGGL(kernel_of(kind), g, t, 0, b->stream, C);
}

int ensure_graph(BatchCtx* b) {
  const int steps = std::max(1, g_tune.graph_steps), blocks = g_tune.max_blocks;
  const int sig = g_tune.gates_per_step * 1000003 + g_tune.gate_items * 101 + g_tune.stream_items +
                  b->layer_w * 7919;
  if (b->exec && b->exec_steps == steps && b->exec_blocks == blocks && b->exec_sig == sig)
    return PP_OK;
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  hipGraph_t graph;
  HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < steps; ++k) launch_step(b, blocks);
  HIP_TRY(hipStreamEndCapture(b->stream, &graph));
  const hipError_t e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(PP_EDEVICE, std::string("graph: ") + hipGetErrorString(e));
  b->exec_steps = steps;
  b->exec_blocks = blocks;
  b->exec_sig = sig;
  return PP_OK;
}

// One instance through a whole program: the kernels of each sub-layer chunk
// are launched ahead (at most two chunks in flight); after each chunk the
// dynamic state is copied to pinned memory behind an event, so the host
// learns of an overflow (or a merge retry) without draining the stream, and
// only then synchronises, grows and relaunches from the op that stopped.
// `resume`: continue from the op the device state names (an instance that
// leaves a batch at a step boundary) instead of starting the program.
// A layer op at pc reported a bucket that did not fit (ST_LAYER; h_dyn is
// fresh and the device idles behind it): grow a crowded store, else run it
// again with fewer buckets (staging slots overflowed) or more (the LDS
// did), at most kLayerRetries times, else run its GATE(S) copies instead.
// After kLayerGiveUp fallbacks the handle runs the copies in place of every
// layer op.
constexpr int kLayerGiveUp = 3;
constexpr int kLayerRetries = 2;   // runs again with other bucket counts before a fallback

int layer_failed(pp_state* s, const Op* ops, size_t len) {
  InstDyn& h = *s->h_dyn;
  h.status &= ~ST_LAYER;
  const uint32_t k = h.pc;
  int rc;
  if (k < len && ops[k].type == OP_LAYER) {
    // a bucket's staging slots overflowed: fewer, larger buckets (a set of
    // strings closed under the rotations may be large); the LDS overflowed:
    // more, smaller buckets
    if (s->layer_fail_pc != k) {              // another op: every boost may be tried again
      for (bool& t : s->layer_tried) t = false;
      s->layer_fail_pc = k;
      s->layer_retries = 0;
    }
    const int32_t step = h.lwhy & 1u ? -1 : 1;
    const int32_t next = h.lboost + step;
    if (!ops[k].fail_test && (h.lwhy & 1u) && (uint64_t)h.M * 3 > s->buf.cap) {
      if ((rc = grow(s))) return rc;           // more staging slots per bucket
    } else if (!ops[k].fail_test && next >= -kLayerMaxBoost && next <= kLayerMaxBoost &&
               !s->layer_tried[next + kLayerMaxBoost] && s->layer_retries < kLayerRetries) {
      ++s->layer_retries;
      s->layer_tried[h.lboost + kLayerMaxBoost] = true;
      h.lboost = next;
      HIP_TRY(hipMemcpyAsync(&s->d_dyn->lboost, &h.lboost, sizeof(int32_t),
                             hipMemcpyHostToDevice, s->stream));
    } else {
      for (bool& t : s->layer_tried) t = false;
      s->fb_lo = k + 1;
      s->fb_hi = k + 1 + ops[k].skip;
      h.pc = k + 1;
      HIP_TRY(hipMemcpyAsync(&s->d_dyn->pc, &h.pc, sizeof(uint32_t), hipMemcpyHostToDevice,
                             s->stream));
      if (++s->layer_fallbacks >= kLayerGiveUp && !ops[k].fail_test && !s->buf.nolayer) {
        s->layer_off = true;
        s->buf.nolayer = 1;
        if ((rc = upload_buf(s))) return rc;
      }
    }
  }
  HIP_TRY(hipMemcpyAsync(&s->d_dyn->status, &h.status, sizeof(uint32_t), hipMemcpyHostToDevice,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return PP_OK;
}

// The fallback copies around pc when a program resumes inside them.
void resume_window(pp_state* s, const Op* ops, size_t len, size_t pc) {
  s->fb_lo = s->fb_hi = 0;
  if (pc >= len || !ops[pc].fallback) return;
  size_t k = pc;
  while (k > 0 && ops[k].type != OP_LAYER) --k;
  if (ops[k].type == OP_LAYER) {
    s->fb_lo = k + 1;
    s->fb_hi = k + 1 + ops[k].skip;
  }
}

int solo_program(pp_state* s, const pp_program* p, double* expectation, bool resume = false) {
  int rc;
  const hipStream_t st = s->stream;
  const Op* ops = p->ops.data();
  const size_t len = p->ops.size();
  s->buf.prog = p->d_ops;
  s->buf.prog_len = (uint32_t)len;
  s->buf.nopart = 0;
  s->buf.nolayer = s->layer_off ? 1u : 0u;
  s->batch_prog = p;
  if ((rc = upload_buf(s))) return rc;
  if (!resume) hipLaunchKernelGGL(k_set_pc, dim3(1), dim3(1), 0, st, s->d_dyn, 0u);
  resume_window(s, ops, len, resume ? s->h_dyn->pc : 0);
  // chunk ends: after every kChunkSubs-th sub-layer (its MERGE and the TRUNC
  // that follows it), or the last op; the host reads the state once per chunk
  std::vector<size_t> ends;
  int subs = 0;
  for (size_t k = 0; k < len; ++k) {
    const bool merge_end = ops[k].type == OP_MERGE && !(k + 1 < len && ops[k + 1].type == OP_TRUNC);
    if (merge_end || ops[k].type == OP_TRUNC) ++subs;
    if (((merge_end || ops[k].type == OP_TRUNC) && subs % kChunkSubs == 0) || k + 1 == len)
      ends.push_back(k + 1);
  }
  if (!s->solo_slots) {
    HIP_TRY(hipHostMalloc((void**)&s->solo_slots, sizeof(InstDyn) * kSoloSlots,
                          hipHostMallocDefault));
    for (auto& e : s->solo_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  size_t next_chunk = 0, launched_to = resume ? s->h_dyn->pc : 0;
  while (next_chunk < ends.size() && ends[next_chunk] <= launched_to) ++next_chunk;
  if (resume && launched_to >= len) {
    if (expectation) *expectation = s->h_dyn->expect;
    return PP_OK;
  }
  std::vector<size_t> inflight;            // chunk indices, oldest first
  for (int guard = 0; guard < 1 << 30; ++guard) {
    while (inflight.size() < kSoloInflight && next_chunk < ends.size()) {
      const size_t end = ends[next_chunk];
      if ((rc = launch_range(s, ops, launched_to, end))) return rc;
      const int slot = (int)(next_chunk % kSoloSlots);
      HIP_TRY(hipMemcpyAsync(&s->solo_slots[slot], s->d_dyn, sizeof(InstDyn),
                             hipMemcpyDeviceToHost, st));
      HIP_TRY(hipEventRecord(s->solo_ev[slot], st));
      inflight.push_back(next_chunk);
      launched_to = end;
      ++next_chunk;
    }
    if (inflight.empty()) break;
    const size_t c = inflight.front();
    inflight.erase(inflight.begin());
    HIP_TRY(hipEventSynchronize(s->solo_ev[c % kSoloSlots]));
    const InstDyn dy = s->solo_slots[c % kSoloSlots];
    if (dy.merge_in > s->m_prev_in && s->m_prev)
      s->m_growth = (double)(dy.merge_in - s->m_prev_in) / (double)s->m_prev;
    s->m_prev_in = dy.merge_in;
    s->m_prev = dy.M;
    s->m_hint = dy.M;
    if (dy.status & ST_RANGE)
      return fail(PP_EINVAL, "a coefficient is not finite or exceeds 2^54 in magnitude");
    if (dy.pc >= ends[c]) {
      if (dy.pc >= len && inflight.empty() && next_chunk >= ends.size()) {
        *s->h_dyn = dy;
        if (expectation) *expectation = dy.expect;
        prof_resolve(s);
        return PP_OK;
      }
      // grow ahead of time when the store is a third full, so that a gate
      // rarely has to stop (and the launches queued behind it idle)
      if ((uint64_t)dy.M * 3 > s->buf.cap && next_chunk < ends.size()) {
        if ((rc = read_dyn(s))) return rc;
        if (s->h_dyn->pc < len && !(s->h_dyn->status & ST_OVERFLOW) &&
            (uint64_t)s->h_dyn->M * 3 > s->buf.cap) {
          if ((rc = grow(s))) return rc;
        }
        inflight.clear();
        if (s->h_dyn->status & ST_OVERFLOW) {
          if ((rc = grow(s))) return rc;
          s->h_dyn->status &= ~ST_OVERFLOW;
          HIP_TRY(hipMemcpyAsync(&s->d_dyn->status, &s->h_dyn->status, sizeof(uint32_t),
                                 hipMemcpyHostToDevice, st));
        }
        if (s->h_dyn->status & ST_LAYER) {
          if ((rc = layer_failed(s, ops, len))) return rc;
        }
        launched_to = s->h_dyn->pc;
        next_chunk = 0;
        while (next_chunk < ends.size() && ends[next_chunk] <= launched_to) ++next_chunk;
        if (s->h_dyn->pc >= len) {
          if (expectation) *expectation = s->h_dyn->expect;
          prof_resolve(s);
          return PP_OK;
        }
      }
      continue;
    }
    // stopped inside chunk c: drain, grow if needed, resume at its pc
    if ((rc = read_dyn(s))) return rc;
    if (s->h_dyn->status & ST_OVERFLOW) {
      if ((rc = grow(s))) return rc;
      s->h_dyn->status &= ~ST_OVERFLOW;
      HIP_TRY(hipMemcpyAsync(&s->d_dyn->status, &s->h_dyn->status, sizeof(uint32_t),
                             hipMemcpyHostToDevice, st));
    }
    if (s->h_dyn->status & ST_LAYER) {
      if ((rc = layer_failed(s, ops, len))) return rc;
    }
    inflight.clear();
    launched_to = s->h_dyn->pc;
    next_chunk = 0;
    while (next_chunk < ends.size() && ends[next_chunk] <= launched_to) ++next_chunk;
  }
  return fail(PP_EDEVICE, "program did not complete");
}

// A finished instance's store holding far more room than its final set
// is compacted into a store just large enough (the batch's finished
// instances keep their sets, not their peaks).
int shrink_finished(pp_state* s) {
  const InstDyn& d = *s->h_dyn;
  const uint64_t want = std::max<uint64_t>(4096, 2ull * d.live);
  if ((uint64_t)s->buf.cap <= 4 * want || s->buf.cap <= (1u << 20)) return PP_OK;
  InstBuf nb;
  std::vector<void*> allocs;
  int rc = alloc_store(s, (uint32_t)want, &nb, &allocs);
  if (rc) return PP_OK;                    // keeping the larger store is correct too
  nb.prog = s->buf.prog;
  nb.prog_len = s->buf.prog_len;
  nb.nopart = s->buf.nopart;
  hipLaunchKernelGGL(k_grow, dim3(launch_blocks(d.M)), dim3(kBlock), 0, s->stream, s->buf, nb,
                     s->d_dyn, s->d_sync);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s->stream));
  free_store(s, s->store);
  s->store = std::move(allocs);
  s->buf = nb;
  if ((rc = upload_buf(s))) return rc;
  return read_dyn(s);
}

// Whether a batched instance runs its program's layer ops (the program has
// some, layer ops are not off for the handle, and its staging exists).
bool batch_layer(pp_state* s, const pp_program* p) {
  if (s->layer_off || !p->has_layer) return false;
  s->buf.lshift = (uint32_t)g_tune.layer_shift;
  return ensure_layer(s) == PP_OK;
}

// Instances whose store has held this many entries leave the batch at the
// next step boundary and finish on the one-instance path (partitioned
// merges, the whole GPU), while the rest of the batch waits.
constexpr uint32_t kPromote = kPartMin;

int batch_common(pp_state* const* states, const pp_program* const* programs, size_t n,
                 void* hip_stream, int max_replays, int* done, double* expectations) {
  if (!states || !programs) return fail(PP_EINVAL, "NULL argument");
  if (n == 0) return PP_OK;
  if (n > (size_t)kMaxInst) return fail(PP_EINVAL, "at most 1024 instances per batch");
  hipStream_t stream = (hipStream_t)hip_stream;
  if (!stream) return fail(PP_EINVAL, "the batched form needs a non-null stream");
  for (size_t i = 0; i < n; ++i) {
    if (!states[i] || !programs[i]) return fail(PP_EINVAL, "NULL state or program");
    if (states[i]->stream != stream) return fail(PP_EINVAL, "state created on another stream");
    if (states[i]->n != programs[i]->n) return fail(PP_EINVAL, "program n differs from state n");
  }
  BatchCtx* b;
  int rc = batch_ctx(stream, &b);
  if (rc) return rc;
  // (re)start instances whose program changed
  for (size_t i = 0; i < n; ++i) {
    pp_state* s = states[i];
    if (s->batch_prog != programs[i]) {
      if (s->h_dyn->status & ST_FAILED) return fail(PP_EINVAL, "state failed in an earlier batch");
      s->shrunk = false;
      s->buf.prog = programs[i]->d_ops;
      s->buf.prog_len = (uint32_t)programs[i]->ops.size();
      s->batch_prog = programs[i];
      s->buf.nopart = 1;                   // the batched steps have no partitioned merge
      s->buf.nolayer = batch_layer(s, programs[i]) ? 0u : 1u;
      if ((rc = upload_buf(s))) return rc;
      hipLaunchKernelGGL(k_set_pc, dim3(1), dim3(1), 0, stream, s->d_dyn, 0u);
    } else if (!s->buf.nopart || s->buf.nolayer != (batch_layer(s, programs[i]) ? 0u : 1u)) {
      s->buf.nopart = 1;
      s->buf.nolayer = batch_layer(s, programs[i]) ? 0u : 1u;
      if ((rc = upload_buf(s))) return rc;
    }
    b->h_bufp[i] = s->d_buf;
    b->h_dynp[i] = s->d_dyn;
  }
  *b->h_ninst = (int)n;
  b->layer_w = 0;
  for (size_t i = 0; i < n; ++i)
    if (!states[i]->buf.nolayer) b->layer_w |= 1 << (states[i]->W - 1);
  HIP_TRY(hipMemcpyAsync(b->d_bufp, b->h_bufp, sizeof(void*) * n, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(b->d_dynp, b->h_dynp, sizeof(void*) * n, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(b->d_ninst, b->h_ninst, sizeof(int), hipMemcpyHostToDevice, stream));
  if ((rc = ensure_graph(b))) return rc;
  for (int rep = 0; max_replays < 0 || rep < max_replays; ++rep) {
    HIP_TRY(hipGraphLaunch(b->exec, stream));
    hipLaunchKernelGGL(k_gather_dyn, dim3((n + 255) / 256), dim3(256), 0, stream, b->d_dynp,
                       b->d_ninst, b->d_gather);
    HIP_TRY(hipMemcpyAsync(b->h_gather, b->d_gather, sizeof(InstDyn) * n, hipMemcpyDeviceToHost,
                           stream));
    HIP_TRY(hipStreamSynchronize(stream));
    bool all_done = true;
    for (size_t i = 0; i < n; ++i) {
      pp_state* s = states[i];
      *s->h_dyn = b->h_gather[i];
      if (s->h_dyn->status & ST_FAILED) continue;
      if ((s->h_dyn->status & ST_OVERFLOW)) {
        // an instance that cannot grow stops (kernels keep skipping it);
        // the others go on
        const int g = grow(s);
        s->h_dyn->status = g ? (s->h_dyn->status | ST_FAILED) : (s->h_dyn->status & ~ST_OVERFLOW);
        HIP_TRY(hipMemcpyAsync(&s->d_dyn->status, &s->h_dyn->status, sizeof(uint32_t),
                               hipMemcpyHostToDevice, stream));
        if (g) {
          s->fail_code = g;
          continue;
        }
      }
      if (s->h_dyn->status & ST_RANGE) {
        s->h_dyn->status |= ST_FAILED | ST_OVERFLOW;
        s->fail_code = PP_EINVAL;
        HIP_TRY(hipMemcpyAsync(&s->d_dyn->status, &s->h_dyn->status, sizeof(uint32_t),
                               hipMemcpyHostToDevice, stream));
        continue;
      }
      if (s->h_dyn->pc < s->buf.prog_len && s->h_dyn->peak >= kPromote) {
        // a large instance: finish it alone, then put it back (finished)
        const pp_program* prog = s->batch_prog;
        double e = 0.0;
        s->m_hint = s->h_dyn->M;
        const int g = solo_program(s, prog, &e, true);
        s->buf.prog = prog->d_ops;
        s->buf.prog_len = (uint32_t)prog->ops.size();
        s->buf.nopart = 1;
        s->buf.nolayer = batch_layer(s, prog) ? 0u : 1u;
        s->batch_prog = prog;
        if (g) {
          s->h_dyn->status |= ST_FAILED | ST_OVERFLOW;
          s->fail_code = g;
          HIP_TRY(hipMemcpyAsync(&s->d_dyn->status, &s->h_dyn->status, sizeof(uint32_t),
                                 hipMemcpyHostToDevice, stream));
          if ((rc = upload_buf(s))) return rc;
          continue;
        }
        if ((rc = upload_buf(s))) return rc;
        b->h_gather[i] = *s->h_dyn;
      }
      if (s->h_dyn->pc >= s->buf.prog_len && !s->shrunk) {
        if ((rc = shrink_finished(s))) return rc;
        s->shrunk = true;
      }
      all_done = all_done && s->h_dyn->pc >= s->buf.prog_len;
    }
    if (all_done) break;
  }
  int first_fail = PP_OK;
  for (size_t i = 0; i < n; ++i) {
    const InstDyn& d = *states[i]->h_dyn;
    const bool failed = (d.status & ST_FAILED) != 0;
    const bool fin = !failed && d.pc >= states[i]->buf.prog_len;
    if (done) done[i] = failed ? -1 : (fin ? 1 : 0);
    if (expectations && fin) expectations[i] = d.expect;
    if (failed && first_fail == PP_OK) first_fail = states[i]->fail_code;
  }
  if (first_fail != PP_OK && !done)
    return fail(first_fail, "an instance of the batch could not grow its term store");
  return PP_OK;
}

}  // namespace

extern "C" {

int pp_batch_run(pp_state* const* states, const pp_program* const* programs, size_t n,
                 void* hip_stream, double* expectations) {
  if (n == 1 && states && programs && states[0] && programs[0]) {
    if (states[0]->stream != (hipStream_t)hip_stream)
      return fail(PP_EINVAL, "state created on another stream");
    if (states[0]->n != programs[0]->n) return fail(PP_EINVAL, "program n differs from state n");
    return solo_program(states[0], programs[0], expectations);
  }
  return batch_common(states, programs, n, hip_stream, -1, nullptr, expectations);
}

int pp_batch_step(pp_state* const* states, const pp_program* const* programs, size_t n,
                  void* hip_stream, int max_steps, int* done, double* expectations) {
  if (max_steps <= 0) return fail(PP_EINVAL, "max_steps must be > 0");
  const int per = std::max(1, g_tune.graph_steps);
  return batch_common(states, programs, n, hip_stream, (max_steps + per - 1) / per, done,
                      expectations);
}

}  // extern "C"
