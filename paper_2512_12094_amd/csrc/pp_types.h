// Internal data layout of the gfx950 Pauli propagation library (shared by
// host and device code).
//
// Term store (per instance, one per handle)
// -----------------------------------------
// Two halves of structure-of-arrays buffers, each of capacity `cap`:
//   x[h][w*cap + i], z[h][w*cap + i]   uint64 words of term i's masks
//   c[h][i]                            coefficient: FP64, or FP32 when
//                                      the handle was created with
//                                      PP_F32_COMPENSATED (f32 != 0)
//   alive[h][p][i]                     uint8 liveness, double-buffered (p)
// Gates update coefficients in place and append new strings at the end of
// the current half; a term that is truncated is only marked dead.  A
// symmetry merge (or a compaction) writes the surviving unique terms into
// the other half and flips `half`.
//
// Gate table: open addressing, linear probing, 2^hg_bits uint64 slots, slot
// value (generation << 32) | index.  A slot whose generation differs from
// the instance's current one is empty, so a rebuild only bumps `gen`.
//
// Merge table: 2^hm_bits slots of (key, sum[, owner]); a merge of M records
// uses only the first 2^b slots, b = ceil(log2(2M)) (at least 10, at most
// hm_bits), so the collect pass scans what the merge can fill.  Keys are the
// representative itself when it fits 64 bits exactly ("narrow"), else a
// 64-bit hash of it with the owning record's full representative kept in
// `wrep` and compared for every record ("wide").  Sums are exact: every
// coefficient becomes a 192-bit two's-complement fixed-point integer with
// kFxFrac fraction bits and the three 64-bit limbs are added with integer
// atomics and carries, so the orbit sum is exact, independent of the order
// of the additions, and rounded to FP64 once.
#pragma once
#include <cstddef>
#include <cstdint>

namespace pp {

constexpr int kMaxW = 2;                   // up to 128 qubits
constexpr int kMaxFuse = 3;                // rotations one gate launch may apply
constexpr uint32_t kNone32 = 0xFFFFFFFFu;
constexpr uint64_t kEmpty64 = ~0ull;
constexpr int kMaxInst = 1024;             // instances per batched launch

enum OpType : uint32_t {
  OP_END = 0,
  OP_GATE = 1,     // one Pauli rotation + exact merge + truncation
  OP_MERGE = 2,    // symmetry merge by orbit representative
  OP_DAMP = 3,     // c *= (1-p)^weight
  OP_TRUNC = 4,    // drop |c| < eps or weight > wmax
  OP_COUNT = 5,    // only recount (live, anticommuting with next gate)
  OP_EXPECT = 6,   // expectation in a symmetric product state
  OP_GATES = 7,    // 2..kMaxFuse mutually commuting rotations in circuit
                   // order, each followed by the exact merge and
                   // truncation, in one pass
  OP_LAYER = 8,    // 4..kLayerMaxRot mutually commuting rotations in circuit
                   // order, each followed by the exact merge and truncation,
                   // applied to buckets of strings closed under all of them
                   // (two launches); its `skip` following ops are the same
                   // rotations as GATE(S) ops, run only if it fails
};

enum : uint32_t { ST_OVERFLOW = 1u, ST_COLLISION = 2u, ST_RANGE = 4u, ST_FAILED = 8u,
                  ST_LAYER = 16u };   // a LAYER op did not fit its buckets

// Contended device-scope atomics on one address serialise (about 12 ns each
// on gfx950), so per-launch counts go to kAccShards accumulators and the
// done counter is a two-level tree of kSyncShards; each shard sits on its
// own 128-byte line (kLineU64 / kLineU32 entries apart).
constexpr int kAccShards = 16;
constexpr int kSyncShards = 16;
constexpr int kLineU64 = 16;
constexpr int kLineU32 = 32;
// done counters: the root line, kSyncShards shard lines, and one line whose
// 64-bit word counts done blocks and their packed counts (kPackedLine)
constexpr int kPackedLine = 1 + kSyncShards;
constexpr size_t kSyncBytes = (2 + kSyncShards) * kLineU32 * sizeof(uint32_t);
constexpr size_t kAccBytes = kAccShards * kLineU64 * sizeof(uint64_t);
// work statistics that no kernel reads back (multi-rotation ops): live terms
// after each rotation but the last, those anticommuting with the next
// rotation, coefficients rewritten; summed over launches, per shard line
enum : int { STAT_LIVE = 0, STAT_ANTI = 1, STAT_RW = 2, kStatKinds = 3 };
constexpr size_t kStatBytes = kStatKinds * kAccShards * kLineU64 * sizeof(uint64_t);

// Partitioned merge (narrow keys except S_n, at least kPartMin records):
//   1. histogram: tiles of kPartTileRec records; each live record's key goes
//      to bucket mix64(key) >> (64 - pbits); per-tile bucket counts;
//   2. column scan: per bucket, the tiles' exclusive offsets and the total;
//      the last block turns the totals into bucket bases and the list of
//      aggregation work items;
//   3. scatter: every record (key, coefficient) to its exact place in the
//      bucket-contiguous staging array, through an LDS counting sort of
//      kPartSub records at a time;
//   4. aggregation: one block per bucket (or per chunk of a bucket holding
//      more than twice the average), LDS table of kPartSlots keys with exact
//      carry-free sums; emits one term per key (chunks of a split bucket add
//      into the global merge table instead, emitted by the collect pass).
// P = 2^pbits buckets, pbits = clamp(ceil(log2(M / 2^pshift)), 6, 12), where
// pshift (records per bucket aimed at, default kPartShift) is a tuning knob.
constexpr uint32_t kPartMin = 1u << 18;
constexpr int kPartTileRec = 32768;
constexpr int kPartSub = 4096;
constexpr int kPartShift = 14;
constexpr int kPartMinBits = 6;
constexpr int kPartMaxBits = 12;
constexpr int kPartSlots = 2048;
constexpr int kPartFill = 1536;
constexpr int kPartChunks = 5;       // 32-bit chunks of a fixed-point sum (160 bits)
constexpr int kPartMaxPasses = 64;   // selector passes over an overfull bucket
constexpr int kPartProbe = 64;       // probes before the LDS table refuses a key

// Layer op (OP_LAYER): a commuting run of r rotations P_1..P_r maps a string
// Q only within the set Q * <P_g : P_g anticommutes with Q>, and every
// member of that set anticommutes with the same P_g.  So the key
//   (anticommutation pattern a, x bits outside the x-support of the
//    anticommuting rotations, z bits outside their z-support)
// is the same for all members, and strings bucketed by a hash of it can be
// rotated bucket by bucket, each bucket in one block's LDS:
//   1. scatter: each live string to its bucket (2^lbits buckets of
//      lslots >> lbits staging slots; a global counter per bucket);
//   2. apply: one block per bucket runs the r rotations with the exact
//      merge and truncation after each, then writes the survivors to the
//      other half of the store.
// Within a bucket each wave takes whole groups (by the key's hash; strings
// that commute with every rotation anywhere), so a wave rotates its strings
// with no barrier between rotations and skips the rotations none of them
// anticommutes with.  A bucket that does not fit its staging slots or a
// wave's share of the LDS fails the op; the host then retries it with more
// buckets, then falls back to the op's GATE(S) copies.
constexpr int kLayerMaxRot = 64;
constexpr int kLayerMinRot = 4;
constexpr int kLayerShift = 8;        // strings per bucket aimed at: 2^8 (default)
constexpr int kLayerMaxBits = 20;
constexpr int kLayerMinSlots = 64;    // staging slots per bucket, at least
constexpr int kLayerMaxBoost = 3;     // bucket bits added or taken after failures
constexpr int kLayerAcc = 8;          // per-shard layer sums (accs line entries 1..8)

constexpr int kFxFrac = 104;   // fixed-point fraction bits of merge sums
constexpr int kFxMaxShift = 105;   // |c| < 2^54 keeps 2^32 addends in range

struct Op {
  uint32_t type;
  uint32_t full_check;   // GATE: re-check |c| and weight of every live term
  uint32_t next_gate;    // index of the next GATE op after this one, or kNone32
  int32_t wmax;          // GATE/TRUNC: weight limit (< 0: off)
  uint32_t force_full;   // MERGE with group NONE: merge duplicates (creation)
  uint32_t trunc;        // MERGE: emit only terms passing eps / wmax (the
                         // sub-layer's truncation, folded into the merge)
  uint32_t fallback;     // GATE(S): copy of a LAYER op's rotations, run only
                         // after that op failed
  uint32_t nrot;         // GATE: 1; GATES, LAYER: rotations in the op
  uint32_t skip;         // LAYER: number of fallback ops that follow it
  uint32_t gtab;         // LAYER: its output gets gate-table entries (no
                         // merge follows before the next gate)
  uint32_t fail_test;    // LAYER: always reports a failure (tests of the
                         // fallback path)
  uint64_t px[kMaxW];    // GATE(S): the (first) rotation's Pauli string
  uint64_t pz[kMaxW];
  double cs, sn;         // GATE(S): cos(theta), sin(theta)
  uint64_t qx[kMaxFuse - 1][kMaxW];   // GATES: rotations 2..nrot
  uint64_t qz[kMaxFuse - 1][kMaxW];
  double qcs[kMaxFuse - 1], qsn[kMaxFuse - 1];
  uint64_t nx[kMaxW];    // the next gate op's (first) rotation, when next_gate
  uint64_t nz[kMaxW];    // != kNone32 (its anticommutation count is tallied here)
  double eps;            // GATE/TRUNC: coefficient threshold (0: off)
  const double* table;   // DAMP: (1-p)^w for w = 0..n;
                         // EXPECT: bx^k, by^k, bz^k for k = 0..n (3 blocks);
                         // LAYER: per rotation kLayerRec doubles: x words,
                         // z words (bit patterns), cos, sin
};

constexpr int kLayerRec = 2 * kMaxW + 2;

struct InstBuf {
  uint64_t* x[2];
  uint64_t* z[2];
  void* c[2];            // double[cap], or float[cap] when f32
  uint8_t* alive[2][2];  // [half][parity]
  uint64_t* gtab;
  uint64_t* mkey;
  uint64_t* mfx;         // 3 limbs per slot: [3*slot + k]
  uint32_t* mown;
  uint64_t* wrep;        // [2W][cap]: x words then z words of each record's rep
  uint32_t* wslot;
  uint64_t* accs;        // kAccShards count accumulators
  uint64_t* stats;       // kStatKinds x kAccShards statistics lines (cumulative)
  // partitioned merge (narrow keys, large sets)
  uint64_t* phash;       // [cap] mix64 of each record's representative key
                         // (mix64(kEmpty64): no record to merge)
  uint64_t* pstage;      // [cap][2]: (mixed key, coefficient bits), bucket-contiguous
  uint32_t* phist;       // [tiles][P]: per-tile counts, then exclusive offsets
  uint32_t* ptot;        // [P] bucket totals
  uint32_t* pbase;       // [P + 1] bucket bases
  uint32_t* pwork;       // aggregation items: bucket | chunk << 16
  uint32_t* plist;       // [2^hm_bits] global merge-table slots in use
  uint32_t pmaxbits;     // largest pbits the staging tables were sized for
  uint32_t pshift;       // log2 of the records per bucket aimed at (tuning)
  // layer op (allocated on first use)
  uint64_t* lstx;        // [W][lslots] staged x words
  uint64_t* lstz;        // [W][lslots] staged z words
  double* lstc;          // [lslots] staged coefficients (exact in FP64)
  uint64_t* lsta;        // [lslots] staged anticommutation patterns (bit g: P_g)
  uint32_t* lsth;        // [lslots] staged low 32 bits of the bucket key's hash
  uint32_t* lcount;      // [2^lmaxbits] strings per bucket (zero between ops)
  uint32_t lslots;       // staging slots (a power of two)
  uint32_t lmaxbits;     // largest bucket bits (lslots >> lmaxbits >= kLayerMinSlots)
  uint32_t lshift;       // log2 of the strings per bucket aimed at (tuning)
  uint32_t nolayer;      // LAYER ops are skipped (their fallback ops run)
  const Op* prog;
  uint32_t prog_len;
  uint32_t cap;
  uint32_t hg_bits;
  uint32_t hm_bits;
  int32_t n;
  int32_t W;
  int32_t group;
  uint32_t narrow;       // merge keys fit 64 bits exactly
  uint32_t f32;          // coefficients stored and rotated in FP32
  uint32_t nopart;       // the partitioned merge's kernels are not launched
  int32_t lx;            // torus width (group 4: translations of lx x n/lx)
  const uint8_t* gperm;  // group 5: gsize rows of n qubit indices
  uint32_t gsize;
};

struct InstDyn {
  uint64_t propagated;   // work counters (see pp_counters, pp_work_counters)
  uint64_t merged;
  uint64_t anti_total;   // sum over gates of the anticommuting live terms
  uint64_t appended;     // strings appended by gates
  uint64_t merge_in;     // records entering symmetry merges / compactions
  uint64_t merge_out;    // representatives leaving them
  uint64_t acc;          // counts folded from the shards by the last block
  uint64_t key_reads;    // sum over gate launches of the live terms entering them
  uint64_t coef_rw;      // sum over gate launches of the entering terms they rotate
  uint64_t special_fx[3];   // narrow merge: the one key equal to kEmpty64
  uint64_t expect_fx[3];    // exact expectation accumulator
 double expect;
  uint32_t M;            // entries in the current half (live and dead)
  uint32_t Mnext;        // append cursor while a gate runs
  uint32_t half;
  uint32_t parity;
  uint32_t gen;          // gate-table generation
  uint32_t pc;           // program counter
  uint32_t status;       // ST_* bits
  uint32_t count;        // live terms anticommuting with gate op `count_for`
  uint32_t count_for;
  uint32_t live;         // live terms
  uint32_t nuniq;        // output cursor of a merge / compaction
  uint32_t mphase;       // merge progress: 0 none, 1 inserted, 2 owned (wide)
  uint32_t seed;         // wide-merge hash seed (bumped on a collision)
  uint32_t special;
  uint32_t failed_pc;
  uint32_t pglobal;      // partitioned merge: some bucket used the global table
  uint32_t pbits;        // partitioned merge: log2 of the bucket count
  uint32_t pnwork;       // partitioned merge: aggregation items
  uint32_t plist_n;      // partitioned merge: global-table slots listed
  uint32_t pchunk;       // partitioned merge: records per item of a split bucket
  // cumulative partitioned-merge statistics (pp_merge_stats)
  uint32_t pruns;        // partitioned merges run
  uint32_t phot;         // buckets split over several blocks (hot representatives)
  uint32_t pover;        // buckets summed in several selector passes
  uint32_t pglob;        // keys that went through the global merge table
  uint32_t peak;         // most entries (live and not yet compacted) the store held
  int32_t lboost;        // layer ops: bucket bits added (or taken) after failures
  uint32_t lwhy;         // layer op: why the last run failed (1 staging slots, 2 LDS)
  uint32_t lops;         // layer ops completed (pp_layer_stats)
  uint32_t lfails;       // layer ops that reported a bucket overflow
  uint32_t lfb;          // layer ops the batched form replaced by their gate copies
  uint32_t lserved;      // batched form: this step's scatter took the instance's layer op
  uint32_t lfail;        // layer op: a bucket overflowed its slots or the LDS
  uint32_t lneed;        // layer op: survivors of an op whose output did not fit
};

}  // namespace pp
