/*
 * pp.h -- C ABI of the MI355X (gfx950) symmetry-merging Pauli propagation
 * library.
 *
 * The library evolves an observable O, stored as a set of Pauli strings
 * with real coefficients, through a circuit of Pauli rotations in the
 * Heisenberg picture and merges strings that are related by a symmetry of
 * the circuit, following "Leveraging Symmetry Merging in Pauli Propagation"
 * (Teng, Chang, Rudolph, Holmes, arXiv:2512.12094): Algorithm 1, the gate
 * rule of Proposition 1, and the lowest-integer representatives of
 * Algorithms 2 (translations Z_n) and 3 (permutations S_n).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - A Pauli string on n qubits is a pair of bit masks (x, z) of W = ceil(n/64)
 *   little-endian uint64 words each; qubit q is bit q%64 of word q/64
 *   (symplectic form, Appendix E.2).  I=(0,0), X=(1,0), Y=(1,1), Z=(0,1).
 *   Row r of an array of strings occupies words [r*W, r*W+W).  Bits at
 *   positions >= n must be zero.
 * - Coefficients are those of unnormalised Pauli operators, O = sum c_s s.
 * - A gate (x, z, theta) is the rotation exp(-i theta/2 P).  In the
 *   Heisenberg picture an anticommuting string Q becomes
 *   cos(theta) Q + sin(theta) (iPQ) and a commuting one is unchanged
 *   (Proposition 1, proof part (2), with the half-angle convention).
 * - Representatives are the lowest-integer members of each orbit
 *   (Definition "lowest integer representation", Appendix E.2): I->0, X->1,
 *   Y->2, Z->3 as the base-4 digit of weight 4^q for qubit q.  For Z_n this
 *   is the minimum over the n cyclic translations (Algorithm 2); for S_n it
 *   is Z^{nZ} Y^{nY} X^{nX} I^{rest} from qubit 0 upward (Algorithm 3); for
 *   the dihedral group D_n (translations and the reflection q -> n-1-q of
 *   the ring, a wider group of the kind the paper's outlook names) it is
 *   the smaller of the Z_n representatives of the string and of its
 *   reflection; for PP_GROUP_TORUS (qubit q = x + lx*y of an lx x ly torus,
 *   the lattice setting of the paper's Fig. 3) it is the minimum over the
 *   lx*ly translations (x, y) -> (x + a, y + b); for PP_GROUP_EXPLICIT (any
 *   finite group of qubit permutations, given by its element list) it is the
 *   minimum over the listed images (Algorithm 2 generalised).  Merging adds
 *   the coefficients of the distinct strings of one orbit.
 * - Supported sizes: PP_GROUP_NONE and PP_GROUP_PERMUTATION for 1 <= n <= 128,
 *   PP_GROUP_TRANSLATION and PP_GROUP_DIHEDRAL for 2 <= n <= 64,
 *   PP_GROUP_TORUS for 2 <= lx*ly <= 64, PP_GROUP_EXPLICIT for 2 <= n <= 64
 *   with at most 1024 group elements.
 *
 * Memory, streams, ownership
 * --------------------------
 * - A handle owns all of its device memory.  It obtains that memory from the
 *   caller's allocator (e.g. PyTorch's caching allocator) or, when the
 *   allocator argument is NULL, from hipMalloc/hipFree.
 * - Every call enqueues its kernels on the handle's HIP stream.  Host arrays
 *   passed in are copied before the call returns; the caller keeps them.
 *   Output arrays are owned by the caller.
 * - Calls that synchronise the stream: pp_create, pp_apply_layer (once, to
 *   learn whether the term store had to grow: the growth of a layer is not
 *   known before its gates run, and the store is grown by the host),
 *   pp_merge_canonicalize (to learn whether every sum stayed in range, so
 *   that a failure can be rolled back), pp_expectation, pp_num_terms,
 *   pp_export_terms, pp_counters, pp_batch_run.  pp_truncate does not
 *   synchronise.  A whole propagation that must not wait on the host runs
 *   as a program (pp_program_create + pp_batch_run): its steps run on the
 *   device and the host only reads the state after each chunk of them.
 * - A handle is not thread-safe; distinct handles are independent.
 *
 * Errors
 * ------
 * Every int-returning function returns PP_OK (0) or a negative code; nothing
 * throws across the ABI.  pp_last_error() returns a thread-local message for
 * the most recent failure.  pp_apply_layer and pp_merge_canonicalize are
 * transactional: after any error (PP_EINVAL, PP_ENOTSYM, PP_ECAPACITY when
 * the store would exceed pp_set_max_terms, PP_ENOMEM, a coefficient out of
 * range) the handle holds exactly its state from before the call (terms,
 * coefficients, counters).  pp_truncate validates its arguments before it
 * changes anything.
 */
#ifndef PP_H
#define PP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pp_state pp_state;
typedef struct pp_program pp_program;

enum {
  PP_GROUP_NONE = 0,         /* plain Pauli propagation (no symmetry merge) */
  PP_GROUP_TRANSLATION = 1,  /* cyclic translations Z_n                     */
  PP_GROUP_PERMUTATION = 2,  /* qubit permutations S_n                      */
  PP_GROUP_DIHEDRAL = 3,     /* ring translations and reflection D_n        */
  PP_GROUP_TORUS = 4,        /* translations of a 2D torus (pp_create_torus) */
  PP_GROUP_EXPLICIT = 5      /* any permutation group (pp_create_group)     */
};

/*
 * Coefficient precision.  PP_F64: coefficients stored and rotated in FP64.
 * PP_F32_COMPENSATED: coefficients stored in FP32 (4 bytes per term) and
 * each rotation computed in FP32 with cos and sin rounded to FP32 once;
 * damping factors are rounded to FP32 the same way.  In both modes every
 * merge sum (inner exact merges and orbit sums, Algorithms 2 and 3) is
 * exact (integer fixed point) and rounded once to FP64, then, in FP32 mode,
 * to FP32; this is at least as accurate as compensated summation.  The
 * expectation is an exact sum of FP64 products, rounded once to FP64.
 */
enum { PP_F64 = 0, PP_F32_COMPENSATED = 1 };

enum {
  PP_OK = 0,
  PP_EINVAL = -1,     /* bad argument                                        */
  PP_ENOTSYM = -2,    /* gate multiset not closed under the handle's group   */
  PP_ENOMEM = -3,     /* the allocator returned NULL                         */
  PP_ECAPACITY = -4,  /* the term store would exceed pp_set_max_terms        */
  PP_EDEVICE = -5     /* a HIP runtime call failed                           */
};

typedef struct {
  /* Returns device memory of at least `bytes` bytes usable on `stream`, or NULL. */
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  /* Releases memory obtained from alloc. */
  void (*free)(void* p, void* stream, void* ctx);
  void* ctx;
} pp_allocator;

/*
 * pp_create -- Algorithm 1, step 1.
 * Builds a handle for n_qubits qubits and merge group `group`, loads the
 * observable rows (obs_x/obs_z: n_obs rows of W words, host memory;
 * obs_coef: n_obs doubles, host), adds duplicate rows, and merges the rows
 * by orbit representative.  dtype is PP_F64 or PP_F32_COMPENSATED (FP32
 * mode rounds each obs_coef to FP32 once).  hip_stream may be NULL
 * (the null stream).  alloc may be NULL (hipMalloc).  On success *out holds
 * the handle; release it with pp_destroy.
 */
int pp_create(pp_state** out, int n_qubits, int group, int dtype,
              const uint64_t* obs_x, const uint64_t* obs_z,
              const double* obs_coef, size_t n_obs, void* hip_stream,
              const pp_allocator* alloc);

/*
 * pp_create_torus -- pp_create for the translation group of an lx x ly
 * torus (group PP_GROUP_TORUS, n_qubits = lx * ly, qubit q = x + lx*y).
 * Arguments, layout, ownership and errors as for pp_create; PP_EINVAL
 * unless 2 <= lx*ly <= 64.  Gate layers applied to the handle must be
 * closed under both unit translations (PP_ENOTSYM otherwise).
 */
int pp_create_torus(pp_state** out, int lx, int ly, int dtype,
                    const uint64_t* obs_x, const uint64_t* obs_z,
                    const double* obs_coef, size_t n_obs, void* hip_stream,
                    const pp_allocator* alloc);

/*
 * pp_create_group -- pp_create for any finite group of qubit permutations
 * (PP_GROUP_EXPLICIT).  perms (host, n_elems rows of n_qubits bytes,
 * row-major) lists every element g: qubit q of g.s carries qubit
 * perms[g*n_qubits + q] of s.  The list must be a group: every row a
 * permutation of 0..n_qubits-1, the identity present, closed under
 * composition, no row repeated; otherwise PP_EINVAL (also unless
 * 2 <= n_qubits <= 64 and 1 <= n_elems <= 1024).  The list is copied to the
 * device before the call returns.  Other arguments as for pp_create.
 * Gate layers applied to the handle must be closed under every element
 * (PP_ENOTSYM otherwise).
 */
int pp_create_group(pp_state** out, int n_qubits, const uint8_t* perms, size_t n_elems,
                    int dtype, const uint64_t* obs_x, const uint64_t* obs_z,
                    const double* obs_coef, size_t n_obs, void* hip_stream,
                    const pp_allocator* alloc);

/*
 * pp_apply_layer -- Algorithm 1, step 2a, for one symmetric (sub-)layer.
 * Applies n_gates rotations in the given order: gate k is
 * exp(-i theta[k]/2 P_k) with P_k = rows k of gate_x/gate_z (host, W words
 * each).  Each gate conjugates the current observable, O <- V_k^dag O V_k,
 * so a caller that holds a time-ordered layer passes it reversed.  After
 * every gate, identical strings are merged (standard PP, Sec. I) and terms
 * with |c| < inner_eps or weight > inner_max_weight are dropped
 * (inner_eps = 0 and inner_max_weight < 0 switch these off).
 * merge_every must be 1.  For a handle whose group is not
 * PP_GROUP_NONE the gate multiset must be closed under the group (every
 * translate / reflection / permutation of each gate present with the same
 * angle), otherwise PP_ENOTSYM.
 */
int pp_apply_layer(pp_state* s, const uint64_t* gate_x, const uint64_t* gate_z,
                   const double* theta, size_t n_gates, int merge_every,
                   double inner_eps, int inner_max_weight);

/*
 * pp_merge_canonicalize -- Algorithm 1, step 2b (Algorithms 2 and 3).
 * Replaces every string by its orbit representative and adds the
 * coefficients per representative.  For PP_GROUP_NONE the set is already
 * free of duplicates and the call only compacts the store.
 */
int pp_merge_canonicalize(pp_state* s);

/*
 * pp_truncate -- damping and truncation (Sec. IV: coefficient truncation of
 * the numerical examples; Fig. 3 caption: depolarising noise damping each
 * Pauli string by its weight after every Trotter step).
 * First multiplies every coefficient by (1 - depol_p)^{weight} (depolarising
 * noise on every qubit, Heisenberg picture; depol_p = 0: no damping), then
 * drops terms with |c| < eps or weight > max_weight (eps = 0 and
 * max_weight < 0: off; weight truncation is not in the paper, its truncated
 * workloads name it).  Does not synchronise.  PP_EINVAL for eps < 0 or
 * depol_p outside [0, 1], before anything changes.
 */
int pp_truncate(pp_state* s, double eps, int max_weight, double depol_p);

/*
 * pp_expectation -- Algorithm 1, step 3.
 * *out = Tr[rho O] for the symmetric product state rho = (|psi><psi|)^{(x)n}
 * whose single-qubit Bloch vector is bloch_xyz = (<X>, <Y>, <Z>):
 * sum_r c_r bx^{nX(r)} by^{nY(r)} bz^{nZ(r)}, reduced in FP64.
 */
int pp_expectation(pp_state* s, const double bloch_xyz[3], double* out);

/*
 * pp_expectation_noalloc -- pp_expectation for callers that cannot allocate
 * device or pinned memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, same result
 * (bitwise: the same products summed exactly and rounded once).  Its
 * working memory is a fixed device array inside the library (about 1.6 MB
 * per GPU, held until the process ends): the powers table, one exact
 * partial sum per 2048 store entries, a done counter and the result.  The
 * first call on a device looks the array up for that device (the handle's
 * device must be current); later calls allocate nothing.  Stores of more
 * than 2^27 entries (live and not yet compacted): PP_EINVAL with a message.
 * Every call on one GPU shares that array, so calls that overlap on one GPU
 * (other threads, other streams) race; calls on one stream are ordered.
 * Synchronises the handle's stream.
 */
int pp_expectation_noalloc(pp_state* s, const double bloch_xyz[3], double* out);

/*
 * Largest number of entries (live terms plus those truncated but not yet
 * compacted) the handle's term store has held since creation: the store
 * size a propagation needed, which the served form's admission learns from.
 * Synchronises.  NULL arguments: PP_EINVAL.
 */
int pp_peak_terms(pp_state* s, size_t* out);

/*
 * Layer-op statistics of a handle (see pp_set_layer_ops): out[0] layer ops
 * completed, out[1] layer-op runs that reported a bucket that did not fit
 * (each was run again with more buckets or replaced by its gate launches),
 * out[2] layer ops replaced by their gate launches, out[3] 1 when the
 * handle runs the gate launches throughout.  Synchronises the handle's
 * stream.
 */
int pp_layer_stats(pp_state* s, uint64_t out[4]);

/*
 * Device bytes of a term store of `cap` entries for a handle of n_qubits,
 * group and dtype (both halves, tables and the merge staging, as the
 * library would allocate them now; no allocation happens).  A handle that
 * has run a layer op (one-instance programs, see pp_set_layer_ops) also
 * carries its staging: 16W + 20 bytes per entry more.  A handle's
 * store grows to hold its largest set with headroom (4x below 2^24
 * entries, 2x below 2^27, 1.5x above), and the old store is freed only
 * after the new one is filled.  PP_EINVAL for a bad group or size.
 */
int pp_store_bytes(int n_qubits, int group, int dtype, size_t cap, size_t* out);

/* Number of live terms. */
int pp_num_terms(pp_state* s, size_t* out);

/*
 * Copies the live terms to caller-owned host arrays (x, z: cap rows of W
 * words, row r at [r*W, r*W + W); coef: cap doubles, FP32 coefficients
 * widened) sorted by key: ascending in the integer of Appendix E.2 (qubit q
 * the base-4 digit of weight 4^q, I, X, Y, Z = 0, 1, 2, 3), the integer
 * whose minimum picks a representative in Algorithms 2 and 3.  After a
 * symmetry merge that is one record per representative in key order.  The
 * sort runs on the device (radix passes over the store, 8 bits of the
 * integer each) in workspace taken from the handle's allocator and freed
 * before the call returns; synchronises the handle's stream.  *n_out =
 * number written.  PP_EINVAL if cap is smaller than the number of live
 * terms or an array is NULL; PP_ENOMEM if the workspace cannot be had;
 * PP_EDEVICE if the liveness flags disagree with the term count.
 */
int pp_export_terms(pp_state* s, uint64_t* x, uint64_t* z, double* coef,
                    size_t cap, size_t* n_out);

/*
 * Work counters since creation: out[0] = propagated = sum over gates of the
 * live terms tested against the gate (Prop. 1's propagation unit);
 * out[1] = merged = sum over merge points of the records entering the merge
 * (after every gate: live terms + anticommuting terms; after a layer: the
 * live terms fed to the symmetry merge).
 */
int pp_counters(pp_state* s, uint64_t out[2]);

/*
 * Finer work counters: out[0] propagated, out[1] merged (as pp_counters),
 * out[2] = sum over gates of the live terms that anticommute with the gate,
 * out[3] = strings appended by gates (children whose partner was absent),
 * out[4] = records entering symmetry merges / compactions,
 * out[5] = representatives leaving them (in programs, after the sub-layer's
 *          truncation, which is applied as the merge emits),
 * out[6] = sum over gate launches of the live terms entering the launch
 *          (keys read; a fused launch of several rotations reads each key once),
 * out[7] = sum over gate launches of the entering terms that anticommute
 *          with one of its rotations (coefficients read and written once).
 * Without fusion out[6] = out[0] and out[7] = out[2].  These are the unit
 * counts of the algorithmic-bytes model of each kernel.
 */
int pp_work_counters(pp_state* s, uint64_t out[8]);

/*
 * Statistics of the partitioned merge (the path large merges of 64-bit keys
 * take, except S_n), cumulative since creation: out[0] = partitioned merges
 * run, out[1] = buckets split over several blocks because a few
 * representatives hold more than twice a bucket's average share of the
 * records, out[2] = buckets with more distinct representatives than one LDS
 * table holds (summed in several selector passes), out[3] = representatives
 * whose sums went through the global merge table (split buckets and
 * overfull passes).  Synchronises.  NULL arguments: PP_EINVAL.
 */
int pp_merge_stats(pp_state* s, uint64_t out[4]);

/* Kernel kinds for per-kernel timing. */
enum {
  PP_K_GATE = 0,          /* one rotation + exact merge + truncation     */
  PP_K_MERGE_NARROW = 1,  /* representative + exact sum, 64-bit keys     */
  PP_K_MERGE_WIDE1 = 2,   /* representative + hash slot, wider keys      */
  PP_K_MERGE_WIDE2 = 3,   /* owner compare + exact sum, wider keys       */
  PP_K_MERGE_COLLECT = 4, /* merge table -> new term store               */
  PP_K_COMPACT = 5,       /* plain-PP layer end: drop dead entries       */
  PP_K_SCAN = 6,          /* damping / truncation / recount / expectation */
  PP_K_GROW = 7,          /* store growth                                */
  PP_K_PART_HIST = 8,     /* partitioned merge 1: bucket counts per tile   */
  PP_K_PART_SCAN = 9,     /* partitioned merge 2: offsets, bucket bases    */
  PP_K_PART_SCATTER = 10, /* partitioned merge 3: bucket-contiguous stage  */
  PP_K_PART_AGG = 11,     /* partitioned merge 4: LDS exact sums per bucket */
  PP_K_LAYER_SCATTER = 12,/* layer op 1: strings to closed buckets        */
  PP_K_LAYER_APPLY = 13,  /* layer op 2: a bucket's rotations in LDS      */
  PP_KERNEL_KINDS = 14
};

/*
 * pp_profile(s, every) resets the per-kernel timing of handle s and, for
 * every > 0, brackets every `every`-th run of back-to-back launches of one
 * kernel kind (for instance the gate launches of one sub-layer) with two HIP
 * events recorded on the handle's stream (1 = every run; 0 = off); the
 * interval counts for each launch of the run, so the average includes the
 * gaps between launches of the run but no event sits between them.
 * pp_profile_read returns, per kernel kind, the number of timed launches
 * and their summed duration in milliseconds (both synchronise).
 * pp_profile(NULL, every) sets the value that handles created afterwards
 * start with (their pp_create included).  The batched form of more than one
 * instance is not timed.
 */
int pp_profile(pp_state* s, int every);
int pp_profile_read(pp_state* s, uint64_t launches[PP_KERNEL_KINDS],
                    double milliseconds[PP_KERNEL_KINDS]);

/* Upper bound on stored terms (live + not yet compacted); 0 = no limit. */
int pp_set_max_terms(pp_state* s, size_t max_terms);

void pp_destroy(pp_state* s);

/* Thread-local message for the most recent error ("" if none). */
const char* pp_last_error(void);

/*
 * Batched form.  A program is a whole propagation described on the host:
 * sub-layers in Heisenberg order (n_sub of them; sub-layer j owns gates
 * [sub_start[j], sub_start[j+1]) of gate_x/gate_z/theta, already in the
 * order they are applied), each with its inner/outer truncation eps[j],
 * max_weight[j] and damping depol_p[j] (applied before its gates), and the
 * final Bloch vector.  The library uploads it once.  Every sub-layer runs
 * damp -> gates (exact merge + truncation after each) -> symmetry merge ->
 * truncation, and the program ends with the expectation value.
 * merge_after: NULL (merge after every sub-layer) or n_sub flags; a 0 skips
 * sub-layer j's symmetry merge (Algorithm 1 step 2b) and keeps only its
 * truncation, as when merging after a full Trotter layer of several
 * symmetric sub-layers (Sec. IV, Ising example): the set then holds
 * non-representative strings until the next merge, and the expectation is
 * the same (Theorem 1 needs only a symmetric state).
 */
int pp_program_create(pp_program** out, int n_qubits, size_t n_sub,
                      const size_t* sub_start, const uint64_t* gate_x,
                      const uint64_t* gate_z, const double* theta,
                      const double* eps, const int* max_weight,
                      const double* depol_p, const double bloch_xyz[3],
                      const int* merge_after);
void pp_program_destroy(pp_program* p);

/*
 * Shape of a created program: out[0] = device operations, out[1] = apply
 * operations a one-instance run launches (a layer op, or a gate launch of
 * up to three fused rotations outside the fallback copies of layer ops),
 * out[2] = rotations, out[3] = layer ops (see pp_set_layer_ops).  NULL
 * arguments: PP_EINVAL.
 */
int pp_program_info(const pp_program* p, uint64_t out[4]);

/*
 * Runs programs[i] on states[i] for i < n (n <= 1024), all instances
 * advancing together: every step is one pass of a fixed sequence of
 * persistent kernels that serve all instances at once, and steps are
 * replayed from a captured HIP graph.  An instance whose store has held
 * 2^18 entries leaves the batch at the next step boundary and finishes
 * alone (the one-instance path, whose large merges are partitioned) while
 * the others wait; results do not depend on it (exact sums).  Each state
 * must have been created on `hip_stream` with the program's n_qubits.  On
 * return
 * expectations[i] (host array, may be NULL) holds Tr[rho O] of instance i.
 */
int pp_batch_run(pp_state* const* states, const pp_program* const* programs,
                 size_t n, void* hip_stream, double* expectations);

/*
 * Incremental form for serving: advances every listed instance by up to
 * max_steps batched steps (graph replays) and sets done[i] = 1 for
 * instances whose program has finished (expectations[i] then valid),
 * 0 for running ones and -1 for one whose term store could not grow
 * (allocator failure or pp_set_max_terms); a failed instance stops, the
 * others continue, and the call still returns PP_OK.  Instances may join or
 * leave between calls.  An instance promoted as in pp_batch_run finishes
 * within the call that promotes it.  A state starts its program at the first
 * pp_batch_step/pp_batch_run call that lists it with that program.
 * pp_batch_run returns the first failure's code instead.
 */
int pp_batch_step(pp_state* const* states, const pp_program* const* programs,
                  size_t n, void* hip_stream, int max_steps, int* done,
                  double* expectations);

/*
 * Launch tuning (process-wide; the autotuner picks it per workload class):
 * terms per thread of the gate kernel and of the streaming kernels (merge,
 * compaction, damping/truncation/expectation) in {1, 2, 4, 8}, the cap on
 * blocks per launch, the batched steps per captured graph, and the gate
 * launches per batched step (1..64).  A 0 keeps the current value.
 * pp_get_tuning returns the five current values in that order.
 */
int pp_set_tuning(int gate_items, int stream_items, int max_blocks, int graph_steps,
                  int gates_per_step);
int pp_get_tuning(int out[5]);

/*
 * Merge tuning (process-wide; the autotuner picks it): the partitioned
 * merge of large sets aims at 2^bucket_log2 records per bucket (10..18;
 * default 14; 0 keeps the current value; applies to term stores allocated
 * afterwards), and its aggregation pass runs on agg_blocks blocks that
 * take the buckets in turn (0: one block per bucket or chunk, the default;
 * at most 4096).  Results do not depend on either (exact sums).
 * pp_get_merge_tuning returns the two current values.
 */
int pp_set_merge_tuning(int bucket_log2, int agg_blocks);
int pp_get_merge_tuning(int out[2]);

/*
 * Gate fusion (process-wide).  Consecutive rotations of a sub-layer whose
 * Pauli strings commute pairwise and are independent (no product of a
 * nonempty subset of them is the identity) are applied by one launch, up to
 * max_rotations of them (2 or 3; 0 or 1 switches fusion off; default 3).
 * Each rotation keeps its own exact merge and truncation in circuit order,
 * as Algorithm 2 prescribes per gate, so results, expectations and the
 * propagated / merged counters are identical with fusion off; the launch
 * count, the keys read and the stored-but-dead strings change.  An op of r
 * fused rotations needs store room for 2^(r-1) (live + anticommuting)
 * terms where a single gate needs live + anticommuting, so near
 * pp_set_max_terms a fused run can report PP_ECAPACITY where an unfused
 * one would not.  Applies to pp_apply_layer and pp_program_create calls
 * made afterwards.  lanes = 1 runs a fused op over a set last seen below
 * 2^19 terms with one lane per member of each group of 2^r strings instead
 * of one thread per term (the same values, bitwise; more blocks, so more
 * contended append atomics); lanes = 0 (default) always uses one thread per
 * term.  Applies to launches made afterwards.  max_rotations outside 0..3
 * or lanes outside 0..1: PP_EINVAL.
 */
int pp_set_gate_fusion(int max_rotations, int lanes);

/*
 * Layer ops (process-wide; programs created afterwards).  A sub-layer of
 * 4 to 64 pairwise commuting rotations (Algorithm 1 step 2a: each rotation
 * of Prop. 1 followed by the exact merge of identical strings and the
 * truncation) is applied by two launches instead of one per group of fused
 * rotations: every live string goes to a bucket keyed by what the
 * sub-layer's rotations cannot change (which rotations it anticommutes
 * with, and its letters outside those rotations' support), so a bucket holds
 * everything its strings can become, and one block applies all the
 * rotations to its bucket in LDS, in circuit order, with the same arithmetic
 * as the gate launches.  Results, expectations and the propagated / merged
 * counters equal those with layer ops off, bitwise.  A bucket that does not
 * fit its staging slots or the block's LDS makes the op run again with
 * twice the buckets, then as its fused gate launches; after eight such
 * fallbacks a handle runs the gate launches throughout.  One-instance
 * programs only (pp_batch_run / pp_batch_step with one instance, and
 * promoted instances); the batched steps run the gate launches.  The store
 * then also carries (16W + 8) bytes of staging per entry.  mode 0: off,
 * 1: on (default), 2: on, but every layer op reports a failure (tests of the
 * fallback path).  Other modes: PP_EINVAL.
 */
int pp_set_layer_ops(int mode);

/*
 * Layer-op tuning knobs (process-wide, launches made afterwards):
 * bucket_log2 = log2 of the strings per bucket aimed at (4..10, default 7;
 * 0 keeps the current value), block = threads per bucket block (256 or 512,
 * default 512; 0 keeps).  Results do not depend on them.  Out of range:
 * PP_EINVAL.  pp_get_layer_tuning returns the two current values.
 */
int pp_set_layer_tuning(int bucket_log2, int block);
int pp_get_layer_tuning(int out[2]);

#ifdef __cplusplus
}
#endif

#endif /* PP_H */
