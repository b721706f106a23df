/*
 * fhs.h -- reduced-history Feynman amplitudes on one AMD MI355X (gfx950).
 *
 * Problem (paper, Section I and Eq. (2)): given a circuit, a sparse input
 * state psi = sum_i coeff_i |b_in_i> and a list of output bitstrings, compute
 * exactly the requested amplitudes <b_out_j| C |psi> =
 * sum_i coeff_i * alpha^{b_in_i, b_out_j}, each transition amplitude being
 * the reduced sum over artificial-source assignments of Eq. (7).
 *
 * Conventions shared by every call:
 *   - Circuit text: one gate per line in time order after "qubits <n>"
 *     (gates H X Y Z S SDG T TDG P RX RY RZ CX CZ SWAP CP RZZ CCX CSWAP MCX MCZ,
 *     angles as C99 hex floats, "~q" marks a control active on 0).
 *   - Bitstrings: W = ceil(n/64) uint64 words each, little-endian: qubit q is
 *     bit (q mod 64) of word q/64.  Bits at positions >= n must be zero.
 *   - Complex numbers: two doubles (re, im), interleaved.
 *   - Evaluation order runs from the output towards the input (Section IV-A);
 *     gate position e in evaluation order is time index G-1-e.  Artificial
 *     source k (k = 0 nearest the output) is bit k of a history index h.
 *   - Every call returns an fhs_status; none aborts, throws or exits.
 *     Argument errors are detected before any work is enqueued and leave all
 *     outputs untouched.
 *   - Device pointers are HIP device memory owned by the caller; "stream" is
 *     a hipStream_t passed as void* (NULL = the null stream).
 */
#ifndef FHS_H
#define FHS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FHS_OK = 0,
    FHS_EINVAL = 1,        /* bad argument (NULL pointer, c1 > c2, NaN/negative threshold, bits >= n) */
    FHS_EUNSUPPORTED = 2,  /* gate or feature outside the supported set */
    FHS_ERANGE = 3,        /* n > 128, A > 62, a size that overflows, or a cost model used outside its training range */
    FHS_ENOMEM = 4,        /* workspace too small, or a host/device allocation failed */
    FHS_EHIP = 5,          /* a HIP runtime call failed (message in fhs_last_error) */
    FHS_ESTATE = 6,        /* call order violated (e.g. evaluate before load) */
    FHS_EPARSE = 7         /* circuit text could not be parsed */
} fhs_status;

/* Partition modes for fhs_choose_partition (Section IV-C). */
enum {
    FHS_PART_NONE = 0,     /* (0,0): no checkpoint, every gate in the suffix */
    FHS_PART_THIRDS = 1,   /* fixed split, a third of the gates per region (Section V, amplitude amplification) */
    FHS_PART_EQ8 = 2,      /* argmin of Eq. (8) over all 0 <= c1 <= c2 <= G, smallest (c1,c2) on ties */
    FHS_PART_MODEL = 3     /* argmin of the loaded cost model's prediction (fhs_load_cost_model) */
};

typedef struct fhs_program fhs_program;  /* host-side reduced-history program; immutable */
typedef struct fhs_ctx fhs_ctx;          /* one device, one loaded program; not thread-safe */

typedef struct {
    uint32_t n_qubits;    /* n */
    uint32_t n_gates;     /* G */
    uint32_t n_sources;   /* A: artificial sources from the backward sweep (Section IV-A) */
    uint32_t n_words;     /* W = ceil(n/64) */
    uint32_t n_leading;   /* gates before the first source gate, evaluation order */
    uint32_t n_branch;    /* branching gates, natural ones included */
    uint32_t forward;     /* 1: sources placed by the forward sweep (FHS_REDUCE_FORWARD) */
} fhs_program_info;

/* Human-readable name of a status code (static storage). */
const char *fhs_status_string(fhs_status s);

/* ---------------------------------------------------------------------
 * Host-only calls (no GPU needed)
 * ------------------------------------------------------------------- */

/* Section II-A and IV-A: parse `text` (len bytes, need not be NUL-terminated),
 * classify every gate from its matrix (diagonal -> wire-preserving, one
 * nonzero per column -> deterministic, else branching), mark natural input
 * segments, place artificial sources by one backward sweep, and emit the
 * straight-line history program.  *out is owned by the caller and released
 * with fhs_program_free.  Errors: FHS_EPARSE, FHS_EUNSUPPORTED, FHS_ERANGE
 * (n > 128 or G >= 2^24).  A > 62 is accepted here (Eq. (8) still works) and
 * rejected by the evaluate calls. */
fhs_status fhs_reduce(const char *text, size_t len, fhs_program **out);

/* fhs_reduce with options; fhs_reduce(t, n, out) == fhs_reduce_ex(t, n,
 * FHS_REDUCE_FUSE | FHS_REDUCE_PAIR, out).  FHS_REDUCE_FUSE folds every
 * ladder of controlled X gates that adds or subtracts one on consecutive
 * qubits (the increment / decrement cascades of the quantum walk, Section V)
 * into one instruction: the same history program step for step, evaluated
 * with a multi-word add instead of one mask test per gate.  FHS_REDUCE_PAIR
 * (only with FHS_REDUCE_FUSE) then merges two folded ladders that are
 * adjacent in evaluation order, act on the same field, and whose controls
 * differ only in the value of one bit outside the field (the walk's shift:
 * +1 for one coin value, -1 for the other) into one instruction that picks
 * the sign from that bit: one carry chain per history instead of two.
 * Positions, sources, cuts, final-bit masks and Eq. (8) are those of the
 * unfused program; fhs_program_work reports the fused work.  flags = 0 keeps
 * one instruction per gate.  FHS_EINVAL on unknown flags or PAIR without
 * FUSE.  (Ladder folding recognises the cascades in evaluation order, so a
 * cascade written most significant bit first is folded only when walked
 * from the output.) */
/* FHS_REDUCE_FORWARD (Section IV-F, Table I's forward column) places the
 * artificial sources by one sweep from the input instead: a branching gate
 * whose output-side segment is not a natural output segment (a wire from the
 * gate to the output with only wire-preserving incidences) gets a source on
 * that segment, numbered from the input.  The evaluation order is then the
 * time order: a history starts from b_in, walks the gates input -> output
 * and is checked against b_out; every evaluation position, cut and source
 * position of this API counts from the input (gate position e is time index
 * e).  The amplitudes are the same; the history indices, and so the valid
 * sets, are those of the forward placement.  Internally the program is the
 * backward one of the transposed circuit (gates reversed, matrices
 * transposed), since <b_out|C|b_in> = <b_in|C^T|b_out>. */
/* FHS_REDUCE_OPTIMAL and FHS_REDUCE_GREEDY (Section IV-B, Fig. 3) place the
 * sources by determinism reachability instead of the sweep: the three
 * internal wires around a CNOT are symmetric (any two fix the third), so
 * some of the backward sweep's sources are implied by the others.  The
 * sources are chosen among the input segments of branching gates, as few
 * as let the relations (CNOT, SWAP, one-qubit deterministic gates) reach
 * every internal wire: OPTIMAL by exhaustive search in increasing size
 * (the first set found with candidates in evaluation order; FHS_ERANGE if
 * the search exceeds its budget), GREEDY adding the candidate that reaches
 * the most wires at each step.  Sources are numbered in evaluation order of
 * their gates.  Every other branching gate's input bit is an affine
 * function over GF(2) of the sources and the boundary bits, evaluated per
 * history (OP_BRANCH_AFF); the evaluation order stays output -> input.
 * Cuts may not separate an affine input from a deeper source its form
 * uses: fhs_set_partition returns FHS_EINVAL for such a cut, and
 * fhs_choose_partition / fhs_candidate_splits avoid them.  Gate set:
 * branching gates on one qubit, deterministic gates on one qubit, CNOT
 * (MCX with one control) and SWAP, diagonal gates of any size; otherwise
 * FHS_EUNSUPPORTED.  Not combinable with FHS_REDUCE_FORWARD. */
enum {
    FHS_REDUCE_FUSE = 1, FHS_REDUCE_PAIR = 2, FHS_REDUCE_FORWARD = 4,
    FHS_REDUCE_OPTIMAL = 8, FHS_REDUCE_GREEDY = 16
};
fhs_status fhs_reduce_ex(const char *text, size_t len, uint32_t flags, fhs_program **out);
void fhs_program_free(fhs_program *prog);
fhs_status fhs_program_get_info(const fhs_program *prog, fhs_program_info *info);

/* Evaluation positions of the gates that carry sources 0..A-1 (ascending),
 * written to eval_pos[0..min(A,cap)-1]. */
fhs_status fhs_program_sources(const fhs_program *prog, uint32_t *eval_pos, uint32_t cap);

/* Whether a cut may fall at evaluation position c (0 <= c <= G): *allowed =
 * 1, or 0 when the cut would put an affine branching input (placement by
 * reachability) in a region evaluated before the region of a source its
 * form uses.  Positions 0 and G, and every position of a program placed by
 * a sweep, are allowed.  A cut below the leading source-free gates acts at
 * their end (n_leading).  fhs_set_partition refuses a split whose acting
 * cuts are not allowed (FHS_EINVAL); fhs_candidate_splits and
 * fhs_choose_partition offer allowed ones only. */
fhs_status fhs_cut_allowed(const fhs_program *prog, uint32_t c, int *allowed);

/* Eq. (8): Gate_ops = 2^Ap (Gp + 2^Ar (Gr + 2^As Gs)) for cuts c1 <= c2 <= G,
 * prefix = evaluation positions [0,c1), root [c1,c2), suffix [c2,G).  The
 * 128-bit result is cost[0] (low word) + 2^64 cost[1].  regions (may be NULL)
 * receives {Gp, Gr, Gs, Ap, Ar, As}. */
fhs_status fhs_partition_cost(const fhs_program *prog, uint32_t c1, uint32_t c2,
                              uint64_t cost[2], uint32_t *regions);

/* Algorithmic work of evaluation positions [e0, e1) for one history, by a
 * fixed per-gate model (a history's backward step through one gate):
 *   int_ops:    32-bit integer operations: controlled permutation or phase
 *               3w+1 (w = state words spanned by its controls, at least 1),
 *               swap 3w+4, one-qubit diagonal 1, two-qubit diagonal 3,
 *               anti-diagonal 2, branching 1 (3 when the gate has zero
 *               entries: the index and its test); a fused ladder 3w+1+1 (1
 *               without controls; the gates folded into it 0) and a paired
 *               ladder 3w+1+2 (2 without common controls; the second ladder
 *               0) for the step, plus 3f (f state words spanned by the
 *               field) once per run of such steps on one field that starts
 *               in [e0, e1) with nothing touching the field in between
 *               (the steps of a run add up and are applied with one carry
 *               chain); when e1 is the end of the program and the final
 *               check compares the whole field of the run still pending
 *               there, that run costs 2 instead of 3f (its count is
 *               compared with the field's residue); a paired step without
 *               controls whose selecting bit holds a source bit set by a
 *               branching gate earlier in [e0, e1) costs 0, its run 2 per
 *               sign of such steps (one popcount of the source index);
 *   fp64_flops: complex multiply of the running amplitude: 6 for a general
 *               factor table, 2 if every entry is purely real or imaginary,
 *               0 if every entry is 0, +-1 or +-i; a negation counts 0; a
 *               branching gate whose four entries are real, nonzero and of
 *               one magnitude (H) counts 0: the product of such magnitudes
 *               over a region is one constant for every history, and only
 *               the sign is per history;
 *   branch:     branching gates (one modulus multiply each when pruning). */
typedef struct {
    uint64_t gates;
    uint64_t int_ops;
    uint64_t fp64_flops;
    uint64_t branch;
    uint64_t src_int_ops;   /* the part of int_ops whose inputs are only the
                               range's own source bits: a source bit into the
                               state (without zero entries), a popcount of the
                               source index, operations on state bits that hold
                               nothing else; the same for every history that
                               shares the range's source assignment */
    uint64_t hoist_int_ops; /* taken as a suffix region (without pruning): the
                               int_ops and fp64_flops of its instructions the
                               compiled consumer evaluates once per root
                               history instead of once per leaf: phases and
                               branching gates on a natural input segment that
                               no source of the range influences and that
                               commute with the instructions before them */
    uint64_t hoist_fp64_flops;
    uint64_t count_int_ops; /* taken as regions of the compiled consumer without
                               pruning whose plan counts two-valued factors
                               (fhs_plan.count_groups > 0): the int32 ops the
                               range's two-valued gates add in their counted
                               form (the step into the history's table index:
                               1 for a diagonal or deterministic gate, 2 for a
                               branching gate, whose selecting bit is then
                               formed too) and the fp64_flops they no longer
                               take; the hoisted part of each below */
    uint64_t count_fp64_flops;
    uint64_t hoist_count_int_ops;
    uint64_t hoist_count_fp64_flops;
} fhs_work;

fhs_status fhs_program_work(const fhs_program *prog, uint32_t e0, uint32_t e1, fhs_work *out);

/* Section IV-C: choose cuts.  FHS_PART_NONE, FHS_PART_THIRDS and
 * FHS_PART_EQ8 need no context; FHS_PART_MODEL needs fhs_choose_partition_ctx
 * (FHS_ESTATE here). */
fhs_status fhs_choose_partition(const fhs_program *prog, int mode, uint32_t *c1, uint32_t *c2);

/* ---------------------------------------------------------------------
 * Device calls
 * ------------------------------------------------------------------- */

/* Create a context on HIP device `device`.  *out is released with
 * fhs_ctx_destroy.  FHS_EHIP when the device cannot be used. */
fhs_status fhs_ctx_create(int device, fhs_ctx **out);
void fhs_ctx_destroy(fhs_ctx *ctx);

/* Message for the last failing call on ctx (valid until the next call). */
const char *fhs_last_error(const fhs_ctx *ctx);

/* Upload the history program to the device (synchronous).  The program may
 * be freed afterwards.  Resets the partition to (0,0). */
fhs_status fhs_load_program(fhs_ctx *ctx, const fhs_program *prog);

/* Set the checkpoint cuts (Section IV-C, Algorithm 2) used by fhs_evaluate.
 * FHS_EINVAL unless c1 <= c2 <= G; FHS_ESTATE before fhs_load_program. */
fhs_status fhs_set_partition(fhs_ctx *ctx, uint32_t c1, uint32_t c2);
fhs_status fhs_get_partition(const fhs_ctx *ctx, uint32_t *c1, uint32_t *c2);

/* Upper bound on the prefix-table bytes one fhs_evaluate call may stage in
 * the workspace (default 1 GiB); output pairs are processed in batches that
 * fit.  Minimum 1 MiB. */
fhs_status fhs_set_table_budget(fhs_ctx *ctx, size_t bytes);

/* Launch shape of the hot kernels (the tile/chunk autotuner's search space;
 * the paper's execution model, Section IV-D, leaves it to the platform).
 * Zero fields mean "default".
 *   histories_per_lane  1 or 2: independent histories each lane walks in
 *                       lockstep through one decoded instruction stream
 *                       (default 2);
 *   chunk               prefix entries per work item of the persistent
 *                       consumer at most, a power of two in [1, 256]
 *                       (default 256); the plan halves it, down to 8, while
 *                       a batch would hold fewer than 128 work items per
 *                       compute unit (fhs_get_plan reports the value used);
 *   blocks_per_cu       persistent workgroups per compute unit, at most the
 *                       occupancy limit (default: the occupancy limit);
 *   dispatch            how the kernels walk the program: 1 one opcode
 *                       dispatch per run of identical opcodes, 2 one per
 *                       instruction, 0 automatic (per run when the program's
 *                       runs average two or more instructions), 3 compiled:
 *                       the consumer's root and suffix regions (and the
 *                       prefix-table build's region, when it also holds at
 *                       most 1024 device instructions) are emitted as
 *                       straight-line code and compiled for gfx950 at the
 *                       first evaluation of each program and split (hipRTC,
 *                       about a second; cached in the context; see
 *                       fhs_precompile) when they hold at most 1024 device
 *                       instructions (else, and for the other kernels, the
 *                       automatic rule).  fhs_evaluate returns
 *                       FHS_EUNSUPPORTED, with the compiler log in
 *                       fhs_last_error, if that compilation fails.
 *   items_per_claim     work items a consumer workgroup takes from the
 *                       queue with one atomic, 1..64 (default: automatic,
 *                       about 2^16 candidate histories per claim, at most
 *                       16 items and at least 64 claims per compute unit;
 *                       fhs_get_plan reports the value used).
 * Affects speed and the grouping of the amplitude sums (so their last bits),
 * never the history counts.  FHS_EINVAL for values out of range. */
typedef struct {
    uint32_t histories_per_lane;
    uint32_t chunk;
    uint32_t blocks_per_cu;
    uint32_t dispatch;
    uint32_t items_per_claim;
} fhs_launch_config;

fhs_status fhs_set_launch_config(fhs_ctx *ctx, const fhs_launch_config *cfg);
fhs_status fhs_get_launch_config(const fhs_ctx *ctx, fhs_launch_config *cfg);

/* Compile ahead of time, under the current launch configuration (dispatch
 * mode 3 only; otherwise nothing to do), the consumers that fhs_evaluate
 * would compile for the n splits (c1[i], c2[i]) at M outputs, S inputs and
 * the given threshold, so that timing many splits (autotuning, the learned
 * split's shortlist, training data) does not pay one compilation per split
 * in turn.  hipRTC serialises compilations inside a process, so they run
 * in up to `threads` child processes of the helper fhs_rtc built next to the
 * library (started with posix_spawn, descriptors from 3 up closed; they make
 * no HIP call), or one at a time in this process when the helper is absent
 * or threads is 1; the modules are loaded on ctx's device and cached in ctx
 * (kept until the next fhs_load_program).  Splits whose plan does not fit (the table budget) or
 * whose consumer is already cached are skipped; *n_compiled (may be NULL)
 * receives the number compiled.  The context's partition is unchanged.
 * FHS_EINVAL for a split outside c1 <= c2 <= G or zero M, S or threads;
 * FHS_ESTATE without a program; FHS_EUNSUPPORTED (log in fhs_last_error) if
 * a compilation fails. */
fhs_status fhs_precompile(fhs_ctx *ctx, const uint32_t *c1, const uint32_t *c2, uint32_t n, uint32_t M,
                          uint32_t S, double threshold, uint32_t threads, uint32_t *n_compiled);

/* Kernel timing.  When enabled, every later evaluation records HIP events
 * around each launch of its hot kernel (the persistent consumer of
 * fhs_evaluate, the plain kernel of fhs_evaluate_plain); fhs_evaluate then
 * enqueues its launch sequence directly on the stream instead of replaying
 * its graph, since events recorded inside a graph carry no timestamps.  After the stream has synchronized, fhs_kernel_times
 * writes the durations in milliseconds of the most recent call's launches to
 * ms[0..min(count,cap)-1] and their number to *count.  FHS_ESTATE if timing
 * is off or nothing was timed; FHS_EHIP if the events have not completed. */
fhs_status fhs_set_kernel_timing(fhs_ctx *ctx, int enable);
fhs_status fhs_kernel_times(fhs_ctx *ctx, float *ms, uint32_t cap, uint32_t *count);

/* Work counts of the most recent fhs_evaluate run in timing mode (Section
 * IV-C, Algorithm 2): prefix-table entries built (M S 2^Ap) and those still
 * consistent after the prefix region, i.e. the entries whose 2^Ar root
 * assignments the consumer evaluates.  Counted by a separate kernel after
 * each table build, outside the timed interval.  Blocks until that count
 * is available.  FHS_ESTATE if timing is off or nothing was timed. */
fhs_status fhs_kernel_counts(fhs_ctx *ctx, uint64_t *prefix_entries, uint64_t *prefix_valid);

/* Per-work-item timestamps of the most recent fhs_evaluate run in timing
 * mode, for the cost distribution over outputs (Section V: time against the
 * number of sources, time per requested bitstring): the persistent
 * consumer's work item (pair p, part j: chunk j / root_parts of its prefix
 * entries, part j % root_parts of that chunk's root tasks) has index
 * p * items_per_pair + j, pairs numbered p = j_out * S + i_in; stamps[2 k]
 * and stamps[2 k + 1] receive the device's constant-rate clock when a
 * workgroup popped item k and when it stored the item's sums (ticks_per_s
 * ticks per second; comparable across compute units).  Writes min(count,
 * cap) items (blocking copy).  The items of a pair the precheck rejected
 * are skipped: their stamps stay 0.
 * FHS_ESTATE if timing is off or the last timed call was not a batched
 * evaluation with sources. */
fhs_status fhs_item_stamps(fhs_ctx *ctx, uint64_t *stamps, size_t cap, size_t *count,
                           uint32_t *items_per_pair, uint64_t *ticks_per_s);

/* Work layout fhs_evaluate would use for M outputs and S inputs.  The cuts
 * are the effective ones: the source-free gates nearest the output run once
 * per pair in the precheck, so a cut below n_leading moves up to it (the
 * source counts per region are unchanged). */
typedef struct {
    uint32_t c1, c2;               /* effective cuts, evaluation order */
    uint32_t Ap, Ar, As;           /* sources per region */
    uint32_t n_batches;            /* launches of the prefix build and the consumer */
    uint32_t pairs_per_batch;      /* (input, output) pairs per batch (last may be fewer) */
    uint32_t chunk;                /* prefix entries per work item */
    uint32_t items_per_pair;       /* work items per pair */
    uint32_t lanes_per_root_task;  /* lanes that share one (entry, h_r) root task */
    uint32_t plain_blocks_per_pair;
    uint64_t table_bytes;          /* prefix-table bytes per batch */
    uint32_t prefix_depth_first;   /* prefix sources enumerated depth first inside a lane */
    uint32_t items_per_claim;      /* work items a consumer workgroup takes from the queue at once */
    uint32_t count_groups;         /* the compiled consumer without pruning: table multiplies per
                                      valid history of the counted two-valued factors (0: none
                                      counted; on only when a class has a gate in the leaf loop and
                                      every class fits the tables) */
    uint32_t count_entries;        /* their tables' entries (16 bytes each, in LDS) */
    uint32_t root_parts;           /* work items per chunk: its root tasks in this many parts
                                      (items_per_pair = chunks per pair * root_parts) */
    uint32_t pair_filter;          /* 1: the precheck applies the pair-level residue test (every
                                      write to one bit field after the leading gates is a
                                      source-selected ladder step and the final check covers it:
                                      a pair whose residue no history's step count reaches is
                                      rejected, its amplitude and statistics zero), and the
                                      consumer skips the items of rejected pairs */
} fhs_plan;

fhs_status fhs_get_plan(const fhs_ctx *ctx, uint32_t M, uint32_t S, fhs_plan *plan);

/* Bytes of device workspace fhs_evaluate / fhs_evaluate_plain need for M
 * outputs and S inputs under the current program and partition. */
fhs_status fhs_workspace_size(const fhs_ctx *ctx, uint32_t M, uint32_t S, size_t *bytes);

/* Batched, checkpointed evaluation (Algorithm 2 on the GPU).
 *   d_inputs  [S*W]  input bitstrings b_in_i          (device, read)
 *   d_coeffs  [S*2]  <b_in_i|psi> as (re,im)          (device, read)
 *   d_outputs [M*W]  requested output bitstrings      (device, read)
 *   threshold        t >= 0, finite; 0 = exact (Section IV-A, threshold pruning)
 *   d_amps    [M*2]  <b_out_j|C|psi>                  (device, written)
 *   d_stats   [M*4]  per output, summed over inputs: number of valid
 *                    histories, sum of their indices h (mod 2^64), xor of
 *                    SplitMix64(h), leaf histories walked: the suffix
 *                    assignments of consistent roots the consumer evaluated
 *                    (those the final field check's residue rules out in
 *                    advance, a pass or a root at a time, are not walked)
 *                    (device, written)
 *   d_ws, ws_bytes   workspace of at least fhs_workspace_size bytes, 256-byte
 *                    aligned (device, scratch; contents undefined afterwards)
 * Enqueued asynchronously on `stream`: one precheck launch, then per batch of
 * output pairs a prefix-table build and one persistent root/suffix launch fed
 * by an atomic work queue, then a deterministic finalize.  The sequence is
 * captured into a HIP graph and replayed when every argument repeats.
 * Results are deterministic (bit-identical across runs).  FHS_ERANGE if
 * A > 62; FHS_ENOMEM if ws_bytes is too small. */
fhs_status fhs_evaluate(fhs_ctx *ctx,
                        const uint64_t *d_inputs, const double *d_coeffs, uint32_t S,
                        const uint64_t *d_outputs, uint32_t M, double threshold,
                        double *d_amps, uint64_t *d_stats,
                        void *d_ws, size_t ws_bytes, void *stream);

/* Plain evaluation (Algorithm 1 on the GPU): no checkpoint, a static grid of
 * one lane per candidate history h over every output pair, no queue, no
 * graph.  Same arguments, results and error behaviour as fhs_evaluate. */
fhs_status fhs_evaluate_plain(fhs_ctx *ctx,
                              const uint64_t *d_inputs, const double *d_coeffs, uint32_t S,
                              const uint64_t *d_outputs, uint32_t M, double threshold,
                              double *d_amps, uint64_t *d_stats,
                              void *d_ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as fhs_evaluate, with no workspace argument.  Its workspace is
 * a static device array of FHS_NOALLOC_SCRATCH_BYTES bytes inside the
 * library, one copy per GPU, held from the library's first use on that GPU
 * until the process ends.  Output pairs are batched so that the whole
 * workspace fits it (smaller batches than fhs_evaluate may use).  The call
 * allocates nothing: no hipMalloc or hipFree, no graph instantiation (the
 * launch sequence is enqueued directly on `stream`), no compilation (dispatch
 * mode 3 uses a consumer only if fhs_evaluate or fhs_precompile already
 * compiled it for this program, split, batch layout and launch shape;
 * otherwise the interpreting kernels run); kernel timing is not recorded.
 * The caller still owns and passes inputs and outputs (device pointers, as
 * for fhs_evaluate).  Every call on one GPU shares that GPU's array and
 * leaves its contents behind (the kernels clear what must start at zero):
 * calls that overlap on one GPU, from any context or stream, race and give
 * undefined results; serialize them.  Errors as fhs_evaluate, plus
 * FHS_ENOMEM when even one output pair per batch does not fit the array,
 * and FHS_EHIP when the array's address could not be obtained on this
 * device. */
#define FHS_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
fhs_status fhs_evaluate_noalloc(fhs_ctx *ctx,
                                const uint64_t *d_inputs, const double *d_coeffs, uint32_t S,
                                const uint64_t *d_outputs, uint32_t M, double threshold,
                                double *d_amps, uint64_t *d_stats, void *stream);

/* ---------------------------------------------------------------------
 * Learned split (cost model).  The paper picks the checkpoint partition by
 * minimising Eq. (8) (Section IV-C); here a small network, trained on the
 * autotuner's measured times, predicts the log run time of each candidate
 * split from split features, and the argmin is used.  Exhaustive timing
 * remains the fallback and the measure of its regret.
 * ------------------------------------------------------------------- */

/* Features of the split (c1, c2) for M outputs and S inputs, FHS_N_FEATURES
 * doubles: A_p, A_r, A_s; log2(1 + work) of the prefix, root and suffix
 * evaluations per pair (int32 ops and FP64 flops each, counts as in Eq. (8):
 * 2^A_p prefixes, 2^(A_p+A_r) roots, 2^A suffixes, work per fhs_program_work,
 * effective cuts); log2 of the prefix-table bytes per pair; log2(M S);
 * 32-bit state words; log2(1 + Eq. (8)); log2 of the root tasks
 * (M S 2^(A_p+A_r)); log2(1 + device instructions) and log2(1 + opcode
 * runs) walked per pair over the three regions (folded gates excluded). */
#define FHS_N_FEATURES 16
fhs_status fhs_split_features(const fhs_program *prog, uint32_t c1, uint32_t c2, uint32_t M,
                              uint32_t S, double *out);

/* The candidate splits the cost model and the exhaustive autotuner search:
 * both cuts taken from {evaluation positions of the source gates} U {G}
 * (moving a cut inside a source-free stretch only moves gates between
 * regions with the same source counts), c1 <= c2: (A+1)(A+2)/2 pairs.
 * Writes min(count, cap) pairs. */
fhs_status fhs_candidate_splits(const fhs_program *prog, uint32_t *c1, uint32_t *c2, uint32_t cap,
                                uint32_t *count);

/* Load a trained cost model into ctx: blob = [n_in, h1, h2, mu[n_in],
 * sd[n_in], lo[n_in], hi[n_in], params...] (doubles; n_in =
 * FHS_N_FEATURES; features are standardised as (f - mu) / sd; [lo, hi] is
 * the per-feature range of the training rows).  params holds K >= 1
 * networks of that shape back to back (K <= 64, from the blob's length);
 * their outputs are averaged into the predicted log(seconds).
 * FHS_EINVAL on a wrong shape or size, sd <= 0 or lo > hi; the blob is
 * copied (the caller keeps ownership). */
fhs_status fhs_load_cost_model(fhs_ctx *ctx, const double *blob, size_t n);

/* fhs_choose_partition with access to the device: FHS_PART_MODEL scores
 * the candidate splits for M outputs and S inputs whose features all lie in
 * the model's training range (each [lo, hi] widened by 5% of its width)
 * with the loaded model (one fhs_mlp_forward on the device) and returns the
 * argmin (smallest (c1, c2) on ties).  FHS_ERANGE, cuts untouched, when
 * no candidate of minimal Eq. (8) cost lies in that range: the model is not
 * trusted there and the caller falls back to timing the candidates.  Other
 * modes behave as fhs_choose_partition.  FHS_ESTATE without a loaded
 * program or model. */
fhs_status fhs_choose_partition_ctx(fhs_ctx *ctx, int mode, uint32_t M, uint32_t S, uint32_t *c1,
                                    uint32_t *c2);

/* The loaded model's predicted log(seconds) of the n splits (c1[i], c2[i])
 * for M outputs and S inputs (host arrays), NaN for a split whose features
 * fall outside the training range.  Lets a tuner shortlist splits by
 * prediction and time only the shortlist.  FHS_EINVAL on a split with
 * c1 > c2 or c2 > G, or M or S = 0; FHS_ESTATE without a program or model. */
fhs_status fhs_predict_splits(fhs_ctx *ctx, uint32_t M, uint32_t S, const uint32_t *c1,
                              const uint32_t *c2, uint32_t n, double *log_seconds);

/* Network x -> tanh(W1 x + b1) -> tanh(W2 a1 + b2) -> w3.a2 + b3 in FP64,
 * n_in, h1, h2 in [1, 64].  Flat parameters, in order: W1 [h1][n_in]
 * row-major, b1 [h1], W2 [h2][h1], b2 [h2], w3 [h2], b3. */
typedef struct {
    uint32_t n_in, h1, h2;
} fhs_mlp_shape;

fhs_status fhs_mlp_param_count(const fhs_mlp_shape *shape, size_t *n);

/* Device workspace fhs_mlp_backward needs for a batch of B rows. */
fhs_status fhs_mlp_workspace_size(const fhs_mlp_shape *shape, uint32_t B, size_t *bytes);

/* y[b] = network(x[b]) for b < B; x is B x n_in row-major.  act (may be
 * NULL) receives the hidden activations, B x (h1 + h2).  Device pointers,
 * asynchronous on `stream`. */
fhs_status fhs_mlp_forward(const fhs_mlp_shape *shape, const double *d_params, const double *d_x,
                           uint32_t B, double *d_y, double *d_act, void *stream);

/* Gradient of the mean squared error (1/B) sum_b (network(x[b]) - t[b])^2
 * with respect to every parameter (d_grad, same layout as the parameters),
 * and the loss itself (d_loss, may be NULL).  Per-tile partial sums are
 * reduced in a fixed order: deterministic. */
fhs_status fhs_mlp_backward(const fhs_mlp_shape *shape, const double *d_params, const double *d_x,
                            const double *d_t, uint32_t B, double *d_grad, double *d_loss,
                            void *d_ws, size_t ws_bytes, void *stream);

/* One Adam step (Kingma & Ba 2015), iteration `step` >= 1, with bias
 * correction: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
fhs_status fhs_mlp_adam(size_t n, double *d_params, const double *d_grad, double *d_m, double *d_v,
                        uint32_t step, double lr, double beta1, double beta2, double eps,
                        void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FHS_H */
