// kernels.hpp -- launch parameters shared by the runtime and the kernels.
#pragma once

#if !defined(__HIPCC_RTC__)
#include <hip/hip_runtime.h>
#endif

#include <cstdint>

#include "program.hpp"

namespace fhs {

// Per-pair precheck results (structure of arrays, P pairs).
struct PreBufs {
    uint32_t *st;      // [NW][P] state after the leading source-free gates
    double2 *amp;      // [P]     partial amplitude (beta_0)
    double *M;         // [P]     running modulus product
    uint32_t *ok;      // [P]     1 = consistent so far
    uint64_t *aff;     // [P]     bit j: the boundary part of affine input j's form
    // The pairs the precheck accepted, per batch of acc_B pairs (listed by
    // the prefix build's first threads):
    // acc_n[b] of them, listed at acc_list[b acc_B ...] by their index in the
    // batch (in no particular order); acc_pos[p] is pair p's place in that
    // list (0xffffffff: rejected).  The consumer's work items cover only them.
    uint32_t *acc_n;
    uint32_t *acc_list;
    uint32_t *acc_pos;
    uint32_t acc_B;
};

// One output pair's finished result.
struct PairRes {
    double2 *amp;      // [P]
    uint64_t *st;      // [P][4] n_valid, sum_h, xor_h, leaves
};

// Checkpoint table for one batch of pairs (structure of arrays).
struct Table {
    uint32_t *st;      // [NW][E]
    double2 *beta;     // [E]
    double *M;         // [E]
    uint32_t *ok;      // [E]
};

// Per-item partial sums.
struct Partials {
    double2 *amp;      // [items]
    uint64_t *st;      // [items][4]
    // timing mode only (else null): per item, the device's constant-rate
    // clock when a workgroup popped it and when its sums were stored
    unsigned long long *stamps;   // [items][2]
};

struct Common {
    const Instr *prog;       // device program, evaluation order
    const double *fac;       // factor table
    const Mask4 *fin;        // [G+1] bits final once e gates are applied
    const uint32_t *src;     // [A] device-program index of source k's gate (ascending)
    const uint64_t *inputs;  // [S][W]
    const uint64_t *outputs; // [M][W]
    uint32_t S, M, W, n;
    uint32_t G, L, A;
    uint32_t c1, c2;         // effective cuts, L <= c1 <= c2 <= G (evaluation positions)
    // The device program drops the gates folded into an OP_ADD, so region
    // bounds are device-program indices: iL, i1, i2, iG of positions L, c1, c2, G.
    uint32_t iL, i1, i2, iG;
    // 1: dispatch once per run of identical opcodes; 0: once per instruction
    // (better when runs are short, e.g. programs dominated by folded ladders)
    uint32_t runs;
    uint32_t Ap, Ar, As;
    uint32_t f_L, f_c1, f_c2, f_G;   // factor-table offsets of evaluation positions L, c1, c2, G
    double thr;
    // 1: the program was placed by the forward sweep and walks the circuit
    // from the input: a history starts from the input bitstring and ends at
    // the check against the output (the roles of the two swap)
    uint32_t fwd;
    // affine branching inputs (sources placed by reachability): per form j,
    // 9 words: input-bit mask [4], output-bit mask [4], constant; and the
    // per-pair boundary bits the precheck derives from them
    const uint32_t *aff_tab;
    uint32_t n_aff;
    const uint64_t *pair_aff;   // [P] (null when n_aff is 0)
    // work items a consumer workgroup claims from the queue at once (>= 1):
    // short items claimed one by one keep the queue's single counter busy
    uint32_t grab;
    // log2 of the lanes that share one root task (the plan's; a compiled
    // consumer is built either for 0 or for any other value)
    uint32_t ss;
    // The pair-level residue test (pair_filter; pf_on 0: none): the
    // precheck rejects a pair whose field residue no history's steps reach,
    // and the consumer skips a rejected pair's items.
    uint32_t pf_on, pf_lo, pf_hi, pf_up, pf_off, pf_span;
    // the accepted pairs of each batch (PreBufs.acc_*)
    const uint32_t *acc_n;
    const uint32_t *acc_list;
    uint32_t acc_B;
    // Work items per chunk of prefix entries: the chunk's root tasks in this
    // many equal parts, so that one pair's work spreads over several
    // workgroups (with the pair-level test, rejected pairs' items are free).
    uint32_t rparts;
};

#if !defined(__HIPCC_RTC__)
// Launchers (kernels.hip).  NW and pruning are dispatched inside.
// k_pair_reduce + k_finalize in one launch (every pair in one batch, S <= 8)
hipError_t launch_reduce_finalize(PreBufs pre, Partials part, uint32_t ipp, uint32_t A, const double *coeffs,
                                  uint32_t S, uint32_t M, double *amps, uint64_t *stats, hipStream_t s);
hipError_t launch_precheck(const Common &c, int NW, PreBufs pre, uint32_t P, uint32_t *zero_words,
                           uint32_t n_zero, hipStream_t s);
// Dp: the last Dp prefix sources are enumerated depth-first inside a lane
// (Dp <= min(Ap, kDfsMax)); B << (Ap - Dp) lanes.
hipError_t launch_prefix(const Common &c, int NW, PreBufs pre, Table tab, uint32_t p0, uint32_t B,
                         uint32_t Dp, hipStream_t s);
// ss: log2 of the number of lanes that share one (entry, h_r) root task, each
// walking a contiguous 2^(As-ss) slice of the suffix assignments.
// H: histories per lane (1 or 2).
hipError_t launch_consume(const Common &c, int NW, int H, Table tab, Partials part, uint32_t p0,
                          uint32_t B, uint32_t chunk, uint32_t ss, uint32_t *counter,
                          uint32_t grid, hipStream_t s);
hipError_t launch_plain(const Common &c, int NW, int H, PreBufs pre, Partials part, uint32_t P,
                        uint32_t blocks_per_pair, hipStream_t s);
hipError_t launch_pair_reduce(PreBufs pre, Partials part, PairRes res, uint32_t p0, uint32_t B,
                              uint32_t items_per_pair, uint32_t A, hipStream_t s);
// Adds the number of nonzero ok[0..n) flags to *out.
hipError_t launch_count_valid(const uint32_t *ok, uint64_t n, unsigned long long *out,
                              hipStream_t s);
hipError_t launch_finalize(PairRes res, const double *coeffs, uint32_t S, uint32_t M,
                           double *amps, uint64_t *stats, hipStream_t s);

#endif  // !__HIPCC_RTC__

// Workgroup size of the persistent consumer and the plain kernel.
constexpr int kConsumeThreads = 256;
constexpr int kPlainThreads = 256;
constexpr int kMaxChunk = 256;   // prefix entries per work item
constexpr int kDfsMax = 4;       // prefix sources enumerated depth-first inside one lane
// Factor slices up to this many doubles are staged in LDS by the hot kernels.
constexpr uint32_t kMaxLdsFactors = 4096;

#if !defined(__HIPCC_RTC__)
// Occupancy-derived persistent grid for the consumer.
int consume_blocks_per_cu(const Common &c, int NW, int H);
#endif

}  // namespace fhs
