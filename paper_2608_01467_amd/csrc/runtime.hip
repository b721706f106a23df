// runtime.hip -- device context, workspace plan, launch sequences and the
// HIP-graph cache behind the C ABI (include/fhs.h).
//
// The paper's execution model (Section IV-D) decomposes the work over output
// bitstrings and balances it dynamically with a server that hands batches of
// outputs to idle workers.  On one GPU the server becomes a device atomic
// counter: the persistent consumer pops (pair, prefix-chunk) work items until
// the counter passes the item count.  The launch sequence of one evaluation
// is captured once into a HIP graph and replayed while its arguments repeat.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <spawn.h>
#include <sys/wait.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <iterator>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fhs.h"
#include "jit.hpp"
#include "kernels.hpp"
#include "program.hpp"

const fhs::HostProgram &fhs_program_host(const fhs_program *p);
fhs_program *fhs_program_clone(const fhs_program *p);

namespace fhs {
hipError_t mlp_forward(const fhs_mlp_shape *s, const double *p, const double *x, uint32_t B,
                       double *y, double *act, hipStream_t st);
}

namespace fhs {
namespace {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct GraphKey {
    const void *inputs, *coeffs, *outputs, *amps, *stats, *ws;
    uint32_t S, M, c1, c2, timing;
    uint64_t thr_bits, ws_bytes, generation;
    bool operator==(const GraphKey &o) const { return std::memcmp(this, &o, sizeof(*this)) == 0; }
};

// Byte layout of one evaluation's workspace.
struct Plan {
    uint32_t P = 0;          // pairs = M * S
    uint32_t c1 = 0, c2 = 0; // effective cuts (>= L)
    uint32_t Ap = 0, Ar = 0, As = 0;
    uint32_t B = 0;          // pairs per batch
    uint32_t n_batches = 0;
    uint32_t chunk = 1;      // prefix entries per work item
    uint32_t nchunks = 1;    // chunks of prefix entries per pair
    uint32_t rparts = 1;     // work items per chunk (parts of its root tasks)
    uint32_t ipp = 1;        // work items per pair: nchunks * rparts
    uint32_t ss = 0;         // log2 lanes per root task
    uint32_t grab = 1;       // work items per claim from the consumer's queue
    uint32_t Dp = 0;         // prefix sources enumerated depth-first inside a lane
    uint32_t bpp = 1;        // plain: blocks per pair
    uint64_t entries = 0;    // table entries per batch
    size_t off_pre_st = 0, off_pre_amp = 0, off_pre_M = 0, off_pre_ok = 0, off_pre_aff = 0;
    size_t off_res_amp = 0, off_res_st = 0;
    size_t off_counters = 0;      // per batch: the queue's counter, then the accepted pairs' count
    size_t off_acc_list = 0, off_acc_pos = 0;
    size_t off_tab_st = 0, off_tab_beta = 0, off_tab_M = 0, off_tab_ok = 0;
    size_t off_part_amp = 0, off_part_st = 0;   // batched mode
    size_t off_plain_amp = 0, off_plain_st = 0; // plain mode
    size_t bytes = 0;
};

}  // namespace
}  // namespace fhs

using namespace fhs;

struct fhs_ctx {
    int device = 0;
    int num_cu = 0;
    std::string err;
    bool loaded = false;
    HostProgram prog;
    Instr *d_prog = nullptr;
    double *d_fac = nullptr;
    Mask4 *d_fin = nullptr;
    uint32_t *d_src = nullptr;   // [max(A,1)] device-program index of each source gate
    uint32_t *d_aff = nullptr;   // [9 per affine input] the forms of affine branching inputs
    std::vector<uint32_t> pos2ins;   // [G+1] evaluation position -> device-program index
    std::vector<Instr> dev_ins;      // host copy of the device program
    std::vector<uint32_t> src_dev;   // device-program index of each source's gate
    std::map<std::string, CompiledConsumer> compiled;   // consumers compiled for this program
    uint32_t c1 = 0, c2 = 0;
    uint32_t grab_override = 0;   // items per claim set by the launch config (0: the plan's)
    size_t table_budget = size_t(1) << 30;
    uint64_t generation = 0;
    hipStream_t cap_stream = nullptr;
    bool have_graph = false;
    GraphKey key{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int ilp = 2;             // histories per lane in the hot kernels
    uint32_t chunk_max = kMaxChunk;
    uint32_t blocks_per_cu = 0;   // 0: occupancy limit
    uint32_t dispatch = 0;        // 0 auto, 1 per run, 2 per instruction
    bool long_runs = true;        // the device program's runs average >= 2 instructions
    const fhs_program *host_prog = nullptr;   // for features (not owned)
    fhs_program *prog_copy = nullptr;         // owned copy used by the cost model
    bool have_model = false;
    fhs_mlp_shape model_shape{0, 0, 0};
    std::vector<double> model_mu, model_sd, model_lo, model_hi;
    double *d_model = nullptr;      // model_k networks, model_np parameters each
    uint32_t model_k = 0;
    size_t model_np = 0;
    bool timing = false;            // record events around hot-kernel launches
    std::vector<hipEvent_t> events; // [2 * launches]: start, end
    uint32_t n_timed = 0;
    unsigned long long *d_valid = nullptr;  // timing mode: consistent prefix entries
    uint64_t n_entries = 0;                 // timing mode: prefix entries built
    void *scratch = nullptr;                // this device's copy of the no-alloc scratch
    bool pf_on = false;                     // the program's pair-level residue test (pair_filter)
    PairFilter pf;
    unsigned long long *d_stamps = nullptr; // timing mode: per work item start/end clock
    size_t stamps_cap = 0;                  // items d_stamps holds
    uint64_t n_stamped = 0;                 // items of the last timed evaluation
    uint32_t stamp_ipp = 0;                 // items per pair of the last timed evaluation
};

// Workspace of fhs_evaluate_noalloc, for callers that cannot allocate: a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host it is only
// a stand-in for the symbol); it uses the address hipGetSymbolAddress gives
// for the current device, looked up once per device when the first context
// on it is created.
static __device__ __align__(256) unsigned char scratch[FHS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];   // per device; nullptr until looked up

// The device address of `scratch` on `device`, which must be current.
hipError_t scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

}  // namespace

namespace {

fhs_status fail(fhs_ctx *c, fhs_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
    return st;
}

fhs_status hip_fail(fhs_ctx *c, hipError_t e, const char *what) {
    return fail(c, FHS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define FHS_HIP(ctx, expr)                                  \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

void free_program(fhs_ctx *c) {
    if (c->d_prog) hipFree(c->d_prog);
    if (c->d_fac) hipFree(c->d_fac);
    if (c->d_fin) hipFree(c->d_fin);
    if (c->d_src) hipFree(c->d_src);
    if (c->d_aff) hipFree(c->d_aff);
    for (auto &kv : c->compiled) release(kv.second);
    c->compiled.clear();
    c->d_prog = nullptr;
    c->d_fac = nullptr;
    c->d_fin = nullptr;
    c->d_src = nullptr;
    c->d_aff = nullptr;
    c->loaded = false;
}

// Make sure 2*n timing events exist (created outside any capture).
hipError_t ensure_events(fhs_ctx *c, uint32_t n) {
    while (c->events.size() < 2 * static_cast<size_t>(n)) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        c->events.push_back(e);
    }
    return hipSuccess;
}

void drop_graph(fhs_ctx *c) {
    if (c->exec) hipGraphExecDestroy(c->exec);
    if (c->graph) hipGraphDestroy(c->graph);
    c->exec = nullptr;
    c->graph = nullptr;
    c->have_graph = false;
}

int nw_of(const HostProgram &P) { return P.NW; }

// Work layout for M outputs x S inputs under the context's program and cuts,
// with pairs batched so that one batch's prefix table fits `budget` bytes.
fhs_status make_plan(const fhs_ctx *c, uint32_t M, uint32_t S, Plan &pl, size_t budget) {
    const HostProgram &P = c->prog;
    const uint64_t pairs = static_cast<uint64_t>(M) * S;
    if (pairs > 0xffffffffull / 4) return FHS_ERANGE;
    pl = Plan{};
    pl.P = static_cast<uint32_t>(pairs);
    const uint32_t L = static_cast<uint32_t>(P.L);
    pl.c1 = std::max(c->c1, L);
    pl.c2 = std::max(c->c2, L);
    for (uint32_t e : P.src_eval) {
        if (e < pl.c1) ++pl.Ap;
        else if (e < pl.c2) ++pl.Ar;
        else ++pl.As;
    }
    const int NW = nw_of(P);
    const uint32_t n_pairs = std::max<uint32_t>(pl.P, 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    pl.off_pre_st = take(sizeof(uint32_t) * NW * n_pairs);
    pl.off_pre_amp = take(sizeof(double2) * n_pairs);
    pl.off_pre_M = take(sizeof(double) * n_pairs);
    pl.off_pre_ok = take(sizeof(uint32_t) * n_pairs);
    pl.off_pre_aff = take(P.aff.empty() ? 0 : sizeof(uint64_t) * n_pairs);
    pl.off_acc_list = take(sizeof(uint32_t) * n_pairs);
    pl.off_acc_pos = take(sizeof(uint32_t) * n_pairs);
    pl.off_res_amp = take(sizeof(double2) * n_pairs);
    pl.off_res_st = take(sizeof(uint64_t) * 4 * n_pairs);
    const size_t common_end = off;

    // batched mode
    if (P.A > 0) {
        if (pl.Ap > 30 || pl.Ar > 30) return FHS_ERANGE;
        const uint64_t per_pair = 1ull << pl.Ap;
        const size_t entry_bytes = sizeof(uint32_t) * NW + sizeof(double2) + sizeof(double) + sizeof(uint32_t);
        if (per_pair * entry_bytes > budget) return FHS_ERANGE;   // one pair's table must fit
        uint64_t B = budget / (per_pair * entry_bytes);
        B = std::max<uint64_t>(1, std::min<uint64_t>(B, n_pairs));
        pl.B = static_cast<uint32_t>(B);
        pl.n_batches = (n_pairs + pl.B - 1) / pl.B;
        // prefix entries per work item: the configured chunk, halved (down to
        // 8) while a batch would hold fewer than 128 items per compute unit,
        // so that when pairs are few and their tables small the costly pairs
        // (those with many valid histories) still spread over several
        // workgroups instead of setting the kernel's length alone
        uint64_t ch = std::min<uint64_t>(per_pair, c->chunk_max);
        const uint64_t want_items = static_cast<uint64_t>(std::max(c->num_cu, 1)) * 128;
        while (ch > 8 && B * ((per_pair + ch - 1) / ch) < want_items) ch >>= 1;
        pl.chunk = static_cast<uint32_t>(ch);
        pl.nchunks = static_cast<uint32_t>((per_pair + pl.chunk - 1) / pl.chunk);
        pl.entries = B * per_pair;
        // lanes sharing one root task: enough root tasks to fill the device
        const uint64_t root_tasks = static_cast<uint64_t>(n_pairs) * per_pair << pl.Ar;
        const uint64_t want = static_cast<uint64_t>(std::max(c->num_cu, 1)) * 2048;
        while (pl.ss < pl.As && (root_tasks << pl.ss) < want) ++pl.ss;
        // prefix sources enumerated depth-first per lane, keeping enough lanes
        pl.Dp = std::min<uint32_t>(pl.Ap, static_cast<uint32_t>(kDfsMax));
        while (pl.Dp > 0 && (static_cast<uint64_t>(pl.B) << (pl.Ap - pl.Dp)) < want) --pl.Dp;
        while (!dfs_allowed(P, pl.c1, pl.Ap, pl.Dp)) --pl.Dp;
        // With the pair-level residue test the pairs it rejects cost nothing
        // in the consumer, so a chunk's root tasks are split into parts of
        // at least one pass of the workgroup: the work of the pairs that
        // remain (often few) spreads over many workgroups.
        pl.rparts = 1;
        if (c->pf_on) {
            const uint64_t pass = static_cast<uint64_t>(std::max(c->ilp, 1)) * kConsumeThreads;
            const uint64_t tasks = static_cast<uint64_t>(pl.chunk) << (pl.Ar + pl.ss);
            pl.rparts = static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(64, tasks / pass)));
        }
        pl.ipp = pl.nchunks * pl.rparts;
        pl.off_counters = take(sizeof(uint32_t) * 2 * pl.n_batches);
        pl.off_tab_st = take(sizeof(uint32_t) * NW * pl.entries);
        pl.off_tab_beta = take(sizeof(double2) * pl.entries);
        pl.off_tab_M = take(sizeof(double) * pl.entries);
        pl.off_tab_ok = take(sizeof(uint32_t) * pl.entries);
        const uint64_t items = static_cast<uint64_t>(pl.B) * pl.ipp;
        if (items > 0xffffffffull) return FHS_ERANGE;
        // short items are claimed several at a time (one atomic on the
        // queue's counter per claim): about 2^16 candidate histories per
        // claim, at most 16 items, and still >= 64 claims per compute unit;
        // the counter may run past the item count by one claim per workgroup
        const uint64_t leaves_item = std::max<uint64_t>(static_cast<uint64_t>(pl.chunk) << (pl.Ar + pl.As), 1);
        uint64_t g = (uint64_t(1) << 16) / leaves_item;
        g = std::min<uint64_t>(g, items / (static_cast<uint64_t>(std::max(c->num_cu, 1)) * 64));
        g = std::min<uint64_t>(g, 16);
        if (items + (g << 20) > 0xffffffffull) g = 1;
        pl.grab = static_cast<uint32_t>(std::max<uint64_t>(g, 1));
        pl.off_part_amp = take(sizeof(double2) * items);
        pl.off_part_st = take(sizeof(uint64_t) * 4 * items);
    }
    const size_t batched_end = off;

    // plain mode reuses the space after the common part
    off = common_end;
    if (P.A > 0) {
        const uint64_t NH = 1ull << std::min<uint32_t>(static_cast<uint32_t>(P.A), 62u);
        const uint64_t max_bpp = std::max<uint64_t>(1, (NH + kPlainThreads - 1) / kPlainThreads);
        const uint64_t target = static_cast<uint64_t>(std::max(c->num_cu, 1)) * 32;
        uint64_t bpp = (target + n_pairs - 1) / n_pairs;
        bpp = std::max<uint64_t>(1, std::min<uint64_t>(bpp, std::min<uint64_t>(max_bpp, 1u << 16)));
        pl.bpp = static_cast<uint32_t>(bpp);
        const uint64_t blocks = static_cast<uint64_t>(n_pairs) * pl.bpp;
        if (blocks > 0x7fffffffull) return FHS_ERANGE;
        pl.off_plain_amp = take(sizeof(double2) * blocks);
        pl.off_plain_st = take(sizeof(uint64_t) * 4 * blocks);
    }
    pl.bytes = std::max(batched_end, off);
    return FHS_OK;
}

fhs_status make_plan(const fhs_ctx *c, uint32_t M, uint32_t S, Plan &pl) {
    return make_plan(c, M, S, pl, c->table_budget);
}

// The plan with the largest table budget (at most the context's) whose whole
// workspace fits `limit` bytes: the budget shrinks by the excess until it
// fits.  FHS_ENOMEM when not even one pair per batch fits.
fhs_status plan_within(const fhs_ctx *c, uint32_t M, uint32_t S, size_t limit, Plan &pl) {
    size_t budget = std::min(c->table_budget, limit);
    for (int it = 0; it < 64; ++it) {
        const fhs_status st = make_plan(c, M, S, pl, budget);
        if (st == FHS_ERANGE && budget < c->table_budget) return FHS_ENOMEM;   // one pair's table no longer fits
        if (st != FHS_OK) return st;
        if (pl.bytes <= limit) return FHS_OK;
        const size_t excess = pl.bytes - limit;
        const size_t next = budget > excess ? std::min(budget - excess, budget - budget / 16) : 0;
        if (next < (size_t(1) << 10)) return FHS_ENOMEM;
        budget = next;
    }
    return FHS_ENOMEM;
}

fhs_status check_eval_args(fhs_ctx *c, const uint64_t *in, const double *cf, uint32_t S,
                           const uint64_t *out, uint32_t M, double thr, double *amps,
                           uint64_t *stats, void *ws, size_t ws_bytes, Plan &pl,
                           bool fit_workspace = false) {
    if (!c) return FHS_EINVAL;
    c->err.clear();
    if (!c->loaded) return fail(c, FHS_ESTATE, "no program loaded");
    if (!(thr >= 0.0) || !std::isfinite(thr)) return fail(c, FHS_EINVAL, "threshold must be finite and >= 0");
    if (c->prog.A > kMaxSources) return fail(c, FHS_ERANGE, "A = %d exceeds %d", c->prog.A, kMaxSources);
    if (M == 0) return FHS_OK;
    if (S == 0) return fail(c, FHS_EINVAL, "S must be >= 1");
    if (!in || !cf || !out || !amps || !stats) return fail(c, FHS_EINVAL, "NULL buffer");
    fhs_status st = fit_workspace ? plan_within(c, M, S, ws_bytes, pl) : make_plan(c, M, S, pl);
    if (st == FHS_ENOMEM)
        return fail(c, st, "the evaluation needs more than the %zu-byte workspace even one pair per batch",
                    ws_bytes);
    if (st != FHS_OK)
        return fail(c, st, "work layout out of range (prefix table of 2^Ap entries exceeds the table budget, or too many pairs)");
    if (!ws || ws_bytes < pl.bytes)
        return fail(c, FHS_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, pl.bytes);
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(c, FHS_EINVAL, "workspace not 256-byte aligned");
    return FHS_OK;
}

template <class T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

Common make_common(const fhs_ctx *c, const Plan &pl, const uint64_t *in, uint32_t S,
                   const uint64_t *out, uint32_t M, double thr, void *ws = nullptr) {
    const HostProgram &P = c->prog;
    Common cm{};
    cm.prog = c->d_prog;
    cm.fac = c->d_fac;
    cm.fin = c->d_fin;
    cm.src = c->d_src;
    cm.inputs = in;
    cm.outputs = out;
    cm.S = S;
    cm.M = M;
    cm.W = static_cast<uint32_t>(P.W);
    cm.n = static_cast<uint32_t>(P.n);
    cm.G = static_cast<uint32_t>(P.G);
    cm.L = static_cast<uint32_t>(P.L);
    cm.A = static_cast<uint32_t>(P.A);
    cm.c1 = pl.c1;
    cm.c2 = pl.c2;
    cm.iL = c->pos2ins[P.L];
    cm.i1 = c->pos2ins[pl.c1];
    cm.i2 = c->pos2ins[pl.c2];
    cm.iG = c->pos2ins[P.G];
    cm.runs = c->dispatch == 1 ? 1u : (c->dispatch == 2 ? 0u : (c->long_runs ? 1u : 0u));
    // mode 3 compiles the consumer; the interpreted kernels (prefix, plain,
    // regions too long to compile) use the automatic rule
    cm.Ap = pl.Ap;
    cm.Ar = pl.Ar;
    cm.As = pl.As;
    cm.f_L = P.fac_begin[P.L];
    cm.f_c1 = P.fac_begin[pl.c1];
    cm.f_c2 = P.fac_begin[pl.c2];
    cm.f_G = P.fac_begin[P.G];
    cm.thr = thr;
    cm.fwd = P.forward ? 1u : 0u;
    cm.aff_tab = c->d_aff;
    cm.n_aff = static_cast<uint32_t>(P.aff.size() / 9);
    cm.pair_aff = (ws && cm.n_aff) ? at<uint64_t>(ws, pl.off_pre_aff) : nullptr;
    cm.acc_n = (ws && P.A > 0) ? at<uint32_t>(ws, pl.off_counters) + pl.n_batches : nullptr;
    cm.acc_list = ws ? at<uint32_t>(ws, pl.off_acc_list) : nullptr;
    cm.acc_B = std::max<uint32_t>(pl.B, 1);
    cm.grab = c->grab_override ? c->grab_override : pl.grab;
    cm.ss = pl.ss;
    cm.rparts = pl.rparts;
    cm.pf_on = c->pf_on ? 1u : 0u;
    cm.pf_lo = c->pf.lo;
    cm.pf_hi = c->pf.hi;
    cm.pf_up = c->pf.up;
    cm.pf_off = c->pf.off;
    cm.pf_span = c->pf.span;
    return cm;
}

PreBufs pre_bufs(void *ws, const Plan &pl) {
    return PreBufs{at<uint32_t>(ws, pl.off_pre_st), at<double2>(ws, pl.off_pre_amp),
                   at<double>(ws, pl.off_pre_M), at<uint32_t>(ws, pl.off_pre_ok),
                   at<uint64_t>(ws, pl.off_pre_aff),
                   pl.off_counters ? at<uint32_t>(ws, pl.off_counters) + pl.n_batches : nullptr,
                   at<uint32_t>(ws, pl.off_acc_list), at<uint32_t>(ws, pl.off_acc_pos), std::max<uint32_t>(pl.B, 1)};
}

PairRes pair_res(void *ws, const Plan &pl) {
    return PairRes{at<double2>(ws, pl.off_res_amp), at<uint64_t>(ws, pl.off_res_st)};
}

// Dynamic LDS of the consumer: the root+suffix factor slice when it fits.
size_t consume_lds_bytes(const Common &cm) {
    const uint32_t n = cm.f_G - cm.f_c1;
    return n <= kMaxLdsFactors ? static_cast<size_t>(n) * sizeof(double) : 0;
}

// Dynamic LDS of the prefix-table build: the prefix region's factors.
size_t prefix_lds_bytes(const Common &cm) {
    const uint32_t n = cm.f_c1 - cm.f_L;
    return n <= kMaxLdsFactors ? static_cast<size_t>(n) * sizeof(double) : 0;
}

// Regions up to this many device instructions are compiled on request.
constexpr uint32_t kMaxCompiledInstr = 1024;

// The consumer compiled for the loaded program, the plan's regions and the
// launch shape (dispatch mode 3), or nullptr when the mode is off or the
// regions are too long; compiled once per program and cached.  Its module
// also holds the prefix-table build when the prefix region is short enough
// (pfn; otherwise the interpreting k_prefix runs).
// Cache key and source of the compiled consumer for `cm` and Dp; false when
// dispatch mode 3 does not apply (mode off, no sources, regions too long).
bool consumer_job(const fhs_ctx *c, const Common &cm, uint32_t Dp, std::string &key, std::string *src,
                  size_t &shm) {
    if (c->dispatch != 3 || c->prog.A == 0 || cm.iG - cm.i1 > kMaxCompiledInstr) return false;
    const bool flds = cm.f_G - cm.f_c1 <= kMaxLdsFactors;
    const bool prune = cm.thr > 0.0;
    const bool prefix_ok = cm.i1 - cm.iL <= kMaxCompiledInstr;
    const bool pflds = cm.f_c1 - cm.f_L <= kMaxLdsFactors;
    const int NW = nw_of(c->prog);
    char buf[192];
    // the cut positions fix the final-bit masks (two cuts inside one folded
    // ladder share device indices but not masks); Dp fixes the prefix's
    // depth-first levels; whether the leaf loop's counter holds every suffix source
    std::snprintf(buf, sizeof(buf), "%u/%u/%u/%u/%u/%u/%u/%u/%d/%d/%d/%d/%u", cm.i1, cm.i2, cm.iG, cm.c1,
                  cm.c2, cm.Ap, cm.Ar, Dp, NW, c->ilp, prune ? 1 : 0, flds ? 1 : 0, cm.ss == 0 ? 0u : 1u);
    key = buf;
    shm = consume_lds_bytes(cm);
    if (src)
        *src = consumer_source(c->dev_ins, c->prog.fac, cm.i1, cm.i2, cm.iG, cm.Ap, cm.Ar,
                               c->prog.final_before[cm.c2], c->prog.final_before[cm.G], NW, c->ilp, prune,
                               flds, flds ? cm.f_c1 : 0u, prefix_ok, cm.iL, c->src_dev, Dp, pflds,
                               pflds ? cm.f_L : 0u, cm.ss);
    return true;
}

fhs_status compiled_consumer(fhs_ctx *c, const Common &cm, uint32_t Dp, const CompiledConsumer **out) {
    *out = nullptr;
    std::string key, src;
    size_t shm = 0;
    if (!consumer_job(c, cm, Dp, key, nullptr, shm)) return FHS_OK;
    auto it = c->compiled.find(key);
    if (it == c->compiled.end()) {
        consumer_job(c, cm, Dp, key, &src, shm);
        CompiledConsumer k;
        std::string log;
        if (!compile_consumer(src, shm, k, log))
            return fail(c, FHS_EUNSUPPORTED, "run-time compilation of the consumer failed: %.400s",
                        log.c_str());
        it = c->compiled.emplace(key, k).first;
    }
    *out = &it->second;
    return FHS_OK;
}

// The batched launch sequence (Algorithm 2): precheck, then per batch the
// prefix-table build, the persistent consumer and the per-pair reduction,
// then Eq. (2).
hipError_t enqueue_batched(fhs_ctx *c, const Plan &pl, const Common &cm, const double *coeffs,
                           double *amps, uint64_t *stats, void *ws, int bpc, bool timed,
                           hipStream_t s, const CompiledConsumer *ck = nullptr) {
    const HostProgram &P = c->prog;
    const int NW = nw_of(P);
    PreBufs pre = pre_bufs(ws, pl);
    PairRes res = pair_res(ws, pl);
    uint32_t *counters = P.A > 0 ? at<uint32_t>(ws, pl.off_counters) : nullptr;
    // (zeroes the queue counters and the accepted pairs' counts)
    hipError_t e = launch_precheck(cm, NW, pre, pl.P, counters, P.A > 0 ? 2 * pl.n_batches : 0, s);
    if (e != hipSuccess) return e;
    if (P.A == 0) {
        e = launch_pair_reduce(pre, Partials{nullptr, nullptr, nullptr}, res, 0, pl.P, 0, 0, s);
        if (e != hipSuccess) return e;
        return launch_finalize(res, coeffs, cm.S, cm.M, amps, stats, s);
    }
    Table tab{at<uint32_t>(ws, pl.off_tab_st), at<double2>(ws, pl.off_tab_beta),
              at<double>(ws, pl.off_tab_M), at<uint32_t>(ws, pl.off_tab_ok)};
    Partials part{at<double2>(ws, pl.off_part_amp), at<uint64_t>(ws, pl.off_part_st), nullptr};
    for (uint32_t b = 0; b < pl.n_batches; ++b) {
        const uint32_t p0 = b * pl.B;
        const uint32_t B = std::min(pl.B, pl.P - p0);
        // timing mode: this batch's items in the stamp buffer (pair-major)
        part.stamps = timed && c->d_stamps ? c->d_stamps + 2ull * p0 * pl.ipp : nullptr;
        const uint64_t items = static_cast<uint64_t>(B) * pl.ipp;
        uint32_t grid = static_cast<uint32_t>(std::max(c->num_cu, 1)) * static_cast<uint32_t>(bpc);
        if (items < grid) grid = static_cast<uint32_t>(items);
        e = (ck && ck->pfn) ? launch_prefix_compiled(*ck, cm, pre, tab, p0, B, pl.Dp, prefix_lds_bytes(cm), s)
                            : launch_prefix(cm, NW, pre, tab, p0, B, pl.Dp, s);
        if (e != hipSuccess) return e;
        if (timed) {
            // outside the timed interval: how many entries the consumer expands
            e = launch_count_valid(tab.ok, static_cast<uint64_t>(B) << pl.Ap, c->d_valid, s);
            if (e != hipSuccess) return e;
            c->n_entries += static_cast<uint64_t>(B) << pl.Ap;
        }
        if (timed && (e = hipEventRecord(c->events[2 * b], s)) != hipSuccess) return e;
        e = ck ? launch_compiled(*ck, cm, tab, part, p0, B, pl.chunk, pl.ss, counters + b, grid,
                                 consume_lds_bytes(cm), s)
               : launch_consume(cm, NW, c->ilp, tab, part, p0, B, pl.chunk, pl.ss, counters + b, grid, s);
        if (e != hipSuccess) return e;
        if (timed && (e = hipEventRecord(c->events[2 * b + 1], s)) != hipSuccess) return e;
        // one batch: the pair sums and Eq. (2) in one launch
        if (pl.n_batches == 1 && cm.S <= 8u)
            return launch_reduce_finalize(pre, part, pl.ipp, cm.A, coeffs, cm.S, cm.M, amps, stats, s);
        e = launch_pair_reduce(pre, part, res, p0, B, pl.ipp, cm.A, s);
        if (e != hipSuccess) return e;
    }
    return launch_finalize(res, coeffs, cm.S, cm.M, amps, stats, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" fhs_status fhs_ctx_create(int device, fhs_ctx **out) {
    if (!out) return FHS_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return FHS_EHIP;
    fhs_ctx *c = new (std::nothrow) fhs_ctx;
    if (!c) return FHS_ENOMEM;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return FHS_EHIP;
    }
    // the no-alloc scratch of this device (a failure only disables
    // fhs_evaluate_noalloc, which then reports it)
    if (scratch_address(device, &c->scratch) != hipSuccess) c->scratch = nullptr;
    *out = c;
    return FHS_OK;
}

extern "C" void fhs_ctx_destroy(fhs_ctx *c) {
    if (!c) return;
    hipSetDevice(c->device);
    drop_graph(c);
    free_program(c);
    fhs_program_free(c->prog_copy);
    if (c->d_model) hipFree(c->d_model);
    if (c->d_valid) hipFree(c->d_valid);
    if (c->d_stamps) hipFree(c->d_stamps);
    for (hipEvent_t e : c->events) hipEventDestroy(e);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    delete c;
}

extern "C" const char *fhs_last_error(const fhs_ctx *c) { return c ? c->err.c_str() : "no context"; }

extern "C" fhs_status fhs_load_program(fhs_ctx *c, const fhs_program *p) {
    if (!c || !p) return FHS_EINVAL;
    c->err.clear();
    FHS_HIP(c, hipSetDevice(c->device));
    drop_graph(c);
    free_program(c);
    const HostProgram &P = fhs_program_host(p);
    c->prog = P;
    fhs_program_free(c->prog_copy);
    c->prog_copy = fhs_program_clone(p);
    // Device copy of the program without the gates folded into an OP_ADD;
    // pos2ins maps evaluation positions to its indices (a position inside a
    // folded ladder maps to the next kept instruction, so the whole ladder
    // runs in the region where it starts).  Runs are recounted.
    std::vector<Instr> dev;
    dev.reserve(P.ins.size());
    c->pos2ins.assign(static_cast<size_t>(P.G) + 1, 0);
    for (int e = 0; e < P.G; ++e) {
        c->pos2ins[e] = static_cast<uint32_t>(dev.size());
        if (op_base(P.ins[e].hdr & 0xffu) != OP_NOP) dev.push_back(P.ins[e]);
    }
    c->pos2ins[P.G] = static_cast<uint32_t>(dev.size());
    size_t n_runs = 0;
    for (size_t i = dev.size(); i-- > 0;) {
        const bool cont = i + 1 < dev.size() && (dev[i + 1].hdr & 0xffu) == (dev[i].hdr & 0xffu);
        dev[i].run = cont ? dev[i + 1].run + 1 : 1;
        if (!cont) ++n_runs;
    }
    c->long_runs = dev.size() >= 2 * n_runs;
    std::vector<uint32_t> src_dev(P.src_eval.size());
    for (size_t k = 0; k < P.src_eval.size(); ++k) src_dev[k] = c->pos2ins[P.src_eval[k]];
    c->dev_ins = dev;
    c->src_dev = src_dev;
    c->pf = PairFilter{};
    c->pf_on = P.A > 0 && pair_filter(dev, P.fac, c->pos2ins[P.L], c->pos2ins[P.G], P.final_before[P.G],
                                      static_cast<uint32_t>(P.A), c->pf);
    const size_t ni = std::max<size_t>(dev.size(), 1), nf = std::max<size_t>(P.fac.size(), 1);
    FHS_HIP(c, hipMalloc(reinterpret_cast<void **>(&c->d_prog), sizeof(Instr) * ni));
    FHS_HIP(c, hipMalloc(reinterpret_cast<void **>(&c->d_fac), sizeof(double) * nf));
    FHS_HIP(c, hipMalloc(reinterpret_cast<void **>(&c->d_fin), sizeof(Mask4) * P.final_before.size()));
    if (!dev.empty())
        FHS_HIP(c, hipMemcpy(c->d_prog, dev.data(), sizeof(Instr) * dev.size(), hipMemcpyHostToDevice));
    if (!P.fac.empty())
        FHS_HIP(c, hipMemcpy(c->d_fac, P.fac.data(), sizeof(double) * P.fac.size(), hipMemcpyHostToDevice));
    FHS_HIP(c, hipMemcpy(c->d_fin, P.final_before.data(), sizeof(Mask4) * P.final_before.size(),
                         hipMemcpyHostToDevice));
    FHS_HIP(c, hipMalloc(reinterpret_cast<void **>(&c->d_src),
                         sizeof(uint32_t) * std::max<size_t>(P.src_eval.size(), 1)));
    if (!src_dev.empty())
        FHS_HIP(c, hipMemcpy(c->d_src, src_dev.data(), sizeof(uint32_t) * src_dev.size(),
                             hipMemcpyHostToDevice));
    if (P.aff.size() / 9 > 64) return fail(c, FHS_ERANGE, "more than 64 affine branching inputs");
    if (!P.aff.empty()) {
        FHS_HIP(c, hipMalloc(reinterpret_cast<void **>(&c->d_aff), sizeof(uint32_t) * P.aff.size()));
        FHS_HIP(c, hipMemcpy(c->d_aff, P.aff.data(), sizeof(uint32_t) * P.aff.size(), hipMemcpyHostToDevice));
    }
    c->c1 = c->c2 = 0;
    c->loaded = true;
    ++c->generation;
    return FHS_OK;
}

constexpr uint32_t kMaxEnsemble = 64;   // networks in one cost model

extern "C" fhs_status fhs_load_cost_model(fhs_ctx *c, const double *blob, size_t n) {
    if (!c || !blob || n < 3) return FHS_EINVAL;
    c->err.clear();
    fhs_mlp_shape sh{static_cast<uint32_t>(blob[0]), static_cast<uint32_t>(blob[1]),
                     static_cast<uint32_t>(blob[2])};
    size_t np = 0;
    if (sh.n_in != FHS_N_FEATURES || fhs_mlp_param_count(&sh, &np) != FHS_OK)
        return fail(c, FHS_EINVAL, "cost model shape");
    const size_t F = sh.n_in;
    // an ensemble of K networks of one shape, predictions averaged
    if (n <= 3 + 4 * F || (n - 3 - 4 * F) % np != 0) return fail(c, FHS_EINVAL, "cost model size");
    const size_t K = (n - 3 - 4 * F) / np;
    if (K > kMaxEnsemble) return fail(c, FHS_EINVAL, "cost model ensemble of %zu > %u networks", K, kMaxEnsemble);
    for (size_t i = 0; i < F; ++i) {
        if (!(blob[3 + F + i] > 0.0)) return fail(c, FHS_EINVAL, "cost model scale must be > 0");
        if (!(blob[3 + 2 * F + i] <= blob[3 + 3 * F + i]))
            return fail(c, FHS_EINVAL, "cost model range: lo > hi for feature %zu", i);
    }
    FHS_HIP(c, hipSetDevice(c->device));
    c->have_model = false;
    if (c->d_model) hipFree(c->d_model);
    c->d_model = nullptr;
    FHS_HIP(c, hipMalloc(reinterpret_cast<void **>(&c->d_model), sizeof(double) * K * np));
    FHS_HIP(c, hipMemcpy(c->d_model, blob + 3 + 4 * F, sizeof(double) * K * np, hipMemcpyHostToDevice));
    c->model_shape = sh;
    c->model_k = static_cast<uint32_t>(K);
    c->model_np = np;
    c->model_mu.assign(blob + 3, blob + 3 + F);
    c->model_sd.assign(blob + 3 + F, blob + 3 + 2 * F);
    c->model_lo.assign(blob + 3 + 2 * F, blob + 3 + 3 * F);
    c->model_hi.assign(blob + 3 + 3 * F, blob + 3 + 4 * F);
    c->have_model = true;
    return FHS_OK;
}

namespace {

// Predicted log(seconds) of the splits (a[i], b[i]) for M outputs and S
// inputs; NaN where a split's features fall outside the model's training
// box (per-feature [lo, hi] widened by 5% of its width).  One forward pass
// of the network on the device for all in-range splits.
fhs_status predict_splits(fhs_ctx *c, uint32_t M, uint32_t S, const uint32_t *a,
                          const uint32_t *b, uint32_t n, double *out) {
    const uint32_t F = c->model_shape.n_in;
    std::vector<double> X;
    std::vector<uint32_t> idx;
    std::vector<double> f(F);
    for (uint32_t i = 0; i < n; ++i) {
        out[i] = std::numeric_limits<double>::quiet_NaN();
        fhs_status st = fhs_split_features(c->prog_copy, a[i], b[i], M, S, f.data());
        if (st != FHS_OK) return fail(c, st, "features of split (%u, %u)", a[i], b[i]);
        bool in = true;
        for (uint32_t k = 0; k < F && in; ++k) {
            const double pad = 0.05 * (c->model_hi[k] - c->model_lo[k]);
            in = f[k] >= c->model_lo[k] - pad && f[k] <= c->model_hi[k] + pad;
        }
        if (!in) continue;
        idx.push_back(i);
        for (uint32_t k = 0; k < F; ++k) X.push_back((f[k] - c->model_mu[k]) / c->model_sd[k]);
    }
    const uint32_t m = static_cast<uint32_t>(idx.size());
    if (m == 0) return FHS_OK;
    const uint32_t K = c->model_k;
    std::vector<double> Y(static_cast<size_t>(K) * m);
    FHS_HIP(c, hipSetDevice(c->device));
    double *dx = nullptr, *dy = nullptr;
    FHS_HIP(c, hipMalloc(reinterpret_cast<void **>(&dx), sizeof(double) * X.size()));
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&dy), sizeof(double) * Y.size());
    if (e == hipSuccess) e = hipMemcpyAsync(dx, X.data(), sizeof(double) * X.size(), hipMemcpyHostToDevice, c->cap_stream);
    for (uint32_t k = 0; k < K && e == hipSuccess; ++k)
        e = mlp_forward(&c->model_shape, c->d_model + k * c->model_np, dx, m, dy + static_cast<size_t>(k) * m,
                        nullptr, c->cap_stream);
    if (e == hipSuccess) e = hipMemcpyAsync(Y.data(), dy, sizeof(double) * Y.size(), hipMemcpyDeviceToHost, c->cap_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->cap_stream);
    hipFree(dx);
    if (dy) hipFree(dy);
    if (e != hipSuccess) return hip_fail(c, e, "cost model inference");
    // mean over the ensemble, in network order
    for (uint32_t j = 0; j < m; ++j) {
        double y = 0.0;
        for (uint32_t k = 0; k < K; ++k) y += Y[static_cast<size_t>(k) * m + j];
        out[idx[j]] = y / K;
    }
    return FHS_OK;
}

}  // namespace

extern "C" fhs_status fhs_predict_splits(fhs_ctx *c, uint32_t M, uint32_t S, const uint32_t *c1,
                                         const uint32_t *c2, uint32_t n, double *log_seconds) {
    if (!c || (n && (!c1 || !c2 || !log_seconds))) return FHS_EINVAL;
    c->err.clear();
    if (!c->loaded || !c->prog_copy) return fail(c, FHS_ESTATE, "no program loaded");
    if (!c->have_model) return fail(c, FHS_ESTATE, "no cost model loaded");
    if (M == 0 || S == 0) return fail(c, FHS_EINVAL, "M and S must be >= 1");
    for (uint32_t i = 0; i < n; ++i)
        if (c1[i] > c2[i] || c2[i] > static_cast<uint32_t>(c->prog.G))
            return fail(c, FHS_EINVAL, "split %u: need c1 <= c2 <= G (%u, %u)", i, c1[i], c2[i]);
    return predict_splits(c, M, S, c1, c2, n, log_seconds);
}

extern "C" fhs_status fhs_choose_partition_ctx(fhs_ctx *c, int mode, uint32_t M, uint32_t S,
                                               uint32_t *c1, uint32_t *c2) {
    if (!c || !c1 || !c2) return FHS_EINVAL;
    c->err.clear();
    if (!c->loaded || !c->prog_copy) return fail(c, FHS_ESTATE, "no program loaded");
    if (mode != FHS_PART_MODEL) return fhs_choose_partition(c->prog_copy, mode, c1, c2);
    if (!c->have_model) return fail(c, FHS_ESTATE, "no cost model loaded");
    if (M == 0 || S == 0) return fail(c, FHS_EINVAL, "M and S must be >= 1");
    uint32_t n = 0;
    fhs_candidate_splits(c->prog_copy, nullptr, nullptr, 0, &n);
    std::vector<uint32_t> a(n), b(n);
    fhs_candidate_splits(c->prog_copy, a.data(), b.data(), n, &n);
    std::vector<double> Y(n);
    fhs_status st = predict_splits(c, M, S, a.data(), b.data(), n, Y.data());
    if (st != FHS_OK) return st;
    // The model is trusted for this program only if some split of minimal
    // Eq. (8) cost lies in its training range.
    uint32_t e1 = 0, e2 = 0;
    uint64_t emin[2] = {0, 0}, cost[2] = {0, 0};
    st = fhs_choose_partition(c->prog_copy, FHS_PART_EQ8, &e1, &e2);
    if (st == FHS_OK) st = fhs_partition_cost(c->prog_copy, e1, e2, emin, nullptr);
    if (st != FHS_OK) return fail(c, st, "Eq. (8) split");
    bool eq8_in = false;
    int best = -1;
    for (uint32_t i = 0; i < n; ++i) {
        if (std::isnan(Y[i])) continue;
        st = fhs_partition_cost(c->prog_copy, a[i], b[i], cost, nullptr);
        if (st != FHS_OK) return fail(c, st, "Eq. (8) cost");
        if (cost[0] == emin[0] && cost[1] == emin[1]) eq8_in = true;
        if (best < 0 || Y[i] < Y[best] ||
            (Y[i] == Y[best] && (a[i] < a[best] || (a[i] == a[best] && b[i] < b[best]))))
            best = static_cast<int>(i);
    }
    if (!eq8_in || best < 0)
        return fail(c, FHS_ERANGE, "split features outside the cost model's training range");
    *c1 = a[best];
    *c2 = b[best];
    return FHS_OK;
}

extern "C" fhs_status fhs_set_partition(fhs_ctx *c, uint32_t c1, uint32_t c2) {
    if (!c) return FHS_EINVAL;
    c->err.clear();
    if (!c->loaded) return fail(c, FHS_ESTATE, "no program loaded");
    if (c1 > c2 || c2 > static_cast<uint32_t>(c->prog.G))
        return fail(c, FHS_EINVAL, "need c1 <= c2 <= G (%u, %u, %d)", c1, c2, c->prog.G);
    const uint32_t L = static_cast<uint32_t>(c->prog.L);
    if (!cut_allowed(c->prog, std::max(c1, L)) || !cut_allowed(c->prog, std::max(c2, L)))
        return fail(c, FHS_EINVAL, "cut (%u, %u) separates an affine branching input from a source its form uses",
                    c1, c2);
    c->c1 = c1;
    c->c2 = c2;
    return FHS_OK;
}

extern "C" fhs_status fhs_get_partition(const fhs_ctx *c, uint32_t *c1, uint32_t *c2) {
    if (!c || !c1 || !c2) return FHS_EINVAL;
    if (!c->loaded) return FHS_ESTATE;
    *c1 = c->c1;
    *c2 = c->c2;
    return FHS_OK;
}

namespace {

// One consumer to compile ahead of time.
struct CompileJob {
    std::string key, src, log;
    size_t shm = 0;
    std::vector<char> code;
    bool ok = false;
};

// Directory of this library: the fhs_rtc helper is built next to it.
std::string library_dir() {
    Dl_info info;
    if (dladdr(reinterpret_cast<void *>(&library_dir), &info) && info.dli_fname) {
        const std::string p(info.dli_fname);
        const size_t k = p.rfind('/');
        if (k != std::string::npos) return p.substr(0, k);
    }
    return ".";
}

bool read_file(const std::string &path, std::vector<char> &out) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    out.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
    return true;
}

// Compile the jobs with up to `procs` fhs_rtc child processes at a time
// (hipRTC serialises compilations inside one process).  The children are
// started with posix_spawn, every descriptor from 3 up closed, and never
// touch the GPU.  Returns false, having compiled nothing, when the helper
// or a temporary directory is not available.
bool compile_in_processes(std::vector<CompileJob> &jobs, uint32_t procs) {
    const std::string helper = library_dir() + "/fhs_rtc";
    if (access(helper.c_str(), X_OK) != 0) return false;
    const char *t = std::getenv("TMPDIR");
    std::string tmpl = std::string(t && *t ? t : "/tmp") + "/fhs_rtc_XXXXXX";
    std::vector<char> dirbuf(tmpl.begin(), tmpl.end());
    dirbuf.push_back('\0');
    if (!mkdtemp(dirbuf.data())) return false;
    const std::string dir(dirbuf.data());
    auto path = [&](size_t i, const char *ext) { return dir + "/" + std::to_string(i) + ext; };
    for (size_t i = 0; i < jobs.size(); ++i) {
        std::ofstream f(path(i, ".hip"), std::ios::binary);
        f << jobs[i].src;
    }
    posix_spawn_file_actions_t fa;
    posix_spawn_file_actions_init(&fa);
    posix_spawn_file_actions_addclosefrom_np(&fa, 3);
    std::vector<std::pair<pid_t, size_t>> running;
    size_t next = 0;
    while (next < jobs.size() || !running.empty()) {
        while (next < jobs.size() && running.size() < procs) {
            const std::string src = path(next, ".hip"), out = path(next, ".co"), log = path(next, ".log");
            char *argv[] = {const_cast<char *>(helper.c_str()), const_cast<char *>(src.c_str()),
                            const_cast<char *>(out.c_str()), const_cast<char *>(log.c_str()), nullptr};
            pid_t pid = 0;
            if (posix_spawn(&pid, helper.c_str(), &fa, nullptr, argv, environ) == 0)
                running.emplace_back(pid, next);
            else
                jobs[next].ok = compile_code(jobs[next].src, jobs[next].code, jobs[next].log);
            ++next;
        }
        bool reaped = false;
        for (size_t r = 0; r < running.size();) {
            int status = 0;
            const pid_t w = waitpid(running[r].first, &status, WNOHANG);
            if (w == 0) {
                ++r;
                continue;
            }
            CompileJob &j = jobs[running[r].second];
            std::vector<char> lg;
            if (read_file(path(running[r].second, ".log"), lg)) j.log.assign(lg.begin(), lg.end());
            j.ok = w > 0 && WIFEXITED(status) && WEXITSTATUS(status) == 0 &&
                   read_file(path(running[r].second, ".co"), j.code) && !j.code.empty();
            if (!j.ok && j.log.empty()) j.log = "fhs_rtc failed";
            running.erase(running.begin() + static_cast<long>(r));
            reaped = true;
        }
        if (!reaped && !running.empty()) usleep(2000);
    }
    posix_spawn_file_actions_destroy(&fa);
    for (size_t i = 0; i < jobs.size(); ++i)
        for (const char *ext : {".hip", ".co", ".log"}) std::remove(path(i, ext).c_str());
    rmdir(dir.c_str());
    return true;
}

}  // namespace

extern "C" fhs_status fhs_precompile(fhs_ctx *c, const uint32_t *c1, const uint32_t *c2, uint32_t n,
                                     uint32_t M, uint32_t S, double threshold, uint32_t threads,
                                     uint32_t *n_compiled) {
    if (!c || (n && (!c1 || !c2)) || M == 0 || S == 0 || !(threshold >= 0.0) || threads == 0)
        return FHS_EINVAL;
    c->err.clear();
    if (!c->loaded) return fail(c, FHS_ESTATE, "no program loaded");
    for (uint32_t i = 0; i < n; ++i)
        if (c1[i] > c2[i] || c2[i] > static_cast<uint32_t>(c->prog.G))
            return fail(c, FHS_EINVAL, "split %u: need c1 <= c2 <= G", i);
    std::vector<CompileJob> jobs;
    const uint32_t s1 = c->c1, s2 = c->c2;
    for (uint32_t i = 0; i < n; ++i) {
        c->c1 = c1[i];
        c->c2 = c2[i];
        Plan pl;
        if (make_plan(c, M, S, pl) != FHS_OK) continue;   // not evaluable at this size: nothing to compile
        const Common cm = make_common(c, pl, nullptr, S, nullptr, M, threshold);
        CompileJob j;
        if (!consumer_job(c, cm, pl.Dp, j.key, nullptr, j.shm) || c->compiled.count(j.key)) continue;
        bool dup = false;
        for (const CompileJob &o : jobs) dup = dup || o.key == j.key;
        if (dup) continue;
        consumer_job(c, cm, pl.Dp, j.key, &j.src, j.shm);
        jobs.push_back(std::move(j));
    }
    c->c1 = s1;
    c->c2 = s2;
    c->err.clear();
    if (jobs.empty() || threads < 2 || !compile_in_processes(jobs, threads))
        for (CompileJob &j : jobs) j.ok = compile_code(j.src, j.code, j.log);
    FHS_HIP(c, hipSetDevice(c->device));
    uint32_t done = 0;
    for (CompileJob &j : jobs) {
        if (!j.ok)
            return fail(c, FHS_EUNSUPPORTED, "run-time compilation of the consumer failed: %.400s",
                        j.log.c_str());
        CompiledConsumer k;
        if (!load_consumer(j.code, j.src.find("fhs_prefix_compiled") != std::string::npos, j.shm, k, j.log))
            return fail(c, FHS_EUNSUPPORTED, "loading the compiled consumer failed: %.400s", j.log.c_str());
        c->compiled.emplace(j.key, k);
        ++done;
    }
    if (n_compiled) *n_compiled = done;
    return FHS_OK;
}

extern "C" fhs_status fhs_set_table_budget(fhs_ctx *c, size_t bytes) {
    if (!c || bytes < (size_t(1) << 20)) return FHS_EINVAL;
    c->table_budget = bytes;
    return FHS_OK;
}

extern "C" fhs_status fhs_set_launch_config(fhs_ctx *c, const fhs_launch_config *cfg) {
    if (!c || !cfg) return FHS_EINVAL;
    const uint32_t h = cfg->histories_per_lane ? cfg->histories_per_lane : 2;
    const uint32_t ch = cfg->chunk ? cfg->chunk : kMaxChunk;
    if (h > 2 || ch > static_cast<uint32_t>(kMaxChunk) || (ch & (ch - 1)) || cfg->blocks_per_cu > 64 ||
        cfg->dispatch > 3 || cfg->items_per_claim > 64)
        return fail(c, FHS_EINVAL, "launch config out of range");
    c->grab_override = cfg->items_per_claim;
    c->ilp = static_cast<int>(h);
    c->chunk_max = ch;
    c->blocks_per_cu = cfg->blocks_per_cu;
    c->dispatch = cfg->dispatch;
    drop_graph(c);
    return FHS_OK;
}

extern "C" fhs_status fhs_get_launch_config(const fhs_ctx *c, fhs_launch_config *cfg) {
    if (!c || !cfg) return FHS_EINVAL;
    cfg->histories_per_lane = static_cast<uint32_t>(c->ilp);
    cfg->chunk = c->chunk_max;
    cfg->blocks_per_cu = c->blocks_per_cu;
    cfg->dispatch = c->dispatch;
    cfg->items_per_claim = c->grab_override;
    return FHS_OK;
}

extern "C" fhs_status fhs_get_plan(const fhs_ctx *c, uint32_t M, uint32_t S, fhs_plan *out) {
    if (!c || !out) return FHS_EINVAL;
    if (!c->loaded) return FHS_ESTATE;
    if (c->prog.A > kMaxSources) return FHS_ERANGE;
    Plan pl;
    fhs_status st = make_plan(c, M, std::max<uint32_t>(S, 1), pl);
    if (st != FHS_OK) return st;
    out->c1 = pl.c1;
    out->c2 = pl.c2;
    out->Ap = pl.Ap;
    out->Ar = pl.Ar;
    out->As = pl.As;
    out->n_batches = pl.n_batches;
    out->pairs_per_batch = pl.B;
    out->chunk = pl.chunk;
    out->items_per_pair = pl.ipp;
    out->root_parts = pl.rparts;
    out->pair_filter = c->pf_on ? 1u : 0u;
    out->lanes_per_root_task = 1u << pl.ss;
    out->plain_blocks_per_pair = pl.bpp;
    out->prefix_depth_first = pl.Dp;
    out->items_per_claim = c->grab_override ? c->grab_override : pl.grab;
    out->count_groups = out->count_entries = 0;
    if (c->prog.A > 0 && pl.c2 <= static_cast<uint32_t>(c->prog.G)) {
        const uint32_t i1 = c->pos2ins[pl.c1], i2 = c->pos2ins[pl.c2], iG = c->pos2ins[c->prog.G];
        const CountPlan cp = count_plan(c->dev_ins, c->prog.fac, i1, i2, iG, hoistable(c->dev_ins, i2, iG, false));
        if (cp.on()) {
            out->count_groups = static_cast<uint32_t>(cp.group_size.size());
            out->count_entries = cp.entries;
        }
    }
    out->table_bytes = pl.entries * (sizeof(uint32_t) * nw_of(c->prog) + sizeof(double2) +
                                     sizeof(double) + sizeof(uint32_t));
    return FHS_OK;
}

extern "C" fhs_status fhs_set_kernel_timing(fhs_ctx *c, int enable) {
    if (!c) return FHS_EINVAL;
    c->err.clear();
    if (enable && !c->d_valid) {
        FHS_HIP(c, hipSetDevice(c->device));
        FHS_HIP(c, hipMalloc(reinterpret_cast<void **>(&c->d_valid), sizeof(unsigned long long)));
    }
    c->timing = enable != 0;
    c->n_timed = 0;
    c->n_entries = 0;
    c->n_stamped = 0;
    drop_graph(c);
    return FHS_OK;
}

extern "C" fhs_status fhs_kernel_counts(fhs_ctx *c, uint64_t *prefix_entries, uint64_t *prefix_valid) {
    if (!c || !prefix_entries || !prefix_valid) return FHS_EINVAL;
    c->err.clear();
    if (!c->timing || c->n_timed == 0) return fail(c, FHS_ESTATE, "no timed launch");
    unsigned long long v = 0;
    FHS_HIP(c, hipSetDevice(c->device));
    FHS_HIP(c, hipMemcpy(&v, c->d_valid, sizeof(v), hipMemcpyDeviceToHost));
    *prefix_entries = c->n_entries;
    *prefix_valid = v;
    return FHS_OK;
}

extern "C" fhs_status fhs_kernel_times(fhs_ctx *c, float *ms, uint32_t cap, uint32_t *count) {
    if (!c || !count || (!ms && cap)) return FHS_EINVAL;
    if (!c->timing || c->n_timed == 0) return fail(c, FHS_ESTATE, "no timed launch");
    *count = c->n_timed;
    for (uint32_t i = 0; i < c->n_timed && i < cap; ++i) {
        hipError_t e = hipEventElapsedTime(&ms[i], c->events[2 * i], c->events[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventElapsedTime");
    }
    return FHS_OK;
}

extern "C" fhs_status fhs_workspace_size(const fhs_ctx *c, uint32_t M, uint32_t S, size_t *bytes) {
    if (!c || !bytes) return FHS_EINVAL;
    if (!c->loaded) return FHS_ESTATE;
    if (c->prog.A > kMaxSources) return FHS_ERANGE;
    Plan pl;
    fhs_status st = make_plan(c, M, std::max<uint32_t>(S, 1), pl);
    if (st != FHS_OK) return st;
    *bytes = pl.bytes;
    return FHS_OK;
}

extern "C" fhs_status fhs_evaluate(fhs_ctx *c, const uint64_t *d_in, const double *d_cf, uint32_t S,
                                   const uint64_t *d_out, uint32_t M, double thr, double *d_amps,
                                   uint64_t *d_stats, void *d_ws, size_t ws_bytes, void *stream) {
    Plan pl;
    fhs_status st = check_eval_args(c, d_in, d_cf, S, d_out, M, thr, d_amps, d_stats, d_ws, ws_bytes, pl);
    if (st != FHS_OK || M == 0) return st;
    FHS_HIP(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    GraphKey key{};
    key.inputs = d_in;
    key.coeffs = d_cf;
    key.outputs = d_out;
    key.amps = d_amps;
    key.stats = d_stats;
    key.ws = d_ws;
    key.S = S;
    key.M = M;
    key.c1 = c->c1;
    key.c2 = c->c2;
    std::memcpy(&key.thr_bits, &thr, sizeof(thr));
    key.ws_bytes = ws_bytes;
    key.generation = c->generation;
    key.timing = 0;
    const bool timed = c->timing && c->prog.A > 0;
    if (c->timing) {
        // Timing mode: the same launch sequence, enqueued directly on the
        // caller's stream with events around every consumer launch (events
        // recorded inside a captured graph carry no usable timestamps).
        const Common cm = make_common(c, pl, d_in, S, d_out, M, thr, d_ws);
        const CompiledConsumer *ck = nullptr;
        if ((st = compiled_consumer(c, cm, pl.Dp, &ck)) != FHS_OK) return st;
        int bpc = c->prog.A > 0 ? (ck ? ck->blocks_per_cu : consume_blocks_per_cu(cm, nw_of(c->prog), c->ilp)) : 1;
        if (c->blocks_per_cu > 0) bpc = std::min<int>(bpc, static_cast<int>(c->blocks_per_cu));
        if (timed) {
            FHS_HIP(c, ensure_events(c, pl.n_batches));
            // not captured: a plain memset is fine here
            FHS_HIP(c, hipMemsetAsync(c->d_valid, 0, sizeof(unsigned long long), s));
            c->n_entries = 0;
            const size_t items = static_cast<size_t>(pl.P) * pl.ipp;
            if (items > c->stamps_cap) {
                FHS_HIP(c, hipStreamSynchronize(s));
                if (c->d_stamps) FHS_HIP(c, hipFree(c->d_stamps));
                c->d_stamps = nullptr;
                c->stamps_cap = 0;
                FHS_HIP(c, hipMalloc(reinterpret_cast<void **>(&c->d_stamps), 2 * sizeof(unsigned long long) * items));
                c->stamps_cap = items;
            }
            // items the consumer skips (pairs the precheck rejected) keep zeros
            if (items) FHS_HIP(c, hipMemsetAsync(c->d_stamps, 0, 2 * sizeof(unsigned long long) * items, s));
            c->n_stamped = items;
            c->stamp_ipp = pl.ipp;
        }
        FHS_HIP(c, enqueue_batched(c, pl, cm, d_cf, d_amps, d_stats, d_ws, bpc, timed, s, ck));
        c->n_timed = timed ? pl.n_batches : 0;
        return FHS_OK;
    }
    if (!(c->have_graph && c->key == key)) {
        drop_graph(c);
        const Common cm = make_common(c, pl, d_in, S, d_out, M, thr, d_ws);
        const CompiledConsumer *ck = nullptr;   // compiled before the capture starts
        if ((st = compiled_consumer(c, cm, pl.Dp, &ck)) != FHS_OK) return st;
        int bpc = c->prog.A > 0 ? (ck ? ck->blocks_per_cu : consume_blocks_per_cu(cm, nw_of(c->prog), c->ilp)) : 1;
        if (c->blocks_per_cu > 0) bpc = std::min<int>(bpc, static_cast<int>(c->blocks_per_cu));
        FHS_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
        hipError_t e = enqueue_batched(c, pl, cm, d_cf, d_amps, d_stats, d_ws, bpc, false, c->cap_stream, ck);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
        if (e != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return hip_fail(c, e, "kernel launch during capture");
        }
        if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
        c->graph = g;
        FHS_HIP(c, hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0));
        c->key = key;
        c->have_graph = true;
    }
    FHS_HIP(c, hipGraphLaunch(c->exec, s));
    return FHS_OK;
}

extern "C" fhs_status fhs_evaluate_plain(fhs_ctx *c, const uint64_t *d_in, const double *d_cf,
                                         uint32_t S, const uint64_t *d_out, uint32_t M, double thr,
                                         double *d_amps, uint64_t *d_stats, void *d_ws,
                                         size_t ws_bytes, void *stream) {
    Plan pl;
    fhs_status st = check_eval_args(c, d_in, d_cf, S, d_out, M, thr, d_amps, d_stats, d_ws, ws_bytes, pl);
    if (st != FHS_OK || M == 0) return st;
    FHS_HIP(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const HostProgram &P = c->prog;
    const int NW = nw_of(P);
    // Algorithm 1 has no checkpoint: every source lives in one region.
    Plan plain = pl;
    plain.c1 = plain.c2 = static_cast<uint32_t>(P.L);
    plain.Ap = plain.Ar = 0;
    plain.As = static_cast<uint32_t>(P.A);
    const Common cm = make_common(c, plain, d_in, S, d_out, M, thr, d_ws);
    PreBufs pre = pre_bufs(d_ws, pl);
    pre.acc_pos = nullptr;   // the plain form's blocks cover every pair
    PairRes res = pair_res(d_ws, pl);
    FHS_HIP(c, launch_precheck(cm, NW, pre, pl.P, nullptr, 0, s));
    if (P.A == 0) {
        FHS_HIP(c, launch_pair_reduce(pre, Partials{nullptr, nullptr, nullptr}, res, 0, pl.P, 0, 0, s));
    } else {
        Partials part{at<double2>(d_ws, pl.off_plain_amp), at<uint64_t>(d_ws, pl.off_plain_st), nullptr};
        if (c->timing) {
            FHS_HIP(c, ensure_events(c, 1));
            FHS_HIP(c, hipEventRecord(c->events[0], s));
        }
        FHS_HIP(c, launch_plain(cm, NW, c->ilp, pre, part, pl.P, pl.bpp, s));
        if (c->timing) FHS_HIP(c, hipEventRecord(c->events[1], s));
        c->n_timed = c->timing ? 1 : 0;
        c->n_stamped = 0;
        FHS_HIP(c, launch_pair_reduce(pre, part, res, 0, pl.P, pl.bpp, cm.A, s));
    }
    FHS_HIP(c, launch_finalize(res, d_cf, S, M, d_amps, d_stats, s));
    return FHS_OK;
}

extern "C" fhs_status fhs_evaluate_noalloc(fhs_ctx *c, const uint64_t *d_in, const double *d_cf,
                                           uint32_t S, const uint64_t *d_out, uint32_t M, double thr,
                                           double *d_amps, uint64_t *d_stats, void *stream) {
    if (!c) return FHS_EINVAL;
    c->err.clear();
    if (!c->scratch) return fail(c, FHS_EHIP, "no-alloc scratch unavailable on device %d", c->device);
    Plan pl;
    fhs_status st = check_eval_args(c, d_in, d_cf, S, d_out, M, thr, d_amps, d_stats, c->scratch,
                                    FHS_NOALLOC_SCRATCH_BYTES, pl, true);
    if (st != FHS_OK || M == 0) return st;
    FHS_HIP(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Common cm = make_common(c, pl, d_in, S, d_out, M, thr, c->scratch);
    // A compiled consumer only if one is already cached for this program,
    // split and launch shape (compiling and loading a module allocates);
    // otherwise the interpreting kernels.
    const CompiledConsumer *ck = nullptr;
    std::string key;
    size_t shm = 0;
    if (consumer_job(c, cm, pl.Dp, key, nullptr, shm)) {
        auto it = c->compiled.find(key);
        if (it != c->compiled.end()) ck = &it->second;
    }
    int bpc = c->prog.A > 0 ? (ck ? ck->blocks_per_cu : consume_blocks_per_cu(cm, nw_of(c->prog), c->ilp)) : 1;
    if (c->blocks_per_cu > 0) bpc = std::min<int>(bpc, static_cast<int>(c->blocks_per_cu));
    // enqueued directly (instantiating a graph allocates), never timed
    FHS_HIP(c, enqueue_batched(c, pl, cm, d_cf, d_amps, d_stats, c->scratch, bpc, false, s, ck));
    return FHS_OK;
}

extern "C" fhs_status fhs_item_stamps(fhs_ctx *c, uint64_t *stamps, size_t cap, size_t *count,
                                      uint32_t *items_per_pair, uint64_t *ticks_per_s) {
    if (!c || !count || (!stamps && cap)) return FHS_EINVAL;
    c->err.clear();
    if (!c->timing || c->n_timed == 0 || c->n_stamped == 0) return fail(c, FHS_ESTATE, "no timed launch");
    FHS_HIP(c, hipSetDevice(c->device));
    *count = c->n_stamped;
    if (items_per_pair) *items_per_pair = c->stamp_ipp;
    if (ticks_per_s) {
        int khz = 0;
        FHS_HIP(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device));
        *ticks_per_s = static_cast<uint64_t>(khz) * 1000u;
    }
    const size_t n = std::min(cap, static_cast<size_t>(c->n_stamped));
    if (n) FHS_HIP(c, hipMemcpy(stamps, c->d_stamps, 2 * sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
    return FHS_OK;
}
