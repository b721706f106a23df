// jit.hpp -- the persistent consumer compiled for one program and split.
//
// The interpreting consumer decodes every instruction of the root and
// suffix regions for every history group it walks.  For short regions (a
// folded walk has a few instructions per region) that decode dominates, so
// the runtime can instead emit the regions as straight-line calls of the
// same per-opcode steps, with every instruction a compile-time constant,
// and compile that consumer with hipRTC at run time.  Same kernel body
// (consume_body in device.hpp), same results.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace fhs {

struct CompiledConsumer {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;    // the consumer
    hipFunction_t pfn = nullptr;   // the prefix-table build (null: the interpreting one is used)
    int blocks_per_cu = 1;   // occupancy limit at the given dynamic LDS size
};

// Source text of the consumer for device-program regions [i1, i2) (root)
// and [i2, iG) (suffix) of `dev`, whose first sources are Ap and Ap + Ar;
// fin_c2 and fin_G are the final-bit masks checked at the ends of the two
// regions; `fac` is the program's factor table, of which the kernel sees
// the slice from fac_lo on (staged in LDS when flds, else read from HBM
// with fac_lo = 0).  Factors whose tables have a shape the device forms in
// registers (a complex-conjugate pair selected by one bit or a parity;
// real entries of one magnitude) are emitted with the table's values as
// constants; the others read their table per lane.  Without pruning, when a
// history can still fail after the root (a final-bit check left, a ladder
// run compared with the output, a zero table entry), the suffix's factor
// multiplications are deferred to the histories that pass the final check
// if their table indices fit in 64 bits.
//
// With prefix_ok, the module also holds the prefix-table build for device
// region [iL, i1): the gates before the first depth-first source
// src_dev[Ap - Dp], then the Dp depth-first levels (src_dev: device index of
// every source's gate); pflds stages the prefix's factors in LDS (from
// pfac_lo on).
std::string consumer_source(const std::vector<Instr> &dev, const std::vector<double> &fac, uint32_t i1,
                            uint32_t i2, uint32_t iG, uint32_t Ap, uint32_t Ar, const Mask4 &fin_c2,
                            const Mask4 &fin_G, int NW, int H, bool prune, bool flds, uint32_t fac_lo,
                            bool prefix_ok, uint32_t iL, const std::vector<uint32_t> &src_dev, uint32_t Dp,
                            bool pflds, uint32_t pfac_lo, uint32_t ss);

// Compile `src` for gfx950 and load it on the current device.  On failure
// returns false and puts the compiler log in `log`.
bool compile_consumer(const std::string &src, size_t shm, CompiledConsumer &out, std::string &log);

// The two halves of compile_consumer: hipRTC to a code object (no HIP
// calls; safe to run for different sources on several threads at once),
// then the module load on the calling thread's current device.
bool compile_code(const std::string &src, std::vector<char> &code, std::string &log);

// A residue test for a whole pair (the precheck): when every write to one
// bit field after the leading source-free gates is a ladder step selected by
// a source bit, and the final check covers the field, the field's step count
// is off0 + 2 P(h) with P(h) in [amin, amax] for every history h.  A pair is
// then feasible only if D = (e - off) << up, e the field residue after the
// leading gates (field_residue), is 2k << up for some k <= span; off =
// off0 + 2 amin.  Returns false when the program has no such field.
struct PairFilter {
    uint32_t lo = 0, hi = 0, up = 0, off = 0, span = 0;
};
bool pair_filter(const std::vector<Instr> &dev, const std::vector<double> &fac, uint32_t iL, uint32_t iG,
                 const Mask4 &fin_G, uint32_t A, PairFilter &out);
bool load_consumer(const std::vector<char> &code, bool has_prefix, size_t shm, CompiledConsumer &out,
                   std::string &log);

void release(CompiledConsumer &k);

// Launch the compiled prefix-table build (k.pfn) with the interpreting
// one's grid: one lane per subtree, B << (Ap - Dp) lanes.
hipError_t launch_prefix_compiled(const CompiledConsumer &k, const Common &c, PreBufs pre, Table tab,
                                  uint32_t p0, uint32_t B, uint32_t Dp, size_t shm, hipStream_t s);

hipError_t launch_compiled(const CompiledConsumer &k, const Common &c, Table tab, Partials part,
                           uint32_t p0, uint32_t B, uint32_t chunk, uint32_t ss, uint32_t *counter,
                           uint32_t grid, size_t shm, hipStream_t s);

}  // namespace fhs
