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
    hipFunction_t fn = nullptr;
    int blocks_per_cu = 1;   // occupancy limit at the given dynamic LDS size
};

// Source text of the consumer for device-program regions [i1, i2) (root)
// and [i2, iG) (suffix) of `dev`, whose first sources are Ap and Ap + Ar;
// fin_c2 and fin_G are the final-bit masks checked at the ends of the two
// regions.  Without pruning, the suffix's factor multiplications are
// deferred to the histories that pass the final check when their table
// indices fit in 64 bits.
std::string consumer_source(const std::vector<Instr> &dev, uint32_t i1, uint32_t i2, uint32_t iG,
                            uint32_t Ap, uint32_t Ar, const Mask4 &fin_c2, const Mask4 &fin_G, int NW,
                            int H, bool prune, bool flds);

// Compile `src` for gfx950 and load it on the current device.  On failure
// returns false and puts the compiler log in `log`.
bool compile_consumer(const std::string &src, size_t shm, CompiledConsumer &out, std::string &log);

void release(CompiledConsumer &k);

hipError_t launch_compiled(const CompiledConsumer &k, const Common &c, Table tab, Partials part,
                           uint32_t p0, uint32_t B, uint32_t chunk, uint32_t ss, uint32_t *counter,
                           uint32_t grid, size_t shm, hipStream_t s);

}  // namespace fhs
