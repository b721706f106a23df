// program.hpp -- the straight-line history program shared by the host reducer
// and the device kernels.
//
// The reducer turns a circuit into one instruction per gate, in evaluation
// order (output -> input, Section IV-A).  A history starts from the output
// bitstring as a complete n-bit time-slice state; walking backward,
//   - a deterministic gate applies its inverse permutation (every permutation
//     used here is an involution) and multiplies its phase,
//   - a wire-preserving (diagonal) gate multiplies the factor selected by the
//     current bits,
//   - a branching gate reads its output bit, takes its input bit from an
//     artificial source (bit k of the history index) or, on a natural input
//     segment, from the input bitstring, multiplies U[out][in] and writes the
//     input bit into the state.
// Consistency with the input boundary is a mask compare at region ends: a
// bit whose natural input segment has been reached can no longer change.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace fhs {

constexpr int kMaxQubits = 128;
constexpr int kMaxWords32 = 4;       // 32-bit words per state on the device
constexpr int kMaxSources = 62;      // history index fits a signed 64-bit range

enum Op : uint8_t {
    OP_PERM = 1,        // if ((s ^ cv) & cm) == 0: flip bit a            (X, CX, CCX, MCX)
    OP_SWAP = 2,        // if ((s ^ cv) & cm) == 0: swap bits a and b      (SWAP, CSWAP)
    OP_DET1 = 3,        // factor fac[2*o .. 2*o+1] with o = bit a, then flip bit a   (Y, phased X)
    OP_DIAG1 = 4,       // factor fac[2*bit a ..]                         (Z S SDG T TDG P RZ)
    OP_DIAG2 = 5,       // factor fac[2*(bit a | bit b << 1) ..]          (CZ CP RZZ)
    OP_MCPHASE = 6,     // if ((s ^ cv) & cm) == 0: amplitude *= -1       (MCZ)
    OP_BRANCH_SRC = 7,  // o = bit a, i = source bit k: factor U[o][i], bit a := i
    OP_BRANCH_NAT = 8,  // o = bit a, i = input bit a:  factor U[o][i], bit a := i
};

// The opcode byte carries the base op in its low 4 bits and the 32-bit
// state word holding bit a (bits 4-5) and bit b (bits 6-7), so the device
// indexes its state registers with compile-time constants only.
constexpr uint8_t op_code(Op base, int a, int b) {
    return static_cast<uint8_t>(base | ((a >> 5) << 4) | ((b >> 5) << 6));
}
constexpr int op_base(uint8_t code) { return code & 15; }

// One instruction, 48 bytes, read wave-uniformly.  Masks are four 32-bit
// words (state bits 0..127).  For branching gates fac points at
// U[o][i] as (re,im) at fac + 2*(2o+i), followed by the four moduli
// min(1,|U[o][i]|) at fac + 8 + (2o+i).
struct alignas(16) Instr {
    uint8_t op, a, b, pad0;   // op: op_code(); a, b: qubit (state bit) indices
    uint32_t k;        // global source index (OP_BRANCH_SRC)
    uint32_t fac;      // offset into the factor table, in doubles
    uint32_t zmask;    // branching: bit (2o+i) set when U[o][i] is exactly zero
    uint32_t cm[4];    // control mask
    uint32_t cv[4];    // control values (subset of cm)
};
static_assert(sizeof(Instr) == 48, "instruction layout");

struct Mask4 {
    uint32_t w[4];
};

struct HostProgram {
    int n = 0;                 // qubits
    int G = 0;                 // gates
    int A = 0;                 // artificial sources
    int W = 1;                 // 64-bit words per bitstring
    int NW = 1;                // 32-bit words per device state (1, 2 or 4)
    int L = 0;                 // leading source-free gates (evaluation order)
    int n_branch = 0;
    std::vector<Instr> ins;            // evaluation order, size G
    std::vector<double> fac;           // factor table
    std::vector<uint32_t> src_eval;    // evaluation position of source k's gate
    std::vector<Mask4> final_before;   // [G+1]: bits final once e gates are applied
    std::vector<uint8_t> role;         // per evaluation position: 0 preserve, 1 det, 2 branch
    std::vector<uint16_t> fp_cost;     // per evaluation position: algorithmic FP64 flops
};

}  // namespace fhs
