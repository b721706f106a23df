// placement.hpp -- artificial-source placement by determinism reachability
// (Section IV-B, Fig. 3) for the host reducer.
//
// The backward sweep (Section IV-A) puts a source at every branching gate
// whose input segment is not natural.  Determinism can also flow the other
// way: the three internal wires around a CNOT are symmetric (any two fix the
// third), and a natural source on a CNOT merges its other two wires, so some
// of those sources are implied by the others.  This analysis picks sources
// among the input segments of branching gates (the values the walk from the
// output has to be given), as few as let the relations reach every internal
// wire: exhaustively (the fewest, first found in evaluation order) or
// greedily (one at a time, the candidate reaching the most wires).
//
// Every other branching gate's input value is then an affine function over
// GF(2) of the sources, the input bits and the output bits, found by
// propagating symbolic values through the same relations (CNOT: t_out =
// t_in ^ c ^ [control active on 0]; one-qubit deterministic gate: out = in ^
// 1; SWAP: the two wires exchanged).  The device evaluates it as
// parity(h & S) ^ (a per-pair constant bit from the boundary bits).
//
// Gate set: branching gates on one qubit; deterministic gates on one qubit,
// CNOT (one control, including MCX with one control) and SWAP; diagonal
// gates of any size.  Anything else is FHS_EUNSUPPORTED.
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/fhs.h"
#include "program.hpp"

namespace fhs {

// An affine form over GF(2): x (input bits), y (output bits), s (sources)
// and a constant.
struct AffineForm {
    uint32_t x[4] = {0, 0, 0, 0};
    uint32_t y[4] = {0, 0, 0, 0};
    uint64_t s = 0;
    uint32_t c = 0;
    void add(const AffineForm &o) {
        for (int w = 0; w < 4; ++w) {
            x[w] ^= o.x[w];
            y[w] ^= o.y[w];
        }
        s ^= o.s;
        c ^= o.c;
    }
};

// How the walk from the output obtains one branching gate's input bit.
struct BranchInput {
    enum Kind { NATURAL, SOURCE, AFFINE } kind = NATURAL;
    int source = -1;      // SOURCE: source number (evaluation order)
    AffineForm form;      // AFFINE
};

// One gate as the analysis sees it (time order).
struct PlaceGate {
    int k = 0;                     // qubits touched
    std::vector<int> q;            // qubits, local bit j <-> q[j]
    bool branch = false;           // branching (one qubit)
    bool det = false;              // deterministic (permutation, maybe with phases)
    std::vector<bool> preserve;    // per local wire: value kept across the gate
    // deterministic two-qubit gates: CNOT (control / target local wires and
    // the control value that flips the target) or SWAP
    bool cnot = false, swap = false;
    int jc = -1, jt = -1, cval = 1;
};

// Places the sources; fills `inputs` (per gate, time order; meaningful for
// branching gates) and the evaluation positions of the sources.  Returns
// FHS_EUNSUPPORTED outside the gate set, FHS_ERANGE if the exhaustive
// search exceeds its budget.
fhs_status place_by_reach(int n, const std::vector<PlaceGate> &gates, bool greedy,
                          std::vector<BranchInput> &inputs, std::vector<uint32_t> &src_eval);

}  // namespace fhs
