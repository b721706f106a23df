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

#include <cstdint>
#if !defined(__HIPCC_RTC__)
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>
#endif

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
    OP_ADD = 9,         // if ((s ^ cv) & cm) == 0: the bit field [a, a+b) += 1 mod 2^b, or -= 1
                        // when zmask bit 0 is set (a folded ladder of controlled X gates)
    OP_NOP = 10,        // a gate folded into the OP_ADD before it (dropped from the device copy)
    OP_ADDSEL = 11,     // if ((s ^ cv) & cm) == 0: the bit field [a, a+b) += 1 or -= 1 mod 2^b,
                        // -= 1 when zmask bit (bit k of the state) is set (two OP_ADDs on one
                        // field whose controls differ only in bit k, outside the field)
    OP_BRANCH_AFF = 12, // o = bit a, i = parity(h & S) ^ bit k of the pair's affine constants
                        // (S = cm[0] | cm[1] << 32): factor U[o][i], bit a := i
};

// The opcode byte carries the base op in its low 4 bits; bits 4-5 and 6-7
// carry 32-bit state-word indices, so the device touches its state registers
// with compile-time indices only:
//   PERM     bits 4-5: word of the target bit, 6-7: highest nonzero control word
//   MCPHASE, ADD  bits 4-5: highest nonzero control word
//   ADDSEL   bits 4-5: highest nonzero control word, 6-7: word of bit k
//   SWAP, DIAG2  bits 4-5: word of bit a, 6-7: word of bit b
//   DET1, DIAG1, BRANCH_*  bits 4-5: word of bit a
constexpr uint8_t op_code(Op base, int w1, int w2) {
    return static_cast<uint8_t>(base | (w1 << 4) | (w2 << 6));
}
constexpr int op_base(uint8_t code) { return code & 15; }

// One instruction, 48 bytes, read wave-uniformly.  Masks are four 32-bit
// words (state bits 0..127).  fac is even (16-byte aligned entries): a
// factor table of complex (re,im) pairs selected by the gate's bits; for
// branching gates U[o][i] sits at fac + 2*(2o+i), followed by the four
// moduli min(1,|U[o][i]|) at fac + 8 + (2o+i).  Factor tables are laid out
// in evaluation order, so a range of gates owns a contiguous slice.
struct alignas(16) Instr {
    // hdr = op | a << 8 | b << 16 | zmask << 24 (one dword, so the device
    // reads it with a scalar load): op = op_code(); a, b = qubit (state bit)
    // indices; zmask (branching gates) has bit (2o+i) set when U[o][i] is
    // exactly zero.
    uint32_t hdr;
    uint32_t k;        // OP_BRANCH_SRC: global source index; OP_PERM: target bit mask;
                       // OP_ADDSEL: the selecting state bit
    uint32_t fac;      // offset into the factor table, in doubles
    uint32_t run;      // instructions from here to the end of this run of identical opcodes
    uint32_t cm[4];    // control mask
    uint32_t cv[4];    // control values (subset of cm)
};
static_assert(sizeof(Instr) == 48, "instruction layout");

constexpr uint32_t pack_hdr(uint32_t op, uint32_t a, uint32_t b, uint32_t zmask) {
    return op | (a << 8) | (b << 16) | (zmask << 24);
}

struct Mask4 {
    uint32_t w[4];
};

#if !defined(__HIPCC_RTC__)
// The state bits an instruction reads or writes (host side: the compiled
// regions' accumulation of ladder steps and its work count follow it).
inline void touched_bits(const Instr &I, uint32_t (&m)[4]) {
    const int base = op_base(static_cast<uint8_t>(I.hdr & 0xffu));
    const uint32_t a = (I.hdr >> 8) & 0xffu, b = (I.hdr >> 16) & 0xffu;
    for (int w = 0; w < 4; ++w) m[w] = 0;
    auto bit = [&](uint32_t q) {
        if (q < 128) m[q >> 5] |= 1u << (q & 31);
    };
    auto controls = [&]() {
        for (int w = 0; w < 4; ++w) m[w] |= I.cm[w];
    };
    switch (base) {
        case OP_PERM: bit(a); controls(); break;
        case OP_SWAP: bit(a); bit(b); controls(); break;
        case OP_DET1:
        case OP_DIAG1:
        case OP_BRANCH_SRC:
        case OP_BRANCH_NAT:
        case OP_BRANCH_AFF: bit(a); break;
        case OP_DIAG2: bit(a); bit(b); break;
        case OP_MCPHASE: controls(); break;
        case OP_ADDSEL: bit(I.k); [[fallthrough]];
        case OP_ADD:
            controls();
            for (uint32_t q = a; q < a + b; ++q) bit(q);
            break;
        default: break;
    }
}

// The state bits an instruction writes (the target of a permutation, both
// swapped bits, the bit a branching gate sets, a ladder step's field).
inline void written_bits(const Instr &I, uint32_t (&m)[4]) {
    const int base = op_base(static_cast<uint8_t>(I.hdr & 0xffu));
    const uint32_t a = (I.hdr >> 8) & 0xffu, b = (I.hdr >> 16) & 0xffu;
    for (int w = 0; w < 4; ++w) m[w] = 0;
    auto bit = [&](uint32_t q) {
        if (q < 128) m[q >> 5] |= 1u << (q & 31);
    };
    switch (base) {
        case OP_PERM:
        case OP_DET1:
        case OP_BRANCH_SRC:
        case OP_BRANCH_NAT:
        case OP_BRANCH_AFF: bit(a); break;
        case OP_SWAP: bit(a); bit(b); break;
        case OP_ADD:
        case OP_ADDSEL:
            for (uint32_t q = a; q < a + b; ++q) bit(q);
            break;
        default: break;
    }
}

// Which state bits hold a source bit of the current region, as the region
// is walked in order: a branching gate with a source sets its bit to source
// k; any other write clears the association.  A ladder step without
// controls whose selecting bit holds source k adds a constant plus +-1 times
// that source bit, so the compiled regions sum such steps' selecting bits
// as a popcount of the region's source index (and the work count follows).
struct SourceBits {
    int src[kMaxQubits];
    SourceBits() {
        for (int &x : src) x = -1;
    }
    void step(const Instr &I, uint32_t kbase) {
        uint32_t m[4];
        written_bits(I, m);
        for (int q = 0; q < kMaxQubits; ++q)
            if ((m[q >> 5] >> (q & 31)) & 1u) src[q] = -1;
        if (op_base(static_cast<uint8_t>(I.hdr & 0xffu)) == OP_BRANCH_SRC)
            src[(I.hdr >> 8) & 0xffu] = static_cast<int>(I.k - kbase);
    }
    // the region-relative source a controls-free paired step selects on, or -1
    int selector_source(const Instr &I) const {
        if (op_base(static_cast<uint8_t>(I.hdr & 0xffu)) != OP_ADDSEL || I.k >= 128) return -1;
        if (I.cm[0] | I.cm[1] | I.cm[2] | I.cm[3]) return -1;
        return src[I.k];
    }
};

// The instructions of a suffix region [lo, hi) (device indices; OP_NOP
// skipped) that can be evaluated once per root history instead of once per
// leaf: phases (DIAG1, DIAG2, MCPHASE) and, without pruning, branching gates
// on a natural input segment (BRANCH_NAT) that commute with every
// instruction before them that stays in the leaf loop (neither writes a
// state bit the other reads or writes; phases write none).  Only staying
// instructions write the bits a source of the region influences, so these
// read none of them.  Their factors are then multiplied before the leaf's
// other factors instead of between them: the same product up to rounding.
// With pruning, branches stay in place (the modulus product's order decides
// pruning).
inline std::vector<uint8_t> hoistable(const std::vector<Instr> &ins, uint32_t lo, uint32_t hi, bool prune) {
    std::vector<uint8_t> out(hi > lo ? hi - lo : 0, 0);
    uint32_t stay_w[4] = {0, 0, 0, 0};   // bits written by an instruction that stays
    uint32_t stay_t[4] = {0, 0, 0, 0};   // bits touched by an instruction that stays
    for (uint32_t x = lo; x < hi; ++x) {
        const Instr &I = ins[x];
        const int base = op_base(static_cast<uint8_t>(I.hdr & 0xffu));
        if (base == OP_NOP) continue;
        uint32_t t[4], w[4];
        touched_bits(I, t);
        written_bits(I, w);
        bool conflict = false;
        for (int k = 0; k < 4; ++k) conflict = conflict || (t[k] & stay_w[k]) || (w[k] & stay_t[k]);
        const bool kind = base == OP_DIAG1 || base == OP_DIAG2 || base == OP_MCPHASE ||
                          (base == OP_BRANCH_NAT && !prune);
        if (kind && !conflict) {
            out[x - lo] = 1;
            continue;
        }
        for (int k = 0; k < 4; ++k) {
            stay_w[k] |= w[k];
            stay_t[k] |= t[k];
        }
    }
    return out;
}

// A gate whose factor table takes exactly two values, a at the table
// indices x where bit x of tt is clear and b where it is set ((a, b) as bit
// patterns of (re, im), in a fixed order so that the same pair is one
// class): phases, diagonal two-qubit gates with two distinct entries (RZZ,
// CZ), branching gates such as RX whose diagonal and off-diagonal entries
// agree.  Branching gates with a zero entry (their histories can fail) and
// real-entry branches of one magnitude (H: a sign per history, collected
// separately) are not counted.
struct TwoValued {
    bool ok = false;
    uint64_t a[2] = {0, 0}, b[2] = {0, 0};
    uint32_t tt = 0;
    uint32_t nx = 0;    // table entries: 2 (one selecting bit) or 4
};

inline TwoValued two_valued(const Instr &I, const std::vector<double> &fac) {
    TwoValued r;
    const int base = op_base(static_cast<uint8_t>(I.hdr & 0xffu));
    const bool branch = base == OP_BRANCH_SRC || base == OP_BRANCH_NAT;
    if (base == OP_DIAG1 || base == OP_DET1) r.nx = 2;
    else if (base == OP_DIAG2 || branch) r.nx = 4;
    else return r;
    if (branch && (I.hdr >> 24) != 0u) return r;
    const double *t = fac.data() + I.fac;
    if (branch) {
        bool real = t[0] != 0.0;
        for (int x = 0; x < 4; ++x) real = real && t[2 * x + 1] == 0.0 && std::fabs(t[2 * x]) == std::fabs(t[0]);
        if (real) return r;
    }
    auto pat = [&](uint32_t x, uint64_t (&v)[2]) { std::memcpy(v, t + 2 * x, sizeof v); };
    uint64_t v0[2], v1[2] = {0, 0};
    pat(0, v0);
    bool second = false;
    uint32_t tt = 0;
    for (uint32_t x = 1; x < r.nx; ++x) {
        uint64_t v[2];
        pat(x, v);
        if (v[0] == v0[0] && v[1] == v0[1]) continue;
        if (!second) {
            v1[0] = v[0];
            v1[1] = v[1];
            second = true;
        } else if (v[0] != v1[0] || v[1] != v1[1]) {
            return r;   // three or more values
        }
        tt |= 1u << x;
    }
    if (!second) return r;   // one value: no selection
    if (v0[0] > v1[0] || (v0[0] == v1[0] && v0[1] > v1[1])) {
        std::swap(v0[0], v1[0]);
        std::swap(v0[1], v1[1]);
        tt = ~tt & ((1u << r.nx) - 1u);
    }
    r.ok = true;
    r.a[0] = v0[0];
    r.a[1] = v0[1];
    r.b[0] = v1[0];
    r.b[1] = v1[1];
    r.tt = tt;
    return r;
}

// Table sizes of the counted factors: entries of one group's table and of
// all groups' (16 bytes each, staged in LDS), and groups, i.e. table
// multiplies per valid history.
constexpr uint32_t kCountGroupMax = 1024;
constexpr uint32_t kCountTabMax = 1024;
constexpr uint32_t kCountGroups = 3;

// Which two-valued gates of the consumer's regions (root [i1, i2), suffix
// [i2, iG); `hoisted[x - i2]` marks the suffix instructions evaluated once
// per root) the compiled consumer counts instead of multiplying.  A class is
// the gates with one pair (a, b); its n gates give a history the product
// a^(n-f) b^f, f the number of b entries taken.  Classes share a group's
// table (the products over every combination of their f) while it stays
// within kCountGroupMax entries; a history's index `ci` holds each group's
// index in a bit field, and a class's gate moves it by its step.  Counting is
// on only when a class has a gate in the leaf loop (else the table multiply
// per valid history would cost more than the root's multiplies it saves)
// and every class fits.
struct CountPlan {
    struct Cls {
        TwoValued v;       // the pair as the class counts it: f = the number of b entries
        uint32_t n = 0;
        bool leaf = false;
        bool flip = false; // the gates' own tt (two_valued) complemented
        uint32_t group = 0, stride = 0, step = 0;
    };
    std::vector<Cls> cls;
    std::vector<int> cls_of;                    // per instruction of [lo, hi): class or -1
    std::vector<uint32_t> group_size, group_base, group_shift;
    uint32_t lo = 0, entries = 0;
    bool on() const { return entries > 0; }
    int of(uint32_t x) const {
        return (on() && x >= lo && x - lo < cls_of.size()) ? cls_of[x - lo] : -1;
    }
    // the truth table gate `v` (of class c) selects b with
    uint32_t tt(int c, const TwoValued &v) const {
        return cls[c].flip ? ~v.tt & ((1u << v.nx) - 1u) : v.tt;
    }
};

inline CountPlan count_plan(const std::vector<Instr> &ins, const std::vector<double> &fac, uint32_t i1,
                            uint32_t i2, uint32_t iG, const std::vector<uint8_t> &hoisted) {
    CountPlan P;
    P.lo = i1;
    P.cls_of.assign(iG > i1 ? iG - i1 : 0, -1);
    bool any_leaf = false;
    for (uint32_t x = i1; x < iG; ++x) {
        const TwoValued v = two_valued(ins[x], fac);
        if (!v.ok) continue;
        int c = -1;
        for (size_t k = 0; k < P.cls.size() && c < 0; ++k) {
            const TwoValued &u = P.cls[k].v;
            if (u.a[0] == v.a[0] && u.a[1] == v.a[1] && u.b[0] == v.b[0] && u.b[1] == v.b[1])
                c = static_cast<int>(k);
        }
        if (c < 0) {
            c = static_cast<int>(P.cls.size());
            P.cls.push_back(CountPlan::Cls{});
            P.cls.back().v = v;
        }
        P.cls_of[x - i1] = c;
        P.cls[c].n += 1;
        if (x >= i2 && (x - i2 >= hoisted.size() || !hoisted[x - i2])) {
            P.cls[c].leaf = true;
            any_leaf = true;
        }
    }
    CountPlan off;
    off.lo = i1;
    if (!any_leaf) return off;
    // count the entry the cheaper form selects (bits that differ, a bit that
    // is set, both set) where most of a class's gates then have that form
    {
        std::vector<int> vote(P.cls.size(), 0);
        for (uint32_t x = i1; x < iG; ++x) {
            const int c = P.cls_of[x - i1];
            if (c < 0) continue;
            const uint32_t t = two_valued(ins[x], fac).tt;
            if (t == 0x9u || t == 0x1u || t == 0x7u) vote[c] += 1;
            else if (t == 0x6u || t == 0x2u || t == 0x8u) vote[c] -= 1;
        }
        for (size_t k = 0; k < P.cls.size(); ++k)
            if (vote[k] > 0) {
                CountPlan::Cls &c = P.cls[k];
                c.flip = true;
                std::swap(c.v.a[0], c.v.b[0]);
                std::swap(c.v.a[1], c.v.b[1]);
            }
    }
    // leaf classes first, then by size
    std::vector<uint32_t> order(P.cls.size());
    for (uint32_t k = 0; k < order.size(); ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        if (P.cls[x].leaf != P.cls[y].leaf) return P.cls[x].leaf;
        return P.cls[x].n > P.cls[y].n;
    });
    uint64_t total = 0;
    for (uint32_t k : order) {
        CountPlan::Cls &c = P.cls[k];
        const uint64_t m = static_cast<uint64_t>(c.n) + 1u;
        bool placed = false;
        for (size_t g = 0; g < P.group_size.size() && !placed; ++g) {
            const uint64_t s = P.group_size[g];
            if (s * m <= kCountGroupMax && total + s * (m - 1u) <= kCountTabMax) {
                c.group = static_cast<uint32_t>(g);
                c.stride = static_cast<uint32_t>(s);
                P.group_size[g] = static_cast<uint32_t>(s * m);
                total += s * (m - 1u);
                placed = true;
            }
        }
        if (!placed && P.group_size.size() < kCountGroups && m <= kCountGroupMax && total + m <= kCountTabMax) {
            c.group = static_cast<uint32_t>(P.group_size.size());
            c.stride = 1u;
            P.group_size.push_back(static_cast<uint32_t>(m));
            total += m;
            placed = true;
        }
        if (!placed) return off;
    }
    uint32_t base = 0, shift = 0;
    for (uint32_t s : P.group_size) {
        P.group_base.push_back(base);
        P.group_shift.push_back(shift);
        base += s;
        uint32_t bits = 0;
        while ((1u << bits) < s) ++bits;
        shift += bits;
    }
    if (shift > 32u) return off;
    for (CountPlan::Cls &c : P.cls) c.step = c.stride << P.group_shift[c.group];
    P.entries = base;
    return P;
}

// Whether `I` ends a pending accumulation of ladder steps on the field
// [lo, hi): it touches a field bit other than as a further step of the same
// field (an add on the field itself only reads its controls and selector).
inline bool ends_field_run(const Instr &I, uint32_t lo, uint32_t hi) {
    const int base = op_base(static_cast<uint8_t>(I.hdr & 0xffu));
    const bool is_add = base == OP_ADD || base == OP_ADDSEL;
    const uint32_t a = (I.hdr >> 8) & 0xffu, b = (I.hdr >> 16) & 0xffu;
    uint32_t m[4];
    if (is_add && a == lo && a + b == hi) {
        for (int w = 0; w < 4; ++w) m[w] = I.cm[w];
        if (base == OP_ADDSEL && I.k < 128) m[I.k >> 5] |= 1u << (I.k & 31);
    } else if (is_add) {
        return true;   // an add on another field
    } else {
        touched_bits(I, m);
    }
    for (uint32_t q = lo; q < hi; ++q)
        if ((m[q >> 5] >> (q & 31)) & 1u) return true;
    return false;
}

constexpr uint32_t kNoPrev = 0xffffffffu;

struct HostProgram {
    int n = 0;                 // qubits
    int G = 0;                 // gates
    int A = 0;                 // artificial sources
    int W = 1;                 // 64-bit words per bitstring
    int NW = 1;                // 32-bit words per device state (1, 2 or 4)
    int L = 0;                 // leading source-free gates (evaluation order)
    int n_branch = 0;
    bool forward = false;      // placed by the forward sweep: evaluation order = time order
    int placement = 0;         // 0 sweep (backward or forward), 1 fewest by reachability, 2 greedy
    // OP_BRANCH_AFF constants: per affine input j, the input-bit and
    // output-bit masks and the constant of its form (4 + 4 + 1 words)
    std::vector<uint32_t> aff;
    // cut_ok[e]: a cut at evaluation position e keeps every affine input in a
    // region no earlier than its sources' (a form may use a source whose own
    // gate lies deeper; the cut may not fall between them)
    std::vector<uint8_t> cut_ok;
    std::vector<Instr> ins;            // evaluation order, size G (fused gates become OP_NOP)
    int n_fused = 0;                   // ladders folded into OP_ADD
    int n_paired = 0;                  // OP_ADD pairs merged into OP_ADDSEL
    std::vector<double> fac;           // factor table
    std::vector<uint32_t> src_eval;    // evaluation position of source k's gate
    std::vector<Mask4> final_before;   // [G+1]: bits final once e gates are applied
    std::vector<uint8_t> role;         // per evaluation position: 0 preserve, 1 det, 2 branch
    std::vector<uint16_t> fp_cost;     // per evaluation position: algorithmic FP64 flops
    // Folded ladders: the carry chain that applies a run of accumulated steps
    // on one field (int32 ops), and the position of the run's previous step
    // (kNoPrev when this step starts the run).
    std::vector<uint16_t> flush_cost;
    std::vector<uint32_t> run_prev;
    // The run still pending after the last position (its last step, or
    // kNoPrev) and whether the final-bit mask there covers its whole field:
    // then the run is compared with the output instead of applied.
    uint32_t tail_last = kNoPrev;
    bool tail_checked = false;
    std::vector<uint16_t> int_cost;    // per evaluation position: algorithmic int32 ops
    std::vector<uint32_t> fac_begin;   // [G+1]: factor-table offset of the first gate at or after e
};

// Whether a cut may fall at evaluation position c.
inline bool cut_allowed(const HostProgram &P, uint32_t c) {
    return P.cut_ok.empty() || c >= P.cut_ok.size() || P.cut_ok[c];
}

// Whether the last Dp of a prefix of Ap sources may be enumerated depth
// first: their bits are set only when the walk reaches their gates, so no
// affine input before cut c1 may use one of them from an earlier position.
inline bool dfs_allowed(const HostProgram &P, uint32_t c1, uint32_t Ap, uint32_t Dp) {
    if (P.aff.empty() || Dp == 0) return true;
    const uint32_t lo_bits = Ap - Dp;
    for (uint32_t e = 0; e < c1 && e < P.ins.size(); ++e) {
        const Instr &I = P.ins[e];
        if (op_base(static_cast<uint8_t>(I.hdr & 0xffu)) != OP_BRANCH_AFF) continue;
        const uint64_t smask = I.cm[0] | (static_cast<uint64_t>(I.cm[1]) << 32);
        for (uint32_t k = lo_bits; k < Ap && k < P.src_eval.size(); ++k)
            if (((smask >> k) & 1u) && P.src_eval[k] > e) return false;
    }
    return true;
}
#endif  // !__HIPCC_RTC__

}  // namespace fhs
