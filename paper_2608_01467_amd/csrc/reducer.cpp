// reducer.cpp -- host-side reduction of a circuit to a history program.
//
// Paper, Section II-A (gate roles), Section IV-A (natural sources, backward
// artificial-source placement), Section IV-C (Eq. (8) and the autotuned
// partition).  Host code only; runs without a GPU.
//
// Moduli min(1,|U|) feed the threshold-pruning decision, which must be
// bit-reproducible: they are computed here once, as sqrt(re*re + im*im)
// with contraction into FMA disabled, and the device only multiplies them.
#pragma STDC FP_CONTRACT OFF
#pragma clang fp contract(off)

#include <algorithm>
#include <cctype>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fhs.h"
#include "placement.hpp"
#include "program.hpp"

struct fhs_program {
    fhs::HostProgram p;
};

namespace fhs {
namespace {

using cd = std::complex<double>;

struct Gate {
    std::string name;
    std::vector<int> q;        // listed qubits (MCX: q[0] is the target)
    std::vector<uint8_t> neg;  // polarity per listed qubit (MCX/MCZ)
    double angle = 0.0;
    bool has_angle = false;
    int k = 0;                 // dense matrix size 2^k (k <= 3), 0 for MCX/MCZ
    cd m[8][8];                // U[out][in], local bit j <-> q[j]
};

bool all_digits(const std::string &s) {
    if (s.empty()) return false;
    for (char c : s)
        if (!std::isdigit(static_cast<unsigned char>(c))) return false;
    return true;
}

// Gate matrix U[out][in] on the listed qubits (local bit j = j-th listed qubit).
fhs_status build_matrix(Gate &g) {
    const std::string &nm = g.name;
    const double h = std::sqrt(0.5);
    auto need = [&](size_t nq, bool ang) {
        return g.q.size() == nq && g.has_angle == ang;
    };
    for (auto ng : g.neg)
        if (ng && nm != "MCX" && nm != "MCZ") return FHS_EPARSE;
    if (nm == "MCX" || nm == "MCZ") {
        if (g.q.empty() || g.has_angle) return FHS_EPARSE;
        if (nm == "MCX" && g.neg[0]) return FHS_EPARSE;
        g.k = 0;
        return FHS_OK;
    }
    int k;
    if (nm == "H" || nm == "X" || nm == "Y" || nm == "Z" || nm == "S" || nm == "SDG" ||
        nm == "T" || nm == "TDG") {
        if (!need(1, false)) return FHS_EPARSE;
        k = 1;
    } else if (nm == "P" || nm == "RX" || nm == "RY" || nm == "RZ") {
        if (!need(1, true)) return FHS_EPARSE;
        k = 1;
    } else if (nm == "CX" || nm == "CZ" || nm == "SWAP") {
        if (!need(2, false)) return FHS_EPARSE;
        k = 2;
    } else if (nm == "CP" || nm == "RZZ") {
        if (!need(2, true)) return FHS_EPARSE;
        k = 2;
    } else if (nm == "CCX" || nm == "CSWAP") {
        if (!need(3, false)) return FHS_EPARSE;
        k = 3;
    } else {
        return FHS_EUNSUPPORTED;
    }
    g.k = k;
    for (auto &row : g.m)
        for (auto &x : row) x = 0.0;
    const double a = g.angle;
    auto bit = [](int x, int j) { return (x >> j) & 1; };
    if (nm == "H") {
        g.m[0][0] = h; g.m[0][1] = h; g.m[1][0] = h; g.m[1][1] = -h;
    } else if (nm == "X") {
        g.m[0][1] = 1.0; g.m[1][0] = 1.0;
    } else if (nm == "Y") {
        g.m[0][1] = cd(0, -1); g.m[1][0] = cd(0, 1);
    } else if (nm == "Z") {
        g.m[0][0] = 1.0; g.m[1][1] = -1.0;
    } else if (nm == "S") {
        g.m[0][0] = 1.0; g.m[1][1] = cd(0, 1);
    } else if (nm == "SDG") {
        g.m[0][0] = 1.0; g.m[1][1] = cd(0, -1);
    } else if (nm == "T") {
        g.m[0][0] = 1.0; g.m[1][1] = cd(h, h);
    } else if (nm == "TDG") {
        g.m[0][0] = 1.0; g.m[1][1] = cd(h, -h);
    } else if (nm == "P") {
        g.m[0][0] = 1.0; g.m[1][1] = cd(std::cos(a), std::sin(a));
    } else if (nm == "RX" || nm == "RY" || nm == "RZ") {
        const double c = std::cos(0.5 * a), s = std::sin(0.5 * a);
        if (nm == "RX") {
            g.m[0][0] = c; g.m[1][1] = c; g.m[0][1] = cd(0, -s); g.m[1][0] = cd(0, -s);
        } else if (nm == "RY") {
            g.m[0][0] = c; g.m[1][1] = c; g.m[0][1] = -s; g.m[1][0] = s;
        } else {
            g.m[0][0] = cd(c, -s); g.m[1][1] = cd(c, s);
        }
    } else if (nm == "CZ") {
        for (int x = 0; x < 4; ++x) g.m[x][x] = (x == 3) ? -1.0 : 1.0;
    } else if (nm == "CP") {
        for (int x = 0; x < 3; ++x) g.m[x][x] = 1.0;
        g.m[3][3] = cd(std::cos(a), std::sin(a));
    } else if (nm == "RZZ") {
        const double c = std::cos(0.5 * a), s = std::sin(0.5 * a);
        for (int x = 0; x < 4; ++x) g.m[x][x] = (bit(x, 0) ^ bit(x, 1)) ? cd(c, s) : cd(c, -s);
    } else {
        for (int x = 0; x < (1 << k); ++x) {
            int y = x;
            if (nm == "CX" && bit(x, 0)) y = x ^ 2;
            if (nm == "SWAP") y = (bit(x, 0) << 1) | bit(x, 1);
            if (nm == "CCX" && bit(x, 0) && bit(x, 1)) y = x ^ 4;
            if (nm == "CSWAP" && bit(x, 0)) y = 1 | (bit(x, 2) << 1) | (bit(x, 1) << 2);
            g.m[y][x] = 1.0;
        }
    }
    return FHS_OK;
}

fhs_status parse(const char *text, size_t len, int &n, std::vector<Gate> &gates) {
    n = -1;
    size_t pos = 0;
    while (pos < len) {
        size_t end = pos;
        while (end < len && text[end] != '\n') ++end;
        std::string line(text + pos, end - pos);
        pos = end + 1;
        size_t hash = line.find('#');
        if (hash != std::string::npos) line.resize(hash);
        std::vector<std::string> tok;
        size_t i = 0;
        while (i < line.size()) {
            while (i < line.size() && std::isspace(static_cast<unsigned char>(line[i]))) ++i;
            size_t j = i;
            while (j < line.size() && !std::isspace(static_cast<unsigned char>(line[j]))) ++j;
            if (j > i) tok.emplace_back(line.substr(i, j - i));
            i = j;
        }
        if (tok.empty()) continue;
        if (tok[0] == "qubits") {
            if (tok.size() != 2 || n >= 0 || !all_digits(tok[1])) return FHS_EPARSE;
            long v = std::strtol(tok[1].c_str(), nullptr, 10);
            if (v < 1 || v > kMaxQubits) return FHS_ERANGE;
            n = static_cast<int>(v);
            continue;
        }
        if (n < 0) return FHS_EPARSE;
        Gate g;
        g.name = tok[0];
        for (size_t t = 1; t < tok.size(); ++t) {
            std::string s = tok[t];
            bool ng = false;
            if (!s.empty() && s[0] == '~') {
                ng = true;
                s = s.substr(1);
            }
            if (all_digits(s)) {
                long q = std::strtol(s.c_str(), nullptr, 10);
                if (q < 0 || q >= n) return FHS_ERANGE;
                for (int prev : g.q)
                    if (prev == q) return FHS_EPARSE;
                g.q.push_back(static_cast<int>(q));
                g.neg.push_back(ng ? 1 : 0);
            } else {
                if (ng || t != tok.size() - 1) return FHS_EPARSE;
                char *e = nullptr;
                double v = std::strtod(s.c_str(), &e);
                if (e == s.c_str() || *e != 0 || !std::isfinite(v)) return FHS_EPARSE;
                g.angle = v;
                g.has_angle = true;
            }
        }
        fhs_status st = build_matrix(g);
        if (st != FHS_OK) return st;
        gates.push_back(std::move(g));
        if (gates.size() >= (1u << 24)) return FHS_ERANGE;
    }
    if (n < 0) return FHS_EPARSE;
    return FHS_OK;
}

inline bool is_zero(const cd &z) { return z.real() == 0.0 && z.imag() == 0.0; }

// Role from the matrix (Section II-A): no off-diagonal nonzero -> wire-
// preserving, exactly one nonzero per column -> deterministic, else branching.
enum Role { R_PRESERVE = 0, R_DET = 1, R_BRANCH = 2 };

Role role_of(const Gate &g) {
    if (g.k == 0) return g.name == "MCX" ? R_DET : R_PRESERVE;
    const int dim = 1 << g.k;
    bool off = false, multi = false;
    for (int x = 0; x < dim; ++x) {
        int nz = 0;
        for (int y = 0; y < dim; ++y) {
            if (is_zero(g.m[y][x])) continue;
            ++nz;
            if (y != x) off = true;
        }
        if (nz > 1) multi = true;
    }
    if (!off) return R_PRESERVE;
    return multi ? R_BRANCH : R_DET;
}

// Local wire j keeps its value across the gate iff every nonzero transition
// has the same bit j on both sides (diagonal gates, control roles).
bool preserves(const Gate &g, int j) {
    if (g.k == 0) return g.name == "MCZ" || j != 0;
    const int dim = 1 << g.k;
    for (int x = 0; x < dim; ++x)
        for (int y = 0; y < dim; ++y)
            if (!is_zero(g.m[y][x]) && (((x ^ y) >> j) & 1)) return false;
    return true;
}

inline void set_bit(uint32_t *w, int q) { w[q >> 5] |= 1u << (q & 31); }

double modulus1(const cd &z) {
    const double re = z.real(), im = z.imag();
    const double m = std::sqrt(re * re + im * im);
    return m > 1.0 ? 1.0 : m;
}

// Algorithmic FP64 flops of multiplying the running amplitude by one factor
// of this table: 0 if every entry is 0, +-1 or +-i, 2 if every entry is purely
// real or purely imaginary, 6 for a general complex multiply.
int flops_of(const std::vector<cd> &tab) {
    bool trivial = true, axis = true;
    for (const cd &z : tab) {
        const double re = z.real(), im = z.imag();
        const bool unit = (re == 0.0 && (im == 0.0 || im == 1.0 || im == -1.0)) ||
                          (im == 0.0 && (re == 1.0 || re == -1.0));
        if (!unit) trivial = false;
        if (re != 0.0 && im != 0.0) axis = false;
    }
    return trivial ? 0 : (axis ? 2 : 6);
}

// The gate as the placement analysis sees it (placement.hpp).
PlaceGate place_gate(const Gate &g) {
    PlaceGate pg;
    pg.q = g.q;
    pg.k = g.k ? g.k : static_cast<int>(g.q.size());
    for (int j = 0; j < pg.k; ++j) pg.preserve.push_back(preserves(g, j));
    const Role r = role_of(g);
    pg.branch = r == R_BRANCH;
    pg.det = r == R_DET;
    if (!pg.det) return pg;
    if (g.k == 0) {                        // MCX: target q[0]
        if (pg.k == 2) {
            pg.cnot = true;
            pg.jt = 0;
            pg.jc = 1;
            pg.cval = g.neg[1] ? 0 : 1;
        }
        return pg;
    }
    if (g.k != 2) return pg;
    if (pg.preserve[0] != pg.preserve[1]) {
        // one wire kept: a controlled flip of the other when the kept wire
        // has one value and nothing for the other value
        const int jc = pg.preserve[0] ? 0 : 1, jt = 1 - jc;
        int flips_for = -1;
        bool ok = true;
        for (int v = 0; v < 2 && ok; ++v) {
            const int x = v << jc;             // target 0
            const bool flip = !is_zero(g.m[x | (1 << jt)][x]);
            const bool stay = !is_zero(g.m[x][x]);
            if (flip == stay) ok = false;
            if (flip) flips_for = flips_for < 0 ? v : 2;
        }
        if (ok && (flips_for == 0 || flips_for == 1)) {
            pg.cnot = true;
            pg.jc = jc;
            pg.jt = jt;
            pg.cval = flips_for;
        }
        return pg;
    }
    bool sw = true;
    for (int x = 0; x < 4; ++x)
        for (int y = 0; y < 4; ++y) {
            const int t = ((x & 1) << 1) | ((x >> 1) & 1);
            if (is_zero(g.m[y][x]) != (y != t)) sw = false;
        }
    pg.swap = sw;
    return pg;
}

// plan (may be null): how each branching gate (time index) gets its input
// bit when the sources are placed by reachability, and the sources'
// evaluation positions; null: the backward sweep.
fhs_status emit(int n, const std::vector<Gate> &gates, HostProgram &P,
                const std::vector<BranchInput> *plan = nullptr,
                const std::vector<uint32_t> *plan_src = nullptr) {
    const int G = static_cast<int>(gates.size());
    P.n = n;
    P.G = G;
    P.W = (n + 63) / 64;
    P.NW = n <= 32 ? 1 : (n <= 64 ? 2 : 4);
    // first non-preserving gate on each wire, time order (-1: none)
    std::vector<int> first_np(n, -1);
    std::vector<Role> role(G);
    for (int t = 0; t < G; ++t) {
        const Gate &g = gates[t];
        role[t] = role_of(g);
        for (size_t j = 0; j < g.q.size(); ++j)
            if (!preserves(g, static_cast<int>(j)) && first_np[g.q[j]] < 0) first_np[g.q[j]] = t;
    }
    P.ins.assign(G, Instr{});
    P.role.assign(G, 0);
    P.fp_cost.assign(G, 0);
    P.int_cost.assign(G, 0);
    P.flush_cost.assign(G, 0);
    P.run_prev.assign(G, kNoPrev);
    P.fac.clear();
    P.src_eval.clear();
    P.final_before.assign(G + 1, Mask4{{0, 0, 0, 0}});
    P.fac_begin.assign(G + 1, 0);
    Mask4 fin{{0, 0, 0, 0}};
    for (int q = 0; q < n; ++q)
        if (first_np[q] < 0) set_bit(fin.w, q);   // wire never changes: b_out[q] must equal b_in[q]
    P.final_before[0] = fin;
    P.n_branch = 0;
    int A = 0;
    for (int e = 0; e < G; ++e) {
        const int t = G - 1 - e;
        const Gate &g = gates[t];
        Instr I{};
        uint32_t op = 0, qa = 0, qb = 0, zmask = 0;
        P.fac_begin[e] = static_cast<uint32_t>(P.fac.size());
        P.role[e] = static_cast<uint8_t>(role[t]);
        auto push_tab = [&](const std::vector<cd> &tab) {
            I.fac = static_cast<uint32_t>(P.fac.size());
            for (const cd &z : tab) {
                P.fac.push_back(z.real());
                P.fac.push_back(z.imag());
            }
            P.fp_cost[e] = static_cast<uint16_t>(flops_of(tab));
        };
        const std::string &nm = g.name;
        if (g.k == 0) {
            // MCX / MCZ: control masks with polarity
            const size_t c0 = (nm == "MCX") ? 1 : 0;
            for (size_t j = c0; j < g.q.size(); ++j) {
                set_bit(I.cm, g.q[j]);
                if (!g.neg[j]) set_bit(I.cv, g.q[j]);
            }
            if (nm == "MCX") {
                op = OP_PERM;
                qa = static_cast<uint32_t>(g.q[0]);
            } else {
                op = OP_MCPHASE;
            }
        } else if (role[t] == R_BRANCH) {
            if (g.k != 1) return FHS_EUNSUPPORTED;   // only single-qubit branching gates
            const int q = g.q[0];
            ++P.n_branch;
            std::vector<cd> tab;
            for (int o = 0; o < 2; ++o)
                for (int i = 0; i < 2; ++i) tab.push_back(g.m[o][i]);
            push_tab(tab);
            for (int o = 0; o < 2; ++o)
                for (int i = 0; i < 2; ++i) {
                    P.fac.push_back(modulus1(g.m[o][i]));
                    if (is_zero(g.m[o][i])) zmask |= 1u << (2 * o + i);
                }
            qa = static_cast<uint32_t>(q);
            if (plan) {
                const BranchInput &b = (*plan)[t];
                if (b.kind == BranchInput::NATURAL) {
                    op = OP_BRANCH_NAT;
                } else if (b.kind == BranchInput::SOURCE) {
                    op = OP_BRANCH_SRC;
                    I.k = static_cast<uint32_t>(b.source);
                } else {
                    // the input bit is an affine form: parity(h & S) on the
                    // device, the boundary part a per-pair constant bit
                    op = OP_BRANCH_AFF;
                    I.k = static_cast<uint32_t>(P.aff.size() / 9);
                    I.cm[0] = static_cast<uint32_t>(b.form.s);
                    I.cm[1] = static_cast<uint32_t>(b.form.s >> 32);
                    for (int w = 0; w < 4; ++w) P.aff.push_back(b.form.x[w]);
                    for (int w = 0; w < 4; ++w) P.aff.push_back(b.form.y[w]);
                    P.aff.push_back(b.form.c);
                }
            } else if (first_np[q] == t) {
                op = OP_BRANCH_NAT;          // input segment is natural: value from b_in
            } else {
                op = OP_BRANCH_SRC;          // artificial source k, numbered in sweep order
                I.k = static_cast<uint32_t>(A++);
                P.src_eval.push_back(static_cast<uint32_t>(e));
            }
        } else if (role[t] == R_PRESERVE) {
            if (g.k == 1) {
                op = OP_DIAG1;
                qa = static_cast<uint32_t>(g.q[0]);
                push_tab({g.m[0][0], g.m[1][1]});
            } else if (g.k == 2) {
                op = OP_DIAG2;
                qa = static_cast<uint32_t>(g.q[0]);
                qb = static_cast<uint32_t>(g.q[1]);
                push_tab({g.m[0][0], g.m[1][1], g.m[2][2], g.m[3][3]});
            } else {
                return FHS_EUNSUPPORTED;
            }
        } else {  // deterministic dense gate
            if (g.k == 1) {
                // anti-diagonal: out bit o comes from in bit 1-o with factor U[o][1-o]
                const bool plain = g.m[0][1] == cd(1.0, 0.0) && g.m[1][0] == cd(1.0, 0.0);
                qa = static_cast<uint32_t>(g.q[0]);
                if (plain) {
                    op = OP_PERM;
                } else {
                    op = OP_DET1;
                    push_tab({g.m[0][1], g.m[1][0]});
                }
            } else if (nm == "CX" || nm == "CCX") {
                op = OP_PERM;
                for (int j = 0; j < g.k - 1; ++j) {
                    set_bit(I.cm, g.q[j]);
                    set_bit(I.cv, g.q[j]);
                }
                qa = static_cast<uint32_t>(g.q[g.k - 1]);
            } else if (nm == "SWAP" || nm == "CSWAP") {
                op = OP_SWAP;
                if (nm == "CSWAP") {
                    set_bit(I.cm, g.q[0]);
                    set_bit(I.cv, g.q[0]);
                }
                qa = static_cast<uint32_t>(g.q[g.k - 2]);
                qb = static_cast<uint32_t>(g.q[g.k - 1]);
            } else {
                return FHS_EUNSUPPORTED;
            }
        }
        {
            // state-word indices carried by the opcode
            auto hiword = [](const uint32_t *m) {
                int w = 0;
                for (int j = 0; j < 4; ++j)
                    if (m[j]) w = j;
                return w;
            };
            const Op base = static_cast<Op>(op);
            int w1 = static_cast<int>(qa >> 5), w2 = static_cast<int>(qb >> 5);
            if (base == OP_PERM) {
                w2 = hiword(I.cm);
                I.k = 1u << (qa & 31);
            } else if (base == OP_MCPHASE) {
                w1 = hiword(I.cm);
                w2 = 0;
            } else if (base != OP_SWAP && base != OP_DIAG2) {
                w2 = 0;
            }
            const bool affine = base == OP_BRANCH_AFF;   // cm holds the source mask, not controls
            I.hdr = pack_hdr(op_code(base, w1, w2), qa, qb, zmask);
            // algorithmic int32 ops of one backward step (fhs_program_work)
            const int wspan = affine ? 1 : hiword(I.cm) + 1;
            int ops = 0;
            switch (base) {
                // the form: the history index masked, its popcount, the
                // pair's constant bit, the bit into the state
                case OP_BRANCH_AFF: ops = zmask ? 6 : 4; break;
                case OP_PERM: ops = (I.cm[0] | I.cm[1] | I.cm[2] | I.cm[3]) ? 3 * wspan + 1 : 1; break;
                case OP_MCPHASE: ops = 3 * wspan + 1; break;
                case OP_SWAP: ops = (I.cm[0] | I.cm[1] | I.cm[2] | I.cm[3]) ? 3 * wspan + 4 : 4; break;
                case OP_DIAG1: ops = 1; break;
                case OP_DIAG2: ops = 3; break;
                case OP_DET1: ops = 2; break;
                // branching: the source (or input) bit into the state; forming
                // the table index and testing it for a zero entry only when
                // the gate has zero entries (the factor itself takes the index
                // where the multiply is made)
                default: ops = zmask ? 3 : 1; break;
            }
            P.int_cost[e] = static_cast<uint16_t>(ops);
        }
        P.ins[e] = I;
        // bits whose natural input segment starts right below this gate
        for (size_t j = 0; j < g.q.size(); ++j)
            if (first_np[g.q[j]] == t) set_bit(fin.w, g.q[j]);
        P.final_before[e + 1] = fin;
    }
    P.fac_begin[G] = static_cast<uint32_t>(P.fac.size());
    // A branching gate whose four entries are real, nonzero and of one
    // magnitude (H) multiplies every history by that magnitude: the product
    // of those magnitudes over a region is one constant for every history,
    // and per history only the entry's sign remains (no flops).
    for (int e = 0; e < G; ++e) {
        const int base = op_base(static_cast<uint8_t>(P.ins[e].hdr & 0xffu));
        if ((base != OP_BRANCH_SRC && base != OP_BRANCH_NAT) || (P.ins[e].hdr >> 24)) continue;
        const double *t = P.fac.data() + P.ins[e].fac;
        bool real = t[0] != 0.0;
        for (int x = 0; x < 4; ++x) real = real && t[2 * x + 1] == 0.0 && std::fabs(t[2 * x]) == std::fabs(t[0]);
        if (real) P.fp_cost[e] = 0;
    }
    if (plan) {
        P.src_eval = *plan_src;
        A = static_cast<int>(P.src_eval.size());
    }
    P.A = A;
    P.L = A > 0 ? static_cast<int>(P.src_eval[0]) : G;
    // a cut between an affine input and a source its form uses whose own
    // gate lies deeper would leave the form without that source
    P.cut_ok.assign(G + 1, 1);
    for (int e = 0; e < G; ++e) {
        const Instr &I = P.ins[e];
        if (op_base(static_cast<uint8_t>(I.hdr & 0xffu)) != OP_BRANCH_AFF) continue;
        const uint64_t smask = I.cm[0] | (static_cast<uint64_t>(I.cm[1]) << 32);
        for (int k = 0; k < A; ++k)
            if ((smask >> k) & 1u)
                for (uint32_t c = static_cast<uint32_t>(e) + 1; c <= P.src_eval[k]; ++c) P.cut_ok[c] = 0;
    }
    // the gates before the first source run once per pair, without sources
    if (!P.cut_ok[P.L]) P.L = 0;
    return FHS_OK;
}

inline bool test_bit(const uint32_t *w, uint32_t q) { return (w[q >> 5] >> (q & 31)) & 1u; }

// Fold ladders of controlled X gates that add or subtract one on a block of
// consecutive qubits into one OP_ADD.  In evaluation order the
// ladder reads (j = 0 .. m-1): X on bit lo+j under the common controls K and
// the controls bits lo .. lo+j-1, all of one polarity v.  Walking backward,
// bit lo+j flips iff K holds and bits lo .. lo+j-1 all equal v after their
// own flips, i.e. iff they all equalled 1-v before: the ladder subtracts one
// from the m-bit field when v = 1 and adds one when v = 0, mod 2^m (one
// OP_ADD, the sign in zmask bit 0; an incrementer built this way is a standard
// reversible-arithmetic circuit).  The folded gates stay in place as OP_NOP,
// so every evaluation position, cut, source index, final-bit mask and Eq. (8)
// count is unchanged; only the work per history drops.
void fuse_ladders(HostProgram &P) {
    const int G = P.G;
    P.n_fused = 0;
    for (int e = 0; e < G;) {
        const Instr &I0 = P.ins[e];
        if (static_cast<Op>(op_base(I0.hdr & 0xffu)) != OP_PERM) {
            ++e;
            continue;
        }
        const uint32_t lo = (I0.hdr >> 8) & 0xffu;
        int m = 1;
        int v = -1;
        while (e + m < G && lo + m < static_cast<uint32_t>(P.n)) {
            const Instr &J = P.ins[e + m];
            if (static_cast<Op>(op_base(J.hdr & 0xffu)) != OP_PERM) break;
            if (((J.hdr >> 8) & 0xffu) != lo + m) break;
            const uint32_t prev = lo + m - 1;      // the new control, bit lo+m-1
            if (!test_bit(J.cm, prev)) break;
            const int pol = test_bit(J.cv, prev) ? 1 : 0;
            if (v >= 0 && pol != v) break;
            // J's controls = I0's controls + bits lo .. lo+m-1 of polarity pol
            bool same = true;
            for (int w = 0; w < 4 && same; ++w) {
                uint32_t field = 0;
                for (uint32_t b = lo; b < lo + static_cast<uint32_t>(m); ++b)
                    if ((b >> 5) == static_cast<uint32_t>(w)) field |= 1u << (b & 31);
                same = J.cm[w] == (I0.cm[w] | field) &&
                       J.cv[w] == (I0.cv[w] | (pol ? field : 0u)) && (I0.cm[w] & field) == 0u;
            }
            if (!same) break;
            v = pol;
            ++m;
        }
        if (m < 2) {
            ++e;
            continue;
        }
        // common controls must not touch the field
        bool clean = true;
        for (uint32_t b = lo; b < lo + static_cast<uint32_t>(m); ++b)
            if (test_bit(I0.cm, b)) clean = false;
        if (!clean) {
            ++e;
            continue;
        }
        Instr A = I0;
        int wspan = 0;
        for (int w = 0; w < 4; ++w)
            if (A.cm[w]) wspan = w;
        A.k = 0;
        A.hdr = pack_hdr(op_code(OP_ADD, wspan, 0), lo, static_cast<uint32_t>(m), v == 1 ? 1u : 0u);
        P.ins[e] = A;
        const int wfield = static_cast<int>(((lo + m - 1) >> 5) - (lo >> 5)) + 1;
        const bool any = (A.cm[0] | A.cm[1] | A.cm[2] | A.cm[3]) != 0u;
        // the step: control test (none without controls) and the masked add of
        // its +-1 to the run's count; the run's carry chain and merge are
        // counted once (flush_cost)
        P.int_cost[e] = static_cast<uint16_t>((any ? 3 * (wspan + 1) + 1 : 0) + 1);
        P.flush_cost[e] = static_cast<uint16_t>(3 * wfield);
        for (int j = 1; j < m; ++j) {
            Instr N{};
            N.hdr = pack_hdr(op_code(OP_NOP, 0, 0), 0, 0, 0);
            P.ins[e + j] = N;
            P.int_cost[e + j] = 0;
            P.flush_cost[e + j] = 0;
        }
        ++P.n_fused;
        e += m;
    }
}

// Pair folded ladders: two OP_ADDs on the same field [lo, lo+m), adjacent in
// evaluation order (only folded gates between them), whose controls have the
// same mask and differ in the value of exactly one bit k, which lies outside
// the field.  At most one of them applies to a history, and neither changes
// a bit the other tests, so their composition is one OP_ADDSEL: add or
// subtract one according to bit k under the common controls.  This is the
// shift of a coined walk (one direction per coin value, Section V), and of
// any controlled add-or-subtract.  The second ladder's position becomes an
// OP_NOP: positions, sources, final-bit masks and Eq. (8) stay as they were;
// a cut inside the pair runs the whole pair in the region where it starts,
// as for a single ladder, which is sound because the pair changes field bits
// only and no field bit can be final before the pair's last gate.
void pair_ladders(HostProgram &P) {
    const int G = P.G;
    P.n_paired = 0;
    auto hiword = [](const uint32_t *m) {
        int w = 0;
        for (int j = 0; j < 4; ++j)
            if (m[j]) w = j;
        return w;
    };
    for (int e = 0; e < G; ++e) {
        const Instr &I1 = P.ins[e];
        if (static_cast<Op>(op_base(I1.hdr & 0xffu)) != OP_ADD) continue;
        int e2 = e + 1;
        while (e2 < G && static_cast<Op>(op_base(P.ins[e2].hdr & 0xffu)) == OP_NOP) ++e2;
        if (e2 >= G) break;
        const Instr &I2 = P.ins[e2];
        if (static_cast<Op>(op_base(I2.hdr & 0xffu)) != OP_ADD) continue;
        const uint32_t lo = (I1.hdr >> 8) & 0xffu, m = (I1.hdr >> 16) & 0xffu;
        if (((I2.hdr >> 8) & 0xffu) != lo || ((I2.hdr >> 16) & 0xffu) != m) continue;
        int nd = 0, q = -1;
        bool same_mask = true;
        for (int w = 0; w < 4; ++w) {
            same_mask = same_mask && I1.cm[w] == I2.cm[w];
            const uint32_t x = I1.cv[w] ^ I2.cv[w];
            nd += __builtin_popcount(x);
            if (x) q = 32 * w + __builtin_ctz(x);
        }
        if (!same_mask || nd != 1) continue;
        if (static_cast<uint32_t>(q) >= lo && static_cast<uint32_t>(q) < lo + m) continue;
        const uint32_t s1 = (I1.hdr >> 24) & 1u, s2 = (I2.hdr >> 24) & 1u;
        const bool q1 = test_bit(I1.cv, static_cast<uint32_t>(q));   // I1 applies when bit q == q1
        const uint32_t z = q1 ? (s2 | (s1 << 1)) : (s1 | (s2 << 1));
        Instr A = I1;
        A.cm[q >> 5] &= ~(1u << (q & 31));
        A.cv[q >> 5] &= ~(1u << (q & 31));
        A.k = static_cast<uint32_t>(q);
        const bool any = (A.cm[0] | A.cm[1] | A.cm[2] | A.cm[3]) != 0u;
        const int wspan = hiword(A.cm);
        A.hdr = pack_hdr(op_code(OP_ADDSEL, wspan, q >> 5), lo, m, z);
        P.ins[e] = A;
        const int wfield = static_cast<int>(((lo + m - 1) >> 5) - (lo >> 5)) + 1;
        // the step: control test, the selecting bit's extraction and its add to
        // the run's count (the sign is a compile-time constant); the run's
        // carry chain and merge are counted once (flush_cost)
        P.int_cost[e] = static_cast<uint16_t>((any ? 3 * (wspan + 1) + 1 : 0) + 2);
        P.flush_cost[e] = static_cast<uint16_t>(3 * wfield);
        Instr N{};
        N.hdr = pack_hdr(op_code(OP_NOP, 0, 0), 0, 0, 0);
        P.ins[e2] = N;
        P.int_cost[e2] = 0;
        P.flush_cost[e2] = 0;
        ++P.n_paired;
        e = e2;
    }
}

// Runs of folded-ladder steps on one field with nothing touching the field
// in between (ends_field_run): the compiled regions accumulate such a run and
// apply it with one carry chain, so each step records the previous step of
// its run (run_prev) and a range's work counts one carry chain per run that
// starts inside it.  A run still pending at the end of the program, on a
// field the final check compares whole, costs a compare of its step count
// with the field's residue instead (kCheckCost).
void set_field_runs(HostProgram &P) {
    bool pending = false;
    uint32_t lo = 0, hi = 0, last = kNoPrev;
    for (int e = 0; e < P.G; ++e) {
        const Instr &I = P.ins[e];
        const int base = op_base(static_cast<uint8_t>(I.hdr & 0xffu));
        if (base == OP_NOP) continue;
        if (pending && ends_field_run(I, lo, hi)) pending = false;
        if (base == OP_ADD || base == OP_ADDSEL) {
            const uint32_t a = (I.hdr >> 8) & 0xffu, b = (I.hdr >> 16) & 0xffu;
            P.run_prev[e] = pending ? last : kNoPrev;
            pending = true;
            lo = a;
            hi = a + b;
            last = static_cast<uint32_t>(e);
        }
    }
    P.tail_last = pending ? last : kNoPrev;
    P.tail_checked = false;
    if (pending) {
        const Mask4 &fin = P.final_before[P.G];
        bool covered = true;
        for (uint32_t q = lo; q < hi; ++q) covered = covered && ((fin.w[q >> 5] >> (q & 31u)) & 1u);
        P.tail_checked = covered;
    }
}

constexpr uint64_t kCheckCost = 2;   // n = pk + 2 pb, and one compare

constexpr uint64_t kPopcountCost = 2;   // the source index masked, its popcount

// Algorithmic int32 ops of evaluation positions [lo, hi) for one history.
// A paired ladder step without controls whose selecting bit holds a source
// bit set earlier in the range (SourceBits) adds a constant plus that bit
// with a fixed sign: such steps cost nothing each, and their run pays one
// popcount of the source index per sign that occurs.
// Work of [lo, hi) per history; *uniform (may be null) receives the part
// whose inputs are only this range's own source bits (and constants): a
// source bit written into the state, a popcount of the source index, and
// operations on state bits that hold nothing else.  That part is the same
// for every history that shares the range's source assignment, whatever
// came before the range.
uint64_t range_int_ops(const HostProgram &P, uint32_t lo, uint32_t hi, uint64_t *uniform = nullptr) {
    uint64_t ops = 0, uni = 0;
    SourceBits sb;
    bool pos_used = false, neg_used = false;
    // state bits whose value is a function of this range's source bits alone
    std::vector<uint8_t> src_only(kMaxQubits, 0);
    auto bits_of = [](const uint32_t (&m)[4], auto &&f) {
        for (int q = 0; q < kMaxQubits; ++q)
            if ((m[q >> 5] >> (q & 31)) & 1u) f(q);
    };
    for (uint32_t e = lo; e < hi; ++e) {
        const Instr &I = P.ins[e];
        const int base = op_base(static_cast<uint8_t>(I.hdr & 0xffu));
        const bool starts_run = P.flush_cost[e] && (P.run_prev[e] == kNoPrev || P.run_prev[e] < lo);
        if (starts_run) pos_used = neg_used = false;
        const int j = sb.selector_source(I);
        sb.step(I, 0);
        uint32_t touched[4], written[4];
        touched_bits(I, touched);
        written_bits(I, written);
        if (j >= 0) {
            const uint32_t z = I.hdr >> 24;
            const int d0 = (z & 1u) ? -1 : 1, d1 = (z & 2u) ? -1 : 1;
            bool &used = d1 > d0 ? pos_used : neg_used;
            if (d1 != d0 && !used) {
                ops += kPopcountCost;
                uni += kPopcountCost;   // the source index alone
                used = true;
            }
            bits_of(written, [&](int q) { src_only[q] = 0; });   // the field: the count joins its old value
        } else {
            bool only = true;   // inputs: this range's sources and source-only bits
            if (base == OP_BRANCH_SRC) {
                only = P.int_cost[e] == 1u || src_only[(I.hdr >> 8) & 0xffu];   // with zero entries it reads o
                bits_of(written, [&](int q) { src_only[q] = 1; });
            } else if (base == OP_BRANCH_NAT || base == OP_BRANCH_AFF) {
                only = false;   // the input bitstring, or forms over the boundary bits
                bits_of(written, [&](int q) { src_only[q] = 0; });
            } else {
                bits_of(touched, [&](int q) { only = only && src_only[q]; });
                bits_of(written, [&](int q) { src_only[q] = only ? 1 : 0; });
            }
            ops += P.int_cost[e];
            if (only) uni += P.int_cost[e];
        }
        if (starts_run) ops += P.flush_cost[e];
    }
    // a range that reaches the final check: the run pending there, from its
    // first step inside the range, is compared instead of applied
    if (hi == static_cast<uint32_t>(P.G) && P.tail_checked && P.tail_last >= lo) {
        uint32_t f = P.tail_last;
        while (P.run_prev[f] != kNoPrev && P.run_prev[f] >= lo) f = P.run_prev[f];
        ops = ops - P.flush_cost[f] + kCheckCost;
    }
    if (uniform) *uniform = uni;
    return ops;
}

// Work of the suffix instructions [lo, hi) the compiled consumer evaluates
// once per root history instead of once per leaf (hoistable, without
// pruning): their integer ops and FP64 flops per evaluation.
void hoisted_work(const HostProgram &P, uint32_t lo, uint32_t hi, uint64_t &iops, uint64_t &flops) {
    iops = flops = 0;
    const std::vector<uint8_t> h = hoistable(P.ins, lo, hi, false);
    for (uint32_t e = lo; e < hi; ++e)
        if (h[e - lo]) {
            iops += P.int_cost[e];
            flops += P.fp_cost[e];
        }
}

// Runs of identical opcodes: the device dispatches once per run.
void set_runs(HostProgram &P) {
    const int G = P.G;
    for (int e = G - 1; e >= 0; --e)
        P.ins[e].run = (e + 1 < G && (P.ins[e + 1].hdr & 0xffu) == (P.ins[e].hdr & 0xffu))
                           ? P.ins[e + 1].run + 1 : 1;
}

void region_sources(const HostProgram &P, uint32_t c1, uint32_t c2, uint32_t out[3]) {
    out[0] = out[1] = out[2] = 0;
    for (uint32_t e : P.src_eval) out[e < c1 ? 0 : (e < c2 ? 1 : 2)]++;
}

unsigned __int128 eq8(uint32_t Ap, uint32_t Ar, uint32_t As, uint64_t Gp, uint64_t Gr,
                      uint64_t Gs) {
    using u128 = unsigned __int128;
    const u128 inner = static_cast<u128>(Gr) + (static_cast<u128>(1) << As) * Gs;
    return (static_cast<u128>(1) << Ap) * (static_cast<u128>(Gp) + (static_cast<u128>(1) << Ar) * inner);
}

}  // namespace
}  // namespace fhs

using namespace fhs;

extern "C" const char *fhs_status_string(fhs_status s) {
    switch (s) {
        case FHS_OK: return "ok";
        case FHS_EINVAL: return "invalid argument";
        case FHS_EUNSUPPORTED: return "unsupported";
        case FHS_ERANGE: return "out of range";
        case FHS_ENOMEM: return "out of memory";
        case FHS_EHIP: return "HIP error";
        case FHS_ESTATE: return "wrong call order";
        case FHS_EPARSE: return "parse error";
    }
    return "unknown status";
}

extern "C" fhs_status fhs_reduce_ex(const char *text, size_t len, uint32_t flags,
                                    fhs_program **out) {
    const uint32_t all = FHS_REDUCE_FUSE | FHS_REDUCE_PAIR | FHS_REDUCE_FORWARD | FHS_REDUCE_OPTIMAL |
                         FHS_REDUCE_GREEDY;
    const uint32_t reach = flags & (FHS_REDUCE_OPTIMAL | FHS_REDUCE_GREEDY);
    if (!text || !out || (flags & ~all) || ((flags & FHS_REDUCE_PAIR) && !(flags & FHS_REDUCE_FUSE)) ||
        reach == (FHS_REDUCE_OPTIMAL | FHS_REDUCE_GREEDY) || (reach && (flags & FHS_REDUCE_FORWARD)))
        return FHS_EINVAL;
    *out = nullptr;
    int n = 0;
    std::vector<Gate> gates;
    fhs_status st = parse(text, len, n, gates);
    if (st != FHS_OK) return st;
    if (flags & FHS_REDUCE_FORWARD) {
        // <b_out|C|b_in> = <b_in|C^T|b_out>: the forward sweep over C is the
        // backward sweep over the transpose, whose gates are C's in reverse
        // order with transposed matrices (MCX and MCZ are symmetric); its
        // natural input segments are C's natural output segments
        std::reverse(gates.begin(), gates.end());
        for (Gate &g : gates)
            for (int a = 0; a < (1 << g.k); ++a)
                for (int b = 0; b < a; ++b) std::swap(g.m[a][b], g.m[b][a]);
    }
    std::vector<BranchInput> plan;
    std::vector<uint32_t> plan_src;
    if (reach) {
        std::vector<PlaceGate> pg;
        pg.reserve(gates.size());
        for (const Gate &g : gates) pg.push_back(place_gate(g));
        st = place_by_reach(n, pg, (flags & FHS_REDUCE_GREEDY) != 0, plan, plan_src);
        if (st != FHS_OK) return st;
    }
    fhs_program *p = new (std::nothrow) fhs_program;
    if (!p) return FHS_ENOMEM;
    st = emit(n, gates, p->p, reach ? &plan : nullptr, reach ? &plan_src : nullptr);
    p->p.forward = (flags & FHS_REDUCE_FORWARD) != 0;
    p->p.placement = (flags & FHS_REDUCE_OPTIMAL) ? 1 : ((flags & FHS_REDUCE_GREEDY) ? 2 : 0);
    if (st != FHS_OK) {
        delete p;
        return st;
    }
    if (flags & FHS_REDUCE_FUSE) fuse_ladders(p->p);
    if (flags & FHS_REDUCE_PAIR) pair_ladders(p->p);
    set_field_runs(p->p);
    set_runs(p->p);
    *out = p;
    return FHS_OK;
}

extern "C" fhs_status fhs_reduce(const char *text, size_t len, fhs_program **out) {
    return fhs_reduce_ex(text, len, FHS_REDUCE_FUSE | FHS_REDUCE_PAIR, out);
}

extern "C" void fhs_program_free(fhs_program *prog) { delete prog; }

extern "C" fhs_status fhs_program_get_info(const fhs_program *prog, fhs_program_info *info) {
    if (!prog || !info) return FHS_EINVAL;
    const HostProgram &P = prog->p;
    info->n_qubits = static_cast<uint32_t>(P.n);
    info->n_gates = static_cast<uint32_t>(P.G);
    info->n_sources = static_cast<uint32_t>(P.A);
    info->n_words = static_cast<uint32_t>(P.W);
    info->n_leading = static_cast<uint32_t>(P.L);
    info->n_branch = static_cast<uint32_t>(P.n_branch);
    info->forward = P.forward ? 1u : 0u;
    return FHS_OK;
}

extern "C" fhs_status fhs_program_sources(const fhs_program *prog, uint32_t *eval_pos, uint32_t cap) {
    if (!prog || (!eval_pos && cap)) return FHS_EINVAL;
    const HostProgram &P = prog->p;
    for (uint32_t k = 0; k < cap && k < P.src_eval.size(); ++k) eval_pos[k] = P.src_eval[k];
    return FHS_OK;
}

extern "C" fhs_status fhs_cut_allowed(const fhs_program *prog, uint32_t c, int *allowed) {
    if (!prog || !allowed) return FHS_EINVAL;
    if (c > static_cast<uint32_t>(prog->p.G)) return FHS_EINVAL;
    *allowed = cut_allowed(prog->p, c) ? 1 : 0;
    return FHS_OK;
}

extern "C" fhs_status fhs_partition_cost(const fhs_program *prog, uint32_t c1, uint32_t c2,
                                         uint64_t cost[2], uint32_t *regions) {
    if (!prog || !cost) return FHS_EINVAL;
    const HostProgram &P = prog->p;
    if (c1 > c2 || c2 > static_cast<uint32_t>(P.G)) return FHS_EINVAL;
    if (P.A > 100) return FHS_ERANGE;
    uint32_t a3[3];
    region_sources(P, c1, c2, a3);
    const unsigned __int128 v = eq8(a3[0], a3[1], a3[2], c1, c2 - c1, P.G - c2);
    cost[0] = static_cast<uint64_t>(v);
    cost[1] = static_cast<uint64_t>(v >> 64);
    if (regions) {
        regions[0] = c1; regions[1] = c2 - c1; regions[2] = P.G - c2;
        regions[3] = a3[0]; regions[4] = a3[1]; regions[5] = a3[2];
    }
    return FHS_OK;
}

extern "C" fhs_status fhs_program_work(const fhs_program *prog, uint32_t e0, uint32_t e1,
                                       fhs_work *out) {
    if (!prog || !out) return FHS_EINVAL;
    const HostProgram &P = prog->p;
    if (e0 > e1 || e1 > static_cast<uint32_t>(P.G)) return FHS_EINVAL;
    fhs_work w{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t e = e0; e < e1; ++e) {
        w.gates += 1;
        w.fp64_flops += P.fp_cost[e];
        w.branch += P.role[e] == 2 ? 1 : 0;
    }
    w.int_ops = range_int_ops(P, e0, e1, &w.src_int_ops);
    hoisted_work(P, e0, e1, w.hoist_int_ops, w.hoist_fp64_flops);
    // the two-valued gates' counted form (the compiled consumer without pruning)
    const std::vector<uint8_t> h = hoistable(P.ins, e0, e1, false);
    for (uint32_t e = e0; e < e1; ++e) {
        if (!two_valued(P.ins[e], P.fac).ok) continue;
        const int base = op_base(static_cast<uint8_t>(P.ins[e].hdr & 0xffu));
        const uint64_t add = (base == OP_BRANCH_SRC || base == OP_BRANCH_NAT) ? 2u : 1u;
        w.count_int_ops += add;
        w.count_fp64_flops += P.fp_cost[e];
        if (h[e - e0]) {
            w.hoist_count_int_ops += add;
            w.hoist_count_fp64_flops += P.fp_cost[e];
        }
    }
    *out = w;
    return FHS_OK;
}

extern "C" fhs_status fhs_split_features(const fhs_program *prog, uint32_t c1, uint32_t c2,
                                         uint32_t M, uint32_t S, double *f) {
    if (!prog || !f) return FHS_EINVAL;
    const HostProgram &P = prog->p;
    const uint32_t G = static_cast<uint32_t>(P.G);
    if (c1 > c2 || c2 > G) return FHS_EINVAL;
    if (P.A > 100) return FHS_ERANGE;
    const uint32_t L = static_cast<uint32_t>(P.L);
    const uint32_t e1 = std::max(c1, L), e2 = std::max(c2, L);
    uint32_t a3[3];
    region_sources(P, c1, c2, a3);
    auto work = [&](uint32_t lo, uint32_t hi, double &iops, double &flops) {
        flops = 0.0;
        for (uint32_t e = lo; e < hi; ++e) flops += P.fp_cost[e];
        iops = static_cast<double>(range_int_ops(P, lo, hi));
    };
    // instructions the device walks (folded gates excluded) and opcode runs
    // among them: the decode work, a first-order cost once ladders are folded
    auto decode = [&](uint32_t lo, uint32_t hi, double &ins, double &runs) {
        ins = runs = 0.0;
        uint32_t prev = 0xffffffffu;
        for (uint32_t e = lo; e < hi; ++e) {
            const uint32_t op = P.ins[e].hdr & 0xffu;
            if (op_base(op) == OP_NOP) continue;
            ins += 1.0;
            if (op != prev) runs += 1.0;
            prev = op;
        }
    };
    double ip, fp, ir, fr, is, fs, dp, rp, dr, rr, ds, rs;
    work(L, e1, ip, fp);
    work(e1, e2, ir, fr);
    work(e2, G, is, fs);
    // the suffix instructions the consumer evaluates once per root history
    uint64_t hi_ops = 0, hi_fl = 0;
    hoisted_work(P, e2, G, hi_ops, hi_fl);
    ir += static_cast<double>(hi_ops);
    fr += static_cast<double>(hi_fl);
    is -= static_cast<double>(hi_ops);
    fs -= static_cast<double>(hi_fl);
    decode(L, e1, dp, rp);
    decode(e1, e2, dr, rr);
    decode(e2, G, ds, rs);
    const double np = std::ldexp(1.0, static_cast<int>(a3[0]));
    const double nr = std::ldexp(1.0, static_cast<int>(a3[0] + a3[1]));
    const double ns = std::ldexp(1.0, P.A);
    const double pairs = std::max(1.0, static_cast<double>(M) * static_cast<double>(S));
    const double entry = 4.0 * P.NW + 16.0 + 8.0 + 4.0;
    const unsigned __int128 e8 = eq8(a3[0], a3[1], a3[2], c1, c2 - c1, G - c2);
    f[0] = a3[0];
    f[1] = a3[1];
    f[2] = a3[2];
    f[3] = std::log2(1.0 + np * ip);
    f[4] = std::log2(1.0 + np * fp);
    f[5] = std::log2(1.0 + nr * ir);
    f[6] = std::log2(1.0 + nr * fr);
    f[7] = std::log2(1.0 + ns * is);
    f[8] = std::log2(1.0 + ns * fs);
    f[9] = a3[0] + std::log2(entry);
    f[10] = std::log2(pairs);
    f[11] = P.NW;
    f[12] = std::log2(1.0 + static_cast<double>(e8));
    f[13] = std::log2(pairs) + a3[0] + a3[1];
    f[14] = std::log2(1.0 + np * dp + nr * dr + ns * ds);
    f[15] = std::log2(1.0 + np * rp + nr * rr + ns * rs);
    return FHS_OK;
}

extern "C" fhs_status fhs_candidate_splits(const fhs_program *prog, uint32_t *c1, uint32_t *c2,
                                           uint32_t cap, uint32_t *count) {
    if (!prog || !count || ((!c1 || !c2) && cap)) return FHS_EINVAL;
    const HostProgram &P = prog->p;
    std::vector<uint32_t> cuts;
    for (uint32_t e : P.src_eval)
        if (cut_allowed(P, e)) cuts.push_back(e);
    cuts.push_back(static_cast<uint32_t>(P.G));
    uint32_t k = 0;
    for (size_t i = 0; i < cuts.size(); ++i)
        for (size_t j = i; j < cuts.size(); ++j) {
            if (k < cap) {
                c1[k] = cuts[i];
                c2[k] = cuts[j];
            }
            ++k;
        }
    *count = k;
    return FHS_OK;
}

extern "C" fhs_status fhs_choose_partition(const fhs_program *prog, int mode, uint32_t *c1,
                                           uint32_t *c2) {
    if (!prog || !c1 || !c2) return FHS_EINVAL;
    const HostProgram &P = prog->p;
    const uint32_t G = static_cast<uint32_t>(P.G);
    if (mode == FHS_PART_NONE) {
        *c1 = 0; *c2 = 0;
        return FHS_OK;
    }
    if (mode == FHS_PART_THIRDS) {
        uint32_t a = G / 3, b = (2 * G) / 3;
        while (!cut_allowed(P, a)) --a;      // position 0 is always allowed
        while (!cut_allowed(P, b)) --b;
        *c1 = a; *c2 = b;
        return FHS_OK;
    }
    if (mode != FHS_PART_EQ8) return mode == FHS_PART_MODEL ? FHS_ESTATE : FHS_EINVAL;
    if (P.A > 100) return FHS_ERANGE;
    // sources strictly before evaluation position e
    std::vector<uint32_t> before(G + 1, 0);
    for (uint32_t e : P.src_eval) before[e + 1]++;
    for (uint32_t e = 1; e <= G; ++e) before[e] += before[e - 1];
    unsigned __int128 best = 0;
    bool have = false;
    uint32_t b1 = 0, b2 = 0;
    const uint32_t A = static_cast<uint32_t>(P.A);
    for (uint32_t x = 0; x <= G; ++x)
        for (uint32_t y = x; y <= G; ++y) {
            if (!cut_allowed(P, x) || !cut_allowed(P, y)) continue;
            const uint32_t ap = before[x], ar = before[y] - before[x], as = A - before[y];
            const unsigned __int128 v = eq8(ap, ar, as, x, y - x, G - y);
            if (!have || v < best) {
                best = v; b1 = x; b2 = y; have = true;
            }
        }
    *c1 = b1; *c2 = b2;
    return FHS_OK;
}

// Internal accessors for the device side.
const fhs::HostProgram &fhs_program_host(const fhs_program *p) { return p->p; }
fhs_program *fhs_program_clone(const fhs_program *p) { return new (std::nothrow) fhs_program(*p); }
