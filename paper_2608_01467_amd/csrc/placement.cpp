// placement.cpp -- source placement by determinism reachability (see
// placement.hpp).
#include "placement.hpp"

#include <algorithm>

#include "../../include/fhs.h"

namespace fhs {
namespace {

// Internal-wire segments: one per (gate, local wire) where the gate does
// not preserve the wire's value, plus the n input segments 0..n-1.
struct Segments {
    std::vector<std::vector<int>> in, out;   // per gate, per local wire
    std::vector<int> out_q;                  // segment carrying each qubit at the output
    int nseg = 0;
};

Segments segments(int n, const std::vector<PlaceGate> &gates) {
    Segments S;
    std::vector<int> cur(n);
    for (int q = 0; q < n; ++q) cur[q] = q;
    int next = n;
    S.in.resize(gates.size());
    S.out.resize(gates.size());
    for (size_t t = 0; t < gates.size(); ++t) {
        const PlaceGate &g = gates[t];
        for (int j = 0; j < g.k; ++j) {
            const int q = g.q[j];
            S.in[t].push_back(cur[q]);
            const int o = g.preserve[j] ? cur[q] : next++;
            S.out[t].push_back(o);
            cur[q] = o;
        }
    }
    S.out_q = cur;
    S.nseg = next;
    return S;
}

// A relation between segments: a pair (b = a ^ k) or a CNOT triple
// (out = in ^ control ^ k); for reachability any two of a triple fix the third.
struct Relation {
    bool triple;
    int a, b, c;     // pair: a, b; triple: control a, target in b, target out c
    uint32_t k;
};

fhs_status relations(const std::vector<PlaceGate> &gates, const Segments &S, std::vector<Relation> &rel) {
    for (size_t t = 0; t < gates.size(); ++t) {
        const PlaceGate &g = gates[t];
        if (g.branch) {
            if (g.k != 1) return FHS_EUNSUPPORTED;
            continue;
        }
        if (!g.det) continue;   // wire-preserving
        if (g.k == 1) {
            rel.push_back({false, S.in[t][0], S.out[t][0], -1, 1u});   // a one-bit permutation flips
        } else if (g.cnot) {
            rel.push_back({true, S.in[t][g.jc], S.in[t][g.jt], S.out[t][g.jt], g.cval ? 0u : 1u});
        } else if (g.swap) {
            rel.push_back({false, S.in[t][0], S.out[t][1], -1, 0u});
            rel.push_back({false, S.in[t][1], S.out[t][0], -1, 0u});
        } else {
            return FHS_EUNSUPPORTED;
        }
    }
    return FHS_OK;
}

// Close `known` under the relations; returns the number of known segments.
int close(const std::vector<Relation> &rel, std::vector<uint8_t> &known) {
    bool changed = true;
    while (changed) {
        changed = false;
        for (const Relation &r : rel) {
            if (!r.triple) {
                if (known[r.a] != known[r.b]) {
                    known[r.a] = known[r.b] = 1;
                    changed = true;
                }
                continue;
            }
            const int nk = known[r.a] + known[r.b] + known[r.c];
            if (nk == 2) {
                known[r.a] = known[r.b] = known[r.c] = 1;
                changed = true;
            }
        }
    }
    int total = 0;
    for (uint8_t v : known) total += v;
    return total;
}

}  // namespace

fhs_status place_by_reach(int n, const std::vector<PlaceGate> &gates, bool greedy,
                          std::vector<BranchInput> &inputs, std::vector<uint32_t> &src_eval) {
    const int G = static_cast<int>(gates.size());
    const Segments S = segments(n, gates);
    std::vector<Relation> rel;
    fhs_status st = relations(gates, S, rel);
    if (st != FHS_OK) return st;
    // candidates: input segments of branching gates that are not input
    // segments, in evaluation order (from the output)
    std::vector<int> cand_seg, cand_gate;
    for (int t = G - 1; t >= 0; --t)
        if (gates[t].branch && S.in[t][0] >= n) {
            cand_seg.push_back(S.in[t][0]);
            cand_gate.push_back(t);
        }
    const int nc = static_cast<int>(cand_seg.size());
    std::vector<uint8_t> base(S.nseg, 0);
    for (int q = 0; q < n; ++q) base[q] = base[S.out_q[q]] = 1;
    auto reached = [&](const std::vector<int> &pick) {
        std::vector<uint8_t> known = base;
        for (int i : pick) known[cand_seg[i]] = 1;
        return close(rel, known);
    };
    std::vector<int> pick;
    if (greedy) {
        std::vector<uint8_t> used(nc, 0);
        while (reached(pick) < S.nseg) {
            int best = -1, best_n = -1;
            for (int i = 0; i < nc; ++i) {
                if (used[i]) continue;
                pick.push_back(i);
                const int m = reached(pick);
                pick.pop_back();
                if (m > best_n) {
                    best_n = m;
                    best = i;
                }
            }
            if (best < 0) return FHS_EUNSUPPORTED;
            used[best] = 1;
            pick.push_back(best);
        }
        std::sort(pick.begin(), pick.end());
    } else {
        // fewest candidates first; within a size, combinations in
        // lexicographic order of evaluation position
        long budget = 2000000;
        bool found = false;
        for (int k = 0; k <= nc && !found; ++k) {
            std::vector<int> c(k);
            for (int i = 0; i < k; ++i) c[i] = i;
            for (;;) {
                if (--budget < 0) return FHS_ERANGE;
                if (reached(c) == S.nseg) {
                    pick = c;
                    found = true;
                    break;
                }
                int i = k - 1;
                while (i >= 0 && c[i] == nc - k + i) --i;
                if (i < 0) break;
                ++c[i];
                for (int j = i + 1; j < k; ++j) c[j] = c[j - 1] + 1;
            }
        }
        if (!found) return FHS_EUNSUPPORTED;
    }
    if (static_cast<int>(pick.size()) > kMaxSources) return FHS_ERANGE;
    // symbolic values: boundary bits, then sources, propagated through the
    // relations until every segment has one
    std::vector<AffineForm> f(S.nseg);
    std::vector<uint8_t> known(S.nseg, 0);
    for (int q = 0; q < n; ++q) {
        f[q].x[q >> 5] |= 1u << (q & 31);
        known[q] = 1;
        const int o = S.out_q[q];
        if (!known[o]) {
            f[o].y[q >> 5] |= 1u << (q & 31);
            known[o] = 1;
        }
    }
    std::vector<int> src_of_seg(S.nseg, -1);
    src_eval.clear();
    for (size_t k = 0; k < pick.size(); ++k) {
        const int seg = cand_seg[pick[k]];
        f[seg] = AffineForm{};
        f[seg].s = 1ull << k;
        known[seg] = 1;
        src_of_seg[seg] = static_cast<int>(k);
        src_eval.push_back(static_cast<uint32_t>(G - 1 - cand_gate[pick[k]]));
    }
    bool changed = true;
    while (changed) {
        changed = false;
        for (const Relation &r : rel) {
            if (!r.triple) {
                if (known[r.a] && !known[r.b]) {
                    f[r.b] = f[r.a];
                    f[r.b].c ^= r.k;
                    known[r.b] = 1;
                    changed = true;
                } else if (known[r.b] && !known[r.a]) {
                    f[r.a] = f[r.b];
                    f[r.a].c ^= r.k;
                    known[r.a] = 1;
                    changed = true;
                }
                continue;
            }
            const int nk = known[r.a] + known[r.b] + known[r.c];
            if (nk != 2) continue;
            // the unknown one is the XOR of the other two and the constant
            const int miss = !known[r.a] ? r.a : (!known[r.b] ? r.b : r.c);
            AffineForm v;
            for (int s2 : {r.a, r.b, r.c})
                if (s2 != miss) v.add(f[s2]);
            v.c ^= r.k;
            f[miss] = v;
            known[miss] = 1;
            changed = true;
        }
    }
    inputs.assign(gates.size(), BranchInput{});
    for (int t = 0; t < G; ++t) {
        if (!gates[t].branch) continue;
        const int seg = S.in[t][0];
        BranchInput &b = inputs[t];
        if (seg < n) {
            b.kind = BranchInput::NATURAL;
        } else if (src_of_seg[seg] >= 0) {
            b.kind = BranchInput::SOURCE;
            b.source = src_of_seg[seg];
        } else {
            if (!known[seg]) return FHS_EUNSUPPORTED;   // cannot happen once every segment is reached
            b.kind = BranchInput::AFFINE;
            b.form = f[seg];
        }
    }
    return FHS_OK;
}

}  // namespace fhs
