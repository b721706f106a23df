// jit.hip -- generation and run-time compilation of the consumer for one
// program and split (see jit.hpp).
#include "jit.hpp"

#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>

#include "program.hpp"

namespace fhs {
namespace {

// device.hpp, kernels.hpp and program.hpp as text (written by the build).
#include "jit_headers.inc"

// A factor taken by a deferred multiply: its table offset and where its
// index sits in dx.
struct Deferred {
    uint32_t fac;
    int off, bits;
};

// Bits of dx a factor op records when deferred (0: no factor).
int factor_bits(int base) {
    switch (base) {
        case OP_BRANCH_SRC:
        case OP_BRANCH_NAT:
        case OP_BRANCH_AFF:
        case OP_DIAG2: return 2;
        case OP_DIAG1:
        case OP_DET1: return 1;
        default: return 0;
    }
}

// How a factor op of the compiled regions forms its factor when it is not
// deferred: from the gate's table as compile-time constants for the shapes
// the device has a step for (op_conj, op_branch_real), else by a per-lane
// table read.
struct FacShape {
    enum Kind { TABLE, CONJ, REAL } kind = TABLE;
    double C = 0.0, S = 0.0;    // CONJ: entry 0 = (C, S), the other = (C, -S)
    double r = 0.0, m = 0.0;    // REAL: magnitude and modulus of every entry
    uint32_t neg = 0;           // REAL: bit x set when entry x is negative
};

FacShape fac_shape(const Instr &I, const std::vector<double> &fac) {
    FacShape f;
    const int base = op_base(I.hdr & 0xffu);
    const double *t = fac.data() + I.fac;
    auto re = [&](int x) { return t[2 * x]; };
    auto im = [&](int x) { return t[2 * x + 1]; };
    auto conj_of = [&](int x, int y) { return re(x) == re(y) && im(x) == -im(y); };
    if (base == OP_DIAG1 && conj_of(0, 1)) {
        f.kind = FacShape::CONJ;
    } else if (base == OP_DIAG2 && re(0) == re(3) && im(0) == im(3) && re(1) == re(2) && im(1) == im(2) &&
               conj_of(0, 1)) {
        f.kind = FacShape::CONJ;
    } else if ((base == OP_BRANCH_SRC || base == OP_BRANCH_NAT) && (I.hdr >> 24) == 0u) {
        bool real = true;
        for (int x = 0; x < 4; ++x)
            real = real && im(x) == 0.0 && std::fabs(re(x)) == std::fabs(re(0)) && t[8 + x] == t[8];
        if (real && re(0) != 0.0) {
            f.kind = FacShape::REAL;
            f.r = std::fabs(re(0));
            f.m = t[8];
            for (int x = 0; x < 4; ++x)
                if (std::signbit(re(x))) f.neg |= 1u << x;
        }
    }
    if (f.kind == FacShape::CONJ) {
        f.C = re(0);
        f.S = im(0);
    }
    return f;
}

// The final field check of a suffix region (flush_check) when its residue is
// the same for every leaf of a root: the run's steps are all selected by
// source bits (a constant plus popcounts of the source index), and nothing
// in the region before the run writes the field.  Then whether a leaf can
// pass depends on the leaf only through the popcounts of its wave-uniform
// source bits, and the consumer can reject whole passes of leaves at once.
struct TailCheck {
    bool ok = false;
    uint32_t lo = 0, hi = 0;    // the field
    int32_t kc = 0;             // the run's constant steps
    std::vector<std::pair<uint64_t, uint64_t>> src;   // (pos, neg) source-bit masks
};

// One block per instruction: the instruction as a constant and the call of
// its backward step with the word indices its opcode carries (wsel maps them
// onto the state registers as the interpreter's dispatch does).  With
// `defer`, factor ops record their table index in dx instead of multiplying
// (the offsets are appended to `deferred`).  Folded and paired ladders on one
// field accumulate in the region's pk counters and are added to the field
// before the next instruction that touches it and at the region's end.  With
// `check` (the final-bit mask that follows the region), a run still pending
// at the end on a field that mask covers whole is compared with the output
// instead (flush_check); its field is returned in `checked`, for the final
// check to leave out.
// Instructions marked in `omit` (indexed from lo) are left out.
// With `defer`, a real-entry branch (FacShape REAL) records only its sign
// (op_branch_real_sign) and its magnitude joins *rdef, the product the valid
// histories are multiplied by at the end (*rsign: some sign was recorded).
// With a count plan, the gates it counts move the history's table index
// instead of multiplying (diagonal ones of a class on one word grouped into
// population counts until the next state write), and the real-entry
// branches' magnitudes are left to the plan's table.
void emit_region(std::string &o, const std::vector<Instr> &dev, const std::vector<double> &fac,
                 uint32_t fac_lo, uint32_t kbase, uint32_t lo, uint32_t hi, bool defer,
                 std::vector<Deferred> &deferred, const Mask4 *check = nullptr, Mask4 *checked = nullptr,
                 double *rdef = nullptr, bool *rsign = nullptr, const std::vector<uint8_t> *omit = nullptr,
                 const CountPlan *cp = nullptr, TailCheck *tail = nullptr) {
    char buf[512];
    int off = 0;
    // the pending run: its first instruction, whether every step is selected
    // by a source bit, its constant steps and its source popcounts
    uint32_t run_first = lo;
    bool run_pure = true;
    int32_t run_kc = 0;
    std::vector<std::pair<uint64_t, uint64_t>> run_src;
    auto run_start = [&](uint32_t x) {
        run_first = x;
        run_pure = true;
        run_kc = 0;
        run_src.clear();
    };
    // grouped counted diagonal gates not yet emitted: class, kind
    // (count_bits), word, distance of the two bits, and the gates' low bits
    struct CRun {
        int cls, kind, word;
        uint32_t dist, mask;
    };
    std::vector<CRun> crun;
    auto add_run = [&](int cls, int kind, int word, uint32_t dist, uint32_t q) {
        for (CRun &r : crun)
            if (r.cls == cls && r.kind == kind && r.word == word && r.dist == dist && !((r.mask >> q) & 1u)) {
                r.mask |= 1u << q;
                return;
            }
        crun.push_back(CRun{cls, kind, word, dist, 1u << q});
    };
    auto flush_count = [&]() {
        std::vector<uint8_t> done(crun.size(), 0);
        for (size_t i = 0; i < crun.size(); ++i) {
            if (done[i]) continue;
            o += "    { uint32_t n[H] = {};";
            for (size_t j = i; j < crun.size(); ++j) {
                if (crun[j].cls != crun[i].cls) continue;
                done[j] = 1;
                std::snprintf(buf, sizeof(buf), " count_bits<NW, H, %d, %d>(L, n, %uu, 0x%08xu);", crun[j].word,
                              crun[j].kind, crun[j].dist, crun[j].mask);
                o += buf;
            }
            std::snprintf(buf, sizeof(buf), " count_take<NW, H>(L, n, %uu); }\n", cp->cls[crun[i].cls].step);
            o += buf;
        }
        crun.clear();
    };
    std::snprintf(buf, sizeof(buf), "    const FacRefC<%uu> Fc{F.p}; (void)Fc;\n"
                                    "    uint32_t sg[H] = {}; (void)sg;\n", fac_lo);
    o += buf;
    bool signs = false;   // a real-entry branch collected a sign to apply at the end
    double rmag = 1.0;    // and the product of their magnitudes, applied there too
    bool pending = false;
    uint32_t plo = 0, phi = 0;
    // ladder steps of the pending run whose selecting bit holds a source bit
    // of this region: their constant parts and the sources they add (+1) or
    // subtract (-1), summed as popcounts of the source index at the flush
    SourceBits sbits;
    int32_t pkc = 0;
    uint64_t spos = 0, sneg = 0;
    auto flush_src = [&]() {
        if (pkc == 0 && spos == 0 && sneg == 0) return;
        std::snprintf(buf, sizeof(buf), "    pend_src<NW, H>(L, pk, pb, pbq, %d, 0x%llxull, 0x%llxull);\n", pkc,
                      static_cast<unsigned long long>(spos), static_cast<unsigned long long>(sneg));
        o += buf;
        run_src.emplace_back(spos, sneg);
        pkc = 0;
        spos = sneg = 0;
    };
    auto flush = [&]() {
        if (!pending) return;
        flush_src();
        std::snprintf(buf, sizeof(buf), "    flush_field<NW, H>(L, %uu, %uu, pk, pb, pbq);\n", plo, phi);
        o += buf;
        pending = false;
    };
    for (uint32_t x = lo; x < hi; ++x) {
        if (omit && (*omit)[x - lo]) continue;   // emitted elsewhere
        const Instr &I = dev[x];
        const uint32_t op = I.hdr & 0xffu;
        const int base = op_base(op);
        const int w1 = static_cast<int>((op >> 4) & 3u), w2 = static_cast<int>((op >> 6) & 3u);
        const bool is_add = base == OP_ADD || base == OP_ADDSEL;
        const uint32_t a = (I.hdr >> 8) & 0xffu, b = (I.hdr >> 16) & 0xffu;
        // the grouped counted gates read the state as it is here
        if (!crun.empty() && base != OP_DIAG1 && base != OP_DIAG2 && base != OP_MCPHASE) flush_count();
        if (pending && ends_field_run(I, plo, phi)) flush();
        const int sel_src = sbits.selector_source(I);
        sbits.step(I, kbase);
        if (sel_src >= 0) {
            // a step selected by source bit j: d0 when the bit is 0, d1 when 1
            const uint32_t z = I.hdr >> 24;
            const int32_t d0 = (z & 1u) ? -1 : 1, d1 = (z & 2u) ? -1 : 1;
            if (!pending) run_start(x);
            pkc += d0;
            run_kc += d0;
            if (d1 > d0) spos |= 1ull << sel_src;
            if (d1 < d0) sneg |= 1ull << sel_src;
            pending = true;
            plo = a;
            phi = a + b;
            continue;
        }
        const int cc = cp ? cp->of(x) : -1;
        if (cc >= 0) {
            TwoValued tv = two_valued(I, fac);
            tv.tt = cp->tt(cc, tv);
            const uint32_t step = cp->cls[cc].step, sa = a & 31u, sb = b & 31u;
            if (base == OP_DIAG1 && (tv.tt == 0x2u || tv.tt == 0x1u)) {
                add_run(cc, tv.tt == 0x2u ? 3 : 4, w1, 0u, sa);
            } else if (base == OP_DIAG2 && w1 == w2 && (tv.tt == 0x6u || tv.tt == 0x9u || tv.tt == 0x8u)) {
                add_run(cc, tv.tt == 0x6u ? 0 : (tv.tt == 0x9u ? 1 : 2), w1, sa > sb ? sa - sb : sb - sa,
                        sa < sb ? sa : sb);
            } else if (base == OP_DIAG1 || base == OP_DIAG2) {
                std::snprintf(buf, sizeof(buf),
                              "    op_count_diag<NW, H, wsel<%d, NW>(), wsel<%d, NW>(), 0x%xu, %s>(L, %uu, %uu, %uu);\n",
                              w1, base == OP_DIAG2 ? w2 : w1, tv.tt, base == OP_DIAG2 ? "true" : "false", sa,
                              base == OP_DIAG2 ? sb : 0u, step);
                o += buf;
            } else if (base == OP_DET1) {
                std::snprintf(buf, sizeof(buf), "    op_det1_count<NW, H, wsel<%d, NW>(), 0x%xu>(L, %uu, %uu);\n", w1,
                              tv.tt, sa, step);
                o += buf;
            } else {
                std::snprintf(buf, sizeof(buf),
                              "    op_branch_count<NW, H, wsel<%d, NW>(), %s, 0x%xu>(L, %uu, %uu, bin, %uu);\n", w1,
                              base == OP_BRANCH_SRC ? "true" : "false", tv.tt, sa,
                              base == OP_BRANCH_SRC ? I.k - kbase : 0u, step);
                o += buf;
            }
            continue;
        }
        std::snprintf(buf, sizeof(buf),
                      "    { constexpr Instr I{0x%08xu, 0x%08xu, 0x%08xu, 0x%08xu, "
                      "{0x%08xu, 0x%08xu, 0x%08xu, 0x%08xu}, {0x%08xu, 0x%08xu, 0x%08xu, 0x%08xu}}; ",
                      I.hdr, I.k, I.fac, I.run, I.cm[0], I.cm[1], I.cm[2], I.cm[3], I.cv[0], I.cv[1],
                      I.cv[2], I.cv[3]);
        o += buf;
        int d = -1;
        char call[512];
        FacShape fs = fac_shape(I, fac);
        const uint32_t sa = a & 31u, sb = b & 31u;
        if (defer && rdef && fs.kind == FacShape::REAL) {
            std::snprintf(call, sizeof(call),
                          "op_branch_real_sign<NW, H, wsel<%d, NW>(), %s>(L, %uu, I.k - kbase, bin, %uu); }\n", w1,
                          base == OP_BRANCH_SRC ? "true" : "false", sa, fs.neg);
            o += call;
            *rdef *= fs.r;
            *rsign = true;
            continue;
        }
        if (defer && factor_bits(base) > 0) {
            d = off;
            deferred.push_back(Deferred{I.fac, off, factor_bits(base)});
            off += factor_bits(base);
            fs = FacShape{};
        }
        if (fs.kind == FacShape::CONJ) {
            std::snprintf(call, sizeof(call),
                          "(void)I; op_conj<NW, H, wsel<%d, NW>(), wsel<%d, NW>(), %s>(L, %uu, %uu, %a, %a); }\n",
                          w1, base == OP_DIAG2 ? w2 : w1, base == OP_DIAG2 ? "true" : "false", sa,
                          base == OP_DIAG2 ? sb : 0u, fs.C, fs.S);
            o += call;
            continue;
        }
        if (fs.kind == FacShape::REAL) {
            std::snprintf(call, sizeof(call),
                          "op_branch_real<NW, H, PRUNE, wsel<%d, NW>(), %s, false>(L, sg, %uu, I.k - kbase, bin, thr, "
                          "%a, %uu, %a); if constexpr (PRUNE) { if (!wave_alive(L)) return; } }\n",
                          w1, base == OP_BRANCH_SRC ? "true" : "false", sa, fs.r, fs.neg, fs.m);
            o += call;
            signs = true;
            rmag *= fs.r;
            continue;
        }
        switch (base) {
            case OP_PERM:
                std::snprintf(call, sizeof(call), "op_perm<NW, H, wsel<%d, NW>(), wsel<%d, NW>()>(L, I); }\n", w1, w2);
                break;
            case OP_BRANCH_SRC:
            case OP_BRANCH_NAT:
                std::snprintf(call, sizeof(call),
                              "op_branch<NW, H, PRUNE, wsel<%d, NW>(), %s, %d>(L, I, Fc, kbase, bin, thr); "
                              "if constexpr (PRUNE) { if (!wave_alive(L)) return; } }\n",
                              w1, base == OP_BRANCH_SRC ? "true" : "false", d);
                break;
            case OP_BRANCH_AFF:
                std::snprintf(call, sizeof(call),
                              "op_branch_aff<NW, H, PRUNE, wsel<%d, NW>(), %d>(L, I, Fc, kbase, thr); "
                              "if constexpr (PRUNE) { if (!wave_alive(L)) return; } }\n",
                              w1, d);
                break;
            case OP_DIAG2:
                std::snprintf(call, sizeof(call),
                              "op_diag2<NW, H, wsel<%d, NW>(), wsel<%d, NW>(), %d>(L, I, Fc); }\n", w1, w2, d);
                break;
            case OP_DIAG1:
                std::snprintf(call, sizeof(call), "op_diag1<NW, H, wsel<%d, NW>(), %d>(L, I, Fc); }\n", w1, d);
                break;
            case OP_MCPHASE:
                std::snprintf(call, sizeof(call), "op_mcphase<NW, H, wsel<%d, NW>()>(L, I); }\n", w1);
                break;
            case OP_SWAP:
                std::snprintf(call, sizeof(call), "op_swap<NW, H, wsel<%d, NW>(), wsel<%d, NW>()>(L, I); }\n", w1, w2);
                break;
            case OP_DET1:
                std::snprintf(call, sizeof(call), "op_det1<NW, H, wsel<%d, NW>(), %d>(L, I, Fc); }\n", w1, d);
                break;
            case OP_ADD:
                std::snprintf(call, sizeof(call), "pend_add<NW, H, wsel<%d, NW>()>(L, I, pk, pb); }\n", w1);
                break;
            case OP_ADDSEL:
                std::snprintf(call, sizeof(call),
                              "pend_addsel<NW, H, wsel<%d, NW>(), wsel<%d, NW>()>(L, I, pk, pb); }\n", w1, w2);
                break;
            default:
                std::snprintf(call, sizeof(call), "(void)I; }\n");
                break;
        }
        o += call;
        if (is_add) {
            if (!pending) run_start(x);
            run_pure = false;   // a step whose controls the leaf may change
            pending = true;
            plo = a;
            phi = a + b;
        }
    }
    flush_count();
    if (pending && check) {
        Mask4 fm{{0u, 0u, 0u, 0u}};
        for (uint32_t q = plo; q < phi; ++q) fm.w[q >> 5] |= 1u << (q & 31u);
        bool covered = true;
        for (int w = 0; w < 4; ++w) covered = covered && (fm.w[w] & ~check->w[w]) == 0u;
        if (covered) {
            flush_src();
            std::snprintf(buf, sizeof(buf), "    flush_check<NW, H>(L, %uu, %uu, pk, pb, pbq, bin);\n", plo, phi);
            o += buf;
            pending = false;
            if (checked) *checked = fm;
            if (tail) {
                bool clean = run_pure;
                for (uint32_t x = lo; x < run_first && clean; ++x) {
                    if (omit && (*omit)[x - lo]) continue;
                    uint32_t wm[4];
                    written_bits(dev[x], wm);
                    for (int w = 0; w < 4; ++w) clean = clean && (wm[w] & fm.w[w]) == 0u;
                }
                tail->ok = clean;
                tail->lo = plo;
                tail->hi = phi;
                tail->kc = run_kc;
                tail->src = run_src;
            }
        }
    }
    flush();
    if (signs) {
        if (rmag != 1.0 && !cp) {
            std::snprintf(buf, sizeof(buf), "    scale_amp<NW, H>(L, %a);\n", rmag);
            o += buf;
        }
        o += "    apply_signs<NW, H>(L, sg);\n";
    }
}

}  // namespace

std::string consumer_source(const std::vector<Instr> &dev, const std::vector<double> &fac, uint32_t i1,
                            uint32_t i2, uint32_t iG, uint32_t Ap, uint32_t Ar, const Mask4 &fin_c2,
                            const Mask4 &fin_G, int NW, int H, bool prune, bool flds, uint32_t fac_lo,
                            bool prefix_ok, uint32_t iL, const std::vector<uint32_t> &src_dev, uint32_t Dp,
                            bool pflds, uint32_t pfac_lo, uint32_t ss) {
    std::vector<Deferred> none, deferred;
    std::string o;
    char buf[512];
    // The final check at G: a pending ladder run the check covers whole is
    // compared with the output instead (flush_check, the `checked` field);
    // a bit whose last write in the suffix is a branching gate on a natural
    // input segment was set from the input and always matches it.
    std::string sfx;
    Mask4 checked{{0u, 0u, 0u, 0u}};
    // suffix instructions evaluated once per root history (suffix_pre)
    const std::vector<uint8_t> hoist = hoistable(dev, i2, iG, prune);
    std::vector<uint8_t> keep(hoist.size());
    bool any_hoist = false;
    for (size_t x = 0; x < hoist.size(); ++x) {
        keep[x] = hoist[x] ? 0 : 1;
        any_hoist = any_hoist || hoist[x];
    }
    // two-valued factors counted instead of multiplied (without pruning: the
    // moduli are then never needed as the walk goes)
    CountPlan cplan;
    if (!prune) cplan = count_plan(dev, fac, i1, i2, iG, hoist);
    const CountPlan *cp = cplan.on() ? &cplan : nullptr;
    TailCheck tail;
    emit_region(sfx, dev, fac, fac_lo, Ap + Ar, i2, iG, false, none, &fin_G, &checked, nullptr, nullptr, &hoist, cp,
                &tail);
    Mask4 natw{{0u, 0u, 0u, 0u}};
    bool zero_entries = false;
    for (uint32_t x = i2; x < iG; ++x) {
        const int base = op_base(dev[x].hdr & 0xffu);
        uint32_t wm[4];
        written_bits(dev[x], wm);
        for (int w = 0; w < 4; ++w) {
            if (base == OP_BRANCH_NAT) natw.w[w] |= wm[w];
            else natw.w[w] &= ~wm[w];
        }
        if ((base == OP_BRANCH_SRC || base == OP_BRANCH_NAT || base == OP_BRANCH_AFF) && (dev[x].hdr >> 24) != 0u)
            zero_entries = true;
    }
    Mask4 fin_rest = fin_G;
    bool check_left = false;
    for (int w = 0; w < 4; ++w) {
        fin_rest.w[w] &= ~(checked.w[w] | natw.w[w]);
        check_left = check_left || fin_rest.w[w] != 0u || checked.w[w] != 0u;
    }
    // Defer the suffix's factors (record their table indices, multiply only
    // for the histories that pass the final check) when nothing needs them
    // during the walk (pruning does), their indices fit in dx, and a history
    // can still fail after the root; when none can, deferring only adds work.
    // (real-entry branches defer only a sign and a constant magnitude)
    int bits = 0;
    for (uint32_t x = i2; x < iG; ++x)
        if (!hoist[x - i2] && fac_shape(dev[x], fac).kind != FacShape::REAL && (!cp || cp->of(x) < 0))
            bits += factor_bits(op_base(dev[x].hdr & 0xffu));
    const bool defer = !prune && bits <= 64 && (check_left || zero_entries);
    double rdef = 1.0;
    bool rsign = false;
    if (defer) {
        sfx.clear();
        tail = TailCheck{};
        emit_region(sfx, dev, fac, fac_lo, Ap + Ar, i2, iG, true, deferred, &fin_G, &checked, &rdef, &rsign, &hoist,
                    cp, &tail);
    }
    o += "#include \"device.hpp\"\nnamespace fhs {\nnamespace {\n";
    std::vector<double> ctab;
    if (cp) {
        // the counted classes' products, group by group; the first group
        // also carries the real-entry branches' magnitudes of the regions
        long double rtotal = 1.0L;
        for (uint32_t x = i1; x < iG; ++x) {
            const FacShape f = fac_shape(dev[x], fac);
            if (f.kind == FacShape::REAL) rtotal *= f.r;
        }
        for (size_t g = 0; g < cp->group_size.size(); ++g) {
            for (uint32_t i = 0; i < cp->group_size[g]; ++i) {
                std::complex<long double> v = g == 0 ? std::complex<long double>(rtotal, 0.0L)
                                                     : std::complex<long double>(1.0L, 0.0L);
                for (const CountPlan::Cls &c : cp->cls) {
                    if (c.group != g) continue;
                    const uint32_t f = (i / c.stride) % (c.n + 1u);
                    double ab[4];
                    std::memcpy(ab, c.v.a, sizeof c.v.a);
                    std::memcpy(ab + 2, c.v.b, sizeof c.v.b);
                    const std::complex<long double> a(ab[0], ab[1]), b(ab[2], ab[3]);
                    for (uint32_t k = 0; k < c.n - f; ++k) v *= a;
                    for (uint32_t k = 0; k < f; ++k) v *= b;
                }
                ctab.push_back(static_cast<double>(v.real()));
                ctab.push_back(static_cast<double>(v.imag()));
            }
        }
        std::snprintf(buf, sizeof(buf), "__constant__ double kCountTab[%zu] = {", ctab.size());
        o += buf;
        for (size_t i = 0; i < ctab.size(); ++i) {
            std::snprintf(buf, sizeof(buf), "%s%a", i ? ", " : "", ctab[i]);
            o += buf;
        }
        o += "};\n";
    }
    o += "struct Compiled {\n";
    // a pure leaf loop: every factor its instructions take is counted or a
    // sign (real-entry branches, MCPHASE), and none is deferred
    bool pure = cp != nullptr && deferred.empty();
    for (uint32_t x = i2; x < iG && pure; ++x) {
        if (hoist[x - i2] || cp->of(x) >= 0) continue;
        const int base = op_base(dev[x].hdr & 0xffu);
        const bool factor = factor_bits(base) > 0;
        if (factor && fac_shape(dev[x], fac).kind != FacShape::REAL) pure = false;
    }
    if (cp) {
        std::snprintf(buf, sizeof(buf),
                      "static constexpr uint32_t kNCT = %uu;\n"
                      "static constexpr bool kLeafPure = %s;\n"
                      "__device__ static __forceinline__ double2 count_entry(uint32_t i) "
                      "{ return make_double2(kCountTab[2u * i], kCountTab[2u * i + 1u]); }\n"
                      "template <int NW, int H>\n"
                      "__device__ static __forceinline__ void count_amp(const double2 *T, Lanes<NW, H> &L, int h) {\n",
                      cp->entries, pure ? "true" : "false");
        o += buf;
        const bool one = cp->group_size.size() == 1;
        for (size_t g = 0; g < cp->group_size.size(); ++g) {
            const uint32_t width = (g + 1 < cp->group_shift.size() ? cp->group_shift[g + 1] : 32u) - cp->group_shift[g];
            // a pure leaf's first product replaces its amplitude (+-1)
            const char *take = (pure && g == 0) ? "count_set(L.re[h], L.im[h], f)" : "cmul(L.re[h], L.im[h], f.x, f.y)";
            if (one)
                std::snprintf(buf, sizeof(buf), "    { const double2 f = T[L.ci[h]]; %s; }\n", take);
            else
                std::snprintf(buf, sizeof(buf), "    { const double2 f = T[%uu + ((L.ci[h] >> %uu) & 0x%xu)]; %s; }\n",
                              cp->group_base[g], cp->group_shift[g],
                              width >= 32u ? 0xffffffffu : (1u << width) - 1u, take);
            o += buf;
        }
        o += "}\n";
    } else {
        o += "static constexpr uint32_t kNCT = 0;\n"
             "static constexpr bool kLeafPure = false;\n"
             "__device__ static __forceinline__ double2 count_entry(uint32_t) { return make_double2(0.0, 0.0); }\n"
             "template <int NW, int H>\n"
             "__device__ static __forceinline__ void count_amp(const double2 *, Lanes<NW, H> &, int) {}\n";
    }
    o += defer ? "static constexpr bool kDefer = true;\n" : "static constexpr bool kDefer = false;\n";
    // a short suffix walks several assignments per pass of the leaf loop
    // (the loop control and the skip of passes without a valid history are
    // paid once per pass); longer ones one at a time, keeping registers
    const int U = iG - i2 <= 24u ? 8 : 1;
    std::snprintf(buf, sizeof(buf), "static constexpr int kUnroll = %d;\n", U);
    o += buf;
    // Whole passes of leaves rejected at once (TailCheck): a leaf passes the
    // final field check only if 2 (P(q) + P(u)) << up equals the root's
    // residue less its constant and lane steps (v), P the source popcounts
    // of the pass's wave-uniform base q and of the leaf's offset u < U; with
    // P(u) in [pmin, pmax], D = v - (2 (P(q) + pmin) << up) must be
    // 2k << up for some k <= pmax - pmin.
    {
        const uint32_t m = tail.hi - tail.lo;
        const uint32_t up = m <= 32u ? 32u - m : 0u;
        int32_t pmin = 0, pmax = 0;
        for (int u = 0; u < U; ++u) {
            int32_t p = 0;
            for (const auto &pn : tail.src)
                p += __builtin_popcountll(static_cast<uint64_t>(u) & pn.first) -
                     __builtin_popcountll(static_cast<uint64_t>(u) & pn.second);
            pmin = u ? std::min(pmin, p) : p;
            pmax = u ? std::max(pmax, p) : p;
        }
        const bool filt = tail.ok && m >= 2u && up <= 30u &&
                          static_cast<uint64_t>(pmax - pmin) + 1u < (1ull << (31u - up));
        // the same over every suffix assignment: per source bit its weight in
        // P, the range the sum of the weights of any subset of bits spans
        int32_t amin = 0, amax = 0;
        const uint32_t As = static_cast<uint32_t>(src_dev.size()) - Ap - Ar;
        for (uint32_t k = 0; k < As && k < 64u; ++k) {
            int32_t wk = 0;
            for (const auto &pn : tail.src)
                wk += static_cast<int32_t>((pn.first >> k) & 1u) - static_cast<int32_t>((pn.second >> k) & 1u);
            if (wk < 0) amin += wk;
            else amax += wk;
        }
        const bool rfilt = filt && static_cast<uint64_t>(amax - amin) + 1u < (1ull << (31u - up));
        std::snprintf(buf, sizeof(buf), "static constexpr uint32_t kRootQ = %uu;\nstatic constexpr int32_t kRootSpan = %d;\n",
                      rfilt ? (2u * static_cast<uint32_t>(amin)) << up : 0u, rfilt ? amax - amin : -1);
        o += buf;
        if (filt) {
            std::snprintf(buf, sizeof(buf),
                          "static constexpr bool kPassFilter = true;\n"
                          "static constexpr uint32_t kPassUp = %uu;\n"
                          "static constexpr uint32_t kPassSpan = %uu;\n"
                          "template <int NW, int H>\n"
                          "__device__ static __forceinline__ void pass_res(const Lanes<NW, H> &R, const uint64_t (&hs)[H], "
                          "const uint32_t (&bin)[NW], uint32_t (&v)[H]) {\n"
                          "    unroll<H>([&](auto hh) {\n"
                          "        constexpr int h = hh.value;\n"
                          "        uint32_t up;\n"
                          "        const uint32_t e = field_residue<NW>(R.s[h], bin, %uu, %uu, up);\n"
                          "        int32_t pb = 0;\n",
                          up, static_cast<uint32_t>(pmax - pmin), tail.lo, tail.hi);
            o += buf;
            for (const auto &pn : tail.src) {
                std::snprintf(buf, sizeof(buf),
                              "        pb += __popcll(hs[h] & 0x%llxull) - __popcll(hs[h] & 0x%llxull);\n",
                              static_cast<unsigned long long>(pn.first), static_cast<unsigned long long>(pn.second));
                o += buf;
            }
            std::snprintf(buf, sizeof(buf),
                          "        v[h] = (e - (%uu + 2u * static_cast<uint32_t>(pb))) << up;\n"
                          "    });\n"
                          "}\n"
                          "template <int UU>\n"
                          "__device__ static __forceinline__ uint32_t pass_q(uint64_t q) {\n"
                          "    int32_t p = UU == 1 ? 0 : %d;\n",
                          static_cast<uint32_t>(tail.kc), pmin);
            o += buf;
            for (const auto &pn : tail.src) {
                std::snprintf(buf, sizeof(buf), "    p += __popcll(q & 0x%llxull) - __popcll(q & 0x%llxull);\n",
                              static_cast<unsigned long long>(pn.first), static_cast<unsigned long long>(pn.second));
                o += buf;
            }
            std::snprintf(buf, sizeof(buf), "    return (2u * static_cast<uint32_t>(p)) << %uu;\n}\n", up);
            o += buf;
        } else {
            o += "static constexpr bool kPassFilter = false;\n"
                 "static constexpr uint32_t kPassUp = 0u;\n"
                 "static constexpr uint32_t kPassSpan = 0u;\n"
                 "template <int NW, int H>\n"
                 "__device__ static __forceinline__ void pass_res(const Lanes<NW, H> &, const uint64_t (&)[H], "
                 "const uint32_t (&)[NW], uint32_t (&)[H]) {}\n"
                 "template <int UU>\n"
                 "__device__ static __forceinline__ uint32_t pass_q(uint64_t) { return 0u; }\n";
        }
    }
    // with one lane per root task, every suffix source lives in the leaf
    // loop's wave-uniform counter: built for that case as constants (with
    // several lanes per root task the lanes' share of the suffix index stays
    // a run-time value; combined with the counter, the compiler then
    // evaluates the suffix's source-only work per lane and per leaf)
    if (ss == 0)
        std::snprintf(buf, sizeof(buf), "static constexpr int kSS = 0;\nstatic constexpr int kAs = %u;\n",
                      static_cast<uint32_t>(src_dev.size()) - Ap - Ar);
    else
        std::snprintf(buf, sizeof(buf), "static constexpr int kSS = -1;\nstatic constexpr int kAs = -1;\n");
    o += buf;
    std::snprintf(buf, sizeof(buf), "static constexpr int kA = %u;\n", static_cast<uint32_t>(src_dev.size()));
    o += buf;
    // the final-bit masks as constants: fully checked words become one compare
    const Mask4 *fm[2] = {&fin_c2, &fin_rest};
    const char *fname[2] = {"final_c2", "final_G"};
    for (int k = 0; k < 2; ++k) {
        std::snprintf(buf, sizeof(buf),
                      "template <int NW>\n"
                      "__device__ static __forceinline__ bool %s(const uint32_t (&s)[NW], "
                      "const uint32_t (&bin)[NW], const Mask4 &) {\n"
                      "    constexpr Mask4 m{{0x%08xu, 0x%08xu, 0x%08xu, 0x%08xu}};\n"
                      "    return check_final<NW>(s, bin, m);\n}\n",
                      fname[k], fm[k]->w[0], fm[k]->w[1], fm[k]->w[2], fm[k]->w[3]);
        o += buf;
    }
    std::snprintf(buf, sizeof(buf),
                  "template <int NW, int H, bool PRUNE>\n"
                  "__device__ static __forceinline__ void root(const Common &c, const FacRef &F, "
                  "Lanes<NW, H> &L, const uint32_t (&bin)[NW]) {\n"
                  "    constexpr uint32_t kbase = %uu; const double thr = c.thr; (void)kbase; (void)thr;\n"
                  "    int32_t pk[H] = {}, pb[H] = {}, pbq = 0; (void)pk; (void)pb; (void)pbq;\n",
                  Ap);
    o += buf;
    emit_region(o, dev, fac, fac_lo, Ap, i1, i2, false, none, nullptr, nullptr, nullptr, nullptr, nullptr, cp);
    o += "}\n";
    std::snprintf(buf, sizeof(buf),
                  "template <int NW, int H, bool PRUNE>\n"
                  "__device__ static __forceinline__ void suffix(const Common &c, const FacRef &F, "
                  "Lanes<NW, H> &L, const uint32_t (&bin)[NW]) {\n"
                  "    constexpr uint32_t kbase = %uu; const double thr = c.thr; (void)kbase; (void)thr;\n"
                  "    int32_t pk[H] = {}, pb[H] = {}, pbq = 0; (void)pk; (void)pb; (void)pbq;\n",
                  Ap + Ar);
    o += buf;
    o += sfx;
    o += "}\n";
    std::snprintf(buf, sizeof(buf),
                  "static constexpr bool kHoist = %s;\n"
                  "template <int NW, int H, bool PRUNE>\n"
                  "__device__ static __forceinline__ void suffix_pre(const Common &c, const FacRef &F, "
                  "Lanes<NW, H> &L, const uint32_t (&bin)[NW]) {\n"
                  "    constexpr uint32_t kbase = %uu; const double thr = c.thr; (void)kbase; (void)thr;\n"
                  "    int32_t pk[H] = {}, pb[H] = {}, pbq = 0; (void)pk; (void)pb; (void)pbq;\n",
                  any_hoist ? "true" : "false", Ap + Ar);
    o += buf;
    if (any_hoist) emit_region(o, dev, fac, fac_lo, Ap + Ar, i2, iG, false, none, nullptr, nullptr, nullptr, nullptr,
                               &keep, cp);
    o += "}\n";
    // the deferred factors, in evaluation order: the same products as the walk
    o += "template <int NW, int H>\n"
         "__device__ static __forceinline__ void suffix_amp(const FacRef &F, Lanes<NW, H> &L, int h) {\n"
         "    (void)F; (void)L; (void)h;\n";
    std::snprintf(buf, sizeof(buf), "    const FacRefC<%uu> Fc{F.p}; (void)Fc;\n", fac_lo);
    o += buf;
    for (const Deferred &d : deferred) {
        std::snprintf(buf, sizeof(buf),
                      "    { const uint32_t x = static_cast<uint32_t>(L.dx[h] >> %d) & %uu; "
                      "const double2 f = Fc.c(%uu + 2u * x); cmul(L.re[h], L.im[h], f.x, f.y); }\n",
                      d.off, (1u << d.bits) - 1u, d.fac);
        o += buf;
    }
    if (rsign && cp) {
        // the real-entry branches' signs (their magnitudes are in the count table)
        o += "    { const uint32_t f = (L.sd[h] & 1u) << 31; "
             "L.re[h] = flip_sign(L.re[h], f); L.im[h] = flip_sign(L.im[h], f); }\n";
    } else if (rsign) {
        // the real-entry branches' magnitudes (one constant) and signs
        std::snprintf(buf, sizeof(buf),
                      "    { const uint32_t f = (L.sd[h] & 1u) << 31; "
                      "L.re[h] = flip_sign(L.re[h] * %a, f); L.im[h] = flip_sign(L.im[h] * %a, f); }\n",
                      rdef, rdef);
        o += buf;
    }
    o += "}\n";
    if (prefix_ok) {
        // the prefix region: head [iL, first depth-first source), then one
        // straight-line case per depth-first level (sources numbered from 0)
        const uint32_t lo_bits = Ap - Dp;
        const uint32_t e_split = Dp ? src_dev[lo_bits] : i1;
        o += "template <int NW, bool PRUNE>\n"
             "__device__ static __forceinline__ void prefix_head(const Common &c, const FacRef &F, "
             "Lanes<NW, 1> &L, const uint32_t (&bin)[NW], uint32_t) {\n"
             "    constexpr int H = 1; constexpr uint32_t kbase = 0u; const double thr = c.thr; "
             "(void)kbase; (void)thr; (void)bin;\n"
             "    int32_t pk[H] = {}, pb[H] = {}, pbq = 0; (void)pk; (void)pb; (void)pbq;\n";
        emit_region(o, dev, fac, pfac_lo, 0u, iL, e_split, false, none);
        o += "}\n";
        o += "template <int NW, bool PRUNE>\n"
             "__device__ static __forceinline__ void prefix_seg(const Common &c, const FacRef &F, "
             "Lanes<NW, 1> &L, const uint32_t (&bin)[NW], uint32_t, uint32_t, uint32_t l) {\n"
             "    constexpr int H = 1; constexpr uint32_t kbase = 0u; const double thr = c.thr; "
             "(void)kbase; (void)thr; (void)bin;\n"
             "    int32_t pk[H] = {}, pb[H] = {}, pbq = 0; (void)pk; (void)pb; (void)pbq;\n"
             "    switch (l) {\n";
        for (uint32_t l = 0; l < Dp; ++l) {
            const uint32_t a = src_dev[lo_bits + l], b = (l + 1 < Dp) ? src_dev[lo_bits + l + 1] : i1;
            std::snprintf(buf, sizeof(buf), "    case %uu: {\n", l);
            o += buf;
            emit_region(o, dev, fac, pfac_lo, 0u, a, b, false, none);
            o += "    } break;\n";
        }
        o += "    default: break;\n    }\n}\n";
    }
    o += "};\n}  // namespace\n}  // namespace fhs\n";
    std::snprintf(buf, sizeof(buf),
                  "extern \"C\" __global__ __launch_bounds__(fhs::kConsumeThreads) void "
                  "fhs_consume_compiled(fhs::Common c, fhs::Table tab, fhs::Partials part, uint32_t p0, "
                  "uint32_t B, uint32_t chunk, uint32_t ss, uint32_t *counter) {\n"
                  "    fhs::consume_body<fhs::Compiled, %d, %d, %s, %s>(c, tab, part, p0, B, chunk, ss, "
                  "counter);\n}\n",
                  NW, H, prune ? "true" : "false", flds ? "true" : "false");
    o += buf;
    if (prefix_ok) {
        std::snprintf(buf, sizeof(buf),
                      "extern \"C\" __global__ __launch_bounds__(256) void "
                      "fhs_prefix_compiled(fhs::Common c, fhs::PreBufs pre, fhs::Table tab, uint32_t p0, "
                      "uint32_t B, uint32_t P, uint32_t Dp) {\n"
                      "    fhs::prefix_body<fhs::Compiled, %d, %s, %s>(c, pre, tab, p0, B, P, Dp);\n}\n",
                      NW, prune ? "true" : "false", pflds ? "true" : "false");
        o += buf;
    }
    return o;
}

bool pair_filter(const std::vector<Instr> &dev, const std::vector<double> &fac, uint32_t iL, uint32_t iG,
                 const Mask4 &fin_G, uint32_t A, PairFilter &out) {
    if (iL >= iG || A == 0) return false;
    // the whole program after the leading gates as one region with global
    // source indices: its final run and what precedes it (the text is not used)
    std::string text;
    std::vector<Deferred> none;
    Mask4 checked{{0u, 0u, 0u, 0u}};
    TailCheck tail;
    emit_region(text, dev, fac, 0u, 0u, iL, iG, false, none, &fin_G, &checked, nullptr, nullptr, nullptr, nullptr,
                &tail);
    if (!tail.ok) return false;
    const uint32_t m = tail.hi - tail.lo;
    const uint32_t up = m <= 32u ? 32u - m : 0u;
    int64_t amin = 0, amax = 0;
    for (uint32_t k = 0; k < A && k < 64u; ++k) {
        int64_t wk = 0;
        for (const auto &pn : tail.src)
            wk += static_cast<int64_t>((pn.first >> k) & 1u) - static_cast<int64_t>((pn.second >> k) & 1u);
        if (wk < 0) amin += wk;
        else amax += wk;
    }
    if (m < 2u || up > 30u || static_cast<uint64_t>(amax - amin) + 1u >= (1ull << (31u - up))) return false;
    out.lo = tail.lo;
    out.hi = tail.hi;
    out.up = up;
    out.off = static_cast<uint32_t>(static_cast<int64_t>(tail.kc) + 2 * amin);
    out.span = static_cast<uint32_t>(amax - amin);
    return true;
}

bool compile_code(const std::string &src, std::vector<char> &code, std::string &log) {
    hiprtcProgram prog = nullptr;
    const char *headers[] = {kSrcProgramHpp, kSrcKernelsHpp, kSrcDeviceHpp};
    const char *names[] = {"program.hpp", "kernels.hpp", "device.hpp"};
    if (hiprtcCreateProgram(&prog, src.c_str(), "fhs_consume_compiled.hip", 3, headers, names) !=
        HIPRTC_SUCCESS) {
        log = "hiprtcCreateProgram failed";
        return false;
    }
    // The same code-generation features as the library build: no packed FP32
    // and no three-input bitwise ops (v_bitop3_b32 was miscompiled for some
    // straight-line history programs by this compiler).
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                          "-Xclang", "-target-feature", "-Xclang", "-bitop3-insts"};
    const hiprtcResult r = hiprtcCompileProgram(prog, static_cast<int>(sizeof(opts) / sizeof(opts[0])), opts);
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    log.assign(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    if (r != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        return false;
    }
    size_t code_size = 0;
    hiprtcGetCodeSize(prog, &code_size);
    code.resize(code_size);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return true;
}

bool load_consumer(const std::vector<char> &code, bool has_prefix, size_t shm, CompiledConsumer &out,
                   std::string &log) {
    if (hipModuleLoadData(&out.mod, code.data()) != hipSuccess) {
        log += "\nhipModuleLoadData failed";
        out.mod = nullptr;
        return false;
    }
    if (hipModuleGetFunction(&out.fn, out.mod, "fhs_consume_compiled") != hipSuccess) {
        log += "\nhipModuleGetFunction failed";
        release(out);
        return false;
    }
    if (has_prefix && hipModuleGetFunction(&out.pfn, out.mod, "fhs_prefix_compiled") != hipSuccess) {
        log += "\nhipModuleGetFunction (prefix) failed";
        release(out);
        return false;
    }
    int nb = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, out.fn, kConsumeThreads, shm) !=
            hipSuccess || nb < 1)
        nb = 1;
    out.blocks_per_cu = nb;
    return true;
}

bool compile_consumer(const std::string &src, size_t shm, CompiledConsumer &out, std::string &log) {
    std::vector<char> code;
    if (!compile_code(src, code, log)) return false;
    return load_consumer(code, src.find("fhs_prefix_compiled") != std::string::npos, shm, out, log);
}

void release(CompiledConsumer &k) {
    if (k.mod) (void)hipModuleUnload(k.mod);
    k.mod = nullptr;
    k.fn = nullptr;
    k.pfn = nullptr;
}

hipError_t launch_prefix_compiled(const CompiledConsumer &k, const Common &c, PreBufs pre, Table tab,
                                  uint32_t p0, uint32_t B, uint32_t Dp, size_t shm, hipStream_t s) {
    if (B == 0) return hipSuccess;
    if (!k.pfn || Dp > c.Ap || Dp > static_cast<uint32_t>(kDfsMax)) return hipErrorInvalidValue;
    const uint64_t NL = static_cast<uint64_t>(B) << (c.Ap - Dp);
    uint64_t blocks = (NL + 255) / 256;
    if (blocks > (1u << 20)) blocks = 1u << 20;
    Common cc = c;
    uint32_t P = c.M * c.S;
    void *args[] = {&cc, &pre, &tab, &p0, &B, &P, &Dp};
    return hipModuleLaunchKernel(k.pfn, static_cast<uint32_t>(blocks), 1, 1, 256, 1, 1,
                                 static_cast<unsigned>(shm), s, args, nullptr);
}

hipError_t launch_compiled(const CompiledConsumer &k, const Common &c, Table tab, Partials part,
                           uint32_t p0, uint32_t B, uint32_t chunk, uint32_t ss, uint32_t *counter,
                           uint32_t grid, size_t shm, hipStream_t s) {
    if (B == 0 || grid == 0) return hipSuccess;
    Common cc = c;
    void *args[] = {&cc, &tab, &part, &p0, &B, &chunk, &ss, &counter};
    return hipModuleLaunchKernel(k.fn, grid, 1, 1, kConsumeThreads, 1, 1, static_cast<unsigned>(shm),
                                 s, args, nullptr);
}

}  // namespace fhs
