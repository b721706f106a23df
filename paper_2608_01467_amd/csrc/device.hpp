// device.hpp -- device-side building blocks of the reduced-history kernels:
// per-history registers, the per-opcode backward steps, the program
// interpreter (run_region), the depth-first region walk, deterministic
// reductions and the persistent consumer's body.  Included by kernels.hip
// and, as source text, by the consumer the runtime compiles for a program.
//
// Each lane owns one history at a time: an n-bit time-slice state held in
// NW 32-bit VGPRs, an FP64 complex partial amplitude and (with pruning) the
// running modulus product M.  The history program is read wave-uniformly
// (scalar loads), so every lane of a wave executes the same gate and only
// the selected matrix element differs.  Source bits are decoded from the
// lane's history index in registers.
#pragma once

#if !defined(__HIPCC_RTC__)
#include <hip/hip_runtime.h>
#endif

#include <cstdint>
#include <type_traits>
#include <utility>

#include "kernels.hpp"

namespace fhs {
namespace {


// The program is read through the constant address space: it is never
// written while a kernel runs, which lets every instruction field arrive by
// scalar load even in kernels that store to global memory.
// (The host compilation pass only parses device code; it gets the plain type.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using Const = const __attribute__((address_space(4))) T;
#else
template <class T>
using Const = const T;
#endif
using ConstInstr = Const<Instr>;

// Read-only kernel inputs (masks, bitstrings) through the constant address
// space, so uniform reads become scalar loads.
template <class T>
__device__ __forceinline__ T ld_const(const T *p, size_t i) {
    return ((Const<T> *)p)[i];
}

// SplitMix64 finaliser (Steele, Lea, Flood 2014): mix64_tail after the
// first multiply.  For z < 2^30 the first shift-xor leaves z unchanged, so
// the first product is linear in z: the consumer forms it per root history
// plus a wave-uniform part per leaf.
constexpr uint64_t kMixC1 = 0xbf58476d1ce4e5b9ULL, kMixC2 = 0x94d049bb133111ebULL;
__device__ __forceinline__ uint64_t mix64_tail(uint64_t z) {
    z = (z ^ (z >> 27)) * kMixC2;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    return mix64_tail((z ^ (z >> 30)) * kMixC1);
}

// State words are only ever indexed with compile-time constants (the word
// holding a gate's bit is part of its opcode), so the state stays in VGPRs.
// H independent histories per lane share every decoded instruction.
template <int W, int NW>
__device__ __forceinline__ constexpr int wsel() {
    return W < NW ? W : 0;
}

template <int V>
using IC = std::integral_constant<int, V>;

// f(IC<0>), ..., f(IC<N-1>): compile-time unrolling, so that register arrays
// are never indexed with a runtime value.
template <class F, int... I>
__device__ __forceinline__ void unroll_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(IC<I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void unroll(F &&f) {
    unroll_impl(f, std::make_integer_sequence<int, N>{});
}

// Call f(IC<w>) for the uniform word index w < NW.
template <int NW, class F>
__device__ __forceinline__ void with_word(uint32_t w, F &&f) {
    if constexpr (NW == 1) {
        f(IC<0>{});
    } else if constexpr (NW == 2) {
        if (w == 0u) f(IC<0>{});
        else f(IC<1>{});
    } else {
        if (w < 2u) {
            if (w == 0u) f(IC<0>{});
            else f(IC<1>{});
        } else {
            if (w == 2u) f(IC<2>{});
            else f(IC<3>{});
        }
    }
}

template <int NW>
__device__ __forceinline__ bool check_final(const uint32_t (&s)[NW], const uint32_t (&bin)[NW],
                                            const Mask4 &m) {
    uint32_t acc = 0;
    unroll<NW>([&](auto jj) {
        constexpr int j = jj.value;
        acc |= (s[j] ^ bin[j]) & m.w[j];
    });
    return acc == 0;
}

__device__ __forceinline__ void cmul(double &re, double &im, double fr, double fi) {
    const double r = fma(re, fr, -(im * fi));
    const double i = fma(re, fi, im * fr);
    re = r;
    im = i;
}

// Bitstring words (uint64, little-endian) -> NW 32-bit state words.
// Returns true when a bit at position >= n is set.
template <int NW>
__device__ __forceinline__ bool load_bits(const uint64_t *src, uint32_t W, uint32_t n,
                                          uint32_t (&s)[NW]) {
    bool bad = false;
    uint64_t w0 = ld_const(src, 0);
    uint64_t w1 = W > 1 ? ld_const(src, 1) : 0;
    if (n < 64) bad = (w0 >> n) != 0;
    else if (n < 128 && W > 1) bad = (w1 >> (n - 64)) != 0;
    s[0] = static_cast<uint32_t>(w0);
    if constexpr (NW >= 2) s[1] = static_cast<uint32_t>(w0 >> 32);
    if constexpr (NW == 4) {
        s[2] = static_cast<uint32_t>(w1);
        s[3] = static_cast<uint32_t>(w1 >> 32);
    }
    return bad;
}

// The bitstrings of pair p = j S + i (output j, input i): a history starts
// from the one at the evaluation order's start (the output; the input for a
// program placed by the forward sweep) and is checked against the other.
__device__ __forceinline__ const uint64_t *start_bits(const Common &c, uint32_t p) {
    return c.fwd ? c.inputs + static_cast<size_t>(p % c.S) * c.W : c.outputs + static_cast<size_t>(p / c.S) * c.W;
}
__device__ __forceinline__ const uint64_t *check_bits(const Common &c, uint32_t p) {
    return c.fwd ? c.outputs + static_cast<size_t>(p / c.S) * c.W : c.inputs + static_cast<size_t>(p % c.S) * c.W;
}

// Per-history registers of H histories.
template <int NW, int H>
struct Lanes {
    uint32_t s[H][NW];
    double re[H], im[H], M[H];
    bool ok[H];
    uint64_t hb[H];     // this region's source bits, per history
    uint64_t dx[H];     // factor-table indices recorded for a deferred multiply
    uint64_t hf[H];     // the source bits of the earlier regions (their global positions)
    uint64_t aff;       // the pair's boundary bits of the affine inputs' forms
    // Wave-uniform parts of this region's source index, on bits disjoint from
    // hb's and from each other: the region's index is hb | hq | hu.  The
    // consumer's suffix loop keeps its counter here (hq the base of an
    // unrolled pass, hu the leaf's offset in it, a compile-time constant
    // there), so what depends only on those sources is scalar work, and the
    // offset's share of it is folded at compile time.
    uint64_t hq;
    uint32_t hu;
    uint32_t sd[H];     // bit 0: the sign of the deferred real factors' product so far
    uint32_t ci[H];     // counted factors: the index into their tables (op_count_*)
};

// Source bit k of a region's index (hb, hq and hu hold disjoint bits).
template <int NW, int H>
__device__ __forceinline__ uint32_t src_bit(const Lanes<NW, H> &L, int h, uint32_t k) {
    return static_cast<uint32_t>((L.hb[h] >> k) & 1u) | static_cast<uint32_t>((L.hq >> k) & 1u) |
           (k < 32u ? (L.hu >> k) & 1u : 0u);
}

// Factor tables: `fac` points at the slice [lo, ...) of the global table,
// staged in LDS by the hot kernels; entries are read per lane.
struct FacRef {
    const double *p;
    uint32_t lo;
    __device__ __forceinline__ double2 c(uint32_t off) const {
        return *reinterpret_cast<const double2 *>(p + (off - lo));
    }
    __device__ __forceinline__ double d(uint32_t off) const { return p[off - lo]; }
};

// The same with the slice's start a compile-time constant (the compiled
// regions): a table entry's address is then the lane's index times 16 plus
// an immediate offset.
template <uint32_t LO>
struct FacRefC {
    const double *p;
    __device__ __forceinline__ double2 c(uint32_t off) const {
        return *reinterpret_cast<const double2 *>(p + (off - LO));
    }
    __device__ __forceinline__ double d(uint32_t off) const { return p[off - LO]; }
};

// Entry x of a gate's factor table (at offset fac) for history h: multiplied
// into the running amplitude now (DEFER < 0), or recorded in bits
// [DEFER, DEFER + 2) of dx[h] and multiplied after the history has passed
// its final check (the same factors in the same order, so the same result).
template <int DEFER, int NW, int H, class FR>
__device__ __forceinline__ void take_factor(Lanes<NW, H> &L, int h, const FR &F, uint32_t fac,
                                            uint32_t x) {
    if constexpr (DEFER < 0) {
        const double2 f = F.c(fac + 2u * x);
        cmul(L.re[h], L.im[h], f.x, f.y);
    } else {
        L.dx[h] |= static_cast<uint64_t>(x) << DEFER;
    }
}

__device__ __forceinline__ uint32_t hdr_a(const Instr &I) { return (I.hdr >> 8) & 0xffu; }
__device__ __forceinline__ uint32_t hdr_b(const Instr &I) { return (I.hdr >> 16) & 0xffu; }
__device__ __forceinline__ uint32_t hdr_z(const Instr &I) { return I.hdr >> 24; }

template <int NW, int H, int TW, int LW>
__device__ __forceinline__ void op_perm(Lanes<NW, H> &L, const Instr &I) {
    constexpr int T = wsel<TW, NW>();
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        uint32_t acc = (L.s[h][0] ^ I.cv[0]) & I.cm[0];
        unroll<NW>([&](auto jj) {
            constexpr int j = jj.value;
            if constexpr (j >= 1 && j <= LW) acc |= (L.s[h][j] ^ I.cv[j]) & I.cm[j];
        });
        L.s[h][T] ^= (acc == 0u) ? I.k : 0u;
    });
}

template <int NW, int H, int LW>
__device__ __forceinline__ void op_mcphase(Lanes<NW, H> &L, const Instr &I) {
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        uint32_t acc = (L.s[h][0] ^ I.cv[0]) & I.cm[0];
        unroll<NW>([&](auto jj) {
            constexpr int j = jj.value;
            if constexpr (j >= 1 && j <= LW) acc |= (L.s[h][j] ^ I.cv[j]) & I.cm[j];
        });
        const bool m = acc == 0u;
        L.re[h] = m ? -L.re[h] : L.re[h];
        L.im[h] = m ? -L.im[h] : L.im[h];
    });
}

// Wave-uniform masks of a bit field [lo, hi) of the state (hi <= 128), as
// four 32-bit words: fm = the field, dp = +2^lo and dn = -2^lo in two's
// complement over 128 bits (every bit from lo up).
struct FieldMasks {
    uint32_t fm[4], dp[4], dn[4];
};
__device__ __forceinline__ FieldMasks field_masks(uint32_t lo, uint32_t hi) {
    FieldMasks f;
    for (int w = 0; w < 4; ++w) {
        const uint32_t b0 = 32u * static_cast<uint32_t>(w);
        // bits of word w below lo / below hi
        const uint32_t blo = lo <= b0 ? 0u : (lo >= b0 + 32u ? ~0u : ((1u << (lo - b0)) - 1u));
        const uint32_t bhi = hi <= b0 ? 0u : (hi >= b0 + 32u ? ~0u : ((1u << (hi - b0)) - 1u));
        f.fm[w] = bhi & ~blo;
        f.dn[w] = ~blo;
        f.dp[w] = (lo >> 5) == static_cast<uint32_t>(w) ? (1u << (lo & 31u)) : 0u;
    }
    return f;
}

// The control test of a controlled op on history h: all of ((s ^ cv) & cm)
// over words 0..LW is zero.
template <int NW, int H, int LW>
__device__ __forceinline__ bool controls_hold(const Lanes<NW, H> &L, int h, const Instr &I) {
    uint32_t acc = (L.s[h][0] ^ I.cv[0]) & I.cm[0];
    unroll<NW>([&](auto jj) {
        constexpr int j = jj.value;
        if constexpr (j >= 1 && j <= LW) acc |= (L.s[h][j] ^ I.cv[j]) & I.cm[j];
    });
    return acc == 0u;
}

// state += d over the state's words with one carry chain, keeping the sum
// only on the field bits fm: no bit below the field changes (d has no bits
// there), and whatever the carry does above the field is discarded.
template <int NW, int H>
__device__ __forceinline__ void add_into_field(Lanes<NW, H> &L, int h, const uint32_t (&d)[NW],
                                               const uint32_t (&fm)[4]) {
    uint32_t carry = 0;
    unroll<NW>([&](auto ww) {
        constexpr int w = ww.value;
        const uint32_t x = L.s[h][w];
        const uint32_t r = __builtin_addc(x, d[w], carry, &carry);
        L.s[h][w] = (x & ~fm[w]) | (r & fm[w]);
    });
}

// Folded ladder (OP_ADD): when the controls match, add one to (zmask bit
// 0: subtract one from) the bit field [lo, lo+m) of the state, mod 2^m, as
// an addition of +-2^lo to the whole state.  A history whose controls do
// not match adds zero: the addend is selected, not the result, so the cost
// is one select per history instead of one per state word.
template <int NW, int H, int LW>
__device__ __forceinline__ void op_add(Lanes<NW, H> &L, const Instr &I) {
    const uint32_t lo = hdr_a(I);
    const FieldMasks f = field_masks(lo, lo + hdr_b(I));
    const bool sub = (hdr_z(I) & 1u) != 0u;
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t gm = controls_hold<NW, H, LW>(L, h, I) ? ~0u : 0u;
        uint32_t d[NW];
        unroll<NW>([&](auto ww) {
            constexpr int w = ww.value;
            d[w] = (sub ? f.dn[w] : f.dp[w]) & gm;
        });
        add_into_field<NW, H>(L, h, d, f.fm);
    });
}

// Paired ladders (OP_ADDSEL): when the controls match, add one to the
// field when state bit k equals s and zmask bit s is clear, subtract one
// when it is set.  Two folded ladders on the same field under controls that
// differ only in bit k (outside the field) are mutually exclusive and
// neither changes what the other tests, so together they are one addition
// of an addend chosen per history: one carry chain instead of two.
template <int NW, int H, int LW, int SW>
__device__ __forceinline__ void op_addsel(Lanes<NW, H> &L, const Instr &I) {
    const uint32_t lo = hdr_a(I);
    const FieldMasks f = field_masks(lo, lo + hdr_b(I));
    const uint32_t z = hdr_z(I), kb = I.k & 31u;
    uint32_t d0[4], dx[4];   // addend when bit k is 0, and its xor with the addend when it is 1
    for (int w = 0; w < 4; ++w) {
        d0[w] = (z & 1u) ? f.dn[w] : f.dp[w];
        dx[w] = d0[w] ^ ((z & 2u) ? f.dn[w] : f.dp[w]);
    }
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t gm = controls_hold<NW, H, LW>(L, h, I) ? ~0u : 0u;
        const uint32_t sel = 0u - ((L.s[h][SW] >> kb) & 1u);   // all ones when bit k is set
        uint32_t d[NW];
        unroll<NW>([&](auto ww) {
            constexpr int w = ww.value;
            d[w] = (d0[w] ^ (dx[w] & sel)) & gm;
        });
        add_into_field<NW, H>(L, h, d, f.fm);
    });
}

// Pending field additions (straight-line regions).  Folded ladders on one
// field, with nothing between them that reads or writes a field bit, add up:
// (x + d1 + d2) mod 2^m = ((x + d1) mod 2^m + d2) mod 2^m.  The compiled
// regions therefore accumulate each history's +-1 steps as signed counts and
// add (pk + 2 pb) * 2^lo to the field with one carry chain (flush_field)
// before the next instruction that touches the field, and at the region's
// end: pk sums the steps' values when their selecting bit is 0, pb counts
// (with sign) the steps whose selecting bit flips that value, so a run of
// steps costs a bit extract and an add each, with no selects.
template <int NW, int H, int LW>
__device__ __forceinline__ void pend_add(const Lanes<NW, H> &L, const Instr &I, int32_t (&pk)[H],
                                         int32_t (&pb)[H]) {
    (void)pb;
    const int32_t d = (hdr_z(I) & 1u) ? -1 : 1;
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const int32_t gm = controls_hold<NW, H, LW>(L, h, I) ? -1 : 0;
        pk[h] += d & gm;
    });
}

template <int NW, int H, int LW, int SW>
__device__ __forceinline__ void pend_addsel(const Lanes<NW, H> &L, const Instr &I, int32_t (&pk)[H],
                                            int32_t (&pb)[H]) {
    const uint32_t z = hdr_z(I), kb = I.k & 31u;
    const int32_t d0 = (z & 1u) ? -1 : 1, d1 = (z & 2u) ? -1 : 1;   // step when bit k is 0 / 1
    const int32_t half = (d1 - d0) / 2;                             // -1, 0 or 1
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const int32_t bit = static_cast<int32_t>((L.s[h][SW] >> kb) & 1u);
        const int32_t gm = controls_hold<NW, H, LW>(L, h, I) ? -1 : 0;
        pk[h] += d0 & gm;
        if (half > 0) pb[h] += bit & gm;
        if (half < 0) pb[h] -= bit & gm;
    });
}

// Ladder steps of a pending run without controls whose selecting bit holds
// a source bit of the region (set by a branching gate earlier in the region,
// not written since): each adds its constant part d0 and, for a source bit
// of 1, d1 - d0 = +-2, so together they add kc to pk and the popcount of the
// source index over `pos` minus that over `neg` to pb (n = pk + 2 pb).
template <int NW, int H>
__device__ __forceinline__ void pend_src(const Lanes<NW, H> &L, int32_t (&pk)[H], int32_t (&pb)[H], int32_t &pbq,
                                         int32_t kc, uint64_t pos, uint64_t neg) {
    // hb and hq hold disjoint bits, so the popcounts split: hb's part per
    // lane into pb, hq's (the same in every lane) into the scalar pbq
    if ((pos | neg) >> 32) {
        pbq += __popcll(L.hq & pos) - __popcll(L.hq & neg);
    } else {
        const uint32_t hq = static_cast<uint32_t>(L.hq);
        if (pos) pbq += __popc(hq & static_cast<uint32_t>(pos));
        if (neg) pbq -= __popc(hq & static_cast<uint32_t>(neg));
    }
    pbq += __popc(L.hu & static_cast<uint32_t>(pos)) - __popc(L.hu & static_cast<uint32_t>(neg));
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        pk[h] += kc;
        if ((pos | neg) >> 32) {
            pb[h] += __popcll(L.hb[h] & pos) - __popcll(L.hb[h] & neg);
        } else {
            const uint32_t hb = static_cast<uint32_t>(L.hb[h]);
            if (pos) pb[h] += __popc(hb & static_cast<uint32_t>(pos));
            if (neg) pb[h] -= __popc(hb & static_cast<uint32_t>(neg));
        }
    });
}

template <int NW, int H>
__device__ __forceinline__ void flush_field(Lanes<NW, H> &L, uint32_t lo, uint32_t hi, int32_t (&pk)[H],
                                            int32_t (&pb)[H], int32_t &pbq) {
    const FieldMasks f = field_masks(lo, hi);
    const uint32_t wl = lo >> 5, sh = lo & 31u;
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const int32_t n = pk[h] + 2 * (pb[h] + pbq);
        // n * 2^lo in two's complement over the state's words
        const int64_t v = static_cast<int64_t>(n) * (static_cast<int64_t>(1) << sh);
        const uint32_t lo32 = static_cast<uint32_t>(static_cast<uint64_t>(v));
        const uint32_t hi32 = static_cast<uint32_t>(static_cast<uint64_t>(v) >> 32);
        const uint32_t sgn = n < 0 ? ~0u : 0u;
        uint32_t d[NW];
        unroll<NW>([&](auto ww) {
            constexpr uint32_t w = static_cast<uint32_t>(ww.value);
            d[w] = w < wl ? 0u : (w == wl ? lo32 : (w == wl + 1u ? hi32 : sgn));
        });
        add_into_field<NW, H>(L, h, d, f.fm);
        pk[h] = 0;
        pb[h] = 0;
    });
    pbq = 0;
}

// The residue (output - state) on the field [lo, hi) in the form the final
// check compares it with a step count n: n matches iff (n << up) == (e << up)
// for the returned e.  For m = hi - lo <= 32 bits, e holds the residue's low 32 bits and
// up = 32 - m (only the field's m low bits count).  For wider fields up = 0
// and e is the residue as an int32 when it is one, else a value no step
// count reaches (|n| is at most the number of steps): n sign-extended to m
// bits equals the residue iff their low 32 bits agree and bits [lo+32, hi)
// all repeat bit 31, and equal int32 values are equal mod 2^32.
template <int NW>
__device__ __forceinline__ uint32_t field_residue(const uint32_t (&s)[NW], const uint32_t (&bin)[NW], uint32_t lo,
                                                  uint32_t hi, uint32_t &up) {
    const FieldMasks f = field_masks(lo, hi);
    const FieldMasks g = field_masks(lo + 32u < hi ? lo + 32u : hi, hi);   // bits [lo+32, hi)
    const uint32_t m = hi - lo, wl = lo >> 5, sh = lo & 31u;
    // bits [lo, hi) of d hold the residue
    uint32_t d[NW], borrow = 0;
    unroll<NW>([&](auto ww) {
        constexpr int w = ww.value;
        d[w] = __builtin_subc(bin[w] & f.fm[w], s[w] & f.fm[w], borrow, &borrow);
    });
    uint32_t x0 = 0, x1 = 0, zhi = 0, ohi = 0;
    unroll<NW>([&](auto ww) {
        constexpr uint32_t w = static_cast<uint32_t>(ww.value);
        if (w == wl) x0 = d[w];
        if (w == wl + 1u) x1 = d[w];
        zhi |= d[w] & g.fm[w];
        ohi |= ~d[w] & g.fm[w];
    });
    const uint32_t e32 = sh ? (x0 >> sh) | (x1 << (32u - sh)) : x0;   // bits [lo, lo+32) of d
    if (m <= 32u) {
        up = 32u - m;
        return e32;
    }
    up = 0u;
    const bool fits = static_cast<int32_t>(e32) < 0 ? ohi == 0u : zhi == 0u;
    return fits ? e32 : 0x80000000u;
}

// The last pending run of a region after which the final check compares
// every bit of the field with the output: (x + n) mod 2^m equals the target
// t iff n = (t - x) mod 2^m, so instead of adding n 2^lo to the field and
// comparing its words, compare the step count n with that residue.  The
// residue reads only the field and the output; when nothing earlier in the
// region writes the field it is the same for every suffix assignment and the
// compiler computes it once per root history, leaving one compare per
// history.  The field's bits are left as they were, so the final check that
// follows must leave them out (nothing else reads them after the region).
// The count is compared as 2 pbq = residue - pk - 2 pb (mod 2^32): the right
// side does not depend on the wave-uniform sources, so inside the suffix
// loop it is computed once per root history and each leaf costs one compare
// against a scalar.
template <int NW, int H>
__device__ __forceinline__ void flush_check(Lanes<NW, H> &L, uint32_t lo, uint32_t hi, int32_t (&pk)[H],
                                            int32_t (&pb)[H], int32_t &pbq, const uint32_t (&bin)[NW]) {
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        uint32_t up;
        const uint32_t e = field_residue<NW>(L.s[h], bin, lo, hi, up);
        // the step count is n = pk + 2 pb + 2 pbq
        const uint32_t nl = static_cast<uint32_t>(pk[h]) + 2u * static_cast<uint32_t>(pb[h]);
        const uint32_t nq = 2u * static_cast<uint32_t>(pbq);
        L.ok[h] = L.ok[h] && (nq << up) == ((e - nl) << up);
        pk[h] = 0;
        pb[h] = 0;
    });
    pbq = 0;
}

template <int NW, int H, int WA, int WB>
__device__ __forceinline__ void op_swap(Lanes<NW, H> &L, const Instr &I) {
    constexpr int A = wsel<WA, NW>(), B = wsel<WB, NW>();
    const uint32_t sa = hdr_a(I) & 31u, sb = hdr_b(I) & 31u;
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        uint32_t acc = 0;
        unroll<NW>([&](auto jj) {
            constexpr int j = jj.value;
            acc |= (L.s[h][j] ^ I.cv[j]) & I.cm[j];
        });
        const uint32_t d = (((L.s[h][A] >> sa) ^ (L.s[h][B] >> sb)) & 1u) & (acc == 0u ? 1u : 0u);
        L.s[h][A] ^= d << sa;
        L.s[h][B] ^= d << sb;
    });
}

template <int NW, int H, int WA, int DEFER = -1, class FR = FacRef>
__device__ __forceinline__ void op_det1(Lanes<NW, H> &L, const Instr &I, const FR &F) {
    constexpr int A = wsel<WA, NW>();
    const uint32_t sh = hdr_a(I) & 31u;
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t o = (L.s[h][A] >> sh) & 1u;
        take_factor<DEFER>(L, h, F, I.fac, o);
        L.s[h][A] ^= 1u << sh;
    });
}

template <int NW, int H, int WA, int DEFER = -1, class FR = FacRef>
__device__ __forceinline__ void op_diag1(Lanes<NW, H> &L, const Instr &I, const FR &F) {
    constexpr int A = wsel<WA, NW>();
    const uint32_t sh = hdr_a(I) & 31u;
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t o = (L.s[h][A] >> sh) & 1u;
        take_factor<DEFER>(L, h, F, I.fac, o);
    });
}

template <int NW, int H, int WA, int WB, int DEFER = -1, class FR = FacRef>
__device__ __forceinline__ void op_diag2(Lanes<NW, H> &L, const Instr &I, const FR &F) {
    constexpr int A = wsel<WA, NW>(), B = wsel<WB, NW>();
    const uint32_t sa = hdr_a(I) & 31u, sb = hdr_b(I) & 31u;
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t x = ((L.s[h][A] >> sa) & 1u) | (((L.s[h][B] >> sb) & 1u) << 1);
        take_factor<DEFER>(L, h, F, I.fac, x);
    });
}

template <int NW, int H, bool PRUNE, int WA, bool SRC, int DEFER = -1, class FR = FacRef>
__device__ __forceinline__ void op_branch(Lanes<NW, H> &L, const Instr &I, const FR &F,
                                          uint32_t kbase, const uint32_t (&bin)[NW], double thr) {
    static_assert(!(PRUNE && DEFER >= 0), "pruning needs the moduli as the walk goes");
    constexpr int A = wsel<WA, NW>();
    const uint32_t sh = hdr_a(I) & 31u;
    const uint32_t ks = I.k - kbase;
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t o = (L.s[h][A] >> sh) & 1u;
        const uint32_t i = SRC ? src_bit(L, h, ks) : (bin[A] >> sh) & 1u;
        const uint32_t x = 2u * o + i;
        take_factor<DEFER>(L, h, F, I.fac, x);
        if (PRUNE) {
            L.M[h] = L.M[h] * F.d(I.fac + 8u + x);
            L.ok[h] = L.ok[h] && !(L.M[h] < thr);
        }
        L.ok[h] = L.ok[h] && !((hdr_z(I) >> x) & 1u);
        L.s[h][A] ^= (o ^ i) << sh;
    });
}

// ---------------------------------------------------------------------------
// Factor steps with the gate's table as compile-time constants (the compiled
// regions): for the table shapes below the factor is formed in registers from
// the selecting bits instead of being read from a table per lane.  Each
// computes the same product as the table step: the same factor entry
// multiplied into the running amplitude in the same order.
// ---------------------------------------------------------------------------

// x with its sign flipped where bit 31 of f is set.
__device__ __forceinline__ double flip_sign(double x, uint32_t f) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x) ^ (static_cast<uint64_t>(f & 0x80000000u) << 32);
    return __builtin_bit_cast(double, b);
}

// Diagonal gate whose two distinct entries are a complex-conjugate pair
// (C, S) and (C, -S), selected by one bit (DIAG1: entry 0 when bit a is 0)
// or by the parity of two (DIAG2 tables {t, u, u, t}: entry 0 when bits a
// and b agree), e.g. RZ and RZZ: the selecting bit moved to bit 31 flips the
// sign of S, then one complex multiply.
template <int NW, int H, int WA, int WB, bool TWO>
__device__ __forceinline__ void op_conj(Lanes<NW, H> &L, uint32_t sa, uint32_t sb, double C, double S) {
    constexpr int A = wsel<WA, NW>(), B = wsel<WB, NW>();
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        uint32_t f = L.s[h][A] << (31u - sa);
        if constexpr (TWO) f ^= L.s[h][B] << (31u - sb);
        cmul(L.re[h], L.im[h], C, flip_sign(S, f));
    });
}

// Branching gate whose four entries U[o][i] are real, of one magnitude r
// and one modulus m (e.g. H): the factor is r times the sign of entry
// x = 2o + i (neg has bit x set when U[o][i] < 0).  The amplitude is
// multiplied by r, and the sign goes into sg: a word whose popcount parity
// is the product of the region's signs so far, applied once at the region's
// end (apply_signs).  Negation is exact and commutes with every rounding of
// the complex and real multiplies, so this is the same amplitude as
// multiplying by the signed entry at the gate.  The input bit comes from the
// source (SRC) or from the input bitstring and replaces bit a of the state.
// No entry is zero.
// With MUL false the magnitude is left out too: every such factor's r is
// the same for every history, so the region multiplies their product in
// once, at its end with the signs (scale_amp).
template <int NW, int H, bool PRUNE, int WA, bool SRC, bool MUL = true>
__device__ __forceinline__ void op_branch_real(Lanes<NW, H> &L, uint32_t (&sg)[H], uint32_t sa, uint32_t ks,
                                               const uint32_t (&bin)[NW], double thr, double r,
                                               uint32_t neg, double m) {
    constexpr int A = wsel<WA, NW>();
    const uint32_t bit = 1u << sa;
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t s0 = L.s[h][A];
        uint32_t snew;
        if constexpr (SRC) {
            const uint32_t i = src_bit(L, h, ks);
            sg[h] ^= (neg >> (((s0 >> sa) & 1u) * 2u + i)) & 1u;   // the entry's sign
            snew = (s0 & ~bit) | (i << sa);
        } else {
            if (neg == 8u) sg[h] ^= s0 & bin[A] & bit;      // negative only at o = i = 1
            else if (neg != 0u) sg[h] ^= (neg >> (((s0 >> sa) & 1u) * 2u + ((bin[A] >> sa) & 1u))) & 1u;
            snew = (s0 & ~bit) | (bin[A] & bit);
        }
        if constexpr (MUL) {
            L.re[h] *= r;
            L.im[h] *= r;
        }
        if (PRUNE) {
            L.M[h] = L.M[h] * m;
            L.ok[h] = L.ok[h] && !(L.M[h] < thr);
        }
        L.s[h][A] = snew;
    });
}

// The signs op_branch_real collected: negate the amplitude where the parity
// of sg is odd, and start over.
// The same gate in a region whose factors are deferred to the histories
// that pass the final check: only the state and the entry's sign (into
// L.sd) change here; the magnitude r is the same for every history and is
// multiplied in once for the valid ones, with the region's other deferred
// factors.
template <int NW, int H, int WA, bool SRC>
__device__ __forceinline__ void op_branch_real_sign(Lanes<NW, H> &L, uint32_t sa, uint32_t ks,
                                                    const uint32_t (&bin)[NW], uint32_t neg) {
    constexpr int A = wsel<WA, NW>();
    const uint32_t bit = 1u << sa;
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t s0 = L.s[h][A];
        const uint32_t i = SRC ? src_bit(L, h, ks) : (bin[A] >> sa) & 1u;
        L.sd[h] ^= (neg >> (((s0 >> sa) & 1u) * 2u + i)) & 1u;
        L.s[h][A] = (s0 & ~bit) | (i << sa);
    });
}

// The region's real-entry magnitudes, one constant (op_branch_real, MUL
// false).
template <int NW, int H>
__device__ __forceinline__ void scale_amp(Lanes<NW, H> &L, double r) {
    unroll<H>([&](auto hh) {
        L.re[hh.value] *= r;
        L.im[hh.value] *= r;
    });
}

template <int NW, int H>
__device__ __forceinline__ void apply_signs(Lanes<NW, H> &L, uint32_t (&sg)[H]) {
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t f = static_cast<uint32_t>(__popc(sg[h])) << 31;
        L.re[h] = flip_sign(L.re[h], f);
        L.im[h] = flip_sign(L.im[h], f);
        sg[h] = 0u;
    });
}

// ---------------------------------------------------------------------------
// Counted factors (the compiled consumer without pruning).  A gate whose
// factor table takes two values, a where bit x of TT is clear and b where it
// is set (x the table index the gate selects), belongs to the class of the
// gates with that pair.  A history's product over a class's n gates is
// a^(n-f) b^f, f the number of b entries it took: the history keeps f, as a
// field of its index ci (a gate of the class moves it by the class's step
// d), and the consumer multiplies in the tabulated product once, for the
// histories that pass the final check.  The same amplitude up to rounding.
// ---------------------------------------------------------------------------

// Whether bit lo | hi << 1 of TT is set, for the truth tables of the common
// gates written as the bit operation they are.
template <uint32_t TT>
__device__ __forceinline__ uint32_t tt_sel(uint32_t lo, uint32_t hi) {
    if constexpr (TT == 0x6u) return lo ^ hi;
    else if constexpr (TT == 0x9u) return (lo ^ hi) ^ 1u;
    else if constexpr (TT == 0x8u) return lo & hi;
    else if constexpr (TT == 0x7u) return (lo & hi) ^ 1u;
    else if constexpr (TT == 0xeu) return lo | hi;
    else if constexpr (TT == 0x1u) return (lo | hi) ^ 1u;
    else if constexpr (TT == 0xau) return lo;
    else if constexpr (TT == 0x5u) return lo ^ 1u;
    else if constexpr (TT == 0xcu) return hi;
    else if constexpr (TT == 0x3u) return hi ^ 1u;
    else return (TT >> (lo | (hi << 1))) & 1u;
}

// A diagonal gate (DIAG1: x = bit a; DIAG2: x = bit a | bit b << 1), counted.
template <int NW, int H, int WA, int WB, uint32_t TT, bool TWO>
__device__ __forceinline__ void op_count_diag(Lanes<NW, H> &L, uint32_t sa, uint32_t sb, uint32_t d) {
    constexpr int A = wsel<WA, NW>(), B = wsel<WB, NW>();
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t lo = (L.s[h][A] >> sa) & 1u;
        const uint32_t hi = TWO ? (L.s[h][B] >> sb) & 1u : 0u;
        L.ci[h] += tt_sel<TT>(lo, hi) * d;
    });
}

// A deterministic one-qubit gate (x = bit a, then bit a flips), counted.
template <int NW, int H, int WA, uint32_t TT>
__device__ __forceinline__ void op_det1_count(Lanes<NW, H> &L, uint32_t sa, uint32_t d) {
    constexpr int A = wsel<WA, NW>();
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        L.ci[h] += tt_sel<TT>((L.s[h][A] >> sa) & 1u, 0u) * d;
        L.s[h][A] ^= 1u << sa;
    });
}

// A branching gate (x = 2o + i, o the state's bit a, i the source's or the
// input's), counted; bit a becomes i.  No entry is zero.
template <int NW, int H, int WA, bool SRC, uint32_t TT>
__device__ __forceinline__ void op_branch_count(Lanes<NW, H> &L, uint32_t sa, uint32_t ks,
                                                const uint32_t (&bin)[NW], uint32_t d) {
    constexpr int A = wsel<WA, NW>();
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t o = (L.s[h][A] >> sa) & 1u;
        const uint32_t i = SRC ? src_bit(L, h, ks) : (bin[A] >> sa) & 1u;
        L.ci[h] += tt_sel<TT>(i, o) * d;
        L.s[h][A] ^= (o ^ i) << sa;
    });
}

// Counted diagonal gates of one class on one state word with no state write
// between them, grouped: b is taken where bit q and bit q + dist differ
// (KIND 0), agree (1) or are both set (2), or, for one-bit gates, where bit
// q is set (3) or clear (4); `mask` has bit q of each gate of the group, and
// n[h] gains their number of b entries, a population count.
template <int NW, int H, int W, int KIND>
__device__ __forceinline__ void count_bits(const Lanes<NW, H> &L, uint32_t (&n)[H], uint32_t dist,
                                           uint32_t mask) {
    constexpr int A = wsel<W, NW>();
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t s = L.s[h][A];
        uint32_t y;
        if constexpr (KIND == 0) y = s ^ (s >> dist);
        else if constexpr (KIND == 1) y = ~(s ^ (s >> dist));
        else if constexpr (KIND == 2) y = s & (s >> dist);
        else if constexpr (KIND == 3) y = s;
        else y = ~s;
        n[h] += static_cast<uint32_t>(__popc(y & mask));
    });
}

// A pure leaf's amplitude is +-1 (its signs) when its counted product is
// taken: the product with that sign replaces it.
__device__ __forceinline__ void count_set(double &re, double &im, double2 f) {
    const uint32_t s = static_cast<uint32_t>(__builtin_bit_cast(uint64_t, re) >> 32) & 0x80000000u;
    re = flip_sign(f.x, s);
    im = flip_sign(f.y, s);
}

template <int NW, int H>
__device__ __forceinline__ void count_take(Lanes<NW, H> &L, const uint32_t (&n)[H], uint32_t d) {
    unroll<H>([&](auto hh) { L.ci[hh.value] += n[hh.value] * d; });
}

// Branching gate whose input bit is an affine form (sources placed by
// reachability): the parity of the history index over the form's sources
// (cm[0], cm[1]), xor the pair's boundary bit k of the form; otherwise as
// op_branch.
template <int NW, int H, bool PRUNE, int WA, int DEFER = -1, class FR = FacRef>
__device__ __forceinline__ void op_branch_aff(Lanes<NW, H> &L, const Instr &I, const FR &F, uint32_t kbase,
                                              double thr) {
    static_assert(!(PRUNE && DEFER >= 0), "pruning needs the moduli as the walk goes");
    constexpr int A = wsel<WA, NW>();
    const uint32_t sh = hdr_a(I) & 31u;
    const uint64_t smask = static_cast<uint64_t>(I.cm[0]) | (static_cast<uint64_t>(I.cm[1]) << 32);
    const uint32_t cbit = static_cast<uint32_t>(L.aff >> I.k) & 1u;
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        const uint32_t o = (L.s[h][A] >> sh) & 1u;
        const uint64_t full = L.hf[h] | ((L.hb[h] | L.hq | L.hu) << kbase);
        const uint32_t i = (static_cast<uint32_t>(__popcll(full & smask)) & 1u) ^ cbit;
        const uint32_t x = 2u * o + i;
        take_factor<DEFER>(L, h, F, I.fac, x);
        if (PRUNE) {
            L.M[h] = L.M[h] * F.d(I.fac + 8u + x);
            L.ok[h] = L.ok[h] && !(L.M[h] < thr);
        }
        L.ok[h] = L.ok[h] && !((hdr_z(I) >> x) & 1u);
        L.s[h][A] ^= (o ^ i) << sh;
    });
}

// The boundary bits of the affine forms for one pair: bit j = parity of the
// check bitstring over form j's input-bit mask, xor the parity of the start
// bitstring over its output-bit mask, xor its constant.
template <int NW>
__device__ __forceinline__ uint64_t affine_bits(const Common &c, const uint32_t (&bin)[NW],
                                                const uint32_t (&bout)[NW]) {
    uint64_t bits = 0;
    for (uint32_t j = 0; j < c.n_aff; ++j) {
        const uint32_t *f = c.aff_tab + 9u * j;
        uint32_t p = f[8];
        unroll<NW>([&](auto ww) {
            constexpr int w = ww.value;
            p ^= static_cast<uint32_t>(__popc(bin[w] & f[w])) ^ static_cast<uint32_t>(__popc(bout[w] & f[4 + w]));
        });
        bits |= static_cast<uint64_t>(p & 1u) << j;
    }
    return bits;
}

// Walk evaluation positions [e0, e1) of the history program backward for H
// histories at once.  Source k of history h reads bit (k - kbase) of hb[h];
// bin is the input bitstring (the same for every history of a lane).  The
// opcode is dispatched once per run of identical opcodes; the case loops
// over the run.
template <int NW, int H, bool PRUNE, bool RUNS>
__device__ __forceinline__ void run_region(const Instr *prog_generic, const FacRef &F,
                                           uint32_t e0, uint32_t e1, Lanes<NW, H> &L,
                                           uint32_t kbase, const uint32_t (&bin)[NW], double thr) {
    ConstInstr *prog = (ConstInstr *)prog_generic;
    uint32_t e = e0;
    while (e < e1) {
        const uint32_t op = prog[e].hdr & 0xffu;
        const uint32_t end = RUNS ? e + min(prog[e].run, e1 - e) : e + 1u;
        const uint32_t w1 = (op >> 4) & 3u, w2 = (op >> 6) & 3u;
        // the instructions of this dispatch: the run, or just prog[e]
        auto each = [&](auto &&f) {
            if constexpr (RUNS) {
                for (uint32_t x = e; x < end; ++x) {
                    const Instr I = prog[x];
                    f(I);
                }
            } else {
                const Instr I = prog[e];
                f(I);
            }
        };
        switch (op & 15u) {
            case OP_PERM:
                with_word<NW>(w1, [&](auto TW) {
                    with_word<NW>(w2, [&](auto LW) {
                        each([&](const Instr &I) { op_perm<NW, H, TW.value, LW.value>(L, I); });
                    });
                });
                break;
            case OP_BRANCH_SRC:
                with_word<NW>(w1, [&](auto WA) {
                    each([&](const Instr &I) { op_branch<NW, H, PRUNE, WA.value, true>(L, I, F, kbase, bin, thr); });
                });
                break;
            case OP_BRANCH_NAT:
                with_word<NW>(w1, [&](auto WA) {
                    each([&](const Instr &I) { op_branch<NW, H, PRUNE, WA.value, false>(L, I, F, kbase, bin, thr); });
                });
                break;
            case OP_BRANCH_AFF:
                with_word<NW>(w1, [&](auto WA) {
                    each([&](const Instr &I) { op_branch_aff<NW, H, PRUNE, WA.value>(L, I, F, kbase, thr); });
                });
                break;
            case OP_DIAG2:
                with_word<NW>(w1, [&](auto WA) {
                    with_word<NW>(w2, [&](auto WB) {
                        each([&](const Instr &I) { op_diag2<NW, H, WA.value, WB.value>(L, I, F); });
                    });
                });
                break;
            case OP_DIAG1:
                with_word<NW>(w1, [&](auto WA) {
                    each([&](const Instr &I) { op_diag1<NW, H, WA.value>(L, I, F); });
                });
                break;
            case OP_MCPHASE:
                with_word<NW>(w1, [&](auto LW) {
                    each([&](const Instr &I) { op_mcphase<NW, H, LW.value>(L, I); });
                });
                break;
            case OP_SWAP:
                with_word<NW>(w1, [&](auto WA) {
                    with_word<NW>(w2, [&](auto WB) {
                        each([&](const Instr &I) { op_swap<NW, H, WA.value, WB.value>(L, I); });
                    });
                });
                break;
            case OP_DET1:
                with_word<NW>(w1, [&](auto WA) {
                    each([&](const Instr &I) { op_det1<NW, H, WA.value>(L, I, F); });
                });
                break;
            case OP_ADD:
                with_word<NW>(w1, [&](auto LW) {
                    each([&](const Instr &I) { op_add<NW, H, LW.value>(L, I); });
                });
                break;
            case OP_ADDSEL:
                with_word<NW>(w1, [&](auto LW) {
                    with_word<NW>(w2, [&](auto SW) {
                        each([&](const Instr &I) { op_addsel<NW, H, LW.value, SW.value>(L, I); });
                    });
                });
                break;
            default:
                break;
        }
        e = end;
        // With pruning, histories die at branching gates; once no history of
        // the wave is alive the rest of the region cannot change any result.
        if constexpr (PRUNE) {
            const uint32_t base = op & 15u;
            if (base == OP_BRANCH_SRC || base == OP_BRANCH_NAT || base == OP_BRANCH_AFF) {
                bool any = false;
                unroll<H>([&](auto hh) { any = any || L.ok[hh.value]; });
                if (!__any(any)) return;
            }
        }
    }
}

// Copy every per-history register of src into dst except the source bits.
template <int NW, int H>
__device__ __forceinline__ void copy_core(Lanes<NW, H> &dst, const Lanes<NW, H> &src) {
    unroll<H>([&](auto hh) {
        constexpr int h = hh.value;
        unroll<NW>([&](auto ww) { dst.s[h][ww.value] = src.s[h][ww.value]; });
        dst.re[h] = src.re[h];
        dst.im[h] = src.im[h];
        dst.M[h] = src.M[h];
        dst.ok[h] = src.ok[h];
    });
}

// Depth-first enumeration of the D <= DMAX consecutive sources k0 ..
// k0+D-1 (evaluation order) of a region that ends at e_end.  On entry L
// holds each history's state just before source k0's gate; its hb carries
// the region's other source bits.  For every one of the 2^D assignments
// (source k0 varying slowest) the histories are carried to e_end and
// leaf(C) is called with C.hb holding the assignment.  The gates between
// source k0+l and the next enumerated source run 2^(l+1) times rather than
// 2^D: the state before each enumerated source is kept in registers and
// reused by every assignment that agrees on the earlier sources (the
// checkpoint idea of Algorithm 2 applied at every source).  Control flow is
// wave-uniform throughout.
template <int NW, int H, int DMAX, class Seg, class Leaf>
__device__ __forceinline__ void dfs_region(uint32_t k0, uint32_t D, const Lanes<NW, H> &L,
                                           uint32_t kbase, Seg &&seg, Leaf &&leaf) {
    Lanes<NW, H> C = L;
    Lanes<NW, H> S[DMAX];      // S[l]: state before level l's source (l >= 1)
    const uint32_t nt = 1u << D;
    for (uint32_t t = 0; t < nt; ++t) {
        uint32_t l0 = 0;
        if (t != 0u) {
            // the levels whose bit changed since t - 1 are l0 .. D-1
            l0 = D - 1u - static_cast<uint32_t>(__builtin_ctz(t));
            unroll<DMAX>([&](auto LV) {
                if (static_cast<uint32_t>(LV.value) == l0) {
                    if constexpr (LV.value == 0) copy_core(C, L);
                    else copy_core(C, S[LV.value]);
                }
            });
        }
        for (uint32_t l = l0; l < D; ++l) {
            const uint32_t kb = k0 + l - kbase;
            const uint64_t bit = static_cast<uint64_t>((t >> (D - 1u - l)) & 1u) << kb;
            unroll<H>([&](auto hh) { C.hb[hh.value] = (C.hb[hh.value] & ~(1ull << kb)) | bit; });
            seg(l, C);   // the gates from level l's source up to the next level's
            if (l + 1u < D) {
                unroll<DMAX>([&](auto LV) {
                    if constexpr (LV.value > 0)
                        if (static_cast<uint32_t>(LV.value) == l + 1u) copy_core(S[LV.value], C);
                });
            }
        }
        leaf(C);
    }
}

// Copy the factor slice [lo, hi) of the global table into LDS.
__device__ __forceinline__ void stage_factors(double *lds, const double *fac, uint32_t lo,
                                              uint32_t hi) {
    for (uint32_t i = threadIdx.x; i < hi - lo; i += blockDim.x) lds[i] = fac[lo + i];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// deterministic workgroup reduction of (amp, 4 counters)
// ---------------------------------------------------------------------------

struct Acc {
    double re, im;
    uint64_t nval, sumh, xorh, leaves;
};

__device__ __forceinline__ void wave_reduce(Acc &a) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a.re += __shfl_xor(a.re, off, 64);
        a.im += __shfl_xor(a.im, off, 64);
        a.nval += __shfl_xor(a.nval, off, 64);
        a.sumh += __shfl_xor(a.sumh, off, 64);
        a.xorh ^= __shfl_xor(a.xorh, off, 64);
        a.leaves += __shfl_xor(a.leaves, off, 64);
    }
}

template <int NT>
__device__ __forceinline__ void block_reduce_store(Acc a, Acc *lds, Partials part, uint32_t idx) {
    wave_reduce(a);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc t = lds[0];
        for (int w = 1; w < NT / 64; ++w) {
            t.re += lds[w].re;
            t.im += lds[w].im;
            t.nval += lds[w].nval;
            t.sumh += lds[w].sumh;
            t.xorh ^= lds[w].xorh;
            t.leaves += lds[w].leaves;
        }
        part.amp[idx] = make_double2(t.re, t.im);
        uint64_t *st = part.st + 4ull * idx;
        st[0] = t.nval;
        st[1] = t.sumh;
        st[2] = t.xorh;
        st[3] = t.leaves;
    }
    __syncthreads();
}

// Regions policy of the interpreting consumer.
template <bool RUNS>
struct Interp {
    static constexpr bool kDefer = false;   // factors are multiplied as the walk goes
    static constexpr int kUnroll = 1;       // suffix assignments per pass of the leaf loop
    static constexpr int kSS = -1;          // lanes per root task: the launch's
    static constexpr int kAs = -1;          // suffix sources: the program's
    static constexpr int kA = -1;           // sources: the program's
    // prefix region: the gates before the first depth-first source, and the
    // gates of depth-first level l (from its source up to the next level's)
    template <int NW, bool PRUNE>
    __device__ static __forceinline__ void prefix_head(const Common &c, const FacRef &F,
                                                       Lanes<NW, 1> &L, const uint32_t (&bin)[NW],
                                                       uint32_t e_split) {
        run_region<NW, 1, PRUNE, RUNS>(c.prog, F, c.iL, e_split, L, 0, bin, c.thr);
    }
    template <int NW, bool PRUNE>
    __device__ static __forceinline__ void prefix_seg(const Common &c, const FacRef &F,
                                                      Lanes<NW, 1> &C, const uint32_t (&bin)[NW],
                                                      uint32_t k0, uint32_t D, uint32_t l) {
        const uint32_t a = ld_const(c.src, k0 + l);
        const uint32_t b = (l + 1u < D) ? ld_const(c.src, k0 + l + 1u) : c.i1;
        run_region<NW, 1, PRUNE, RUNS>(c.prog, F, a, b, C, 0, bin, c.thr);
    }
    template <int NW, int H>
    __device__ static __forceinline__ void suffix_amp(const FacRef &, Lanes<NW, H> &, int) {}
    // counted factors: none here (kNCT table entries; kLeafPure: the leaf
    // loop multiplies no factor but the counted ones and signs)
    static constexpr uint32_t kNCT = 0;
    static constexpr bool kLeafPure = false;
    __device__ static __forceinline__ double2 count_entry(uint32_t) { return make_double2(0.0, 0.0); }
    template <int NW, int H>
    __device__ static __forceinline__ void count_amp(const double2 *, Lanes<NW, H> &, int) {}
    // whole passes of leaves rejected by the final field check: not here
    static constexpr bool kPassFilter = false;
    static constexpr uint32_t kPassUp = 0u;
    static constexpr uint32_t kPassSpan = 0u;
    static constexpr uint32_t kRootQ = 0u;
    static constexpr int32_t kRootSpan = -1;
    template <int NW, int H>
    __device__ static __forceinline__ void pass_res(const Lanes<NW, H> &, const uint64_t (&)[H],
                                                    const uint32_t (&)[NW], uint32_t (&)[H]) {}
    template <int UU>
    __device__ static __forceinline__ uint32_t pass_q(uint64_t) { return 0u; }
    // suffix instructions evaluated once per root history: none here
    static constexpr bool kHoist = false;
    template <int NW, int H, bool PRUNE>
    __device__ static __forceinline__ void suffix_pre(const Common &, const FacRef &, Lanes<NW, H> &,
                                                      const uint32_t (&)[NW]) {}
    // final-bit checks at c2 and G with the masks read from the program
    template <int NW>
    __device__ static __forceinline__ bool final_c2(const uint32_t (&s)[NW], const uint32_t (&bin)[NW],
                                                    const Mask4 &m) {
        return check_final<NW>(s, bin, m);
    }
    template <int NW>
    __device__ static __forceinline__ bool final_G(const uint32_t (&s)[NW], const uint32_t (&bin)[NW],
                                                   const Mask4 &m) {
        return check_final<NW>(s, bin, m);
    }
    template <int NW, int H, bool PRUNE>
    __device__ static __forceinline__ void root(const Common &c, const FacRef &F, Lanes<NW, H> &L,
                                                const uint32_t (&bin)[NW]) {
        run_region<NW, H, PRUNE, RUNS>(c.prog, F, c.i1, c.i2, L, c.Ap, bin, c.thr);
    }
    template <int NW, int H, bool PRUNE>
    __device__ static __forceinline__ void suffix(const Common &c, const FacRef &F, Lanes<NW, H> &L,
                                                  const uint32_t (&bin)[NW]) {
        run_region<NW, H, PRUNE, RUNS>(c.prog, F, c.i2, c.iG, L, c.Ap + c.Ar, bin, c.thr);
    }
};

// Once no history of the wave is alive (pruning), stop walking the region.
template <int NW, int H>
__device__ __forceinline__ bool wave_alive(const Lanes<NW, H> &L) {
    bool any = false;
    unroll<H>([&](auto hh) { any = any || L.ok[hh.value]; });
    return __any(any);
}

// The prefix-table build (Algorithm 2, first loop) over a Walk policy
// (Interp, or the run-time compiled regions): one lane per subtree of prefix
// assignments; the lane's index fixes the first Ap - Dp prefix sources, the
// last Dp are enumerated depth-first, 2^Dp entries per lane.
template <class Walk, int NW, bool PRUNE, bool FLDS>
__device__ __forceinline__ void prefix_body(Common c, PreBufs pre, Table tab, uint32_t p0,
                                            uint32_t B, uint32_t P, uint32_t Dp) {
    extern __shared__ __attribute__((aligned(16))) double l_fac[];  // 16-byte entries: ds_read_b128
    FacRef F{c.fac, 0u};
    if constexpr (FLDS) {
        stage_factors(l_fac, c.fac, c.f_L, c.f_c1);
        F = FacRef{l_fac, c.f_L};
    }
    // the batch's pairs the precheck accepted, listed for the consumer
    // (PreBufs.acc_*; one atomic per wave): the first B threads of the grid
    if (pre.acc_n && static_cast<uint64_t>(blockIdx.x) * blockDim.x < B) {
        const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x, lane = threadIdx.x & 63u;
        const uint32_t bidx = p0 / pre.acc_B;
        const bool in = g < B;
        const bool a = in && pre.ok[p0 + g] == 1u;
        const uint64_t take = __ballot(a);
        uint32_t base = 0;
        if (lane == 0u && take) base = atomicAdd(pre.acc_n + bidx, static_cast<uint32_t>(__popcll(take)));
        base = __shfl(base, 0);
        if (in) {
            uint32_t slot = 0xffffffffu;
            if (a) {
                slot = base + static_cast<uint32_t>(__popcll(take & ((1ull << lane) - 1ull)));
                pre.acc_list[static_cast<size_t>(bidx) * pre.acc_B + slot] = g;
            }
            pre.acc_pos[p0 + g] = slot;
        }
    }
    const uint32_t lo_bits = c.Ap - Dp;
    const uint64_t NL = static_cast<uint64_t>(B) << lo_bits;
    const uint64_t lomask = (1ull << lo_bits) - 1ull;
    const uint32_t e_split = Dp ? ld_const(c.src, lo_bits) : c.i1;
    const Mask4 fin_c1 = ld_const(c.fin, c.c1);
    for (uint64_t lb = static_cast<uint64_t>(blockIdx.x) * blockDim.x; lb < NL;
         lb += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t l_raw = lb + threadIdx.x;
        const bool live = l_raw < NL;
        const uint64_t li = live ? l_raw : NL - 1;   // clamp so every lane reads in bounds
        const uint64_t pl = li >> lo_bits;
        const uint32_t p = p0 + static_cast<uint32_t>(pl);
        Lanes<NW, 1> L;
        uint32_t bin[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) L.s[0][w] = pre.st[static_cast<size_t>(w) * P + p];
        load_bits<NW>(check_bits(c, p), c.W, c.n, bin);
        const double2 a = pre.amp[p];
        L.re[0] = a.x;
        L.im[0] = a.y;
        L.M[0] = pre.M[p];
        L.ok[0] = pre.ok[p] == 1u;
        L.hb[0] = li & lomask;
        L.dx[0] = 0;
        L.hf[0] = 0;
        L.hq = 0;
        L.hu = 0;
        L.sd[0] = 0;
        L.aff = c.n_aff ? pre.aff[p] : 0ull;
        Walk::template prefix_head<NW, PRUNE>(c, F, L, bin, e_split);
        const uint64_t ebase = pl << c.Ap;
        const uint64_t E = static_cast<uint64_t>(B) << c.Ap;
        dfs_region<NW, 1, kDfsMax>(
            lo_bits, Dp, L, 0u,
            [&](uint32_t l, Lanes<NW, 1> &C) {
                Walk::template prefix_seg<NW, PRUNE>(c, F, C, bin, lo_bits, Dp, l);
            },
            [&](Lanes<NW, 1> &C) {
                const bool ok = C.ok[0] && check_final<NW>(C.s[0], bin, fin_c1);
                if (live) {
                    const uint64_t e = ebase | C.hb[0];
#pragma unroll
                    for (int w = 0; w < NW; ++w) tab.st[static_cast<size_t>(w) * E + e] = C.s[0][w];
                    tab.beta[e] = make_double2(C.re[0], C.im[0]);
                    if (PRUNE) tab.M[e] = C.M[0];
                    tab.ok[e] = ok ? 1u : 0u;
                }
            });
    }
}

// The persistent consumer (Algorithm 2, inner loops) over a Regions policy
// that walks the root region [c1, c2) and the suffix region [c2, G) of a
// history: Interp decodes the program at run time; the runtime can also
// compile a policy with the regions' instructions as straight-line code,
// which may defer the suffix's factor multiplications (kDefer) to the
// histories that pass the final check (suffix_amp).
template <class Regions, int NW, int H, bool PRUNE, bool FLDS>
__device__ __forceinline__ void consume_body(Common c, Table tab, Partials part, uint32_t p0,
                                             uint32_t B, uint32_t chunk, uint32_t ss,
                                             uint32_t *counter) {
    constexpr int NT = kConsumeThreads;
    extern __shared__ __attribute__((aligned(16))) double l_fac[];  // 16-byte entries: ds_read_b128
    __shared__ uint32_t s_item;
    __shared__ uint32_t l_st[NW][kMaxChunk];
    __shared__ double2 l_beta[kMaxChunk];
    __shared__ double l_M[kMaxChunk];
    __shared__ uint32_t l_hp[kMaxChunk];
    __shared__ uint32_t l_wcount[NT / 64];
    __shared__ Acc l_red[NT / 64];
    // the counted factors' products
    __shared__ double2 l_ct[Regions::kNCT > 0 ? Regions::kNCT : 1];
    if constexpr (Regions::kNCT > 0) {
        for (uint32_t i = threadIdx.x; i < Regions::kNCT; i += NT) l_ct[i] = Regions::count_entry(i);
        __syncthreads();
    }

    FacRef F{c.fac, 0u};
    if constexpr (FLDS) {
        stage_factors(l_fac, c.fac, c.f_c1, c.f_G);
        F = FacRef{l_fac, c.f_c1};
    }
    const uint32_t per_pair = 1u << c.Ap;
    const uint32_t nchunks = (per_pair + chunk - 1) / chunk;
    const uint32_t rparts = c.rparts > 0u ? c.rparts : 1u;   // items per chunk
    const uint32_t ipp = nchunks * rparts;                   // items per pair
    // the batch's pairs the precheck accepted (written before this launch)
    const uint32_t bidx = p0 / c.acc_B;
    const uint32_t n_items = c.acc_n[bidx] * ipp;
    const uint64_t E = static_cast<uint64_t>(B) << c.Ap;
    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    const uint32_t rmask = (1u << c.Ar) - 1u;
    if constexpr (Regions::kSS >= 0) ss = static_cast<uint32_t>(Regions::kSS);   // compiled for it
    const uint32_t smask = (1u << ss) - 1u;
    const uint32_t As = Regions::kAs >= 0 ? static_cast<uint32_t>(Regions::kAs) : c.As;
    const uint64_t n_suffix = 1ull << (As - ss);   // suffix assignments per task
    const uint32_t sshift = c.Ap + c.Ar;
    // history indices below 2^30: the valid-set hash's first product split
    // into a per-root and a per-leaf part (mix64)
    const bool small_h = Regions::kA >= 0 ? Regions::kA <= 30 : sshift + As <= 30u;
    const Mask4 fin_c2 = ld_const(c.fin, c.c2), fin_G = ld_const(c.fin, c.G);

    const uint32_t grab = c.grab > 0u ? c.grab : 1u;
    // Each workgroup's first run of items is fixed (workgroup b: items
    // [b grab, (b + 1) grab)); the counter hands out the items after the
    // grid's first runs, so a launch starts without one atomic per
    // workgroup on the one counter.
    const uint32_t first_runs = gridDim.x * grab;
    uint32_t item = 0, left = 0;   // the claimed run of items not yet done (uniform)
    bool first = true;
    for (;; ++item, --left) {
        if (left == 0u) {
            if (first) {
                item = blockIdx.x * grab;
                first = false;
            } else {
                // every item was in the grid's first runs: nothing to claim
                if (first_runs >= n_items) break;
                // the previous claim was last read before the barrier in the
                // block reduction of its last item
                if (t == 0) s_item = atomicAdd(counter, grab);
                __syncthreads();
                item = s_item + first_runs;
            }
            left = grab;
        }
        if (item >= n_items) break;
        const uint32_t f = item / ipp, rem = item - f * ipp, ch = rem / rparts, rp = rem - ch * rparts;
        const uint32_t pl = c.acc_list[static_cast<size_t>(bidx) * c.acc_B + f];
        const uint32_t p = p0 + pl;
        // timing stamps by pair (pair-major), the pair's item rem
        const uint64_t sidx = static_cast<uint64_t>(pl) * ipp + rem;
        if (part.stamps && t == 0) part.stamps[2ull * sidx] = wall_clock64();
        const uint32_t hp0 = ch * chunk;
        const uint32_t cnt = min(chunk, per_pair - hp0);

        // stage the chunk HBM -> registers -> LDS, compacting valid entries
        bool v = false;
        uint32_t es[NW];
        double2 eb = make_double2(0.0, 0.0);
        double em = 1.0;
        if (t < cnt) {
            const uint64_t e = (static_cast<uint64_t>(pl) << c.Ap) + hp0 + t;
            v = tab.ok[e] != 0u;
#pragma unroll
            for (int w = 0; w < NW; ++w) es[w] = tab.st[static_cast<size_t>(w) * E + e];
            eb = tab.beta[e];
            if (PRUNE) em = tab.M[e];
        }
        const uint64_t bal = __ballot(v);
        const uint32_t rank = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) l_wcount[wave] = __popcll(bal);
        __syncthreads();
        uint32_t base = 0, nv = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            const uint32_t cw = l_wcount[w];
            base += (static_cast<uint32_t>(w) < wave) ? cw : 0u;
            nv += cw;
        }
        if (v) {
            const uint32_t d = base + rank;
#pragma unroll
            for (int w = 0; w < NW; ++w) l_st[w][d] = es[w];
            l_beta[d] = eb;
            l_M[d] = em;
            l_hp[d] = hp0 + t;
        }
        __syncthreads();

        uint32_t bin[NW];
        load_bits<NW>(check_bits(c, p), c.W, c.n, bin);
        const uint64_t paff = c.n_aff ? c.pair_aff[p] : 0ull;
        Acc acc{0.0, 0.0, 0, 0, 0, 0};
        // this item's part of the chunk's root tasks: whole passes of the
        // workgroup (uniform loop bounds: the program counter inside stays
        // wave-uniform)
        const uint64_t step = static_cast<uint64_t>(H) * NT;
        const uint64_t ntask_all = static_cast<uint64_t>(nv) << (c.Ar + ss);
        const uint64_t per_part = ((ntask_all + rparts - 1u) / rparts + step - 1u) / step * step;
        const uint64_t t_lo = min(ntask_all, static_cast<uint64_t>(rp) * per_part);
        const uint64_t ntask = min(ntask_all, t_lo + per_part);
        for (uint64_t tb = t_lo; tb < ntask; tb += step) {
            Lanes<NW, H> R;
            uint64_t hbase[H], hs0[H];
            unroll<H>([&](auto jj) {
                constexpr int j = jj.value;
                const uint64_t task = tb + t + static_cast<uint64_t>(j) * NT;
                const bool valid = task < ntask;
                const uint32_t jx = valid ? static_cast<uint32_t>(task >> (c.Ar + ss)) : 0u;
                const uint32_t hr = static_cast<uint32_t>(task >> ss) & rmask;
                hs0[j] = static_cast<uint64_t>(task & smask) * n_suffix;
                unroll<NW>([&](auto ww) { R.s[j][ww.value] = l_st[ww.value][jx]; });
                const double2 b = l_beta[jx];
                R.re[j] = b.x;
                R.im[j] = b.y;
                R.M[j] = l_M[jx];
                R.ok[j] = valid;
                R.hb[j] = hr;
                R.hf[j] = l_hp[jx];
                R.sd[j] = 0;
                R.ci[j] = 0;
                hbase[j] = static_cast<uint64_t>(l_hp[jx]) | (static_cast<uint64_t>(hr) << c.Ap);
            });
            R.aff = paff;
            R.hq = 0;
            R.hu = 0;
            Regions::template root<NW, H, PRUNE>(c, F, R, bin);
            bool any = false;
            unroll<H>([&](auto jj) {
                constexpr int j = jj.value;
                R.ok[j] = R.ok[j] && Regions::template final_c2<NW>(R.s[j], bin, fin_c2);
                any = any || R.ok[j];
            });
            if (!__any(any)) continue;   // wave-uniform skip
            // a pure leaf loop starts each leaf from amplitude +1: a leaf's
            // value is then its sign times its counted product, and the
            // root's amplitude multiplies their sum once
            double ar[H], ai[H], sre[H], sim[H];
            if constexpr (Regions::kLeafPure) {
                unroll<H>([&](auto jj) {
                    constexpr int j = jj.value;
                    ar[j] = R.re[j];
                    ai[j] = R.im[j];
                    R.re[j] = 1.0;
                    R.im[j] = 0.0;
                    sre[j] = sim[j] = 0.0;
                });
            }
            // a pass of leaves can hold a valid history only where the final
            // field check's residue v (per root) is within reach of the
            // pass's source popcounts (the compiled regions' pass_res/pass_q)
            uint32_t pv[H];
            if constexpr (Regions::kPassFilter) Regions::template pass_res<NW, H>(R, hs0, bin, pv);
            auto may_pass = [&](uint64_t qq, auto uu) {
                constexpr int UU = decltype(uu)::value;
                constexpr uint32_t up = Regions::kPassUp;
                constexpr uint32_t span = UU == 1 ? 0u : Regions::kPassSpan;
                const uint32_t pq = Regions::template pass_q<UU>(qq);
                bool may = false;
                unroll<H>([&](auto jj) {
                    constexpr int j = jj.value;
                    const uint32_t D = pv[j] - pq;
                    may = may || (R.ok[j] && (D & ((2u << up) - 1u)) == 0u && (D >> (up + 1u)) <= span);
                });
                return __any(may);
            };
            if constexpr (Regions::kPassFilter && Regions::kRootSpan >= 0) {
                // no suffix assignment at all within reach: skip the root's leaves
                constexpr uint32_t up = Regions::kPassUp;
                bool may = false;
                unroll<H>([&](auto jj) {
                    constexpr int j = jj.value;
                    const uint32_t D = pv[j] - Regions::kRootQ;
                    may = may || (R.ok[j] && (D & ((2u << up) - 1u)) == 0u &&
                                  (D >> (up + 1u)) <= static_cast<uint32_t>(Regions::kRootSpan));
                });
                if (!__any(may)) continue;
            }
            // the leaves walked: every suffix assignment of a consistent root
            // that no filter rejected before its walk
            auto walked = [&](uint64_t n) {
                unroll<H>([&](auto jj) { acc.leaves += R.ok[jj.value] ? n : 0u; });
            };
            uint64_t hm[H];   // the root's part of the hash's first product
            unroll<H>([&](auto jj) {
                constexpr int j = jj.value;
                hm[j] = small_h ? (hbase[j] + (hs0[j] << sshift)) * kMixC1 : 0u;
                // opaque to the compiler, which would otherwise fold the two
                // parts back into one product per leaf
                asm volatile("" : "+v"(hm[j]));
            });
            // the suffix instructions no suffix source influences, once per root
            if constexpr (Regions::kHoist) Regions::template suffix_pre<NW, H, PRUNE>(c, F, R, bin);
            // one leaf: the suffix region for assignment q (wave-uniform: the
            // lanes differ in hs0 only), then its final check
            auto walk_leaf = [&](Lanes<NW, H> &S2, uint64_t q, uint32_t u) {
                unroll<H>([&](auto jj) {
                    S2.hb[jj.value] = hs0[jj.value];   // multiples of n_suffix
                    S2.dx[jj.value] = 0;
                    S2.sd[jj.value] = 0;
                    S2.hf[jj.value] = hbase[jj.value];
                });
                S2.hq = q;                              // below n_suffix, the same in every lane
                S2.hu = u;
                Regions::template suffix<NW, H, PRUNE>(c, F, S2, bin);
                unroll<H>([&](auto jj) {
                    constexpr int j = jj.value;
                    S2.ok[j] = S2.ok[j] && Regions::template final_G<NW>(S2.s[j], bin, fin_G);
                });
            };
            auto count_leaf = [&](Lanes<NW, H> &S2, uint64_t q) {
                unroll<H>([&](auto jj) {
                    constexpr int j = jj.value;
                    if (S2.ok[j]) {
                        // a policy that deferred the suffix's factors applies them
                        // now, for the histories that count
                        if constexpr (Regions::kDefer) Regions::template suffix_amp<NW, H>(F, S2, j);
                        if constexpr (Regions::kNCT > 0) Regions::template count_amp<NW, H>(l_ct, S2, j);
                        const uint64_t h = hbase[j] | ((hs0[j] + q) << sshift);
                        if constexpr (Regions::kLeafPure) {
                            sre[j] += S2.re[j];
                            sim[j] += S2.im[j];
                        } else {
                            acc.re += S2.re[j];
                            acc.im += S2.im[j];
                        }
                        acc.nval += 1;
                        acc.sumh += h;
                        if (small_h) acc.xorh ^= mix64_tail(hm[j] + (q << sshift) * kMixC1);
                        else acc.xorh ^= mix64(h);
                    }
                });
            };
            constexpr int U = Regions::kUnroll;
            uint64_t q = 0;
            if constexpr (U > 1) {
                // U leaves per pass: their checks first, then one wave-uniform
                // test skips the pass when no lane has a valid history in it
                for (; q + U <= n_suffix; q += U) {   // q stays a multiple of U
                    if constexpr (Regions::kPassFilter) {
                        if (!may_pass(q, IC<U>{})) continue;
                    }
                    walked(U);
                    Lanes<NW, H> S2[U];
                    bool any = false;
                    unroll<U>([&](auto uu) {
                        constexpr int u = uu.value;
                        S2[u] = R;
                        walk_leaf(S2[u], q, static_cast<uint32_t>(u));
                        unroll<H>([&](auto jj) { any = any || S2[u].ok[jj.value]; });
                    });
                    if (!__any(any)) continue;
                    unroll<U>([&](auto uu) { count_leaf(S2[uu.value], q + uu.value); });
                }
            }
            for (; q < n_suffix; ++q) {
                if constexpr (Regions::kPassFilter) {
                    if (!may_pass(q, IC<1>{})) continue;
                }
                walked(1);
                Lanes<NW, H> S2 = R;
                walk_leaf(S2, q, 0u);
                count_leaf(S2, q);
            }
            if constexpr (Regions::kLeafPure) {
                unroll<H>([&](auto jj) {
                    constexpr int j = jj.value;
                    acc.re += fma(ar[j], sre[j], -(ai[j] * sim[j]));
                    acc.im += fma(ar[j], sim[j], ai[j] * sre[j]);
                });
            }
        }
        block_reduce_store<NT>(acc, l_red, part, item);
        if (part.stamps && t == 0) part.stamps[2ull * sidx + 1] = wall_clock64();
    }
}

}  // namespace
}  // namespace fhs
