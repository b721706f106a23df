// kernels.hip -- CDNA4 (gfx950) kernels of the reduced-history path.
//
// Each lane owns one history at a time: an n-bit time-slice state held in
// NW 32-bit VGPRs, an FP64 complex partial amplitude and (with pruning) the
// running modulus product M.  The history program is read wave-uniformly
// (scalar loads), so every lane of a wave executes the same gate and only
// the selected matrix element differs.  Source bits are decoded from the
// lane's history index in registers.
//
//   k_precheck  once per (b_in, b_out) pair: the source-free gates nearest
//               the output, plus every boundary-only consistency check
//               (Algorithm 1, SetBoundaryWires/PropagateKnownValues);
//   k_prefix    one lane per prefix assignment h_p: runs the prefix region
//               and writes the checkpoint table (state, beta, M, valid) in
//               structure-of-arrays form (Algorithm 2, first loop);
//   k_consume   persistent: work items (pair, chunk of prefix entries) are
//               popped from an atomic counter, the chunk is staged into LDS
//               and compacted, then each lane takes (entry, h_r), runs the
//               root once and the suffix for every h_s (Algorithm 2, inner
//               loops); the workgroup reduces its sums deterministically;
//   k_plain     Algorithm 1: one lane per candidate history, static grid;
//   k_pair_reduce / k_finalize: fixed-order sums, then Eq. (2).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fhs {
namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // SplitMix64 finaliser (Steele, Lea, Flood 2014)
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// State words are only ever indexed with compile-time constants (the word
// holding a gate's bit is part of its opcode), so the state stays in VGPRs.
template <int W, int NW>
__device__ __forceinline__ constexpr int wsel() {
    return W < NW ? W : 0;
}

template <int NW>
__device__ __forceinline__ bool matches(const uint32_t (&s)[NW], const Instr &I) {
    uint32_t acc = (s[0] ^ I.cv[0]) & I.cm[0];
#pragma unroll
    for (int j = 1; j < NW; ++j)
        if (I.cm[j] != 0u) acc |= (s[j] ^ I.cv[j]) & I.cm[j];
    return acc == 0u;
}

template <int NW>
__device__ __forceinline__ bool check_final(const uint32_t (&s)[NW], const uint32_t (&bin)[NW],
                                            const Mask4 &m) {
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < NW; ++j) acc |= (s[j] ^ bin[j]) & m.w[j];
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
    uint64_t w0 = src[0];
    uint64_t w1 = W > 1 ? src[1] : 0;
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

// 4-way select of a complex table entry fac[2x], fac[2x+1].
__device__ __forceinline__ void pick4(const double *f, uint32_t x, double &fr, double &fi) {
    const double a0 = f[0], a1 = f[1], b0 = f[2], b1 = f[3];
    const double c0 = f[4], c1 = f[5], d0 = f[6], d1 = f[7];
    fr = (x & 2u) ? ((x & 1u) ? d0 : c0) : ((x & 1u) ? b0 : a0);
    fi = (x & 2u) ? ((x & 1u) ? d1 : c1) : ((x & 1u) ? b1 : a1);
}

template <int NW, int WA>
__device__ __forceinline__ void op_perm(uint32_t (&s)[NW], const Instr &I) {
    constexpr int A = wsel<WA, NW>();
    const bool m = matches<NW>(s, I);
    const uint32_t bm = 1u << (I.a & 31u);
    s[A] ^= m ? bm : 0u;
}

template <int NW, int WA, int WB>
__device__ __forceinline__ void op_swap(uint32_t (&s)[NW], const Instr &I) {
    constexpr int A = wsel<WA, NW>(), B = wsel<WB, NW>();
    const bool m = matches<NW>(s, I);
    const uint32_t sa = I.a & 31u, sb = I.b & 31u;
    const uint32_t d = (((s[A] >> sa) ^ (s[B] >> sb)) & 1u) & (m ? 1u : 0u);
    s[A] ^= d << sa;
    s[B] ^= d << sb;
}

template <int NW, int WA>
__device__ __forceinline__ void op_det1(uint32_t (&s)[NW], const Instr &I, const double *fac,
                                        double &re, double &im) {
    constexpr int A = wsel<WA, NW>();
    const uint32_t o = (s[A] >> (I.a & 31u)) & 1u;
    const double *f = fac + I.fac;
    const double f0r = f[0], f0i = f[1], f1r = f[2], f1i = f[3];
    cmul(re, im, o ? f1r : f0r, o ? f1i : f0i);
    s[A] ^= 1u << (I.a & 31u);
}

template <int NW, int WA>
__device__ __forceinline__ void op_diag1(const uint32_t (&s)[NW], const Instr &I, const double *fac,
                                         double &re, double &im) {
    constexpr int A = wsel<WA, NW>();
    const uint32_t o = (s[A] >> (I.a & 31u)) & 1u;
    const double *f = fac + I.fac;
    const double f0r = f[0], f0i = f[1], f1r = f[2], f1i = f[3];
    cmul(re, im, o ? f1r : f0r, o ? f1i : f0i);
}

template <int NW, int WA, int WB>
__device__ __forceinline__ void op_diag2(const uint32_t (&s)[NW], const Instr &I, const double *fac,
                                         double &re, double &im) {
    constexpr int A = wsel<WA, NW>(), B = wsel<WB, NW>();
    const uint32_t x = ((s[A] >> (I.a & 31u)) & 1u) | (((s[B] >> (I.b & 31u)) & 1u) << 1);
    double fr, fi;
    pick4(fac + I.fac, x, fr, fi);
    cmul(re, im, fr, fi);
}

template <int NW, bool PRUNE, int WA, bool SRC>
__device__ __forceinline__ void op_branch(uint32_t (&s)[NW], const Instr &I, const double *fac,
                                          double &re, double &im, double &M, bool &ok,
                                          uint64_t hb, uint32_t kbase, const uint32_t (&bin)[NW],
                                          double thr) {
    constexpr int A = wsel<WA, NW>();
    const uint32_t sh = I.a & 31u;
    const uint32_t o = (s[A] >> sh) & 1u;
    const uint32_t i = SRC ? static_cast<uint32_t>((hb >> (I.k - kbase)) & 1u)
                           : (bin[A] >> sh) & 1u;
    const uint32_t x = 2u * o + i;
    const double *f = fac + I.fac;
    double fr, fi;
    pick4(f, x, fr, fi);
    cmul(re, im, fr, fi);
    if (PRUNE) {
        const double m0 = f[8], m1 = f[9], m2 = f[10], m3 = f[11];
        const double md = (x & 2u) ? ((x & 1u) ? m3 : m2) : ((x & 1u) ? m1 : m0);
        M = M * md;
        ok = ok && !(M < thr);
    }
    ok = ok && !((I.zmask >> x) & 1u);
    s[A] ^= (o ^ i) << sh;
}

// Walk evaluation positions [e0, e1) of the history program backward from
// the state s.  hb holds this region's source bits: source k reads bit
// (k - kbase).  bin is the input bitstring.
template <int NW, bool PRUNE>
__device__ __forceinline__ void run_region(const Common &c, uint32_t e0, uint32_t e1,
                                           uint32_t (&s)[NW], double &re, double &im, double &M,
                                           bool &ok, uint64_t hb, uint32_t kbase,
                                           const uint32_t (&bin)[NW]) {
    const Instr *__restrict__ prog = c.prog;
    const double *__restrict__ fac = c.fac;
    const double thr = c.thr;
    for (uint32_t e = e0; e < e1; ++e) {
        const Instr I = prog[e];
        switch (I.op) {
#define FHS_A_CASES(WA)                                                                      \
    case OP_PERM | ((WA) << 4): op_perm<NW, WA>(s, I); break;                                \
    case OP_DET1 | ((WA) << 4): op_det1<NW, WA>(s, I, fac, re, im); break;                   \
    case OP_DIAG1 | ((WA) << 4): op_diag1<NW, WA>(s, I, fac, re, im); break;                 \
    case OP_BRANCH_SRC | ((WA) << 4):                                                        \
        op_branch<NW, PRUNE, WA, true>(s, I, fac, re, im, M, ok, hb, kbase, bin, thr); break; \
    case OP_BRANCH_NAT | ((WA) << 4):                                                        \
        op_branch<NW, PRUNE, WA, false>(s, I, fac, re, im, M, ok, hb, kbase, bin, thr); break;
#define FHS_AB_CASES(WA, WB)                                                                 \
    case OP_SWAP | ((WA) << 4) | ((WB) << 6): op_swap<NW, WA, WB>(s, I); break;              \
    case OP_DIAG2 | ((WA) << 4) | ((WB) << 6): op_diag2<NW, WA, WB>(s, I, fac, re, im); break;
            FHS_A_CASES(0)
            FHS_AB_CASES(0, 0)
            case OP_MCPHASE:
                if (matches<NW>(s, I)) {
                    re = -re;
                    im = -im;
                }
                break;
            default:
                if constexpr (NW >= 2) {
                    switch (I.op) {
                        FHS_A_CASES(1)
                        FHS_AB_CASES(0, 1)
                        FHS_AB_CASES(1, 0)
                        FHS_AB_CASES(1, 1)
                        default:
                            if constexpr (NW == 4) {
                                switch (I.op) {
                                    FHS_A_CASES(2)
                                    FHS_A_CASES(3)
                                    FHS_AB_CASES(0, 2)
                                    FHS_AB_CASES(0, 3)
                                    FHS_AB_CASES(1, 2)
                                    FHS_AB_CASES(1, 3)
                                    FHS_AB_CASES(2, 0)
                                    FHS_AB_CASES(2, 1)
                                    FHS_AB_CASES(2, 2)
                                    FHS_AB_CASES(2, 3)
                                    FHS_AB_CASES(3, 0)
                                    FHS_AB_CASES(3, 1)
                                    FHS_AB_CASES(3, 2)
                                    FHS_AB_CASES(3, 3)
                                    default:
                                        break;
                                }
                            }
                            break;
                    }
                }
                break;
#undef FHS_A_CASES
#undef FHS_AB_CASES
        }
    }
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

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

template <int NW, bool PRUNE>
__global__ __launch_bounds__(256) void k_precheck(Common c, PreBufs pre, uint32_t P,
                                                  uint32_t *zero_words, uint32_t n_zero) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n_zero) zero_words[p] = 0u;
    if (p >= P) return;
    const uint32_t j = p / c.S, i = p % c.S;
    uint32_t s[NW], bin[NW];
    const bool bad_o = load_bits<NW>(c.outputs + static_cast<size_t>(j) * c.W, c.W, c.n, s);
    const bool bad_i = load_bits<NW>(c.inputs + static_cast<size_t>(i) * c.W, c.W, c.n, bin);
    double re = 1.0, im = 0.0, M = 1.0;
    bool ok = !(bad_o || bad_i);
    run_region<NW, PRUNE>(c, 0, c.L, s, re, im, M, ok, 0, 0, bin);
    ok = ok && check_final<NW>(s, bin, c.fin[c.L]);
#pragma unroll
    for (int w = 0; w < NW; ++w) pre.st[static_cast<size_t>(w) * P + p] = s[w];
    pre.amp[p] = make_double2(re, im);
    pre.M[p] = M;
    pre.ok[p] = (ok ? 1u : 0u) | ((bad_o || bad_i) ? 2u : 0u);
}

template <int NW, bool PRUNE>
__global__ __launch_bounds__(256) void k_prefix(Common c, PreBufs pre, Table tab, uint32_t p0,
                                                uint32_t B, uint32_t P) {
    const uint64_t E = static_cast<uint64_t>(B) << c.Ap;
    const uint64_t hmask = (1ull << c.Ap) - 1ull;
    for (uint64_t e = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < E;
         e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t p = p0 + static_cast<uint32_t>(e >> c.Ap);
        const uint64_t hp = e & hmask;
        uint32_t s[NW], bin[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) s[w] = pre.st[static_cast<size_t>(w) * P + p];
        load_bits<NW>(c.inputs + static_cast<size_t>(p % c.S) * c.W, c.W, c.n, bin);
        const double2 a = pre.amp[p];
        double re = a.x, im = a.y, M = pre.M[p];
        bool ok = pre.ok[p] == 1u;
        if (ok) {
            run_region<NW, PRUNE>(c, c.L, c.c1, s, re, im, M, ok, hp, 0, bin);
            ok = ok && check_final<NW>(s, bin, c.fin[c.c1]);
        }
#pragma unroll
        for (int w = 0; w < NW; ++w) tab.st[static_cast<size_t>(w) * E + e] = s[w];
        tab.beta[e] = make_double2(re, im);
        if (PRUNE) tab.M[e] = M;
        tab.ok[e] = ok ? 1u : 0u;
    }
}

template <int NW, bool PRUNE>
__global__ __launch_bounds__(kConsumeThreads) void k_consume(Common c, Table tab, Partials part,
                                                             uint32_t p0, uint32_t B,
                                                             uint32_t chunk, uint32_t ss,
                                                             uint32_t *counter) {
    constexpr int NT = kConsumeThreads;
    __shared__ uint32_t s_item;
    __shared__ uint32_t l_st[NW][kMaxChunk];
    __shared__ double2 l_beta[kMaxChunk];
    __shared__ double l_M[kMaxChunk];
    __shared__ uint32_t l_hp[kMaxChunk];
    __shared__ uint32_t l_wcount[NT / 64];
    __shared__ Acc l_red[NT / 64];

    const uint32_t per_pair = 1u << c.Ap;
    const uint32_t nchunks = (per_pair + chunk - 1) / chunk;
    const uint32_t n_items = B * nchunks;
    const uint64_t E = static_cast<uint64_t>(B) << c.Ap;
    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    const uint32_t rmask = (1u << c.Ar) - 1u;
    const uint32_t smask = (1u << ss) - 1u;
    const uint64_t n_suffix = 1ull << (c.As - ss);   // suffix assignments per task

    for (;;) {
        if (t == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= n_items) break;
        const uint32_t pl = item / nchunks, ch = item - pl * nchunks;
        const uint32_t p = p0 + pl;
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
        load_bits<NW>(c.inputs + static_cast<size_t>(p % c.S) * c.W, c.W, c.n, bin);
        Acc acc{0.0, 0.0, 0, 0, 0, 0};
        const uint64_t ntask = static_cast<uint64_t>(nv) << (c.Ar + ss);
        for (uint64_t task = t; task < ntask; task += NT) {
            const uint32_t jx = static_cast<uint32_t>(task >> (c.Ar + ss));
            const uint32_t hr = static_cast<uint32_t>(task >> ss) & rmask;
            const uint64_t hs0 = static_cast<uint64_t>(task & smask) * n_suffix;
            uint32_t s[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) s[w] = l_st[w][jx];
            const double2 b = l_beta[jx];
            double re = b.x, im = b.y, M = l_M[jx];
            bool ok = true;
            run_region<NW, PRUNE>(c, c.c1, c.c2, s, re, im, M, ok, hr, c.Ap, bin);
            ok = ok && check_final<NW>(s, bin, c.fin[c.c2]);
            if (ok) {
                const uint64_t hbase = static_cast<uint64_t>(l_hp[jx]) |
                                       (static_cast<uint64_t>(hr) << c.Ap);
                for (uint64_t hs = hs0; hs < hs0 + n_suffix; ++hs) {
                    uint32_t s2[NW];
#pragma unroll
                    for (int w = 0; w < NW; ++w) s2[w] = s[w];
                    double re2 = re, im2 = im, M2 = M;
                    bool ok2 = true;
                    run_region<NW, PRUNE>(c, c.c2, c.G, s2, re2, im2, M2, ok2, hs, c.Ap + c.Ar, bin);
                    ok2 = ok2 && check_final<NW>(s2, bin, c.fin[c.G]);
                    acc.leaves += 1;
                    if (ok2) {
                        const uint64_t h = hbase | (hs << (c.Ap + c.Ar));
                        acc.re += re2;
                        acc.im += im2;
                        acc.nval += 1;
                        acc.sumh += h;
                        acc.xorh ^= mix64(h);
                    }
                }
            }
        }
        block_reduce_store<NT>(acc, l_red, part, item);
    }
}

template <int NW, bool PRUNE>
__global__ __launch_bounds__(kPlainThreads) void k_plain(Common c, PreBufs pre, Partials part,
                                                         uint32_t P, uint32_t bpp) {
    constexpr int NT = kPlainThreads;
    __shared__ Acc l_red[NT / 64];
    const uint32_t p = blockIdx.x / bpp, b = blockIdx.x - p * bpp;
    Acc acc{0.0, 0.0, 0, 0, 0, 0};
    if (pre.ok[p] == 1u) {
        uint32_t s0[NW], bin[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) s0[w] = pre.st[static_cast<size_t>(w) * P + p];
        load_bits<NW>(c.inputs + static_cast<size_t>(p % c.S) * c.W, c.W, c.n, bin);
        const double2 a = pre.amp[p];
        const double M0 = pre.M[p];
        const uint64_t NH = 1ull << c.A;
        for (uint64_t h = static_cast<uint64_t>(b) * NT + threadIdx.x; h < NH;
             h += static_cast<uint64_t>(bpp) * NT) {
            uint32_t s[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) s[w] = s0[w];
            double re = a.x, im = a.y, M = M0;
            bool ok = true;
            run_region<NW, PRUNE>(c, c.L, c.G, s, re, im, M, ok, h, 0, bin);
            ok = ok && check_final<NW>(s, bin, c.fin[c.G]);
            acc.leaves += 1;
            if (ok) {
                acc.re += re;
                acc.im += im;
                acc.nval += 1;
                acc.sumh += h;
                acc.xorh ^= mix64(h);
            }
        }
    }
    block_reduce_store<NT>(acc, l_red, part, blockIdx.x);
}

__global__ void k_pair_reduce(PreBufs pre, Partials part, PairRes res, uint32_t p0, uint32_t B,
                              uint32_t ipp, uint32_t A) {
    const uint32_t pl = blockIdx.x * blockDim.x + threadIdx.x;
    if (pl >= B) return;
    const uint32_t p = p0 + pl;
    const uint32_t okv = pre.ok[p];
    double re = 0.0, im = 0.0;
    uint64_t nv = 0, sh = 0, xh = 0, lv = 0;
    if (A == 0) {
        if (okv == 1u) {
            const double2 a = pre.amp[p];
            re = a.x;
            im = a.y;
            nv = 1;
            lv = 1;
            xh = mix64(0);
        }
    } else {
        for (uint32_t k = 0; k < ipp; ++k) {
            const size_t it = static_cast<size_t>(pl) * ipp + k;
            const double2 a = part.amp[it];
            re += a.x;
            im += a.y;
            const uint64_t *st = part.st + 4 * it;
            nv += st[0];
            sh += st[1];
            xh ^= st[2];
            lv += st[3];
        }
    }
    if (okv & 2u) lv = ~0ull;
    res.amp[p] = make_double2(re, im);
    uint64_t *o = res.st + 4ull * p;
    o[0] = nv;
    o[1] = sh;
    o[2] = xh;
    o[3] = lv;
}

__global__ void k_finalize(PairRes res, const double *coeffs, uint32_t S, uint32_t M,
                           double *amps, uint64_t *stats) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    double re = 0.0, im = 0.0;
    uint64_t nv = 0, sh = 0, xh = 0, lv = 0;
    bool bad = false;
    for (uint32_t i = 0; i < S; ++i) {
        const size_t p = static_cast<size_t>(j) * S + i;
        const double2 a = res.amp[p];
        const double cr = coeffs[2 * i], ci = coeffs[2 * i + 1];
        re += cr * a.x - ci * a.y;
        im += cr * a.y + ci * a.x;
        const uint64_t *st = res.st + 4 * p;
        nv += st[0];
        sh += st[1];
        xh ^= st[2];
        if (st[3] == ~0ull) bad = true;
        lv += st[3];
    }
    amps[2 * j] = re;
    amps[2 * j + 1] = im;
    stats[4ull * j] = nv;
    stats[4ull * j + 1] = sh;
    stats[4ull * j + 2] = xh;
    stats[4ull * j + 3] = bad ? ~0ull : lv;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define FHS_DISPATCH(NWV, PR, ...)                                              \
    do {                                                                        \
        if ((NWV) == 1) {                                                       \
            if (PR) { constexpr int NW_ = 1; constexpr bool PR_ = true; __VA_ARGS__; }  \
            else { constexpr int NW_ = 1; constexpr bool PR_ = false; __VA_ARGS__; }    \
        } else if ((NWV) == 2) {                                                \
            if (PR) { constexpr int NW_ = 2; constexpr bool PR_ = true; __VA_ARGS__; }  \
            else { constexpr int NW_ = 2; constexpr bool PR_ = false; __VA_ARGS__; }    \
        } else {                                                                \
            if (PR) { constexpr int NW_ = 4; constexpr bool PR_ = true; __VA_ARGS__; }  \
            else { constexpr int NW_ = 4; constexpr bool PR_ = false; __VA_ARGS__; }    \
        }                                                                       \
    } while (0)

hipError_t launch_precheck(const Common &c, int NW, PreBufs pre, uint32_t P, uint32_t *zero_words,
                           uint32_t n_zero, hipStream_t s) {
    const uint32_t n = P > n_zero ? P : n_zero;
    const uint32_t blocks = (n + 255) / 256;
    if (blocks == 0) return hipSuccess;
    const bool pr = c.thr > 0.0;
    FHS_DISPATCH(NW, pr, k_precheck<NW_, PR_><<<blocks, 256, 0, s>>>(c, pre, P, zero_words, n_zero));
    return hipGetLastError();
}

hipError_t launch_prefix(const Common &c, int NW, PreBufs pre, Table tab, uint32_t p0, uint32_t B,
                         hipStream_t s) {
    const uint64_t E = static_cast<uint64_t>(B) << c.Ap;
    if (E == 0) return hipSuccess;
    uint64_t blocks = (E + 255) / 256;
    if (blocks > (1u << 20)) blocks = 1u << 20;
    const bool pr = c.thr > 0.0;
    const uint32_t P = c.M * c.S;
    FHS_DISPATCH(NW, pr, k_prefix<NW_, PR_><<<static_cast<uint32_t>(blocks), 256, 0, s>>>(c, pre, tab, p0, B, P));
    return hipGetLastError();
}

hipError_t launch_consume(const Common &c, int NW, Table tab, Partials part, uint32_t p0,
                          uint32_t B, uint32_t chunk, uint32_t ss, uint32_t *counter,
                          uint32_t grid, hipStream_t s) {
    if (B == 0 || grid == 0) return hipSuccess;
    const bool pr = c.thr > 0.0;
    FHS_DISPATCH(NW, pr, k_consume<NW_, PR_><<<grid, kConsumeThreads, 0, s>>>(c, tab, part, p0, B, chunk, ss, counter));
    return hipGetLastError();
}

hipError_t launch_plain(const Common &c, int NW, PreBufs pre, Partials part, uint32_t P,
                        uint32_t bpp, hipStream_t s) {
    const uint64_t blocks = static_cast<uint64_t>(P) * bpp;
    if (blocks == 0) return hipSuccess;
    const bool pr = c.thr > 0.0;
    FHS_DISPATCH(NW, pr, k_plain<NW_, PR_><<<static_cast<uint32_t>(blocks), kPlainThreads, 0, s>>>(c, pre, part, P, bpp));
    return hipGetLastError();
}

hipError_t launch_pair_reduce(PreBufs pre, Partials part, PairRes res, uint32_t p0, uint32_t B,
                              uint32_t ipp, uint32_t A, hipStream_t s) {
    if (B == 0) return hipSuccess;
    k_pair_reduce<<<(B + 255) / 256, 256, 0, s>>>(pre, part, res, p0, B, ipp, A);
    return hipGetLastError();
}

hipError_t launch_finalize(PairRes res, const double *coeffs, uint32_t S, uint32_t M, double *amps,
                           uint64_t *stats, hipStream_t s) {
    if (M == 0) return hipSuccess;
    k_finalize<<<(M + 255) / 256, 256, 0, s>>>(res, coeffs, S, M, amps, stats);
    return hipGetLastError();
}

int consume_blocks_per_cu(int NW, bool prune) {
    int nb = 0;
    hipError_t e = hipSuccess;
    FHS_DISPATCH(NW, prune, e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                &nb, reinterpret_cast<const void *>(k_consume<NW_, PR_>),
                                kConsumeThreads, 0));
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

}  // namespace fhs
