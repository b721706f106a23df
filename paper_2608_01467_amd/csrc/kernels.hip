// kernels.hip -- CDNA4 (gfx950) kernels of the reduced-history path (the
// per-history machinery they share is in device.hpp).
//
//   k_precheck  once per (b_in, b_out) pair: the source-free gates nearest
//               the output, plus every boundary-only consistency check
//               (Algorithm 1, SetBoundaryWires/PropagateKnownValues);
//   k_prefix    one lane per subtree of prefix assignments: runs the prefix
//               region and writes the checkpoint table (state, beta, M,
//               valid) in structure-of-arrays form (Algorithm 2, first loop);
//   k_consume   persistent: work items (pair, chunk of prefix entries) are
//               popped from an atomic counter, the chunk is staged into LDS
//               and compacted, then each lane takes (entry, h_r), runs the
//               root once and the suffix for every h_s (Algorithm 2, inner
//               loops); the workgroup reduces its sums deterministically;
//   k_plain     Algorithm 1: one lane per candidate history, static grid;
//   k_pair_reduce / k_finalize: fixed-order sums, then Eq. (2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace fhs {
namespace {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

template <int NW, bool PRUNE>
__global__ __launch_bounds__(256) void k_precheck(Common c, PreBufs pre, uint32_t P,
                                                  uint32_t *zero_words, uint32_t n_zero) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n_zero) zero_words[p] = 0u;
    if (p >= P) return;
    Lanes<NW, 1> L;
    uint32_t bin[NW];
    const bool bad_o = load_bits<NW>(start_bits(c, p), c.W, c.n, L.s[0]);
    const bool bad_i = load_bits<NW>(check_bits(c, p), c.W, c.n, bin);
    L.re[0] = 1.0;
    L.im[0] = 0.0;
    L.M[0] = 1.0;
    L.ok[0] = !(bad_o || bad_i);
    L.hb[0] = 0;
    L.hf[0] = 0;
    L.hq = 0;
    L.hu = 0;
    L.sd[0] = 0;
    L.aff = 0;
    if (c.n_aff) {
        L.aff = affine_bits<NW>(c, bin, L.s[0]);   // the start bits, before any gate
        pre.aff[p] = L.aff;
    }
    const FacRef F{c.fac, 0u};
    run_region<NW, 1, PRUNE, true>(c.prog, F, 0, c.iL, L, 0, bin, c.thr);
    bool ok = L.ok[0] && check_final<NW>(L.s[0], bin, ld_const(c.fin, c.L));
    if (c.pf_on) {
        // the field's residue against every step count the histories reach
        uint32_t up;
        const uint32_t e = field_residue<NW>(L.s[0], bin, c.pf_lo, c.pf_hi, up);
        const uint32_t D = (e - c.pf_off) << up;
        ok = ok && (D & ((2u << up) - 1u)) == 0u && (D >> (up + 1u)) <= c.pf_span;
    }
#pragma unroll
    for (int w = 0; w < NW; ++w) pre.st[static_cast<size_t>(w) * P + p] = L.s[0][w];
    pre.amp[p] = make_double2(L.re[0], L.im[0]);
    pre.M[p] = L.M[0];
    pre.ok[p] = (ok ? 1u : 0u) | ((bad_o || bad_i) ? 2u : 0u);
}

template <int NW, bool PRUNE, bool FLDS, bool RUNS>
__global__ __launch_bounds__(256) void k_prefix(Common c, PreBufs pre, Table tab, uint32_t p0,
                                                uint32_t B, uint32_t P, uint32_t Dp) {
    prefix_body<Interp<RUNS>, NW, PRUNE, FLDS>(c, pre, tab, p0, B, P, Dp);
}

template <int NW, int H, bool PRUNE, bool FLDS, bool RUNS>
__global__ __launch_bounds__(kConsumeThreads) void k_consume(Common c, Table tab, Partials part,
                                                             uint32_t p0, uint32_t B,
                                                             uint32_t chunk, uint32_t ss,
                                                             uint32_t *counter) {
    consume_body<Interp<RUNS>, NW, H, PRUNE, FLDS>(c, tab, part, p0, B, chunk, ss, counter);
}

template <int NW, int H, bool PRUNE, bool FLDS, bool RUNS>
__global__ __launch_bounds__(kPlainThreads) void k_plain(Common c, PreBufs pre, Partials part,
                                                         uint32_t P, uint32_t bpp) {
    constexpr int NT = kPlainThreads;
    extern __shared__ __attribute__((aligned(16))) double l_fac[];  // 16-byte entries: ds_read_b128
    __shared__ Acc l_red[NT / 64];
    FacRef F{c.fac, 0u};
    if constexpr (FLDS) {
        stage_factors(l_fac, c.fac, c.f_L, c.f_G);
        F = FacRef{l_fac, c.f_L};
    }
    const uint32_t p = blockIdx.x / bpp, b = blockIdx.x - p * bpp;
    const Mask4 fin_G = ld_const(c.fin, c.G);
    Acc acc{0.0, 0.0, 0, 0, 0, 0};
    if (pre.ok[p] == 1u) {
        uint32_t s0[NW], bin[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) s0[w] = pre.st[static_cast<size_t>(w) * P + p];
        load_bits<NW>(check_bits(c, p), c.W, c.n, bin);
        const double2 a = pre.amp[p];
        const double M0 = pre.M[p];
        const uint64_t NH = 1ull << c.A;
        const uint64_t stride = static_cast<uint64_t>(bpp) * NT;
        for (uint64_t hb0 = static_cast<uint64_t>(b) * NT; hb0 < NH; hb0 += H * stride) {
            const uint64_t h0 = hb0 + threadIdx.x;
            Lanes<NW, H> L;
            unroll<H>([&](auto jj) {
                constexpr int j = jj.value;
                unroll<NW>([&](auto ww) { L.s[j][ww.value] = s0[ww.value]; });
                L.re[j] = a.x;
                L.im[j] = a.y;
                L.M[j] = M0;
                L.hb[j] = h0 + j * stride;
                L.hf[j] = 0;
                L.sd[j] = 0;
                L.ok[j] = L.hb[j] < NH;
            });
            L.aff = c.n_aff ? pre.aff[p] : 0ull;
            L.hq = 0;
            L.hu = 0;
            run_region<NW, H, PRUNE, RUNS>(c.prog, F, c.iL, c.iG, L, 0, bin, c.thr);
            unroll<H>([&](auto jj) {
                constexpr int j = jj.value;
                const bool inrange = L.hb[j] < NH;
                const bool ok = L.ok[j] && check_final<NW>(L.s[j], bin, fin_G);
                acc.leaves += inrange ? 1u : 0u;
                if (ok) {
                    acc.re += L.re[j];
                    acc.im += L.im[j];
                    acc.nval += 1;
                    acc.sumh += L.hb[j];
                    acc.xorh ^= mix64(L.hb[j]);
                }
            });
        }
    }
    block_reduce_store<NT>(acc, l_red, part, blockIdx.x);
}

// Number of nonzero flags in ok[0..n): one ballot per wave, one global
// (vector) atomic add per wave.  Used only when kernel timing is on, to
// report how many prefix-table entries the consumer expands.
__global__ __launch_bounds__(256) void k_count_valid(const uint32_t *ok, uint64_t n,
                                                     unsigned long long *out) {
    uint64_t cnt = 0;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t base = static_cast<uint64_t>(blockIdx.x) * blockDim.x; base < n; base += stride) {
        const uint64_t i = base + threadIdx.x;
        const bool v = i < n && ok[i] != 0u;
        cnt += static_cast<uint64_t>(__popcll(__ballot(v)));
    }
    if ((threadIdx.x & 63u) == 0u && cnt) atomicAdd(out, static_cast<unsigned long long>(cnt));
}

// One pair's sums over its items, in item order.
__device__ __forceinline__ void pair_sums(const PreBufs &pre, const Partials &part, uint32_t p0, uint32_t pl,
                                          uint32_t ipp, uint32_t A, double2 &amp, uint64_t (&o)[4]) {
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
    } else if (okv == 1u) {
        // the consumer's items cover only the accepted pairs, listed (the
        // plain form's blocks cover every pair)
        const uint32_t f = pre.acc_pos ? pre.acc_pos[p] : pl;
        const double2 *pa = part.amp + static_cast<size_t>(f) * ipp;
        const uint64_t *ps = part.st + 4ull * f * ipp;
        // items in groups of 8: a group's loads are all issued before the
        // first is used (one memory round trip per group, not per item);
        // the sums still run in item order
        constexpr uint32_t G = 8;
        for (uint32_t k0 = 0; k0 < ipp; k0 += G) {
            const uint32_t n = ipp - k0 < G ? ipp - k0 : G;
            double2 a[G];
            ulonglong4 s[G];
#pragma unroll
            for (uint32_t j = 0; j < G; ++j) {
                if (j < n) {
                    a[j] = pa[k0 + j];
                    s[j] = *reinterpret_cast<const ulonglong4 *>(ps + 4ull * (k0 + j));
                }
            }
#pragma unroll
            for (uint32_t j = 0; j < G; ++j) {
                if (j < n) {
                    re += a[j].x;
                    im += a[j].y;
                    nv += s[j].x;
                    sh += s[j].y;
                    xh ^= s[j].z;
                    lv += s[j].w;
                }
            }
        }
    }
    if (okv & 2u) lv = ~0ull;
    amp = make_double2(re, im);
    o[0] = nv;
    o[1] = sh;
    o[2] = xh;
    o[3] = lv;
}

__global__ void k_pair_reduce(PreBufs pre, Partials part, PairRes res, uint32_t p0, uint32_t B,
                              uint32_t ipp, uint32_t A) {
    const uint32_t pl = blockIdx.x * blockDim.x + threadIdx.x;
    if (pl >= B) return;
    double2 a;
    uint64_t o[4];
    pair_sums(pre, part, p0, pl, ipp, A, a, o);
    const uint32_t p = p0 + pl;
    res.amp[p] = a;
    uint64_t *r = res.st + 4ull * p;
    for (int k = 0; k < 4; ++k) r[k] = o[k];
}

// Eq. (2) over the inputs of one output.
__device__ __forceinline__ void combine(uint32_t j, const double2 *pa, const uint64_t *pst, size_t stride,
                                        const double *coeffs, uint32_t S, double *amps, uint64_t *stats) {
    double re = 0.0, im = 0.0;
    uint64_t nv = 0, sh = 0, xh = 0, lv = 0;
    bool bad = false;
    for (uint32_t i = 0; i < S; ++i) {
        const double2 a = pa[i];
        const double cr = coeffs[2 * i], ci = coeffs[2 * i + 1];
        re += cr * a.x - ci * a.y;
        im += cr * a.y + ci * a.x;
        const uint64_t *st = pst + stride * i;
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

// k_pair_reduce and k_finalize in one launch when every pair is in one
// batch: the same sums in the same order.
__global__ void k_reduce_finalize(PreBufs pre, Partials part, uint32_t ipp, uint32_t A, const double *coeffs,
                                  uint32_t S, uint32_t M, double *amps, uint64_t *stats) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    constexpr uint32_t kMaxS = 8;
    if (S > kMaxS) return;   // the launcher takes the two-kernel path then
    double2 pa[kMaxS];
    uint64_t pst[4 * kMaxS];
    for (uint32_t i = 0; i < S; ++i) {
        uint64_t o[4];
        pair_sums(pre, part, 0u, j * S + i, ipp, A, pa[i], o);
        for (int k = 0; k < 4; ++k) pst[4 * i + k] = o[k];
    }
    combine(j, pa, pst, 4, coeffs, S, amps, stats);
}

__global__ void k_finalize(PairRes res, const double *coeffs, uint32_t S, uint32_t M,
                           double *amps, uint64_t *stats) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const size_t p = static_cast<size_t>(j) * S;
    combine(j, res.amp + p, res.st + 4 * p, 4, coeffs, S, amps, stats);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <class F>
void dispatch_nw(int NW, F &&f) {
    if (NW == 1) f(IC<1>{});
    else if (NW == 2) f(IC<2>{});
    else f(IC<4>{});
}

template <class F>
void dispatch_bool(bool b, F &&f) {
    if (b) f(std::true_type{});
    else f(std::false_type{});
}

template <class F>
void dispatch_h(int H, F &&f) {
    if (H <= 1) f(IC<1>{});
    else f(IC<2>{});
}

size_t lds_bytes(uint32_t lo, uint32_t hi) { return static_cast<size_t>(hi - lo) * sizeof(double); }

bool fits_lds(uint32_t lo, uint32_t hi) { return hi - lo <= kMaxLdsFactors; }

hipError_t launch_precheck(const Common &c, int NW, PreBufs pre, uint32_t P, uint32_t *zero_words,
                           uint32_t n_zero, hipStream_t s) {
    const uint32_t n = P > n_zero ? P : n_zero;
    const uint32_t blocks = (n + 255) / 256;
    if (blocks == 0) return hipSuccess;
    dispatch_nw(NW, [&](auto nw) {
        dispatch_bool(c.thr > 0.0, [&](auto pr) {
            k_precheck<nw.value, pr.value><<<blocks, 256, 0, s>>>(c, pre, P, zero_words, n_zero);
        });
    });
    return hipGetLastError();
}

hipError_t launch_prefix(const Common &c, int NW, PreBufs pre, Table tab, uint32_t p0, uint32_t B,
                         uint32_t Dp, hipStream_t s) {
    if (B == 0) return hipSuccess;
    if (Dp > c.Ap || Dp > static_cast<uint32_t>(kDfsMax)) return hipErrorInvalidValue;
    const uint64_t NL = static_cast<uint64_t>(B) << (c.Ap - Dp);
    uint64_t blocks = (NL + 255) / 256;
    if (blocks > (1u << 20)) blocks = 1u << 20;
    const uint32_t P = c.M * c.S;
    const bool flds = fits_lds(c.f_L, c.f_c1);
    const size_t shm = flds ? lds_bytes(c.f_L, c.f_c1) : 0;
    dispatch_nw(NW, [&](auto nw) {
        dispatch_bool(c.thr > 0.0, [&](auto pr) {
            dispatch_bool(flds, [&](auto fl) {
                dispatch_bool(c.runs != 0u, [&](auto ru) {
                    k_prefix<nw.value, pr.value, fl.value, ru.value>
                        <<<static_cast<uint32_t>(blocks), 256, shm, s>>>(c, pre, tab, p0, B, P, Dp);
                });
            });
        });
    });
    return hipGetLastError();
}

hipError_t launch_consume(const Common &c, int NW, int H, Table tab, Partials part, uint32_t p0,
                          uint32_t B, uint32_t chunk, uint32_t ss, uint32_t *counter,
                          uint32_t grid, hipStream_t s) {
    if (B == 0 || grid == 0) return hipSuccess;
    const bool flds = fits_lds(c.f_c1, c.f_G);
    const size_t shm = flds ? lds_bytes(c.f_c1, c.f_G) : 0;
    dispatch_nw(NW, [&](auto nw) {
        dispatch_h(H, [&](auto hh) {
            dispatch_bool(c.thr > 0.0, [&](auto pr) {
                dispatch_bool(flds, [&](auto fl) {
                    dispatch_bool(c.runs != 0u, [&](auto ru) {
                        k_consume<nw.value, hh.value, pr.value, fl.value, ru.value>
                            <<<grid, kConsumeThreads, shm, s>>>(c, tab, part, p0, B, chunk, ss, counter);
                    });
                });
            });
        });
    });
    return hipGetLastError();
}

hipError_t launch_plain(const Common &c, int NW, int H, PreBufs pre, Partials part, uint32_t P,
                        uint32_t bpp, hipStream_t s) {
    const uint64_t blocks = static_cast<uint64_t>(P) * bpp;
    if (blocks == 0) return hipSuccess;
    const bool flds = fits_lds(c.f_L, c.f_G);
    const size_t shm = flds ? lds_bytes(c.f_L, c.f_G) : 0;
    dispatch_nw(NW, [&](auto nw) {
        dispatch_h(H, [&](auto hh) {
            dispatch_bool(c.thr > 0.0, [&](auto pr) {
                dispatch_bool(flds, [&](auto fl) {
                    dispatch_bool(c.runs != 0u, [&](auto ru) {
                        k_plain<nw.value, hh.value, pr.value, fl.value, ru.value>
                            <<<static_cast<uint32_t>(blocks), kPlainThreads, shm, s>>>(c, pre, part, P, bpp);
                    });
                });
            });
        });
    });
    return hipGetLastError();
}

hipError_t launch_pair_reduce(PreBufs pre, Partials part, PairRes res, uint32_t p0, uint32_t B,
                              uint32_t ipp, uint32_t A, hipStream_t s) {
    if (B == 0) return hipSuccess;
    k_pair_reduce<<<(B + 255) / 256, 256, 0, s>>>(pre, part, res, p0, B, ipp, A);
    return hipGetLastError();
}

hipError_t launch_count_valid(const uint32_t *ok, uint64_t n, unsigned long long *out,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 4096);
    k_count_valid<<<static_cast<uint32_t>(blocks), 256, 0, s>>>(ok, n, out);
    return hipGetLastError();
}

hipError_t launch_reduce_finalize(PreBufs pre, Partials part, uint32_t ipp, uint32_t A, const double *coeffs,
                                  uint32_t S, uint32_t M, double *amps, uint64_t *stats, hipStream_t s) {
    if (M == 0) return hipSuccess;
    k_reduce_finalize<<<(M + 255) / 256, 256, 0, s>>>(pre, part, ipp, A, coeffs, S, M, amps, stats);
    return hipGetLastError();
}

hipError_t launch_finalize(PairRes res, const double *coeffs, uint32_t S, uint32_t M, double *amps,
                           uint64_t *stats, hipStream_t s) {
    if (M == 0) return hipSuccess;
    k_finalize<<<(M + 255) / 256, 256, 0, s>>>(res, coeffs, S, M, amps, stats);
    return hipGetLastError();
}

int consume_blocks_per_cu(const Common &c, int NW, int H) {
    int nb = 0;
    hipError_t e = hipSuccess;
    const bool flds = fits_lds(c.f_c1, c.f_G);
    const size_t shm = flds ? lds_bytes(c.f_c1, c.f_G) : 0;
    dispatch_nw(NW, [&](auto nw) {
        dispatch_h(H, [&](auto hh) {
            dispatch_bool(c.thr > 0.0, [&](auto pr) {
                dispatch_bool(flds, [&](auto fl) {
                    dispatch_bool(c.runs != 0u, [&](auto ru) {
                        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb,
                            reinterpret_cast<const void *>(
                                k_consume<nw.value, hh.value, pr.value, fl.value, ru.value>),
                            kConsumeThreads, shm);
                    });
                });
            });
        });
    });
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

}  // namespace fhs
