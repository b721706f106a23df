// probe_valu_issue -- VALU issue-rate probe for the ALU rooflines.
//
// The consumer kernels are bound by VALU issue, and the chip's published
// figures give only the FP32 and FP64 vector rates.  This probe measures
// the throughput of the instruction kinds the compiled history programs are
// made of: every lane runs 8 independent chains of one instruction kind
// (inline asm on registers only, so the compiler can neither fuse nor
// vectorise them; no memory operation inside the asm), 8 blocks of 256
// threads per compute unit (8 waves per SIMD).  It prints lane-instructions
// per clock per CU at the 2.4 GHz peak engine clock, timed with HIP events
// over the second of two identical launches.
//
//     paper_2608_01467_amd/probe_valu_issue
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int kIters = 4096;
constexpr int kChains = 8;

enum Kind {
    ADD_U32, XOR_B32, AND_B32, LSHL_B32, BFE_U32, CNDMASK_B32, ADD3_U32, BFI_B32, BCNT_U32, FMA_F64, MUL_F64,
    FMA_F64_ADD_U32, CNDMASK_SGPR
};

template <int K>
__global__ __launch_bounds__(256) void probe(uint32_t *out, uint32_t seed) {
    uint32_t a[kChains];
    double d[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        a[i] = threadIdx.x * 7u + static_cast<uint32_t>(i) + seed;
        d[i] = 1.0 + 1e-9 * (threadIdx.x + i);
    }
    const uint32_t k = seed | 1u;
    const double m = 1.0000001, c = 1e-12;
    uint64_t msk = 0;   // a lane mask in an SGPR pair, written by a compare as in the history programs
    if constexpr (K == CNDMASK_SGPR) asm volatile("v_cmp_ne_u32_e64 %0, 0, %1" : "=s"(msk) : "v"(a[0] & 1u));
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) {
            if constexpr (K == ADD_U32) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[i]) : "v"(k));
            if constexpr (K == XOR_B32) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[i]) : "v"(k));
            if constexpr (K == AND_B32) asm volatile("v_and_b32 %0, %0, %1" : "+v"(a[i]) : "v"(k));
            if constexpr (K == LSHL_B32) asm volatile("v_lshlrev_b32 %0, 1, %0" : "+v"(a[i]));
            if constexpr (K == BFE_U32) asm volatile("v_bfe_u32 %0, %0, 3, 5" : "+v"(a[i]));
            if constexpr (K == CNDMASK_B32) asm volatile("v_cndmask_b32 %0, %0, %1, vcc" : "+v"(a[i]) : "v"(k));
            if constexpr (K == CNDMASK_SGPR)
                asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(a[i]) : "v"(k), "s"(msk));
            if constexpr (K == ADD3_U32) asm volatile("v_add3_u32 %0, %0, %1, %1" : "+v"(a[i]) : "v"(k));
            if constexpr (K == BFI_B32) asm volatile("v_bfi_b32 %0, %1, %0, %1" : "+v"(a[i]) : "v"(k));
            if constexpr (K == BCNT_U32) asm volatile("v_bcnt_u32_b32 %0, %0, %1" : "+v"(a[i]) : "v"(k));
            if constexpr (K == FMA_F64) asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(d[i]) : "v"(m), "v"(c));
            if constexpr (K == MUL_F64) asm volatile("v_mul_f64 %0, %0, %1" : "+v"(d[i]) : "v"(m));
            if constexpr (K == FMA_F64_ADD_U32) {
                asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(d[i]) : "v"(m), "v"(c));
                asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[i]) : "v"(k));
            }
        }
    }
    uint32_t s = 0;
    double ds = 0.0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        s += a[i];
        ds += d[i];
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = s + (ds > 3.0 ? 1u : 0u);
}

bool ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return false;
}

template <int K>
bool run(const char *name, int instr_per_step, uint32_t *d_out, int nblk, int ncu) {
    hipEvent_t e0, e1;
    if (!ok(hipEventCreate(&e0), "hipEventCreate") || !ok(hipEventCreate(&e1), "hipEventCreate")) return false;
    probe<K><<<nblk, 256>>>(d_out, 1u);
    if (!ok(hipDeviceSynchronize(), name)) return false;
    if (!ok(hipEventRecord(e0), "hipEventRecord")) return false;
    probe<K><<<nblk, 256>>>(d_out, 2u);
    if (!ok(hipEventRecord(e1), "hipEventRecord") || !ok(hipEventSynchronize(e1), name)) return false;
    float ms = 0.0f;
    if (!ok(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) return false;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double lane_instr = static_cast<double>(nblk) * 256 * kIters * kChains * instr_per_step;
    const double per_s = lane_instr / (ms * 1e-3);
    std::printf("%-30s %8.3f ms  %.3e lane-instr/s  %6.1f lanes/clk/CU at 2.4 GHz\n", name, ms, per_s,
                per_s / (ncu * 2.4e9));
    return true;
}

}  // namespace

int main() {
    int ncu = 0, khz = 0;
    if (!ok(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0), "attribute")) return 1;
    (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, 0);
    std::printf("CUs %d, max engine clock %d kHz; %d chains x %d steps per lane, 8 waves per SIMD\n", ncu, khz,
                kChains, kIters);
    const int nblk = ncu * 8;
    uint32_t *d_out = nullptr;
    if (!ok(hipMalloc(&d_out, sizeof(uint32_t) * nblk * 256), "hipMalloc")) return 1;
    const bool good = run<ADD_U32>("v_add_u32", 1, d_out, nblk, ncu) && run<XOR_B32>("v_xor_b32", 1, d_out, nblk, ncu) &&
                      run<AND_B32>("v_and_b32", 1, d_out, nblk, ncu) &&
                      run<LSHL_B32>("v_lshlrev_b32", 1, d_out, nblk, ncu) &&
                      run<BFE_U32>("v_bfe_u32", 1, d_out, nblk, ncu) &&
                      run<CNDMASK_B32>("v_cndmask_b32 (mask in vcc)", 1, d_out, nblk, ncu) &&
                      run<CNDMASK_SGPR>("v_cndmask_b32_e64 (mask in s[])", 1, d_out, nblk, ncu) &&
                      run<ADD3_U32>("v_add3_u32", 1, d_out, nblk, ncu) &&
                      run<BFI_B32>("v_bfi_b32", 1, d_out, nblk, ncu) &&
                      run<BCNT_U32>("v_bcnt_u32_b32", 1, d_out, nblk, ncu) &&
                      run<FMA_F64>("v_fma_f64", 1, d_out, nblk, ncu) && run<MUL_F64>("v_mul_f64", 1, d_out, nblk, ncu) &&
                      run<FMA_F64_ADD_U32>("v_fma_f64 + v_add_u32 (pairs)", 2, d_out, nblk, ncu);
    (void)hipFree(d_out);
    return good ? 0 : 1;
}
