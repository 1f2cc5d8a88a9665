// issue_rates.hip -- measured issue costs of the instruction classes the grid morph
// kernels spend their time in: the diagnostic behind pdmp_issue_rates, with which the
// benchmark states its ceilings from this device instead of assumed rates.
//
// Each probe kernel runs a fixed loop of one instruction class in eight independent
// dependency chains per lane (enough waves per SIMD that issue, not latency, binds)
// and is timed with HIP events; the shader clock over the same kernel comes from the
// ratio of the shader-clock counter (s_memtime) to the 100 MHz real-time counter.  A
// class's cost is then cycles / (instructions issued per SIMD).  The two mixed probes
// interleave independent chains of two classes, so their per-iteration cost shows
// whether the classes overlap (co-issue) or add.
#include "mfma_split.h"
#include "pdmp_common.h"

namespace pdmp {

constexpr int kProbeIters = 1024;

enum ProbeOp {
    kPFma = 0,     // v_fma_f32
    kPExp = 1,     // v_exp_f32
    kPCvt = 2,     // v_cvt_pk_f16_f32
    kPMix = 3,     // v_fma_mix_f32
    kPExpFma = 4,  // 4 v_exp_f32 + 4 v_fma_f32, independent chains
    kPMfma = 5,    // v_mfma_f32_32x32x16_f16, 4 independent accumulators
    kPMfmaFma = 6  // 4 v_mfma_f32_32x32x16_f16 + 32 v_fma_f32, independent
};

template <int OP>
__global__ void __launch_bounds__(256) k_probe(float *sink, uint64_t *clk) {
    float r[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = 0.5f + 0.01f * j + 1e-7f * threadIdx.x;
    float a = 0.999f, b = 0.001f, m1 = -1.0f;
    asm volatile("" : "+v"(a), "+v"(b), "+v"(m1));
    f16x8_t ha, hb;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        ha[j] = (_Float16)(0.01f * j);
        hb[j] = (_Float16)(0.02f * j);
    }
    f32x16_t acc[4] = {};
    const uint64_t t0 = __builtin_amdgcn_s_memtime();
    const uint64_t w0 = __builtin_amdgcn_s_memrealtime();
    for (int it = 0; it < kProbeIters; ++it) {
        if (OP == kPFma) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(r[j]) : "v"(a), "v"(b));
        } else if (OP == kPExp) {
#pragma unroll
            for (int j = 0; j < 8; ++j) asm volatile("v_exp_f32 %0, -%0" : "+v"(r[j]));
        } else if (OP == kPCvt) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                asm volatile("v_cvt_pk_f16_f32 %0, %0, %1" : "+v"(r[j]) : "v"(a));
        } else if (OP == kPMix) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                asm volatile("v_fma_mix_f32 %0, %0, %1, %2 op_sel_hi:[1,0,0]"
                             : "+v"(r[j]) : "v"(m1), "v"(a));
        } else if (OP == kPExpFma) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                asm volatile("v_exp_f32 %0, -%0" : "+v"(r[j]));
                asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(r[j + 4]) : "v"(a), "v"(b));
            }
        } else if (OP == kPMfma) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ha, hb, acc[j], 0, 0, 0);
        } else if (OP == kPMfmaFma) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ha, hb, acc[j], 0, 0, 0);
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(r[k]) : "v"(a), "v"(b));
            }
        }
    }
    const uint64_t t1 = __builtin_amdgcn_s_memtime();
    const uint64_t w1 = __builtin_amdgcn_s_memrealtime();
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += r[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) s += acc[j][0];
    sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
    if (threadIdx.x == 0) {
        clk[2 * (size_t)blockIdx.x] = t1 - t0;
        clk[2 * (size_t)blockIdx.x + 1] = w1 - w0;
    }
}

struct ProbeSpec {
    int op, waves_per_simd;
    double instr_per_iter;  // per wave, of the class the cost is quoted for
};

template <int OP>
static hipError_t run_probe(int blocks, float *sink, uint64_t *clk, hipEvent_t e0, hipEvent_t e1,
                            float &ms) {
    hipLaunchKernelGGL(k_probe<OP>, dim3(blocks), dim3(256), 0, nullptr, sink, clk);  // warm-up
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_probe<OP>, dim3(blocks), dim3(256), 0, nullptr, sink, clk);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    return e;
}

}  // namespace pdmp

using namespace pdmp;

extern "C" int32_t pdmp_issue_rates(double *out, int32_t n_out) {
    PDMP_REQUIRE(out != nullptr && n_out >= 1, "out NULL or n_out < 1");
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cus < 1) {
        set_error("device query: %s", hipGetErrorString(e));
        return PDMP_EDEVICE;
    }
    const ProbeSpec specs[] = {{kPFma, 8, 8},  {kPExp, 8, 8},      {kPCvt, 8, 8}, {kPMix, 8, 8},
                               {kPExpFma, 8, 1}, {kPMfma, 4, 4}, {kPMfmaFma, 4, 1}};
    constexpr int kSpecs = 7;
    const int max_blocks = cus * 8;
    float *sink = nullptr;
    uint64_t *clk = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipMalloc(&sink, sizeof(float) * 256 * (size_t)max_blocks);
    if (e == hipSuccess) e = hipMalloc(&clk, sizeof(uint64_t) * 2 * (size_t)max_blocks);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double res[kSpecs + 1] = {};
    double clock_sum = 0.0;
    for (int k = 0; k < kSpecs && e == hipSuccess; ++k) {
        const ProbeSpec &p = specs[k];
        const int blocks = cus * p.waves_per_simd;  // 4 waves per block, one on each SIMD
        float ms = 0.0f;
        switch (p.op) {
            case kPFma: e = run_probe<kPFma>(blocks, sink, clk, e0, e1, ms); break;
            case kPExp: e = run_probe<kPExp>(blocks, sink, clk, e0, e1, ms); break;
            case kPCvt: e = run_probe<kPCvt>(blocks, sink, clk, e0, e1, ms); break;
            case kPMix: e = run_probe<kPMix>(blocks, sink, clk, e0, e1, ms); break;
            case kPExpFma: e = run_probe<kPExpFma>(blocks, sink, clk, e0, e1, ms); break;
            case kPMfma: e = run_probe<kPMfma>(blocks, sink, clk, e0, e1, ms); break;
            default: e = run_probe<kPMfmaFma>(blocks, sink, clk, e0, e1, ms); break;
        }
        if (e != hipSuccess) break;
        uint64_t c0[2];
        e = hipMemcpy(c0, clk, sizeof(c0), hipMemcpyDeviceToHost);
        if (e != hipSuccess) break;
        // the real-time counter runs at 100 MHz
        const double ghz = c0[1] ? (double)c0[0] / (double)c0[1] * 0.1 : 0.0;
        clock_sum += ghz;
        const double issued = (double)p.waves_per_simd * kProbeIters * p.instr_per_iter;
        res[k] = (double)ms * 1e-3 * ghz * 1e9 / issued;
    }
    res[kSpecs] = clock_sum / kSpecs;
    if (sink) (void)hipFree(sink);
    if (clk) (void)hipFree(clk);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        set_error("issue-rate probe: %s", hipGetErrorString(e));
        return PDMP_EDEVICE;
    }
    for (int k = 0; k < n_out && k <= kSpecs; ++k) out[k] = res[k];
    return PDMP_OK;
}
