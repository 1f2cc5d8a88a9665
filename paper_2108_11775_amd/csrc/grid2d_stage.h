// grid2d_stage.h -- per-block staging of the 2-D grid kernels with 32-sample waves
// (the fused morph and the log-det / inverse kernel): the kappa-scaled hinge axes and
// W in MFMA fragment order on the block's split scheme (mfma_split.h).
#pragma once

#include "mfma_split.h"

namespace pdmp {

// gxs[16 KS]: x-coordinates (kappa units), padding far away so that its features are
// 0 on both schemes (its weights are 0); gys[32 TB]: y-coordinates, padding 0.
// frag[(p * KS + ks) * TB * 64 + t * 64 + lane] = part p of
//   W[b = 32t + lane%32][a = 16ks + 8(lane/32) + j], j < 8 (0 outside the grid):
// three bf16 parts of W, or -- with ALLOW16 and the scheme test passed -- two FP16
// parts of 2^sw W.  fraw holds 3 KS TB 64 16-byte fragments.  All 64 kSplitWaves
// threads of the block call it; it synchronises the block before returning the
// block's scheme (fp16 == 0: BF16 parts).  Requires g0 <= 16 KS and g1 <= 32 TB.
template <int TB, int KS, bool ALLOW16>
__device__ __forceinline__ SplitScheme g2_stage(uint4 *fraw, float *gxs, float *gys,
                                                SplitRange &rg, const float *__restrict__ hinges,
                                                const float *__restrict__ weights, int g0, int g1,
                                                float kappa) {
    constexpr int kThreads = 64 * kSplitWaves;
    const int M = g0 * g1;
    for (int a = threadIdx.x; a < 16 * KS; a += kThreads)
        gxs[a] = a < g0 ? kappa * hinges[a] : 1e18f;
    for (int b = threadIdx.x; b < 32 * TB; b += kThreads)
        gys[b] = b < g1 ? kappa * hinges[(size_t)M + (size_t)g0 * b] : 0.0f;
    // this thread's share of W in fragment order, kept in registers through the range
    // check, and its largest and smallest nonzero magnitude
    constexpr int kNI = (KS * TB * 64 + kThreads - 1) / kThreads;
    float wv8[kNI][8];
    uint32_t mx = 0, mn = 0xffffffffu;
#pragma unroll
    for (int it = 0; it < kNI; ++it) {
        const int idx = threadIdx.x + it * kThreads;
        const int ln = idx & 63, t = (idx >> 6) % TB, ks = idx / (64 * TB);
        const int b = 32 * t + (ln & 31);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int a = 16 * ks + 8 * (ln >> 5) + j;
            const float w = (idx < KS * TB * 64 && a < g0 && b < g1)
                                ? weights[a + (int64_t)g0 * b] : 0.0f;
            wv8[it][j] = w;
            const uint32_t u = __float_as_uint(w) & 0x7fffffffu;
            mx = max(mx, u);
            if (u != 0) mn = min(mn, u);
        }
    }
    SplitScheme sc = {0, 0, 0.0f, 0.0f};
    if (ALLOW16) sc = split_decide(mx, mn, hinges, g0, kappa, rg);
#pragma unroll
    for (int it = 0; it < kNI; ++it) {
        const int idx = threadIdx.x + it * kThreads;
        if (idx >= KS * TB * 64) break;
        const int ln = idx & 63, t = (idx >> 6) % TB, ks = idx / (64 * TB);
        if (ALLOW16 && sc.fp16) {
            f16x8_t *frag = reinterpret_cast<f16x8_t *>(fraw);
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = ldexpf(wv8[it][j], sc.sw);
            f16x8_t p1, p2;
            split2h(v, p1, p2);
            frag[(0 * KS + ks) * TB * 64 + t * 64 + ln] = p1;
            frag[(1 * KS + ks) * TB * 64 + t * 64 + ln] = p2;
        } else {
            bf16x8_t *frag = reinterpret_cast<bf16x8_t *>(fraw);
            bf16x8_t p1, p2, p3;
            split3(wv8[it], p1, p2, p3);
            frag[(0 * KS + ks) * TB * 64 + t * 64 + ln] = p1;
            frag[(1 * KS + ks) * TB * 64 + t * 64 + ln] = p2;
            frag[(2 * KS + ks) * TB * 64 + t * 64 + ln] = p3;
        }
    }
    __syncthreads();
    return sc;
}

}  // namespace pdmp
