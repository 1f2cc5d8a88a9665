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

// ---- exact-zero skipping on the FP16 scheme (the ordered kernels) ----
//
// The wave-level tests of the ordered morph (grid2d.hip, where the argument for the
// morph's sums is set out) and of the ordered log-det / inverse: a k-step is skipped
// when every sample lies at dx^2 >= c + lim0 from its hinges' x-range, an 8-row group
// when every sample lies kYReach beyond its rows.  lim0 = 30 zeroes the FP16 parts of
// the B operands 2^c ex and 2^c ex dx.  The Hessian's third operand 2^(c-k) ex dx^2
// (k >= 0) is 2^(c - dx^2 + 2 log2|dx| - k): below the FP16 zero (2^-25) when dx^2 >=
// c + 35 for |dx| < 32, and for |dx| >= 32 since dx^2 - 2 log2|dx| >= 1014 exceeds
// c + 25 (c <= 271), so the Hessian's evaluations take lim0 = 35.  On the y side the
// Hessian's factors ey dy^2 vanish with ey, as ey dy does.
constexpr int kSortParts = 8;  // parts of an ordered batch, one per XCD
constexpr float kYReach = 12.5f;

// Samples per part: ceil(n / 8).
__host__ __device__ __forceinline__ int64_t sort_part(int64_t n) {
    return (n + kSortParts - 1) / kSortParts;
}

// The wave-uniform frame of the tests: each k-step's hinge x-range and each 8-row
// group's widened y-range (kappa units; padding excluded: a group of padding rows
// only is never needed, its weights being zero), in scalar registers.
template <int TB, int KS>
struct SkipFrame {
    float klo[KS], khi[KS], ga[4 * TB], gb[4 * TB];
    bool group_test;
};

template <int TB, int KS>
__device__ __forceinline__ void skip_frame(const float *gxs, const float *gys, int g0, int g1,
                                           SkipFrame<TB, KS> &f) {
    // one coordinate per lane, reduced over its k-step's 16 lanes and its group's 8
    const int lane = threadIdx.x & 63;
    const bool xin = lane < g0, yin = lane < g1;  // g0 <= 16 KS, g1 <= 32 TB
    const float gx = gxs[min(lane, 16 * KS - 1)], gy = gys[min(lane, 32 * TB - 1)];
    float xlo = xin ? gx : INFINITY, xhi = xin ? gx : -INFINITY;
    float ylo = yin ? gy : INFINITY, yhi = yin ? gy : -INFINITY;
    float ymag = yin ? fabsf(gy) : 0.0f;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        if (off < 16) {
            xlo = fminf(xlo, __shfl_xor(xlo, off, 64));
            xhi = fmaxf(xhi, __shfl_xor(xhi, off, 64));
        }
        if (off < 8) {
            ylo = fminf(ylo, __shfl_xor(ylo, off, 64));
            yhi = fmaxf(yhi, __shfl_xor(yhi, off, 64));
        }
        ymag = fmaxf(ymag, __shfl_xor(ymag, off, 64));
    }
    auto lane_f = [](float v, int l) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
    };
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        f.klo[ks] = lane_f(xlo, 16 * ks);
        f.khi[ks] = lane_f(xhi, 16 * ks);
    }
#pragma unroll
    for (int g = 0; g < 4 * TB; ++g) {
        f.ga[g] = lane_f(ylo, 8 * g) - kYReach;
        f.gb[g] = lane_f(yhi, 8 * g) + kYReach;
    }
    f.group_test = lane_f(ymag, 0) < 0x1p20f;
}

// The wave's kept k-steps (km, bit ks) and 8-row groups (gm, bit g) at the prescaled
// points (xs, ys), with lim = c + lim0 (per lane).
template <int TB, int KS>
__device__ __forceinline__ void skip_masks(const SkipFrame<TB, KS> &f, float xs, float ys,
                                           float lim, uint32_t &km, uint32_t &gm) {
    km = 0;
    gm = 0;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const float d = fmaxf(fmaxf(f.klo[ks] - xs, xs - f.khi[ks]), 0.0f);
        km |= (__ballot(d * d < lim) != 0 ? 1u : 0u) << ks;
    }
#pragma unroll
    for (int g = 0; g < 4 * TB; ++g)
        gm |= ((__ballot(!(ys <= f.ga[g])) & __ballot(!(ys >= f.gb[g]))) != 0 ? 1u : 0u) << g;
    if (!f.group_test || __ballot(!__builtin_isfinite(xs) || !__builtin_isfinite(ys)) != 0) {
        km = (1u << KS) - 1u;
        gm = (1u << (4 * TB)) - 1u;
    }
    km = __builtin_amdgcn_readfirstlane(km);
    gm = __builtin_amdgcn_readfirstlane(gm);
}

// Tiles (bit t) with at least one kept group.
template <int TB>
__device__ __forceinline__ uint32_t skip_tiles(uint32_t gm) {
    uint32_t tm = 0;
#pragma unroll
    for (int t = 0; t < TB; ++t) tm |= (((gm >> (4 * t)) & 15u) != 0 ? 1u : 0u) << t;
    return tm;
}

}  // namespace pdmp
