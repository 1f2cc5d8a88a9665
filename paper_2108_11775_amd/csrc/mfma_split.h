// mfma_split.h -- FP32-accurate contractions on BF16 or FP16 MFMA (gfx950), and the
// per-block choice between the two for the grid kernels.
//
// BF16 scheme.  Each FP32 operand v is split, rounding to nearest even, into three bf16 parts
// v = v1 + v2 + v3 + r with |v2| <= 2^-8 |v|, |v3| <= 2^-16 |v| and |r| <= 2^-24 |v|
// (bf16 carries 8 significant bits; every difference is exact in FP32) while the
// parts are normal numbers, |v| >= 2^-110; below, |r| is at most 2^-133.  Of the nine
// products of the parts of two operands, the six with v_i w_j, i + j <= 4, are kept:
// the three dropped ones are below 2^-24 of the product.  Products of bf16 parts are
// exact and v_mfma_f32_32x32x16_bf16 accumulates them in FP32, so a contraction
// carries FP32-class error (a few units of 2^-24 of the sum of absolute products) at
// 6 x 16 = 96 bf16 flops per FP32 multiply-add; the dense BF16 MFMA rate is 16 times
// the FP32 one, so the contraction takes 6/16 of the matrix-core time of
// v_mfma_f32_32x32x2_f32, and the splitting adds about 5.5 VALU per operand value.
// Layout of v_mfma_f32_32x32x16_bf16: lane l holds A[i = l%32][k = 8(l/32) + j] and
// B[k = 8(l/32) + j][n = l%32], j < 8; the accumulator (D) is lane l, register v ->
// row 8(v/4) + 4(l/32) + v%4, column l%32.
#pragma once

#include <hip/hip_runtime.h>

namespace pdmp {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

// v = p1 + p2 + p3 + r, each part rounded to nearest even in bf16.
__device__ __forceinline__ void split3(const float (&v)[8], bf16x8_t &p1, bf16x8_t &p2,
                                       bf16x8_t &p3) {
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
        const f32x2_t a = {v[j], v[j + 1]};
        const bf16x2_t h = __builtin_convertvector(a, bf16x2_t);
        const f32x2_t r = a - __builtin_convertvector(h, f32x2_t);
        const bf16x2_t m = __builtin_convertvector(r, bf16x2_t);
        const f32x2_t r2 = r - __builtin_convertvector(m, f32x2_t);
        const bf16x2_t l = __builtin_convertvector(r2, bf16x2_t);
        p1[j] = h[0];
        p1[j + 1] = h[1];
        p2[j] = m[0];
        p2[j + 1] = m[1];
        p3[j] = l[0];
        p3[j + 1] = l[1];
    }
}

// acc += (a1 + a2 + a3)(b1 + b2 + b3) to FP32 accuracy: the six leading products,
// smallest first.
__device__ __forceinline__ f32x16_t mfma_x6(const bf16x8_t &a1, const bf16x8_t &a2,
                                            const bf16x8_t &a3, const bf16x8_t &b1,
                                            const bf16x8_t &b2, const bf16x8_t &b3,
                                            f32x16_t acc) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3, b1, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, b2, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b3, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, b1, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b2, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc, 0, 0, 0);
}

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

// The same six products on v_mfma_f32_16x16x32_bf16 (lane l holds A[i = l%16][k =
// 8(l/16) + j] and B[k = 8(l/16) + j][n = l%16]; D: lane l, register v -> row
// 4(l/16) + v, column l%16).
__device__ __forceinline__ f32x4_t mfma16_x6(const bf16x8_t &a1, const bf16x8_t &a2,
                                             const bf16x8_t &a3, const bf16x8_t &b1,
                                             const bf16x8_t &b2, const bf16x8_t &b3,
                                             f32x4_t acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, b1, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b2, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b3, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b1, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b2, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc, 0, 0, 0);
}

// ---- FP16 scheme: two-part FP16 splits (for operands whose range has been brought
// inside FP16's by power-of-two scaling) ----
//
// FP16 carries 11 significant bits, so two parts hold 22 and three products of them
// reach what six products of three bf16 parts do: 3 x 16 = 48 FP16 flops per FP32
// multiply-add (half the matrix-core time of the BF16 scheme) and about 2 VALU per
// operand value for the split.
//
// v = h1 + h2 + r with both parts FP16 rounded to nearest even: |h2| <= 2^-11 |v| and
// |r| <= max(2^-22 |v|, 2^-25), 2^-25 being half the FP16 subnormal spacing, for any
// |v| <= 65504.  The residual v - h1 is exact in FP32.  Of the four products of two split operands the three with h1 are kept:
// the dropped h2 g2 is below 2^-22 of the product, so a product carries at most
// 3 x 2^-22 of its magnitude, and the FP16 products are exact in the FP32
// accumulator.  Values above 65504 overflow: callers scale both operands by powers
// of two first.
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));

// The residual v - h1 is one v_fma_mix_f32 (h1 read as FP16 from its half of the
// packed register, times -1 from a register, plus v; exact), which the compiler forms
// for only some of the values by itself.
__device__ __forceinline__ void split2h(const float (&v)[8], f16x8_t &p1, f16x8_t &p2) {
    float neg1 = -1.0f;
    asm volatile("" : "+v"(neg1));  // a register operand: no inline constant in the mix
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
        const f32x2_t a = {v[j], v[j + 1]};
        const f16x2_t h = __builtin_convertvector(a, f16x2_t);
        float r0, r1;
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[1,0,0]"
            : "=v"(r0) : "v"(h), "v"(neg1), "v"(v[j]));
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
            : "=v"(r1) : "v"(h), "v"(neg1), "v"(v[j + 1]));
        const f32x2_t r = {r0, r1};
        const f16x2_t l = __builtin_convertvector(r, f16x2_t);
        p1[j] = h[0];
        p1[j + 1] = h[1];
        p2[j] = l[0];
        p2[j + 1] = l[1];
    }
}

// acc += (a1 + a2)(b1 + b2) less a2 b2 on v_mfma_f32_32x32x16_f16 (the bf16 layout
// above), smallest product first.
__device__ __forceinline__ f32x16_t mfma_h3(const f16x8_t &a1, const f16x8_t &a2,
                                            const f16x8_t &b1, const f16x8_t &b2,
                                            f32x16_t acc) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a2, b1, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1, b2, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a1, b1, acc, 0, 0, 0);
}

// The same three products on v_mfma_f32_16x16x32_f16 (the 16x16x32 bf16 layout above).
__device__ __forceinline__ f32x4_t mfma16_h3(const f16x8_t &a1, const f16x8_t &a2,
                                             const f16x8_t &b1, const f16x8_t &b2,
                                             f32x4_t acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, b1, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, b2, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, b1, acc, 0, 0, 0);
}

// ---- choosing a grid contraction's split scheme ----
//
// A grid kernel contracts W (rows: the other axes' hinges, k: the x-axis hinges a)
// with the x-side operands ex_a = 2^-(xs - gx_a)^2 and ex_a (xs - gx_a) of each point
// (kappa units).  The FP16 scheme needs both inside FP16's exponent range after
// power-of-two scaling; every block of a launch decides from the same data, so all
// reach the same choice:
//  * W is scaled by 2^sw so that 2^14 <= max|W| < 2^15; every nonzero |W| must be at
//    least 2^-19 max|W| (its two FP16 parts then stay normal, or their rounding within
//    2^-19 of it) and all of W finite;
//  * a point's x-side operands are scaled by 2^c, c = 15 - k + floor(m), m the squared
//    distance of xs from the hinge x-range [gmin, gmax] and 2^k > sqrt(m): the largest
//    2^c ex_a is at most 2^15 and at least 2^(14-k) outside the range, and
//    2^c ex_a |dx_a| stays below 2^15; inside the range every point lies within 3 of a
//    hinge when no two consecutive hinge x-coordinates are more than 6 apart, so the
//    largest 2^15 ex_a is at least 2^6;
//  * the sums are scaled back by 2^-(sw + c) with ldexp (exact).
// Otherwise the kernel takes the three-part BF16 splits, which have FP32's range.
constexpr int kSplitRangeLog2 = 19;   // nonzero |W| >= 2^-19 max|W|
constexpr float kSplitMaxGap = 6.0f;  // consecutive hinge x-coordinates, kappa units
constexpr int kSplitWaves = 4;        // the grid kernels' 256-thread blocks

struct SplitRange {
    uint32_t wmax[kSplitWaves], wmin[kSplitWaves];
    float gmin, gmax, gap;
};

// The block's scheme: FP16 parts with W scaled by 2^sw and the hinge x-range
// [gmin, gmax] (kappa units), or (fp16 == 0) BF16 parts.
struct SplitScheme {
    int fp16, sw;
    float gmin, gmax;
};

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}

// The scheme from each thread's largest and smallest nonzero weight magnitude (FP32
// bit patterns, which order like the values for non-negative numbers and put NaN
// above infinity) and the g0 <= 64 hinge x-coordinates xaxis[0..g0).  Every thread of
// the 256-thread block calls it; it synchronises the block once.
__device__ __forceinline__ SplitScheme split_decide(uint32_t mx, uint32_t mn,
                                                    const float *__restrict__ xaxis, int g0,
                                                    float kappa, SplitRange &rg) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    mx = wave_max_u32(mx);
    mn = wave_min_u32(mn);
    if (lane == 0) {
        rg.wmax[wv] = mx;
        rg.wmin[wv] = mn;
    }
    if (wv == 0) {
        // one hinge x-coordinate per lane; the next larger coordinate of each by a
        // scan over the lanes
        const bool act = lane < g0;
        const float g = act ? kappa * xaxis[lane] : 0.0f;
        float lo = act ? g : INFINITY, hi = act ? g : -INFINITY, nxt = INFINITY;
        for (int b = 0; b < g0; ++b) {
            const float o = __builtin_bit_cast(float, __builtin_amdgcn_readlane(
                                                          __builtin_bit_cast(int, g), b));
            if (o > g) nxt = fminf(nxt, o);
        }
        float gap = act && nxt < INFINITY ? nxt - g : 0.0f;
        if (act && !(g == g)) gap = INFINITY;  // a NaN coordinate fails the check
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            lo = fminf(lo, __shfl_xor(lo, off, 64));
            hi = fmaxf(hi, __shfl_xor(hi, off, 64));
            gap = fmaxf(gap, __shfl_xor(gap, off, 64));
        }
        if (lane == 0) {
            rg.gmin = lo;
            rg.gmax = hi;
            rg.gap = gap;
        }
    }
    __syncthreads();
    uint32_t wmx = rg.wmax[0], wmn = rg.wmin[0];
#pragma unroll
    for (int w = 1; w < kSplitWaves; ++w) {
        wmx = max(wmx, rg.wmax[w]);
        wmn = min(wmn, rg.wmin[w]);
    }
    SplitScheme sc = {0, 0, rg.gmin, rg.gmax};
    bool ok = wmx < 0x7f800000u && rg.gap <= kSplitMaxGap && sc.gmax - sc.gmin < INFINITY;
    if (ok && wmx != 0) {
        int e;
        (void)frexpf(__uint_as_float(wmx), &e);  // max|W| = f 2^e, f in [0.5, 1)
        sc.sw = 15 - e;
        ok = __uint_as_float(wmn) >= ldexpf(__uint_as_float(wmx), -kSplitRangeLog2);
    }
    sc.fp16 = __builtin_amdgcn_readfirstlane((int)ok);
    return sc;
}

// A point's FP16 operand scale exponent c (above), with k returned for operands that
// carry a second factor dx (2^(c-k) ex dx^2 stays below 2^15 as well).  m is capped at
// 256, where every feature underflows anyway.
__device__ __forceinline__ int split_scale_exp(float xs, float gmin, float gmax, int &k) {
    const float dist = fmaxf(fmaxf(gmin - xs, xs - gmax), 0.0f);
    const float m = floorf(fminf(dist * dist, 256.0f));
    (void)frexpf(dist, &k);  // dist < 2^k
    k = max(k, 0);
    return 15 - k + (int)m;
}
__device__ __forceinline__ int split_scale_exp(float xs, float gmin, float gmax) {
    int k;
    return split_scale_exp(xs, gmin, gmax, k);
}

}  // namespace pdmp
