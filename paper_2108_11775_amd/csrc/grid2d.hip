// grid2d.hip -- the occupancy and the fused T-step morph for hinges on a regular 2-D
// grid, as a dense contraction on the matrix cores.
//
// With hinges h_{a + G0 b} = (gx_a, gy_b) the RBF feature factorises,
//   phi_ab(x) = ex_a(x) ey_b(y),  ex_a = exp(-(x - gx_a)^2 / (2 l^2)),
// so with W[b][a] = w_{a + G0 b}
//   s      = sum_b ey_b U_b + beta,         U_b = sum_a W[b][a] ex_a
//   ds/dx  = -(1/l^2) sum_b ey_b V_b,       V_b = sum_a W[b][a] ex_a (x - gx_a)
//   ds/dy  = -(1/l^2) sum_b ey_b (y - gy_b) U_b
// which is the same s and grad s as the pairwise sum (rounding aside).  Per sample
// and step that is G0 + G1 exponentials and two G1 x G0 matrix-vector products,
// instead of G0 G1 exponentials.  The products for 32 samples at a time run on the
// matrix cores with A = W (rows b, k = a) and B = [ex | ex * dx] (k = a, column =
// sample); each lane computes the exponentials of its own B entries, so none is
// evaluated twice, and W is staged once per block in LDS in fragment order.  The y
// contraction runs on the accumulator layout: lane l owns rows b = 8(v/4) + 4(l/32)
// + v%4 of sample l%32, evaluates ey_b for them and the two lanes of a sample are
// summed by one xor-32 exchange (bit-identical in both lanes).  The T-step loop
// runs in registers.
#include "grid2d_stage.h"
#include "mfma_split.h"
#include "pdmp_common.h"

// Every rounding in this file is the one its source states (multiply-adds are written
// as fmaf): the spatially ordered kernel below must reproduce the unordered kernel's
// bits, which holds only if the compiler fuses neither kernel's products on its own.
#pragma clang fp contract(off)

namespace pdmp {

constexpr int kG2Block = 256;   // 4 waves, 32 samples each
static_assert(kG2Block == 64 * kSplitWaves, "the scheme test's block");

// The contractions run at FP32 accuracy on the matrix cores, on one of two split
// schemes (mfma_split.h): two-part FP16 splits with three products where the
// operands' range allows, three-part BF16 splits with six products otherwise.  Morphs
// only -- a single evaluation, whose blocks mostly stage W, keeps the BF16 scheme and
// skips the check.  The FP16 scheme needs half the matrix-core work and about half
// the splitting VALU.

// The x-side operands of k-step ks for this lane: ex and ex * dx at a = 16ks + 8half + j.
__device__ __forceinline__ void x6_operands(const float *gxs, float xs, int ks, int half,
                                            bf16x8_t (&e)[3], bf16x8_t (&de)[3]) {
    float ev[8], dv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float d = xs - gxs[16 * ks + 8 * half + j];
        ev[j] = exp2_fast(-d * d);
        dv[j] = ev[j] * d;
    }
    split3(ev, e[0], e[1], e[2]);
    split3(dv, de[0], de[1], de[2]);
}

// The same operands scaled by 2^c (c folded into the exponent) as FP16 pairs.
__device__ __forceinline__ void h3_operands(const float *gxs, float xs, float cf, int ks,
                                            int half, f16x8_t (&e)[2], f16x8_t (&de)[2]) {
    float ev[8], dv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float d = xs - gxs[16 * ks + 8 * half + j];
        ev[j] = exp2_fast(fmaf(-d, d, cf));
        dv[j] = ev[j] * d;
    }
    split2h(ev, e[0], e[1]);
    split2h(dv, de[0], de[1]);
}

// One sample's outputs, written by the lower lane of its pair: the morphed point, or
// the logit / occupancy / gradient of a single evaluation.
template <int MODE>
__device__ __forceinline__ void g2_finish(float s, float sx, float sy, float beta, float gscale,
                                          float x, float y, int half, int64_t i, int64_t n,
                                          float *c_out, float *s_out, float *g_out,
                                          float *x_out) {
    if (half != 0 || i >= n) return;
    if (MODE == kMorph) {
        x_out[i] = x;
        x_out[(size_t)n + i] = y;
    } else {
        const float sv = s + beta;
        float c, sp;
        sigmoid_and_slope(sv, c, sp);
        if (c_out) c_out[i] = c;
        if (MODE == kEval) {
            if (s_out) s_out[i] = sv;
        } else {
            g_out[i] = -sp * gscale * sx;
            g_out[(size_t)n + i] = -sp * gscale * sy;
        }
    }
}

// The y contraction on the accumulator layout and the xor-32 sum of the lane pair.
template <int TB>
__device__ __forceinline__ void g2_ysum(const float *gys, float ys, int half,
                                        const f32x16_t (&U)[TB], const f32x16_t (&V)[TB],
                                        float &s, float &sx, float &sy) {
    s = 0.0f;
    sx = 0.0f;
    sy = 0.0f;
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int b = 32 * t + 8 * (v >> 2) + 4 * half + (v & 3);
            const float d = ys - gys[b];
            const float e = exp2_fast(-d * d);
            s = fmaf(e, U[t][v], s);
            sx = fmaf(e, V[t][v], sx);
            sy = fmaf(e * d, U[t][v], sy);
        }
    s += __shfl_xor(s, 32, 64);
    sx += __shfl_xor(sx, 32, 64);
    sy += __shfl_xor(sy, 32, 64);
}

template <int TB, int KS, int MODE>
__global__ void __launch_bounds__(kG2Block) __attribute__((amdgpu_waves_per_eu(2)))
k_grid2d_mfma(const float *__restrict__ hinges, const float *__restrict__ weights, int g0, int g1,
              float kappa, float gscale, const float *x_in, int64_t n, int T, float eta,
              float *c_out, float *s_out, float *g_out, float *x_out, Traj tr) {
    // the FP16 scheme's per-block range check pays off over a morph's steps; a single
    // evaluation, whose blocks mostly stage W, keeps the BF16 scheme without it
    constexpr bool allow_fp16 = MODE == kMorph;
    // fragments and axes: grid2d_stage.h
    __shared__ uint4 fraw[3 * KS * TB * 64];
    __shared__ float gxs[16 * KS];
    __shared__ float gys[32 * TB];
    __shared__ SplitRange rg;
    const int M = g0 * g1;
    const int lane = threadIdx.x & 63, half = lane >> 5, wv = threadIdx.x >> 6;
    const SplitScheme sc =
        g2_stage<TB, KS, allow_fp16>(fraw, gxs, gys, rg, hinges, weights, g0, g1, kappa);
    const bool fp16 = allow_fp16 && sc.fp16;
    const int sw = sc.sw;
    const float gmin = sc.gmin, gmax = sc.gmax;

    const int64_t wave = (int64_t)blockIdx.x * (kG2Block / 64) + wv;
    const int64_t i = wave * 32 + (lane & 31);
    const int64_t ic = i < n ? i : n - 1;
    float x = x_in[ic], y = x_in[(size_t)n + ic];
    const float beta = weights[M];
    const int steps = MODE == kMorph ? T : 1;
    float s = 0.0f, sx = 0.0f, sy = 0.0f;
    int64_t tc;
    const bool rec = MODE == kMorph && half == 0 && traj_col(tr, i, n, tc);

    if (fp16) {
        const f16x8_t *frag = reinterpret_cast<const f16x8_t *>(fraw);
        for (int st = 0; st < steps; ++st) {
            if (rec) traj_put<2>(tr, st, tc, {x, y});
            const float xs = kappa * x, ys = kappa * y;
            // the operand scale 2^c of this sample (both lanes of the pair agree)
            const int c = split_scale_exp(xs, gmin, gmax);
            f32x16_t U[TB], V[TB];
            int ln = lane;  // opaque: keeps the fragment reads inside the step loop
            asm volatile("" : "+v"(ln));
            f16x8_t e[2], de[2];
            h3_operands(gxs, xs, (float)c, 0, half, e, de);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                f16x8_t ec[2] = {e[0], e[1]}, dc[2] = {de[0], de[1]};
                if (ks + 1 < KS) h3_operands(gxs, xs, (float)c, ks + 1, half, e, de);
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    const f16x8_t a1 = frag[(0 * KS + ks) * TB * 64 + t * 64 + ln];
                    const f16x8_t a2 = frag[(1 * KS + ks) * TB * 64 + t * 64 + ln];
                    const f32x16_t zero = {};
                    U[t] = mfma_h3(a1, a2, ec[0], ec[1], ks == 0 ? zero : U[t]);
                    V[t] = mfma_h3(a1, a2, dc[0], dc[1], ks == 0 ? zero : V[t]);
                }
            }
            g2_ysum<TB>(gys, ys, half, U, V, s, sx, sy);
            const int un = -(sw + c);
            s = ldexpf(s, un);
            sx = ldexpf(sx, un);
            sy = ldexpf(sy, un);
            if (MODE == kMorph) {
                float cc, sp;
                sigmoid_and_slope(s + beta, cc, sp);
                const float step = eta * sp * gscale;
                x = fmaf(step, sx, x);
                y = fmaf(step, sy, y);
            }
        }
    } else {
        const bf16x8_t *frag = reinterpret_cast<const bf16x8_t *>(fraw);
        for (int st = 0; st < steps; ++st) {
            if (rec) traj_put<2>(tr, st, tc, {x, y});
            const float xs = kappa * x, ys = kappa * y;
            f32x16_t U[TB], V[TB];
            // an opaque copy of the lane index keeps the fragment reads inside the step
            // loop (hoisted, the loop-invariant W parts would take 96 registers)
            int ln = lane;
            asm volatile("" : "+v"(ln));
            // the operands of k-step ks + 1 are formed while k-step ks's products run;
            // k-step 0 starts the accumulators from the zero constant
            bf16x8_t e[3], de[3];
            x6_operands(gxs, xs, 0, half, e, de);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                bf16x8_t ec[3] = {e[0], e[1], e[2]}, dc[3] = {de[0], de[1], de[2]};
                if (ks + 1 < KS) x6_operands(gxs, xs, ks + 1, half, e, de);
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    const bf16x8_t a1 = frag[(0 * KS + ks) * TB * 64 + t * 64 + ln];
                    const bf16x8_t a2 = frag[(1 * KS + ks) * TB * 64 + t * 64 + ln];
                    const bf16x8_t a3 = frag[(2 * KS + ks) * TB * 64 + t * 64 + ln];
                    const f32x16_t zero = {};
                    U[t] = mfma_x6(a1, a2, a3, ec[0], ec[1], ec[2], ks == 0 ? zero : U[t]);
                    V[t] = mfma_x6(a1, a2, a3, dc[0], dc[1], dc[2], ks == 0 ? zero : V[t]);
                }
            }
            g2_ysum<TB>(gys, ys, half, U, V, s, sx, sy);
            if (MODE == kMorph) {
                float c, sp;
                sigmoid_and_slope(s + beta, c, sp);
                const float step = eta * sp * gscale;
                x = fmaf(step, sx, x);
                y = fmaf(step, sy, y);
            }
        }
    }
    if (rec) traj_put<2>(tr, steps, tc, {x, y});
    g2_finish<MODE>(s, sx, sy, beta, gscale, x, y, half, i, n, c_out, s_out, g_out, x_out);
}

// ---- large batches in spatial order: the same sums, exact zeros skipped ----
//
// A workspace morph of a large batch first orders the samples by a 32 x 32 cell grid
// over the hinge axes' range (a counting sort into a permutation), so that the 32
// samples of a wave lie close together.  Every step, the wave then finds, from its
// samples' distances to each k-step's hinge x-range and to each 8-row group's y-range:
//  * k-steps whose B operands are zero for all its samples: on the FP16 scheme an
//    operand 2^c ex_a or 2^c ex_a |dx_a| = 2^(c - dx^2 + log2|dx|) rounds (both split
//    parts) to the FP16 zero at or below 2^-25, which every hinge of the k-step is
//    when the sample's nearest one lies at dx^2 >= c + 30 (kappa units): for |dx| <
//    32, log2|dx| < 5 leaves a margin far above the rounding of the exponential and
//    its argument, and for |dx| >= 32, dx^2 >= 1024 exceeds c + 25 + log2|dx| since
//    c <= 271;
//  * 8-row groups whose ey_b = exp2(-dy^2) are zero for all its samples: a sample at
//    least kYReach = 12.5 below the group's lowest row or above its highest has
//    dy^2 > 154 for every row, past FP32's smallest subnormal (the 0.5 over sqrt(150)
//    covers the rounding of the coordinates while the rows lie within 2^20 of 0; rows
//    beyond that switch the group test off), and row tiles with no such group take no
//    products at all.
// Their products and contractions add exact zeros to accumulators that start at +0
// (an MFMA with an all-zero B column leaves that column of C unchanged; fma(0, U, s)
// = s, and the sums never hold -0), so skipping them gives each sample the bits of
// the unordered kernel, in any grouping.  A wave with a non-finite coordinate in any
// lane skips nothing (there the unordered kernel's zero features multiply NaN or
// infinite factors).  The BF16 scheme (for operands of FP32 range, whose features
// need not underflow) takes the dense path, only through the permutation.
//
// The order is kept per part: the batch is cut into kSortParts = 8 contiguous parts,
// each sorted on its own, and block b of the morph takes its samples from part b mod
// 8.  Workgroups are handed to the eight XCDs in turn, so each part's samples are
// read and written by one XCD, whose L2 then holds the part's lines while its waves
// gather and scatter single coordinates through the permutation: HBM sees about one
// read and one write of each line instead of one per coordinate.
constexpr int kSortCells = 32;  // per axis (kSortParts, the parts: grid2d_stage.h)

// A wave-uniform value kept in a scalar register.
__device__ __forceinline__ float uniform_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// The y contraction of the 8-row groups of one 32-row tile set in gm (bit j: rows
// 32t + 8j .. 32t + 8j + 7), from this lane's rows gy[j][r] = gy_b, b = 32t + 8j +
// 4 half + r.
__device__ __forceinline__ void g2_ysum_tile(const f32x4_t (&gy)[4], float ys, uint32_t gm,
                                             const f32x16_t &U, const f32x16_t &V, float &s,
                                             float &sx, float &sy) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!((gm >> j) & 1u)) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int v = 4 * j + r;
            const float d = ys - gy[j][r];
            const float e = exp2_fast(-d * d);
            s = fmaf(e, U[v], s);
            sx = fmaf(e, V[v], sx);
            sy = fmaf(e * d, U[v], sy);
        }
    }
}

template <int TB, int KS>
__global__ void __launch_bounds__(kG2Block) __attribute__((amdgpu_waves_per_eu(3)))
k_grid2d_sorted(const float *__restrict__ hinges, const float *__restrict__ weights, int g0,
                int g1, float kappa, float gscale, const float *x_in, int64_t n, int T, float eta,
                const uint32_t *__restrict__ perm, int64_t part, float *x_out, Traj tr) {
    __shared__ uint4 fraw[3 * KS * TB * 64];
    __shared__ float gxs[16 * KS];
    __shared__ __align__(16) float gys[32 * TB];
    __shared__ SplitRange rg;
    const int M = g0 * g1;
    const int lane = threadIdx.x & 63, half = lane >> 5, wv = threadIdx.x >> 6;
    const SplitScheme sc = g2_stage<TB, KS, true>(fraw, gxs, gys, rg, hinges, weights, g0, g1, kappa);
    // part p = b mod 8 holds sorted places [p part, min((p + 1) part, n))
    const int64_t p = blockIdx.x % kSortParts;
    const int64_t k = ((int64_t)(blockIdx.x / kSortParts) * (kG2Block / 64) + wv) * 32 + (lane & 31);
    const int64_t slot = p * part + k;
    const bool live = k < part && slot < n;
    const uint32_t ic = perm[live ? slot : n - 1];
    const uint32_t i = live ? ic : (uint32_t)n;  // n (< 2^32 here): a tail lane, writes nothing
    float x = x_in[ic], y = x_in[(size_t)n + ic];
    const float beta = weights[M];
    float s = 0.0f, sx = 0.0f, sy = 0.0f;
    int64_t tc64;
    const bool rec = half == 0 && traj_col(tr, (int64_t)i, n, tc64);
    const uint32_t tc = (uint32_t)tc64;  // a column below n < 2^32

    if (sc.fp16) {
        const f16x8_t *frag = reinterpret_cast<const f16x8_t *>(fraw);
        SkipFrame<TB, KS> fr;
        skip_frame<TB, KS>(gxs, gys, g0, g1, fr);
        for (int st = 0; st < T; ++st) {
            if (rec) traj_put<2>(tr, st, (int64_t)tc, {x, y});
            const float xs = kappa * x, ys = kappa * y;
            const int c = split_scale_exp(xs, sc.gmin, sc.gmax);
            uint32_t km, gm;
            skip_masks<TB, KS>(fr, xs, ys, (float)(c + 30), km, gm);
            const uint32_t tm = skip_tiles<TB>(gm);
            f32x16_t U[TB], V[TB];
            int ln = lane;  // opaque: keeps the fragment reads inside the step loop
            asm volatile("" : "+v"(ln));
            // the kept k-steps in order, j-th kept one in operand buffer j % 2: its
            // successor's operands are formed while its products run, and the first
            // starts the accumulators from the zero constant
            f16x8_t eb[2][2], db[2][2];
            uint32_t rem = km;
            int ksn = rem ? __builtin_ctz(rem) : 0;
            if (rem) h3_operands(gxs, xs, (float)c, ksn, half, eb[0], db[0]);
#pragma unroll
            for (int j = 0; j < KS; ++j) {
                if (!rem) break;
                const int ks = ksn;
                rem &= rem - 1u;
                if (rem) {
                    ksn = __builtin_ctz(rem);
                    h3_operands(gxs, xs, (float)c, ksn, half, eb[(j + 1) & 1], db[(j + 1) & 1]);
                }
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    if (!((tm >> t) & 1u)) continue;
                    const f16x8_t a1 = frag[(0 * KS + ks) * TB * 64 + t * 64 + ln];
                    const f16x8_t a2 = frag[(1 * KS + ks) * TB * 64 + t * 64 + ln];
                    const f32x16_t zero = {};
                    U[t] = mfma_h3(a1, a2, eb[j & 1][0], eb[j & 1][1], j == 0 ? zero : U[t]);
                    V[t] = mfma_h3(a1, a2, db[j & 1][0], db[j & 1][1], j == 0 ? zero : V[t]);
                }
            }
            s = 0.0f;
            sx = 0.0f;
            sy = 0.0f;
            if (km) {
                // this lane's rows, all read before the group branches (one wait for
                // the LDS reads instead of one per group)
                f32x4_t gy[TB][4];
#pragma unroll
                for (int t = 0; t < TB; ++t) {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        gy[t][j] = *reinterpret_cast<const f32x4_t *>(&gys[32 * t + 8 * j + 4 * half]);
                    asm volatile("" ::"v"(gy[t][0]), "v"(gy[t][1]), "v"(gy[t][2]), "v"(gy[t][3]));
                }
#pragma unroll
                for (int t = 0; t < TB; ++t)
                    if ((tm >> t) & 1u)
                        g2_ysum_tile(gy[t], ys, (gm >> (4 * t)) & 15u, U[t], V[t], s, sx, sy);
            }
            s += __shfl_xor(s, 32, 64);
            sx += __shfl_xor(sx, 32, 64);
            sy += __shfl_xor(sy, 32, 64);
            const int un = -(sc.sw + c);
            s = ldexpf(s, un);
            sx = ldexpf(sx, un);
            sy = ldexpf(sy, un);
            float cc, sp;
            sigmoid_and_slope(s + beta, cc, sp);
            const float step = eta * sp * gscale;
            x = fmaf(step, sx, x);
            y = fmaf(step, sy, y);
        }
    } else {
        const bf16x8_t *frag = reinterpret_cast<const bf16x8_t *>(fraw);
        for (int st = 0; st < T; ++st) {
            if (rec) traj_put<2>(tr, st, (int64_t)tc, {x, y});
            const float xs = kappa * x, ys = kappa * y;
            f32x16_t U[TB], V[TB];
            int ln = lane;
            asm volatile("" : "+v"(ln));
            bf16x8_t e[3], de[3];
            x6_operands(gxs, xs, 0, half, e, de);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                bf16x8_t ec[3] = {e[0], e[1], e[2]}, dc[3] = {de[0], de[1], de[2]};
                if (ks + 1 < KS) x6_operands(gxs, xs, ks + 1, half, e, de);
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    const bf16x8_t a1 = frag[(0 * KS + ks) * TB * 64 + t * 64 + ln];
                    const bf16x8_t a2 = frag[(1 * KS + ks) * TB * 64 + t * 64 + ln];
                    const bf16x8_t a3 = frag[(2 * KS + ks) * TB * 64 + t * 64 + ln];
                    const f32x16_t zero = {};
                    U[t] = mfma_x6(a1, a2, a3, ec[0], ec[1], ec[2], ks == 0 ? zero : U[t]);
                    V[t] = mfma_x6(a1, a2, a3, dc[0], dc[1], dc[2], ks == 0 ? zero : V[t]);
                }
            }
            g2_ysum<TB>(gys, ys, half, U, V, s, sx, sy);
            float cc, sp;
            sigmoid_and_slope(s + beta, cc, sp);
            const float step = eta * sp * gscale;
            x = fmaf(step, sx, x);
            y = fmaf(step, sy, y);
        }
    }
    if (rec) traj_put<2>(tr, T, (int64_t)tc, {x, y});
    g2_finish<kMorph>(s, sx, sy, beta, gscale, x, y, half, (int64_t)i, n, nullptr, nullptr, nullptr,
                      x_out);
}

// ---- the spatial order: a counting sort of the samples into 32 x 32 cells ----

// The cell grid over the hinge axes' range (unscaled coordinates): origin and cells
// per unit on each axis, from the axis entries of the hinge array.
__device__ __forceinline__ void sort_frame(const float *__restrict__ hinges, int g0, int g1,
                                           float (&f)[4], float *red) {
    const int M = g0 * g1;
    float xlo = INFINITY, xhi = -INFINITY, ylo = INFINITY, yhi = -INFINITY;
    for (int a = threadIdx.x; a < g0; a += blockDim.x) {
        xlo = fminf(xlo, hinges[a]);
        xhi = fmaxf(xhi, hinges[a]);
    }
    for (int b = threadIdx.x; b < g1; b += blockDim.x) {
        const float v = hinges[(size_t)M + (size_t)g0 * b];
        ylo = fminf(ylo, v);
        yhi = fmaxf(yhi, v);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        xlo = fminf(xlo, __shfl_xor(xlo, off, 64));
        xhi = fmaxf(xhi, __shfl_xor(xhi, off, 64));
        ylo = fminf(ylo, __shfl_xor(ylo, off, 64));
        yhi = fmaxf(yhi, __shfl_xor(yhi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        const int w = threadIdx.x >> 6;
        red[4 * w] = xlo;
        red[4 * w + 1] = xhi;
        red[4 * w + 2] = ylo;
        red[4 * w + 3] = yhi;
    }
    __syncthreads();
    xlo = red[0], xhi = red[1], ylo = red[2], yhi = red[3];
    for (int w = 1; w < (int)blockDim.x / 64; ++w) {
        xlo = fminf(xlo, red[4 * w]);
        xhi = fmaxf(xhi, red[4 * w + 1]);
        ylo = fminf(ylo, red[4 * w + 2]);
        yhi = fmaxf(yhi, red[4 * w + 3]);
    }
    f[0] = xlo;
    f[1] = xhi > xlo ? (float)kSortCells / (xhi - xlo) : 0.0f;
    f[2] = ylo;
    f[3] = yhi > ylo ? (float)kSortCells / (yhi - ylo) : 0.0f;
}

// A point's cell (clamped; a NaN coordinate takes cell 0 of its axis).
__device__ __forceinline__ int sort_cell(float x, float y, const float (&f)[4]) {
    const float cx = fminf(fmaxf((x - f[0]) * f[1], 0.0f), (float)(kSortCells - 1));
    const float cy = fminf(fmaxf((y - f[2]) * f[3], 0.0f), (float)(kSortCells - 1));
    return (int)cy * kSortCells + (int)cx;
}

constexpr int kSortBlock = 256, kSortChunk = 4096;
constexpr int kSortKeys = kSortParts * kSortCells * kSortCells;

// Chunks of kSortChunk samples are cut within each part, as the morph's places are:
// block b takes chunk b / 8 of part b mod 8, so a part's reads of x and writes of its
// counters and permutation entries all come from one XCD.
__host__ __device__ __forceinline__ int64_t sort_chunks_per_part(int64_t n) {
    return (sort_part(n) + kSortChunk - 1) / kSortChunk;
}

__global__ void __launch_bounds__(kSortBlock) k_sort_zero(uint32_t *counts) {
    for (int b = threadIdx.x; b < kSortKeys; b += kSortBlock) counts[b] = 0;
}

// This block's chunk [lo, hi) of part p in an LDS histogram over the cells.
__device__ __forceinline__ void sort_chunk_hist(const float *__restrict__ hinges, int g0, int g1,
                                                const float *__restrict__ x, int64_t n,
                                                int64_t part, uint32_t *hist, float *red,
                                                float (&f)[4], int64_t &p, int64_t &lo,
                                                int64_t &hi) {
    sort_frame(hinges, g0, g1, f, red);
    for (int b = threadIdx.x; b < kSortCells * kSortCells; b += kSortBlock) hist[b] = 0;
    __syncthreads();
    p = blockIdx.x % kSortParts;
    lo = p * part + (int64_t)(blockIdx.x / kSortParts) * kSortChunk;
    hi = min(min(lo + kSortChunk, (p + 1) * part), n);
    for (int64_t i = lo + threadIdx.x; i < hi; i += kSortBlock)
        atomicAdd(&hist[sort_cell(x[i], x[(size_t)n + i], f)], 1u);
    __syncthreads();
}

__global__ void __launch_bounds__(kSortBlock)
k_sort_count(const float *__restrict__ hinges, int g0, int g1, const float *__restrict__ x, int64_t n,
             int64_t part, uint32_t *counts) {
    __shared__ uint32_t hist[kSortCells * kSortCells];
    __shared__ float red[4 * kSortBlock / 64];
    float f[4];
    int64_t p, lo, hi;
    sort_chunk_hist(hinges, g0, g1, x, n, part, hist, red, f, p, lo, hi);
    for (int b = threadIdx.x; b < kSortCells * kSortCells; b += kSortBlock)
        if (hist[b]) atomicAdd(&counts[p * kSortCells * kSortCells + b], hist[b]);
}

// Exclusive prefix sum of the 8 x 1024 part-cell counts, in place (one block of 1024
// threads, eight consecutive keys each).
__global__ void __launch_bounds__(1024) k_sort_scan(uint32_t *counts) {
    __shared__ uint32_t sh[1024];
    constexpr int kPer = kSortKeys / 1024;
    const int t = threadIdx.x;
    uint32_t v[kPer], run = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        v[j] = counts[kPer * t + j];
        run += v[j];
    }
    sh[t] = run;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t u = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += u;
        __syncthreads();
    }
    uint32_t base = t > 0 ? sh[t - 1] : 0u;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        counts[kPer * t + j] = base;
        base += v[j];
    }
}

__global__ void __launch_bounds__(kSortBlock)
k_sort_scatter(const float *__restrict__ hinges, int g0, int g1, const float *__restrict__ x,
               int64_t n, int64_t part, uint32_t *cursor, uint32_t *perm) {
    __shared__ uint32_t hist[kSortCells * kSortCells];
    __shared__ float red[4 * kSortBlock / 64];
    float f[4];
    int64_t p, lo, hi;
    sort_chunk_hist(hinges, g0, g1, x, n, part, hist, red, f, p, lo, hi);
    // this block's range in each of its part's cells, then the samples' places in it
    for (int b = threadIdx.x; b < kSortCells * kSortCells; b += kSortBlock)
        hist[b] = hist[b] ? atomicAdd(&cursor[p * kSortCells * kSortCells + b], hist[b]) : 0u;
    __syncthreads();
    for (int64_t i = lo + threadIdx.x; i < hi; i += kSortBlock)
        perm[atomicAdd(&hist[sort_cell(x[i], x[(size_t)n + i], f)], 1u)] = (uint32_t)i;
}

// ---- small batches: 16 samples per wave on the 16x16x32 MFMAs (f16 or bf16) ----
//
// A batch of fewer than 2^17 samples gives the 32-sample waves above fewer than four
// waves per SIMD, and a lone wave's T-step chain is then its latency.  Here four lanes
// share a sample (lane l: sample l%16, group g = l/16): each lane forms the B entries
// ex_a, ex_a dx_a of a = 32kb + 8g + j (j < 8) and, in the accumulator layout, owns the
// rows b = 16t + 4g + v (v < 4) of every 16-row tile t; the four lanes of a sample are
// summed by xor-16 and xor-32 exchanges (the same value in all four).  A lane forms
// half the B entries and owns half the rows of the 32-wide kernel's lanes, so a step's
// chain is about half as long, and the batch spreads over twice as many waves.  The
// split scheme is chosen as in the 32-sample kernel (only morphs come here).
constexpr int kG2sBlock = 256;  // 4 waves, 16 samples each

// The y contraction on the 16x16 accumulator layout and the sum over the four lanes
// of a sample.
template <int TB16>
__device__ __forceinline__ void g2s_ysum(const float *gys, float ys, int grp,
                                         const f32x4_t (&U)[TB16], const f32x4_t (&V)[TB16],
                                         float &s, float &sx, float &sy) {
    s = 0.0f;
    sx = 0.0f;
    sy = 0.0f;
#pragma unroll
    for (int t = 0; t < TB16; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int b = 16 * t + 4 * grp + v;
            const float d = ys - gys[b];
            const float e = exp2_fast(-d * d);
            s = fmaf(e, U[t][v], s);
            sx = fmaf(e, V[t][v], sx);
            sy = fmaf(e * d, U[t][v], sy);
        }
    s += __shfl_xor(s, 16, 64);
    sx += __shfl_xor(sx, 16, 64);
    sy += __shfl_xor(sy, 16, 64);
    s += __shfl_xor(s, 32, 64);
    sx += __shfl_xor(sx, 32, 64);
    sy += __shfl_xor(sy, 32, 64);
}

template <int TB16, int KB, int MODE>
__global__ void __launch_bounds__(kG2sBlock)
k_grid2d_small(const float *__restrict__ hinges, const float *__restrict__ weights, int g0,
               int g1, float kappa, float gscale, const float *x_in, int64_t n, int T, float eta,
               float *c_out, float *s_out, float *g_out, float *x_out, Traj tr) {
    static_assert(kG2sBlock == kG2Block, "the scheme test assumes the large kernel's block");
    // fragments: frag[(p * KB + kb) * TB16 + t][lane] = part p of
    //   W[b = 16t + lane%16][a = 32kb + 8(lane/16) + j], j < 8 (0 outside the grid);
    // three bf16 parts of W or two FP16 parts of 2^sw W (the large kernel's schemes)
    __shared__ uint4 fraw[3 * KB * TB16 * 64];
    __shared__ float gxs[32 * KB];
    __shared__ float gys[16 * TB16];
    __shared__ SplitRange rg;
    const int M = g0 * g1;
    // padding x-coordinates far away: their features are 0 on both schemes
    for (int a = threadIdx.x; a < 32 * KB; a += kG2sBlock)
        gxs[a] = a < g0 ? kappa * hinges[a] : 1e18f;
    for (int b = threadIdx.x; b < 16 * TB16; b += kG2sBlock)
        gys[b] = b < g1 ? kappa * hinges[(size_t)M + (size_t)g0 * b] : 0.0f;
    constexpr int kNI = (KB * TB16 * 64 + kG2sBlock - 1) / kG2sBlock;
    float wv8[kNI][8];
    uint32_t mx = 0, mn = 0xffffffffu;
#pragma unroll
    for (int it = 0; it < kNI; ++it) {
        const int idx = threadIdx.x + it * kG2sBlock;
        const int ln = idx & 63, t = (idx >> 6) % TB16, kb = idx / (64 * TB16);
        const int b = 16 * t + (ln & 15);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int a = 32 * kb + 8 * (ln >> 4) + j;
            const float w = (idx < KB * TB16 * 64 && a < g0 && b < g1)
                                ? weights[a + (int64_t)g0 * b] : 0.0f;
            wv8[it][j] = w;
            const uint32_t u = __float_as_uint(w) & 0x7fffffffu;
            mx = max(mx, u);
            if (u != 0) mn = min(mn, u);
        }
    }
    const SplitScheme sc = split_decide(mx, mn, hinges, g0, kappa, rg);
#pragma unroll
    for (int it = 0; it < kNI; ++it) {
        const int idx = threadIdx.x + it * kG2sBlock;
        if (idx >= KB * TB16 * 64) break;
        const int ln = idx & 63, t = (idx >> 6) % TB16, kb = idx / (64 * TB16);
        if (sc.fp16) {
            f16x8_t *frag = reinterpret_cast<f16x8_t *>(fraw);
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = ldexpf(wv8[it][j], sc.sw);
            f16x8_t p1, p2;
            split2h(v, p1, p2);
            frag[(0 * KB + kb) * TB16 * 64 + t * 64 + ln] = p1;
            frag[(1 * KB + kb) * TB16 * 64 + t * 64 + ln] = p2;
        } else {
            bf16x8_t *frag = reinterpret_cast<bf16x8_t *>(fraw);
            bf16x8_t p1, p2, p3;
            split3(wv8[it], p1, p2, p3);
            frag[(0 * KB + kb) * TB16 * 64 + t * 64 + ln] = p1;
            frag[(1 * KB + kb) * TB16 * 64 + t * 64 + ln] = p2;
            frag[(2 * KB + kb) * TB16 * 64 + t * 64 + ln] = p3;
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, grp = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * (kG2sBlock / 64) + (threadIdx.x >> 6);
    const int64_t i = wave * 16 + (lane & 15);
    const int64_t ic = i < n ? i : n - 1;
    float x = x_in[ic], y = x_in[(size_t)n + ic];
    const float beta = weights[M];

    float s = 0.0f, sx = 0.0f, sy = 0.0f;
    const int steps = MODE == kMorph ? T : 1;
    int64_t tc;
    const bool rec = MODE == kMorph && grp == 0 && traj_col(tr, i, n, tc);
    for (int st = 0; st < steps; ++st) {
        if (rec) traj_put<2>(tr, st, tc, {x, y});
        const float xs = kappa * x, ys = kappa * y;
        int ln = lane;  // opaque: keeps the fragment reads inside the step loop
        asm volatile("" : "+v"(ln));
        f32x4_t U[TB16], V[TB16];
        if (sc.fp16) {
            const f16x8_t *frag = reinterpret_cast<const f16x8_t *>(fraw);
            const int c = split_scale_exp(xs, sc.gmin, sc.gmax);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                float ev[8], dv[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float d = xs - gxs[32 * kb + 8 * grp + j];
                    ev[j] = exp2_fast(fmaf(-d, d, (float)c));
                    dv[j] = ev[j] * d;
                }
                f16x8_t e1, e2, d1, d2;
                split2h(ev, e1, e2);
                split2h(dv, d1, d2);
#pragma unroll
                for (int t = 0; t < TB16; ++t) {
                    const f16x8_t a1 = frag[(0 * KB + kb) * TB16 * 64 + t * 64 + ln];
                    const f16x8_t a2 = frag[(1 * KB + kb) * TB16 * 64 + t * 64 + ln];
                    const f32x4_t zero = {};
                    U[t] = mfma16_h3(a1, a2, e1, e2, kb == 0 ? zero : U[t]);
                    V[t] = mfma16_h3(a1, a2, d1, d2, kb == 0 ? zero : V[t]);
                }
            }
            g2s_ysum<TB16>(gys, ys, grp, U, V, s, sx, sy);
            const int un = -(sc.sw + c);
            s = ldexpf(s, un);
            sx = ldexpf(sx, un);
            sy = ldexpf(sy, un);
        } else {
            const bf16x8_t *frag = reinterpret_cast<const bf16x8_t *>(fraw);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                float ev[8], dv[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float d = xs - gxs[32 * kb + 8 * grp + j];
                    ev[j] = exp2_fast(-d * d);
                    dv[j] = ev[j] * d;
                }
                bf16x8_t e1, e2, e3, d1, d2, d3;
                split3(ev, e1, e2, e3);
                split3(dv, d1, d2, d3);
#pragma unroll
                for (int t = 0; t < TB16; ++t) {
                    const bf16x8_t a1 = frag[(0 * KB + kb) * TB16 * 64 + t * 64 + ln];
                    const bf16x8_t a2 = frag[(1 * KB + kb) * TB16 * 64 + t * 64 + ln];
                    const bf16x8_t a3 = frag[(2 * KB + kb) * TB16 * 64 + t * 64 + ln];
                    const f32x4_t zero = {};
                    U[t] = mfma16_x6(a1, a2, a3, e1, e2, e3, kb == 0 ? zero : U[t]);
                    V[t] = mfma16_x6(a1, a2, a3, d1, d2, d3, kb == 0 ? zero : V[t]);
                }
            }
            g2s_ysum<TB16>(gys, ys, grp, U, V, s, sx, sy);
        }
        if (MODE == kMorph) {
            float c, sp;
            sigmoid_and_slope(s + beta, c, sp);
            const float step = eta * sp * gscale;
            x = fmaf(step, sx, x);
            y = fmaf(step, sy, y);
        }
    }
    if (rec) traj_put<2>(tr, steps, tc, {x, y});
    if (grp != 0 || i >= n) return;
    if (MODE == kMorph) {
        x_out[i] = x;
        x_out[(size_t)n + i] = y;
    } else {
        const float sv = s + beta;
        float c, sp;
        sigmoid_and_slope(sv, c, sp);
        if (c_out) c_out[i] = c;
        if (MODE == kEval) {
            if (s_out) s_out[i] = sv;
        } else {
            g_out[i] = -sp * gscale * sx;
            g_out[(size_t)n + i] = -sp * gscale * sy;
        }
    }
}

// The split scheme the 2-D grid morphs take for these operands (every block of those
// kernels decides the same from the same data): one block runs their staging and
// writes 2 (two-part FP16 splits) or 1 (three-part BF16 splits).
template <int TB, int KS>
__global__ void __launch_bounds__(kG2Block)
k_grid2d_scheme(const float *__restrict__ hinges, const float *__restrict__ weights, int g0, int g1,
                float kappa, int32_t *out) {
    __shared__ uint4 fraw[3 * KS * TB * 64];
    __shared__ float gxs[16 * KS];
    __shared__ float gys[32 * TB];
    __shared__ SplitRange rg;
    const SplitScheme sc =
        g2_stage<TB, KS, true>(fraw, gxs, gys, rg, hinges, weights, g0, g1, kappa);
    if (threadIdx.x == 0) *out = sc.fp16 ? 2 : 1;
}

int32_t launch_grid2d_scheme(const float *hinges, const float *weights, int g0, int g1,
                             float kappa, int32_t *out, hipStream_t st) {
    if (g0 < 1 || g1 < 1 || g0 > 64 || g1 > 64) return PDMP_EUNSUPPORTED;
    // the morph kernels' own tile counts (the staging pads to them)
#define PDMP_G2Q(TB, KS)                                                                     \
    hipLaunchKernelGGL((k_grid2d_scheme<TB, KS>), dim3(1), dim3(kG2Block), 0, st, hinges,    \
                       weights, g0, g1, kappa, out)
    const int ks = (g0 + 15) / 16;
    if (g1 <= 32) {
        if (ks == 1) PDMP_G2Q(1, 1); else if (ks == 2) PDMP_G2Q(1, 2);
        else if (ks == 3) PDMP_G2Q(1, 3); else PDMP_G2Q(1, 4);
    } else {
        if (ks == 1) PDMP_G2Q(2, 1); else if (ks == 2) PDMP_G2Q(2, 2);
        else if (ks == 3) PDMP_G2Q(2, 3); else PDMP_G2Q(2, 4);
    }
#undef PDMP_G2Q
    return check_launch("k_grid2d_scheme");
}

// Morphs of fewer samples than this take the 16-sample waves.
constexpr int64_t kG2SmallBatch = (int64_t)1 << 17;

static int32_t launch_grid2d_small(const RbfArgs &a, int g0, int g1, hipStream_t st) {
    const int64_t blocks = (a.n + 63) / 64;
    if (int32_t e = grid_guard(blocks, kG2sBlock, "k_grid2d_small")) return e;
    const dim3 grid((unsigned)blocks), blk(kG2sBlock);
#define PDMP_G2S(TB, KB)                                                                         \
    hipLaunchKernelGGL((k_grid2d_small<TB, KB, kMorph>), grid, blk, 0, st, a.hinges, a.weights, g0, \
                       g1, a.kappa, a.gscale, a.x_in, a.n, a.T, a.eta, a.c_out, a.s_out,          \
                       a.g_out, a.x_out, a.traj)
#define PDMP_G2S_T(KB)                             \
    switch ((g1 + 15) / 16) {                      \
        case 1: PDMP_G2S(1, KB); break;            \
        case 2: PDMP_G2S(2, KB); break;            \
        case 3: PDMP_G2S(3, KB); break;            \
        default: PDMP_G2S(4, KB); break;           \
    }
    if (g0 <= 32) {
        PDMP_G2S_T(1)
    } else {
        PDMP_G2S_T(2)
    }
#undef PDMP_G2S_T
#undef PDMP_G2S
    return check_launch("k_grid2d_small");
}

// Returns PDMP_EUNSUPPORTED (without launching) when the grid does not fit.
int32_t launch_grid2d(int mode, const RbfArgs &a, int g0, int g1, hipStream_t st) {
    if (g0 < 1 || g1 < 1 || g0 > 64 || g1 > 64 || (int64_t)g0 * g1 != a.M)
        return PDMP_EUNSUPPORTED;
    if (mode != kEval && mode != kGrad && mode != kMorph) return PDMP_EUNSUPPORTED;
    // a single evaluation would pay the per-block staging of W twice over: only the
    // multi-step morph takes the 16-sample waves
    if (a.n < kG2SmallBatch && mode == kMorph && a.T > 1) return launch_grid2d_small(a, g0, g1, st);
    const int64_t blocks = (a.n + 127) / 128;
    if (int32_t e = grid_guard(blocks, kG2Block, "k_grid2d_mfma")) return e;
    const dim3 grid((unsigned)blocks), blk(kG2Block);
#define PDMP_G2(TB, KS, MODE)                                                                  \
    hipLaunchKernelGGL((k_grid2d_mfma<TB, KS, MODE>), grid, blk, 0, st, a.hinges, a.weights, g0, \
                       g1, a.kappa, a.gscale, a.x_in, a.n, a.T, a.eta, a.c_out, a.s_out,        \
                       a.g_out, a.x_out, a.traj)
#define PDMP_G2_KS(TB, MODE)                      \
    switch ((g0 + 15) / 16) {                     \
        case 1: PDMP_G2(TB, 1, MODE); break;      \
        case 2: PDMP_G2(TB, 2, MODE); break;      \
        case 3: PDMP_G2(TB, 3, MODE); break;      \
        default: PDMP_G2(TB, 4, MODE); break;     \
    }
    if (g1 <= 32) {
        if (mode == kEval) PDMP_G2_KS(1, kEval)
        else if (mode == kGrad) PDMP_G2_KS(1, kGrad)
        else PDMP_G2_KS(1, kMorph)
    } else {
        if (mode == kEval) PDMP_G2_KS(2, kEval)
        else if (mode == kGrad) PDMP_G2_KS(2, kGrad)
        else PDMP_G2_KS(2, kMorph)
    }
#undef PDMP_G2_KS
#undef PDMP_G2
    return check_launch("k_grid2d");
}

// Workspace bytes of the ordered morph (0: the batch takes another path).
size_t grid2d_sorted_ws_bytes(int g0, int g1, int64_t n, int T) {
    if (g0 < 1 || g1 < 1 || g0 > 64 || g1 > 64 || n < kG2SmallBatch || T < 1 || n > 0xffffffffll)
        return 0;
    return (((size_t)kSortKeys * sizeof(uint32_t) + 255) & ~(size_t)255) +
           (size_t)n * sizeof(uint32_t);
}

// The spatial order of x [2][n] (a workspace of grid2d_sorted_ws_bytes): *perm, the
// permutation (each part's places in cell order), and *part, the samples per part.
int32_t launch_sort2d(const float *hinges, int g0, int g1, const float *x, int64_t n, void *ws,
                      hipStream_t st, const uint32_t **perm_out, int64_t *part_out) {
    uint32_t *cursor = (uint32_t *)ws;
    uint32_t *perm =
        (uint32_t *)((char *)ws + (((size_t)kSortKeys * sizeof(uint32_t) + 255) & ~(size_t)255));
    const int64_t part = sort_part(n);
    const unsigned nb = (unsigned)(kSortParts * sort_chunks_per_part(n));
    hipLaunchKernelGGL(k_sort_zero, dim3(1), dim3(kSortBlock), 0, st, cursor);
    hipLaunchKernelGGL(k_sort_count, dim3(nb), dim3(kSortBlock), 0, st, hinges, g0, g1, x, n, part,
                       cursor);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, st, cursor);
    hipLaunchKernelGGL(k_sort_scatter, dim3(nb), dim3(kSortBlock), 0, st, hinges, g0, g1, x, n,
                       part, cursor, perm);
    *perm_out = perm;
    *part_out = part;
    return check_launch("k_sort");
}

// The morph of a large batch in spatial order (PDMP_EUNSUPPORTED: not this path).
int32_t launch_grid2d_sorted(const RbfArgs &a, int g0, int g1, void *ws, hipStream_t st) {
    if (!grid2d_sorted_ws_bytes(g0, g1, a.n, a.T) || (int64_t)g0 * g1 != a.M)
        return PDMP_EUNSUPPORTED;
    if (int32_t e = grid_guard(kSortParts * ((sort_part(a.n) + 127) / 128), kG2Block,
                               "k_grid2d_sorted"))
        return e;
    const uint32_t *perm;
    int64_t part;
    if (int32_t e = launch_sort2d(a.hinges, g0, g1, a.x_in, a.n, ws, st, &perm, &part)) return e;
    // kSortParts interleaved runs of blocks, each covering one part
    const dim3 grid((unsigned)(kSortParts * ((part + 127) / 128))), blk(kG2Block);
#define PDMP_G2O(TB, KS)                                                                         \
    hipLaunchKernelGGL((k_grid2d_sorted<TB, KS>), grid, blk, 0, st, a.hinges, a.weights, g0, g1, \
                       a.kappa, a.gscale, a.x_in, a.n, a.T, a.eta, perm, part, a.x_out, a.traj)
    const int ks = (g0 + 15) / 16;
    if (g1 <= 32) {
        if (ks == 1) PDMP_G2O(1, 1); else if (ks == 2) PDMP_G2O(1, 2);
        else if (ks == 3) PDMP_G2O(1, 3); else PDMP_G2O(1, 4);
    } else {
        if (ks == 1) PDMP_G2O(2, 1); else if (ks == 2) PDMP_G2O(2, 2);
        else if (ks == 3) PDMP_G2O(2, 3); else PDMP_G2O(2, 4);
    }
#undef PDMP_G2O
    return check_launch("k_grid2d_sorted");
}

}  // namespace pdmp
