// morph_inverse.hip -- the inverse of the morph and the log-determinant of its
// Jacobian (Sec. 3.2).  The flow's inverse integrates the reversed field; for the
// explicit-Euler map the exact inverse of one step x_{k+1} = x_k - eta grad c(x_k) is
// the fixed point x_k = x_{k+1} + eta grad c(x_k), a contraction when
// eta Lip(grad c) < 1.  The density of the morphed samples follows from the change of
// variables, p_z(z) = p_y(y) / prod_k |det(I - eta Hc(x_k))|.
//
// Per step of the inverse: x^(0) = x_{k+1}, x^(j+1) = x_{k+1} + eta grad c(x^(j)) for
// j < iters, x_k = x^(iters); one more evaluation at x_k gives the fixed-point residual
// and the Hessian for the log-determinant.  The forward variant evaluates the Hessian
// at every x_k of the plain morph.
//
// Hessian of c = sigma(s):  Hc = sigma' Hs + sigma'' grad s grad s^T, with
//   Hs = sum_j w_j phi_j ((x - h_j)(x - h_j)^T / l^4 - I / l^2).
// Grid path (2-D hinges on a tensor grid): the G1 x G0 products U = W ex, V = W ex dx
// of the plain morph and a third one, Q = W ex dx^2, on the matrix cores at FP32
// accuracy (the split schemes of mfma_split.h: two-part FP16 splits and three
// products where the operands' range allows, three-way bf16 splits and six products
// otherwise); the y sums run on the accumulator layout as in the plain morph (same
// lane mapping, same xor-32 pair sum).  A large batch with a workspace runs in the
// spatial order of the ordered morph (grid2d.hip: counting sort, then every
// evaluation skips, wave by wave, the k-steps and 8-row groups that are exact zeros
// for all the wave's samples; grid2d_stage.h), with the same bits per sample.
// Pairwise path (any hinges, 2-D or 3-D): one point per thread, hinges staged in LDS
// tiles.
#include "grid2d_stage.h"
#include "mfma_split.h"
#include "pdmp_common.h"

// No FMA contraction beyond the written fmaf calls: the ordered and unordered grid
// kernels then round every sample's arithmetic alike.
#pragma clang fp contract(off)

namespace pdmp {

constexpr int kIvBlock = 256;
static_assert(kIvBlock == 64 * kSplitWaves, "the scheme test's block");

// log|det(I - eta Hc)| for a 2 x 2 or 3 x 3 Hc (row-major).
template <int DIM>
__device__ __forceinline__ float step_logdet(const float (&H)[DIM][DIM], float eta) {
    float A[DIM][DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) A[a][b] = (a == b ? 1.0f : 0.0f) - eta * H[a][b];
    float det;
    if (DIM == 2) {
        det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
    } else {
        det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
              A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
              A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    }
    return logf(fabsf(det));
}

// ------------------------------------------------------------ grid path ---

// The x-side B operands of k-step ks for this lane (a = 16ks + 8half + j): ex, ex dx
// and, with HESS, ex dx^2, each split into three bf16 parts.
template <bool HESS>
__device__ __forceinline__ void g2i_operands(const float *gxs, float xs, int ks, int half,
                                             bf16x8_t (&e)[3], bf16x8_t (&de)[3],
                                             bf16x8_t (&dde)[3]) {
    float ev[8], dv[8], ddv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float d = xs - gxs[16 * ks + 8 * half + j];
        ev[j] = exp2_fast(-d * d);
        dv[j] = ev[j] * d;
        ddv[j] = dv[j] * d;
    }
    split3(ev, e[0], e[1], e[2]);
    split3(dv, de[0], de[1], de[2]);
    if (HESS) split3(ddv, dde[0], dde[1], dde[2]);
}

// The same operands on the FP16 scheme: 2^c ex, 2^c ex dx and 2^(c-k) ex dx^2
// (mfma_split.h), each as two FP16 parts.
template <bool HESS>
__device__ __forceinline__ void g2i_operands_h(const float *gxs, float xs, float cf, float sk,
                                               int ks, int half, f16x8_t (&e)[2],
                                               f16x8_t (&de)[2], f16x8_t (&dde)[2]) {
    float ev[8], dv[8], ddv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float d = xs - gxs[16 * ks + 8 * half + j];
        ev[j] = exp2_fast(fmaf(-d, d, cf));
        dv[j] = ev[j] * d;
        ddv[j] = dv[j] * (d * sk);
    }
    split2h(ev, e[0], e[1]);
    split2h(dv, de[0], de[1]);
    if (HESS) split2h(ddv, dde[0], dde[1]);
}

// Sums at the prescaled point (xs, ys): s' (without beta), (sx, sy) with
// grad s = -gscale (sx, sy), and with HESS (sxx, sxy, syy) with
// Hs = gscale^2 [[sxx, sxy], [sxy, syy]] - (1/l^2) s' I, on the block's split scheme.
template <int TB, int KS, bool HESS, bool F16>
__device__ __forceinline__ void g2i_eval(const uint4 *fraw, const SplitScheme &sc,
                                         const float *gxs, const float *gys, float xs, float ys,
                                         float &s, float &sx, float &sy, float &sxx, float &sxy,
                                         float &syy) {
    const int lane0 = threadIdx.x & 63, half = lane0 >> 5;
    int lane = lane0;  // opaque: the fragment reads stay inside the callers' loops
    asm volatile("" : "+v"(lane));
    f32x16_t U[TB], V[TB], Q[TB];
    // the operands of k-step ks + 1 are formed while k-step ks's products run; k-step 0
    // starts the accumulators from the zero constant
    int c = 0, k = 0;
    if (F16) {
        const f16x8_t *frag = reinterpret_cast<const f16x8_t *>(fraw);
        c = split_scale_exp(xs, sc.gmin, sc.gmax, k);
        const float cf = (float)c, sk = ldexpf(1.0f, -k);
        f16x8_t e[2], de[2], dde[2];
        g2i_operands_h<HESS>(gxs, xs, cf, sk, 0, half, e, de, dde);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            f16x8_t ec[2] = {e[0], e[1]}, dc[2] = {de[0], de[1]}, qc[2] = {dde[0], dde[1]};
            if (ks + 1 < KS) g2i_operands_h<HESS>(gxs, xs, cf, sk, ks + 1, half, e, de, dde);
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const f16x8_t a1 = frag[(0 * KS + ks) * TB * 64 + t * 64 + lane];
                const f16x8_t a2 = frag[(1 * KS + ks) * TB * 64 + t * 64 + lane];
                const f32x16_t zero = {};
                U[t] = mfma_h3(a1, a2, ec[0], ec[1], ks == 0 ? zero : U[t]);
                V[t] = mfma_h3(a1, a2, dc[0], dc[1], ks == 0 ? zero : V[t]);
                if (HESS) Q[t] = mfma_h3(a1, a2, qc[0], qc[1], ks == 0 ? zero : Q[t]);
            }
        }
    } else {
        const bf16x8_t *frag = reinterpret_cast<const bf16x8_t *>(fraw);
        bf16x8_t e[3], de[3], dde[3];
        g2i_operands<HESS>(gxs, xs, 0, half, e, de, dde);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            bf16x8_t ec[3] = {e[0], e[1], e[2]}, dc[3] = {de[0], de[1], de[2]},
                     qc[3] = {dde[0], dde[1], dde[2]};
            if (ks + 1 < KS) g2i_operands<HESS>(gxs, xs, ks + 1, half, e, de, dde);
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const bf16x8_t a1 = frag[(0 * KS + ks) * TB * 64 + t * 64 + lane];
                const bf16x8_t a2 = frag[(1 * KS + ks) * TB * 64 + t * 64 + lane];
                const bf16x8_t a3 = frag[(2 * KS + ks) * TB * 64 + t * 64 + lane];
                const f32x16_t zero = {};
                U[t] = mfma_x6(a1, a2, a3, ec[0], ec[1], ec[2], ks == 0 ? zero : U[t]);
                V[t] = mfma_x6(a1, a2, a3, dc[0], dc[1], dc[2], ks == 0 ? zero : V[t]);
                if (HESS) Q[t] = mfma_x6(a1, a2, a3, qc[0], qc[1], qc[2], ks == 0 ? zero : Q[t]);
            }
        }
    }
    s = sx = sy = sxx = sxy = syy = 0.0f;
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int b = 32 * t + 8 * (v >> 2) + 4 * half + (v & 3);
            const float d = ys - gys[b];
            const float e = exp2_fast(-d * d);
            const float ed = e * d;
            s = fmaf(e, U[t][v], s);
            sx = fmaf(e, V[t][v], sx);
            sy = fmaf(ed, U[t][v], sy);
            if (HESS) {
                sxx = fmaf(e, Q[t][v], sxx);
                sxy = fmaf(ed, V[t][v], sxy);
                syy = fmaf(ed * d, U[t][v], syy);
            }
        }
    s += __shfl_xor(s, 32, 64);
    sx += __shfl_xor(sx, 32, 64);
    sy += __shfl_xor(sy, 32, 64);
    if (HESS) {
        sxx += __shfl_xor(sxx, 32, 64);
        sxy += __shfl_xor(sxy, 32, 64);
        syy += __shfl_xor(syy, 32, 64);
    }
    if (F16) {
        const int un = -(sc.sw + c);
        s = ldexpf(s, un);
        sx = ldexpf(sx, un);
        sy = ldexpf(sy, un);
        if (HESS) {
            sxx = ldexpf(sxx, un + k);
            sxy = ldexpf(sxy, un);
            syy = ldexpf(syy, un);
        }
    }
}

// g2i_eval on the FP16 scheme with the wave's exact-zero skipping (grid2d_stage.h):
// the kept k-steps in order, the j-th kept one's operands in buffer j % NB (with two
// buffers its successor's are formed while its products run; the first starts the
// accumulators from the zero constant), and the kept 8-row groups of the kept tiles.
// Each sum gets the bits of g2i_eval<.., true>'s: every sum is a separate accumulator
// over the same terms in the same order, the skipped ones being exact zeros.  gys
// 16-byte aligned.
template <int TB, int KS, bool HESS>
__device__ __forceinline__ void g2i_eval_skip(const uint4 *fraw, const SplitScheme &sc,
                                              const SkipFrame<TB, KS> &fr, const float *gxs,
                                              const float *gys, float xs, float ys, float &s,
                                              float &sx, float &sy, float &sxx, float &sxy,
                                              float &syy) {
    const int lane0 = threadIdx.x & 63, half = lane0 >> 5;
    int lane = lane0;  // opaque: the fragment reads stay inside the callers' loops
    asm volatile("" : "+v"(lane));
    const f16x8_t *frag = reinterpret_cast<const f16x8_t *>(fraw);
    int k = 0;
    const int c = split_scale_exp(xs, sc.gmin, sc.gmax, k);
    const float cf = (float)c, sk = ldexpf(1.0f, -k);
    uint32_t km, gm;
    skip_masks<TB, KS>(fr, xs, ys, (float)(c + (HESS ? 35 : 30)), km, gm);
    const uint32_t tm = skip_tiles<TB>(gm);
    f32x16_t U[TB], V[TB], Q[TB];
    // with the Hessian's third operand set one buffer (the operands of each kept
    // k-step formed just before its products): two would not fit beside U, V and Q
    constexpr int NB = HESS ? 1 : 2;
    f16x8_t e[NB][2], de[NB][2], dde[NB][2];
    uint32_t rem = km;
    int ksn = rem ? __builtin_ctz(rem) : 0;
    if (rem && NB == 2) g2i_operands_h<HESS>(gxs, xs, cf, sk, ksn, half, e[0], de[0], dde[0]);
#pragma unroll
    for (int j = 0; j < KS; ++j) {
        if (!rem) break;
        const int ks = ksn;
        const int cur = j % NB;
        rem &= rem - 1u;
        if (NB == 1) {
            g2i_operands_h<HESS>(gxs, xs, cf, sk, ks, half, e[0], de[0], dde[0]);
            if (rem) ksn = __builtin_ctz(rem);
        } else if (rem) {
            ksn = __builtin_ctz(rem);
            g2i_operands_h<HESS>(gxs, xs, cf, sk, ksn, half, e[(j + 1) % NB], de[(j + 1) % NB],
                                 dde[(j + 1) % NB]);
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            if (!((tm >> t) & 1u)) continue;
            const f16x8_t a1 = frag[(0 * KS + ks) * TB * 64 + t * 64 + lane];
            const f16x8_t a2 = frag[(1 * KS + ks) * TB * 64 + t * 64 + lane];
            const f32x16_t zero = {};
            U[t] = mfma_h3(a1, a2, e[cur][0], e[cur][1], j == 0 ? zero : U[t]);
            V[t] = mfma_h3(a1, a2, de[cur][0], de[cur][1], j == 0 ? zero : V[t]);
            if (HESS) Q[t] = mfma_h3(a1, a2, dde[cur][0], dde[cur][1], j == 0 ? zero : Q[t]);
        }
    }
    s = sx = sy = sxx = sxy = syy = 0.0f;
    if (km) {
        // this lane's rows b = 32t + 8g + 4 half + r, read before the group branches
        f32x4_t gy[TB][4];
#pragma unroll
        for (int t = 0; t < TB; ++t) {
#pragma unroll
            for (int g = 0; g < 4; ++g)
                gy[t][g] = *reinterpret_cast<const f32x4_t *>(&gys[32 * t + 8 * g + 4 * half]);
            asm volatile("" ::"v"(gy[t][0]), "v"(gy[t][1]), "v"(gy[t][2]), "v"(gy[t][3]));
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            if (!((tm >> t) & 1u)) continue;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                if (!((gm >> (4 * t + g)) & 1u)) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int v = 4 * g + r;
                    const float d = ys - gy[t][g][r];
                    const float ey = exp2_fast(-d * d);
                    const float ed = ey * d;
                    s = fmaf(ey, U[t][v], s);
                    sx = fmaf(ey, V[t][v], sx);
                    sy = fmaf(ed, U[t][v], sy);
                    if (HESS) {
                        sxx = fmaf(ey, Q[t][v], sxx);
                        sxy = fmaf(ed, V[t][v], sxy);
                        syy = fmaf(ed * d, U[t][v], syy);
                    }
                }
            }
        }
    }
    s += __shfl_xor(s, 32, 64);
    sx += __shfl_xor(sx, 32, 64);
    sy += __shfl_xor(sy, 32, 64);
    if (HESS) {
        sxx += __shfl_xor(sxx, 32, 64);
        sxy += __shfl_xor(sxy, 32, 64);
        syy += __shfl_xor(syy, 32, 64);
    }
    const int un = -(sc.sw + c);
    s = ldexpf(s, un);
    sx = ldexpf(sx, un);
    sy = ldexpf(sy, un);
    if (HESS) {
        sxx = ldexpf(sxx, un + k);
        sxy = ldexpf(sxy, un);
        syy = ldexpf(syy, un);
    }
}

// MODE kLogdet: forward morph with the log-determinant.  MODE kInverse: inverse by
// fixed point (iters per step) with residual and log-determinant.  The lane reads
// sample ic and writes sample i (i >= n: a tail lane, writes nothing); with ORD (the
// ordered kernel on the FP16 scheme) each evaluation skips the wave's exact zeros by
// the frame fr.
template <int TB, int KS, int MODE, bool F16, bool ORD>
__device__ __forceinline__ void g2i_body(const uint4 *fraw, const SplitScheme &sc,
                                         const float *gxs, const float *gys, float beta,
                                         float kappa, float gscale, const float *x_in, int64_t n,
                                         int T, float eta, int iters, float *x_out,
                                         float *logdet_out, float *resid_out, int64_t i,
                                         int64_t ic, const SkipFrame<TB, KS> &fr) {
    const int lane = threadIdx.x & 63, half = lane >> 5;
    float x = x_in[ic], y = x_in[(size_t)n + ic];
    const float il2 = gscale * kappa;  // 1 / l^2
    const float g2 = gscale * gscale;
    float ld = 0.0f, rmax = 0.0f;
    // one evaluation at (x, y): s' and the sums of the gradient (and with HESS the
    // Hessian), on the block's scheme, skipping the wave's exact zeros with ORD
    auto eval = [&](auto hess, float &s, float &sx, float &sy, float &sxx, float &sxy,
                    float &syy) {
        constexpr bool H = decltype(hess)::value;
        if constexpr (F16 && ORD)
            g2i_eval_skip<TB, KS, H>(fraw, sc, fr, gxs, gys, kappa * x, kappa * y, s, sx, sy, sxx,
                                     sxy, syy);
        else
            g2i_eval<TB, KS, H, F16>(fraw, sc, gxs, gys, kappa * x, kappa * y, s, sx, sy, sxx,
                                     sxy, syy);
    };
    for (int st = 0; st < T; ++st) {
        const float zx = x, zy = y;
        if (MODE == kInverse) {
            // the fixed-point iterations: gradient only
            for (int j = 0; j < iters; ++j) {
                float s, sx, sy, sxx = 0.0f, sxy = 0.0f, syy = 0.0f;
                eval(std::false_type{}, s, sx, sy, sxx, sxy, syy);
                float c, sp;
                sigmoid_and_slope(s + beta, c, sp);
                const float gx = -gscale * sx, gy = -gscale * sy;  // grad s
                const float cx = sp * gx, cy = sp * gy;            // grad c
                x = fmaf(eta, cx, zx);
                y = fmaf(eta, cy, zy);
            }
        }
        // the evaluation with the Hessian: the step's log-determinant, then the residual
        // (inverse) or the Euler step (forward)
        float s, sx, sy, sxx = 0.0f, sxy = 0.0f, syy = 0.0f;
        eval(std::true_type{}, s, sx, sy, sxx, sxy, syy);
        float c, sp;
        sigmoid_and_slope(s + beta, c, sp);
        const float gx = -gscale * sx, gy = -gscale * sy;  // grad s
        const float spp = sp * (1.0f - 2.0f * c);
        float H[2][2];
        H[0][0] = sp * fmaf(g2, sxx, -il2 * s) + spp * gx * gx;
        H[0][1] = sp * g2 * sxy + spp * gx * gy;
        H[1][0] = H[0][1];
        H[1][1] = sp * fmaf(g2, syy, -il2 * s) + spp * gy * gy;
        ld += step_logdet<2>(H, eta);
        const float cx = sp * gx, cy = sp * gy;  // grad c
        if (MODE == kInverse) {
            const float rx = fabsf(x - fmaf(eta, cx, zx)), ry = fabsf(y - fmaf(eta, cy, zy));
            rmax = fmaxf(rmax, fmaxf(rx, ry));
        } else {
            x = fmaf(-eta, cx, x);
            y = fmaf(-eta, cy, y);
        }
    }
    if (half != 0 || i >= n) return;
    x_out[i] = x;
    x_out[(size_t)n + i] = y;
    if (logdet_out) logdet_out[i] = ld;
    if (resid_out) resid_out[i] = rmax;
}

template <int TB, int KS, int MODE>
__global__ void __launch_bounds__(kIvBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_grid2d_inv(const float *__restrict__ hinges, const float *__restrict__ weights, int g0, int g1,
             float kappa, float gscale, const float *x_in, int64_t n, int T, float eta, int iters,
             float *x_out, float *logdet_out, float *resid_out) {
    // fragments and axes (grid2d_stage.h); every launch here runs T steps, so the
    // scheme test is always made
    __shared__ uint4 fraw[3 * KS * TB * 64];
    __shared__ float gxs[16 * KS];
    __shared__ float gys[32 * TB];
    __shared__ SplitRange rg;
    const int M = g0 * g1;
    const SplitScheme sc =
        g2_stage<TB, KS, true>(fraw, gxs, gys, rg, hinges, weights, g0, g1, kappa);
    const float beta = weights[M];
    const int64_t wave = (int64_t)blockIdx.x * (kIvBlock / 64) + (threadIdx.x >> 6);
    const int64_t i = wave * 32 + (threadIdx.x & 31);
    const int64_t ic = i < n ? i : n - 1;
    const SkipFrame<TB, KS> none = {};  // not read without ORD
    if (sc.fp16)
        g2i_body<TB, KS, MODE, true, false>(fraw, sc, gxs, gys, beta, kappa, gscale, x_in, n, T,
                                            eta, iters, x_out, logdet_out, resid_out, i, ic, none);
    else
        g2i_body<TB, KS, MODE, false, false>(fraw, sc, gxs, gys, beta, kappa, gscale, x_in, n, T,
                                             eta, iters, x_out, logdet_out, resid_out, i, ic, none);
}

// The same in spatial order (perm, part: launch_sort2d; block b takes its samples from
// part b mod kSortParts, so that each part stays on one XCD).
// (Two waves per SIMD: with three, the 168 registers hold the U, V and Q
// accumulators and the skip tests' wave-uniform frame only with spills, even with the
// Hessian's products in a separate pass; measured slower or no faster.)
template <int TB, int KS, int MODE>
__global__ void __launch_bounds__(kIvBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_grid2d_inv_sorted(const float *__restrict__ hinges, const float *__restrict__ weights, int g0,
                    int g1, float kappa, float gscale, const float *x_in, int64_t n, int T,
                    float eta, int iters, const uint32_t *__restrict__ perm, int64_t part,
                    float *x_out, float *logdet_out, float *resid_out) {
    __shared__ uint4 fraw[3 * KS * TB * 64];
    __shared__ float gxs[16 * KS];
    __shared__ __align__(16) float gys[32 * TB];
    __shared__ SplitRange rg;
    const int M = g0 * g1;
    const SplitScheme sc =
        g2_stage<TB, KS, true>(fraw, gxs, gys, rg, hinges, weights, g0, g1, kappa);
    const float beta = weights[M];
    const int64_t p = blockIdx.x % kSortParts;
    const int64_t k =
        ((int64_t)(blockIdx.x / kSortParts) * (kIvBlock / 64) + (threadIdx.x >> 6)) * 32 +
        (threadIdx.x & 31);
    const int64_t slot = p * part + k;
    const bool live = k < part && slot < n;
    const int64_t ic = perm[live ? slot : n - 1];
    const int64_t i = live ? ic : n;  // n: a tail lane
    SkipFrame<TB, KS> fr = {};
    if (sc.fp16) {
        skip_frame<TB, KS>(gxs, gys, g0, g1, fr);
        g2i_body<TB, KS, MODE, true, true>(fraw, sc, gxs, gys, beta, kappa, gscale, x_in, n, T,
                                           eta, iters, x_out, logdet_out, resid_out, i, ic, fr);
    } else {
        g2i_body<TB, KS, MODE, false, false>(fraw, sc, gxs, gys, beta, kappa, gscale, x_in, n, T,
                                             eta, iters, x_out, logdet_out, resid_out, i, ic, fr);
    }
}

// -------------------------------------------------------- pairwise path ---

constexpr int kIvTile = 1024;  // hinges per LDS tile

// One point per thread; s' (without beta), grad s and Hs at x.
template <int DIM>
__device__ __forceinline__ void rbfi_eval(const float *__restrict__ hinges,
                                          const float *__restrict__ weights, int M, float i2l2,
                                          float il2, float *sh_h, float *sh_w, const float (&x)[DIM],
                                          float &s, float (&g)[DIM], float (&Hs)[DIM][DIM]) {
    s = 0.0f;
    float hx[DIM][DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        g[a] = 0.0f;
#pragma unroll
        for (int b = 0; b < DIM; ++b) hx[a][b] = 0.0f;
    }
    for (int j0 = 0; j0 < M; j0 += kIvTile) {
        const int cnt = M - j0 < kIvTile ? M - j0 : kIvTile;
        __syncthreads();
        for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) sh_h[k * kIvTile + j] = hinges[(size_t)k * M + j0 + j];
            sh_w[j] = weights[j0 + j];
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            float d[DIM], r2 = 0.0f;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                d[k] = x[k] - sh_h[k * kIvTile + j];
                r2 = fmaf(d[k], d[k], r2);
            }
            const float wp = sh_w[j] * __expf(-r2 * i2l2);
            s += wp;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                g[a] = fmaf(wp, d[a], g[a]);
#pragma unroll
                for (int b = a; b < DIM; ++b) hx[a][b] = fmaf(wp * d[a], d[b], hx[a][b]);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        g[a] *= -il2;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const float v = a <= b ? hx[a][b] : hx[b][a];
            Hs[a][b] = v * il2 * il2 - (a == b ? il2 * s : 0.0f);
        }
    }
}

template <int DIM, int MODE>
__global__ void __launch_bounds__(kIvBlock)
k_rbf_inv(const float *__restrict__ hinges, const float *__restrict__ weights, int M, float ell,
          const float *x_in, int64_t n, int T, float eta, int iters, float *x_out,
          float *logdet_out, float *resid_out) {
    __shared__ float sh_h[DIM * kIvTile], sh_w[kIvTile];
    const int64_t i = (int64_t)blockIdx.x * kIvBlock + threadIdx.x;
    const int64_t ic = i < n ? i : n - 1;
    const float il2 = 1.0f / (ell * ell), i2l2 = 0.5f * il2;
    const float beta = weights[M];
    float x[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) x[k] = x_in[(size_t)k * n + ic];
    float ld = 0.0f, rmax = 0.0f;
    for (int st = 0; st < T; ++st) {
        float z[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) z[k] = x[k];
        const int evals = MODE == kInverse ? iters + 1 : 1;
        for (int j = 0; j < evals; ++j) {
            const bool last = j == evals - 1;
            float s, g[DIM], Hs[DIM][DIM];
            rbfi_eval<DIM>(hinges, weights, M, i2l2, il2, sh_h, sh_w, x, s, g, Hs);
            float c, sp;
            sigmoid_and_slope(s + beta, c, sp);
            if (last) {
                const float spp = sp * (1.0f - 2.0f * c);
                float H[DIM][DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a)
#pragma unroll
                    for (int b = 0; b < DIM; ++b) H[a][b] = sp * Hs[a][b] + spp * g[a] * g[b];
                ld += step_logdet<DIM>(H, eta);
            }
            if (MODE == kInverse) {
                if (!last) {
#pragma unroll
                    for (int k = 0; k < DIM; ++k) x[k] = fmaf(eta, sp * g[k], z[k]);
                } else {
#pragma unroll
                    for (int k = 0; k < DIM; ++k)
                        rmax = fmaxf(rmax, fabsf(x[k] - fmaf(eta, sp * g[k], z[k])));
                }
            } else {
#pragma unroll
                for (int k = 0; k < DIM; ++k) x[k] = fmaf(-eta, sp * g[k], x[k]);
            }
        }
    }
    if (i >= n) return;
#pragma unroll
    for (int k = 0; k < DIM; ++k) x_out[(size_t)k * n + i] = x[k];
    if (logdet_out) logdet_out[i] = ld;
    if (resid_out) resid_out[i] = rmax;
}

// mode kLogdet or kInverse; grid (nullable) selects the MFMA path for a 2-D grid.
int32_t launch_morph_inverse(int dim, int mode, const float *hinges, const float *weights, int M,
                             const int *grid, float ell, const float *x_in, int64_t n, int T,
                             float eta, int iters, float *x_out, float *logdet, float *resid,
                             hipStream_t st, void *ws) {
    float kappa, gscale;
    derive_scales(ell, kappa, gscale);
    if (dim == 2 && grid && grid[0] >= 1 && grid[1] >= 1 && grid[0] <= 64 && grid[1] <= 64 &&
        grid[0] * grid[1] == M) {
        const int g0 = grid[0], g1 = grid[1];
        const uint32_t *perm = nullptr;
        int64_t part = 0;
        const bool ord = ws && grid2d_sorted_ws_bytes(g0, g1, n, T) != 0;
        if (int32_t e = grid_guard(ord ? kSortParts * ((sort_part(n) + 127) / 128)
                                       : (n + 127) / 128,
                                   kIvBlock, "k_grid2d_inv"))
            return e;
        if (ord) {
            if (int32_t e = launch_sort2d(hinges, g0, g1, x_in, n, ws, st, &perm, &part)) return e;
        }
        // the ordered kernel: kSortParts interleaved runs of blocks, one per part
        const dim3 blocks((unsigned)(ord ? kSortParts * ((part + 127) / 128) : (n + 127) / 128)),
            blk(kIvBlock);
#define PDMP_G2I(TB, KS, MD)                                                                     \
    if (ord)                                                                                     \
        hipLaunchKernelGGL((k_grid2d_inv_sorted<TB, KS, MD>), blocks, blk, 0, st, hinges, weights, \
                           g0, g1, kappa, gscale, x_in, n, T, eta, iters, perm, part, x_out,     \
                           logdet, resid);                                                       \
    else                                                                                         \
        hipLaunchKernelGGL((k_grid2d_inv<TB, KS, MD>), blocks, blk, 0, st, hinges, weights, g0,  \
                           g1, kappa, gscale, x_in, n, T, eta, iters, x_out, logdet, resid)
#define PDMP_G2I_KS(TB, MD)                      \
    switch ((g0 + 15) / 16) {                    \
        case 1: PDMP_G2I(TB, 1, MD); break;      \
        case 2: PDMP_G2I(TB, 2, MD); break;      \
        case 3: PDMP_G2I(TB, 3, MD); break;      \
        default: PDMP_G2I(TB, 4, MD); break;     \
    }
        if (g1 <= 32) {
            if (mode == kInverse) PDMP_G2I_KS(1, kInverse)
            else PDMP_G2I_KS(1, kLogdet)
        } else {
            if (mode == kInverse) PDMP_G2I_KS(2, kInverse)
            else PDMP_G2I_KS(2, kLogdet)
        }
#undef PDMP_G2I_KS
#undef PDMP_G2I
        return check_launch("k_grid2d_inv");
    }
    if (int32_t e = grid_guard((n + kIvBlock - 1) / kIvBlock, kIvBlock, "k_rbf_inv")) return e;
    const dim3 blocks((unsigned)((n + kIvBlock - 1) / kIvBlock)), blk(kIvBlock);
#define PDMP_RI(D, MD)                                                                        \
    hipLaunchKernelGGL((k_rbf_inv<D, MD>), blocks, blk, 0, st, hinges, weights, M, ell, x_in, n, \
                       T, eta, iters, x_out, logdet, resid)
    if (dim == 2) {
        if (mode == kInverse) PDMP_RI(2, kInverse);
        else PDMP_RI(2, kLogdet);
    } else {
        if (mode == kInverse) PDMP_RI(3, kInverse);
        else PDMP_RI(3, kLogdet);
    }
#undef PDMP_RI
    return check_launch("k_rbf_inv");
}

}  // namespace pdmp
