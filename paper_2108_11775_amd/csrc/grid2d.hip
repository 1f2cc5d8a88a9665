// grid2d.hip -- the occupancy and the fused T-step morph for hinges on a regular 2-D
// grid, as a dense FP32 MFMA contraction.
//
// With hinges h_{a + G0 b} = (gx_a, gy_b) the RBF feature factorises,
//   phi_ab(x) = ex_a(x) ey_b(y),  ex_a = exp(-(x - gx_a)^2 / (2 l^2)),
// so with W[b][a] = w_{a + G0 b}
//   s      = sum_b ey_b U_b + beta,         U_b = sum_a W[b][a] ex_a
//   ds/dx  = -(1/l^2) sum_b ey_b V_b,       V_b = sum_a W[b][a] ex_a (x - gx_a)
//   ds/dy  = -(1/l^2) sum_b ey_b (y - gy_b) U_b
// which is the same s and grad s as the pairwise sum (rounding aside).  Per sample
// and step that is G0 + G1 exponentials and two G1 x G0 matrix-vector products,
// instead of G0 G1 exponentials.  The products for 32 samples at a time are
// v_mfma_f32_32x32x2_f32: A = W (rows b, k = a), B = [ex | ex * dx] (k = a, column =
// sample).  Lane l computes the exponentials of its own B entries (a = 2kk + l/32,
// sample l%32), so no exponential is evaluated twice; W is staged once per block in
// LDS in MFMA fragment order (one conflict-free ds_read per fragment).  The y
// contraction runs on the accumulator layout: lane l owns rows b = 8(v/4) + 4(l/32)
// + v%4 of sample l%32, evaluates ey_b for them and the two lanes of a sample are
// summed by one xor-32 exchange (bit-identical in both lanes).  The T-step loop
// runs in registers.
#include "pdmp_common.h"

namespace pdmp {

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

constexpr int kG2Block = 256;   // 4 waves, 32 samples each
constexpr int kG2MaxKS = 32;    // G0 <= 64
constexpr int kG2MaxTB = 2;     // G1 <= 64

template <int TB, int MODE>
__global__ void __launch_bounds__(kG2Block) __attribute__((amdgpu_waves_per_eu(3)))
k_grid2d(const float *__restrict__ hinges, const float *__restrict__ weights, int g0, int g1,
         float kappa, float gscale, const float *x_in, int64_t n, int T, float eta, float *c_out,
         float *s_out, float *g_out, float *x_out) {
    // fragments: frag[kk][t][lane] = W[b = 32t + lane%32][a = 2kk + lane/32] (0 outside)
    // one k-step of padding so that the next step's operands can always be read ahead
    __shared__ float frag[(kG2MaxKS + 1) * TB * 64];
    __shared__ float gxs[2 * (kG2MaxKS + 1)];
    __shared__ float gys[32 * TB];
    const int M = g0 * g1;
    const int ks = (g0 + 1) / 2;
    for (int idx = threadIdx.x; idx < (ks + 1) * TB * 64; idx += kG2Block) {
        const int ln = idx & 63, t = (idx >> 6) % TB, kk = idx / (64 * TB);
        const int b = 32 * t + (ln & 31), a = 2 * kk + (ln >> 5);
        frag[idx] = (a < g0 && b < g1) ? weights[a + (int64_t)g0 * b] : 0.0f;
    }
    for (int a = threadIdx.x; a < 2 * (ks + 1); a += kG2Block)
        gxs[a] = a < g0 ? kappa * hinges[a] : 0.0f;
    for (int b = threadIdx.x; b < 32 * TB; b += kG2Block)
        gys[b] = b < g1 ? kappa * hinges[(size_t)M + (size_t)g0 * b] : 0.0f;
    __syncthreads();

    const int lane = threadIdx.x & 63, half = lane >> 5;
    const int64_t wave = (int64_t)blockIdx.x * (kG2Block / 64) + (threadIdx.x >> 6);
    const int64_t i = wave * 32 + (lane & 31);
    const int64_t ic = i < n ? i : n - 1;
    float x = x_in[ic], y = x_in[(size_t)n + ic];
    const float beta = weights[M];

    float s = 0.0f, sx = 0.0f, sy = 0.0f;
    const int steps = MODE == kMorph ? T : 1;
    for (int st = 0; st < steps; ++st) {
        const float xs = kappa * x, ys = kappa * y;
        f32x16_t U[TB], V[TB];
        // k-step 0 starts the accumulators from the zero constant (no register clears);
        // the LDS operands of step kk + 1 are read while step kk's products run
        float gx_n = gxs[half], w_n[TB];
#pragma unroll
        for (int t = 0; t < TB; ++t) w_n[t] = frag[t * 64 + lane];
        {
            const float d = xs - gx_n;
            const float e = exp2_fast(-d * d);
            const float de = e * d;
            float w_c[TB];
#pragma unroll
            for (int t = 0; t < TB; ++t) w_c[t] = w_n[t];
            gx_n = gxs[2 + half];
#pragma unroll
            for (int t = 0; t < TB; ++t) w_n[t] = frag[(TB + t) * 64 + lane];
            const f32x16_t zero = {};
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                U[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(w_c[t], e, zero, 0, 0, 0);
                V[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(w_c[t], de, zero, 0, 0, 0);
            }
        }
        for (int kk = 1; kk < ks; ++kk) {
            const float d = xs - gx_n;
            float w_c[TB];
#pragma unroll
            for (int t = 0; t < TB; ++t) w_c[t] = w_n[t];
            gx_n = gxs[2 * (kk + 1) + half];
#pragma unroll
            for (int t = 0; t < TB; ++t) w_n[t] = frag[((kk + 1) * TB + t) * 64 + lane];
            const float e = exp2_fast(-d * d);
            const float de = e * d;
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                U[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(w_c[t], e, U[t], 0, 0, 0);
                V[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(w_c[t], de, V[t], 0, 0, 0);
            }
        }
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
        if (MODE == kMorph) {
            float c, sp;
            sigmoid_and_slope(s + beta, c, sp);
            const float step = eta * sp * gscale;  // x - eta sigma' grad s, grad s = -gscale (sx, sy)
            x = fmaf(step, sx, x);
            y = fmaf(step, sy, y);
        }
    }
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

// Returns PDMP_EUNSUPPORTED (without launching) when the grid does not fit.
int32_t launch_grid2d(int mode, const RbfArgs &a, int g0, int g1, hipStream_t st) {
    if (g0 < 1 || g1 < 1 || g0 > 2 * kG2MaxKS || g1 > 32 * kG2MaxTB || (int64_t)g0 * g1 != a.M)
        return PDMP_EUNSUPPORTED;
    if (mode != kEval && mode != kGrad && mode != kMorph) return PDMP_EUNSUPPORTED;
    const int64_t blocks = (a.n + 127) / 128;
    const dim3 grid((unsigned)blocks), blk(kG2Block);
#define PDMP_G2(TB, MODE)                                                                      \
    hipLaunchKernelGGL((k_grid2d<TB, MODE>), grid, blk, 0, st, a.hinges, a.weights, g0, g1, \
                       a.kappa, a.gscale, a.x_in, a.n, a.T, a.eta, a.c_out, a.s_out, a.g_out,  \
                       a.x_out)
    if (g1 <= 32) {
        if (mode == kEval) PDMP_G2(1, kEval);
        else if (mode == kGrad) PDMP_G2(1, kGrad);
        else PDMP_G2(1, kMorph);
    } else {
        if (mode == kEval) PDMP_G2(2, kEval);
        else if (mode == kGrad) PDMP_G2(2, kGrad);
        else PDMP_G2(2, kMorph);
    }
#undef PDMP_G2
    return check_launch("k_grid2d");
}

}  // namespace pdmp
