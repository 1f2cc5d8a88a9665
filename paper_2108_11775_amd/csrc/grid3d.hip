// grid3d.hip -- occupancy, joint-space morph and body-point check for hinges on a
// regular 3-D grid with 16 points on the y axis, as dense contractions on the matrix
// cores (BF16 MFMA at FP32 accuracy, mfma_split.h).
//
// With hinges h_{a + G0 (b + 16 c)} = (X_a, Y_b, Z_c) the feature factorises,
// phi = ex_a ey_b ez_c, so with rows r = b + 16 c of W[r][a] = w_{a + G0 r}
//   U_r = sum_a W[r][a] ex_a,   V_r = sum_a W[r][a] ex_a (x - X_a)        (MFMA)
//   s        = sum_c ez_c sum_b ey_b U_r + beta
//   ds/dx    = -(1/l^2) sum_c ez_c sum_b ey_b V_r
//   ds/dy    = -(1/l^2) sum_c ez_c sum_b ey_b (y - Y_b) U_r
//   ds/dz    = -(1/l^2) sum_c ez_c (z - Z_c) sum_b ey_b U_r
// the same s and grad s as the pairwise sum (rounding aside) for G0 + 16 + G2
// exponentials and two (16 G2) x G0 matrix-vector products per point.  32 points
// per wave go through v_mfma_f32_32x32x16_bf16 (A = W rows, B = [ex | ex dx] of the
// lane's own point, k = a, G0 = 16 in one k-step; three-way bf16 splits of both, six
// products per contraction); each 32-row tile holds two z-planes (c = 2t, 2t+1), so
// in the accumulator layout lane l owns the fixed y indices b = (8(v/4) + 4(l/32)
// + v%4) mod 16 and the y/z contractions need only per-lane tables of ey and ez.
// The two lanes of a point are summed by one xor-32 exchange (bit-identical).
//
// Arm mapping: a wave carries 4 configurations x 8 body points of one link at a
// time (lane = 8*config + point, mirrored in the upper 32 lanes), walks the links
// from the tip down, and keeps only the running suffix sums of the Eq. 3 pull-back.
#include "mfma_split.h"
#include "pdmp_common.h"

namespace pdmp {

constexpr int kG3Y = 16;  // points on the y axis (two z-planes per 32-row MFMA tile)

template <int G0, int G2>
struct G3 {
    static_assert(G0 == 16, "G0 = 16: one 16-wide k-step");
    static_assert(G2 % 2 == 0 && G2 <= 32, "G2 even, <= 32");
    static constexpr int TB = kG3Y * G2 / 32;  // 32-row tiles
    static constexpr int FRAG = 3 * TB * 64;   // bf16x8 fragments: 3 parts x TB tiles
};

// Stage W fragments (frag[(p*TB + t)*64 + lane] = part p of W[32t + lane%32][8(lane/32)
// + j], j < 8) and the prescaled axes into LDS.
template <int G0, int G2>
__device__ __forceinline__ void g3_stage(bf16x8_t *frag, float *ax, float *ay, float *az,
                                         const float *__restrict__ hinges,
                                         const float *__restrict__ weights, float kappa) {
    using C = G3<G0, G2>;
    constexpr int M = G0 * kG3Y * G2;
    for (int idx = threadIdx.x; idx < C::TB * 64; idx += blockDim.x) {
        const int ln = idx & 63, t = idx >> 6;
        const int r = 32 * t + (ln & 31);
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = weights[8 * (ln >> 5) + j + G0 * r];
        bf16x8_t p1, p2, p3;
        split3(v, p1, p2, p3);
        frag[(0 * C::TB + t) * 64 + ln] = p1;
        frag[(1 * C::TB + t) * 64 + ln] = p2;
        frag[(2 * C::TB + t) * 64 + ln] = p3;
    }
    for (int i = threadIdx.x; i < G0; i += blockDim.x) ax[i] = kappa * hinges[i];
    for (int i = threadIdx.x; i < kG3Y; i += blockDim.x) ay[i] = kappa * hinges[M + G0 * i];
    for (int i = threadIdx.x; i < G2; i += blockDim.x) az[i] = kappa * hinges[2 * M + G0 * kG3Y * i];
}

// s (without beta) and, with GRAD, the unscaled logit-gradient sums (sx, sy, sz) at the
// prescaled point (xs, ys, zs) this lane shares with its xor-32 partner.
template <int G0, int G2, bool GRAD>
__device__ __forceinline__ void g3_point(const bf16x8_t *frag, const float *ax, const float *ay,
                                         const float *az, float xs, float ys, float zs, float &s,
                                         float &sx, float &sy, float &sz) {
    using C = G3<G0, G2>;
    const int lane0 = threadIdx.x & 63, h = lane0 >> 5;
    // The weight fragments are the same at every call; an opaque copy of the lane
    // index keeps the compiler from hoisting their LDS reads out of the callers'
    // loops into registers.
    int lane = lane0;
    asm volatile("" : "+v"(lane));
    bf16x8_t e1, e2, e3, d1, d2, d3;
    {
        float e[8], de[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float d = xs - ax[8 * h + j];
            e[j] = exp2_fast(-d * d);
            de[j] = e[j] * d;
        }
        split3(e, e1, e2, e3);
        if (GRAD) split3(de, d1, d2, d3);
    }
    float ey[8], dey[8];  // the lane's 8 distinct y indices
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int b = 8 * (u >> 2) + 4 * h + (u & 3);
        const float d = ys - ay[b];
        ey[u] = exp2_fast(-d * d);
        dey[u] = ey[u] * d;
    }
    s = sx = sy = sz = 0.0f;
#pragma unroll
    for (int t = 0; t < C::TB; ++t) {
        // the two z-planes of this tile
        float ez[2], dez[2];
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const float d = zs - az[2 * t + cc];
            ez[cc] = exp2_fast(-d * d);
            dez[cc] = ez[cc] * d;
        }
        // one k-step (G0 = 16) from the zero accumulator
        const f32x16_t zero = {};
        const bf16x8_t a1 = frag[(0 * C::TB + t) * 64 + lane];
        const bf16x8_t a2 = frag[(1 * C::TB + t) * 64 + lane];
        const bf16x8_t a3 = frag[(2 * C::TB + t) * 64 + lane];
        const f32x16_t U = mfma_x6(a1, a2, a3, e1, e2, e3, zero);
        f32x16_t V;
        if (GRAD) V = mfma_x6(a1, a2, a3, d1, d2, d3, zero);
        // row i = 8(v/4) + 4h + v%4 of tile t: b = i mod 16 (table slot v%8), c = 2t + v/8;
        // the y sums of each z-plane first, then one ez (dez) factor per plane
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            float py = 0.0f, pyx = 0.0f, pdy = 0.0f;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int v = 8 * c + u;
                py = fmaf(ey[u], U[v], py);
                if (GRAD) {
                    pyx = fmaf(ey[u], V[v], pyx);
                    pdy = fmaf(dey[u], U[v], pdy);
                }
            }
            s = fmaf(ez[c], py, s);
            if (GRAD) {
                sx = fmaf(ez[c], pyx, sx);
                sy = fmaf(ez[c], pdy, sy);
                sz = fmaf(dez[c], py, sz);
            }
        }
    }
    s += __shfl_xor(s, 32, 64);
    if (GRAD) {
        sx += __shfl_xor(sx, 32, 64);
        sy += __shfl_xor(sy, 32, 64);
        sz += __shfl_xor(sz, 32, 64);
    }
}

// ---- workspace points [3][n]: eval / grad / morph, 32 points per wave ----
template <int G0, int G2, int MODE>
__global__ void __launch_bounds__(256)
k_grid3d_ws(const float *__restrict__ hinges, const float *__restrict__ weights, float kappa,
            float gscale, const float *x_in, int64_t n, int T, float eta, float *c_out,
            float *s_out, float *g_out, float *x_out) {
    using C = G3<G0, G2>;
    __shared__ bf16x8_t frag[C::FRAG];
    __shared__ float ax[G0], ay[kG3Y], az[G2];
    g3_stage<G0, G2>(frag, ax, ay, az, hinges, weights, kappa);
    __syncthreads();
    constexpr int M = G0 * kG3Y * G2;
    const int lane = threadIdx.x & 63;
    const int64_t i = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32 + (lane & 31);
    const int64_t ic = i < n ? i : n - 1;
    float x = x_in[ic], y = x_in[(size_t)n + ic], z = x_in[2 * (size_t)n + ic];
    const float beta = weights[M];
    float s, sx, sy, sz;
    const int steps = MODE == kMorph ? T : 1;
    for (int st = 0; st < steps; ++st) {
        g3_point<G0, G2, MODE != kEval>(frag, ax, ay, az, kappa * x, kappa * y, kappa * z, s, sx,
                                        sy, sz);
        if (MODE == kMorph) {
            float c, sp;
            sigmoid_and_slope(s + beta, c, sp);
            const float step = eta * sp * gscale;
            x = fmaf(step, sx, x);
            y = fmaf(step, sy, y);
            z = fmaf(step, sz, z);
        }
    }
    if ((lane >> 5) != 0 || i >= n) return;
    if (MODE == kMorph) {
        x_out[i] = x;
        x_out[(size_t)n + i] = y;
        x_out[2 * (size_t)n + i] = z;
    } else {
        float c, sp;
        sigmoid_and_slope(s + beta, c, sp);
        if (c_out) c_out[i] = c;
        if (MODE == kEval) {
            if (s_out) s_out[i] = s + beta;
        } else {
            const float f = -sp * gscale;
            g_out[i] = f * sx;
            g_out[(size_t)n + i] = f * sy;
            g_out[2 * (size_t)n + i] = f * sz;
        }
    }
}

// FP32 DH chain (same convention as the pairwise arm kernel).
template <int NDOF>
__device__ __forceinline__ void g3_chain(const pdmp_arm &arm, const float (&q)[NDOF],
                                         float (&o)[NDOF + 1][3], float (&z)[NDOF][3]) {
    float R[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    o[0][0] = o[0][1] = o[0][2] = 0.0f;
#pragma unroll
    for (int i = 0; i < NDOF; ++i) {
        z[i][0] = R[0][2];
        z[i][1] = R[1][2];
        z[i][2] = R[2][2];
        float st, ct, sa, ca;
        sincosf(arm.theta0[i] + q[i], &st, &ct);
        sincosf(arm.alpha[i], &sa, &ca);
        const float a = arm.a[i], d = arm.d[i];
        const float lx = a * ct, ly = a * st;
#pragma unroll
        for (int r = 0; r < 3; ++r) o[i + 1][r] = o[i][r] + R[r][0] * lx + R[r][1] * ly + R[r][2] * d;
        float N[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            N[r][0] = R[r][0] * ct + R[r][1] * st;
            N[r][1] = -R[r][0] * st * ca + R[r][1] * ct * ca + R[r][2] * sa;
            N[r][2] = R[r][0] * st * sa - R[r][1] * ct * sa + R[r][2] * ca;
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) R[r][c] = N[r][c];
    }
}

__device__ __forceinline__ float sum8(float v) {
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    return v;
}

// ---- joint-space morph (MORPH) or largest body-point occupancy (check) ----
// 4 configurations per wave; lane%32 = 8*cfg + k, body point k of every link.
template <int NDOF, int G0, int G2, bool MORPH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_arm_grid3d(pdmp_arm arm, const float *__restrict__ hinges, const float *__restrict__ weights,
             float kappa, float gscale, const float *q_in, float *q_out, int64_t n, int T,
             float eta, const uint32_t *__restrict__ n_active, float thresh, float *maxc_out,
             uint8_t *flag_out) {
    using C = G3<G0, G2>;
    constexpr int KIN = 3 * (NDOF + 1) + 3 * NDOF + NDOF;  // o, z, grad_q per configuration
    __shared__ bf16x8_t frag[C::FRAG];
    __shared__ float ax[G0], ay[kG3Y], az[G2];
    __shared__ float kin[16 * KIN];
    const int64_t n_eff = n_active ? min((int64_t)*n_active, n) : n;
    if ((int64_t)blockIdx.x * 16 >= n_eff) return;  // whole block idle (uniform)
    g3_stage<G0, G2>(frag, ax, ay, az, hinges, weights, kappa);
    __syncthreads();
    constexpr int M = G0 * kG3Y * G2;
    const int lane = threadIdx.x & 63;
    const int k = lane & 7;
    const int slot = (threadIdx.x >> 6) * 4 + ((lane & 31) >> 3);  // configuration in block
    float *ko = kin + slot * KIN, *kz = ko + 3 * (NDOF + 1), *kg = kz + 3 * NDOF;
    const bool writer = (lane & 39) == 0;  // k == 0 in the lower half-wave
    const int64_t cfg = (int64_t)blockIdx.x * 16 + slot;
    const int64_t cs = cfg < n_eff ? cfg : n_eff - 1;
    const int P = arm.pts_per_link;
    const bool own = k < P;
    const float frac = own ? (float)(k + 1) / (float)P : 0.0f;
    float q[NDOF];
#pragma unroll
    for (int j = 0; j < NDOF; ++j) q[j] = q_in[(size_t)j * n + cs];
    const float beta = weights[M];

    const int steps = MORPH ? T : 1;
    float mc = -1.0f;
    for (int st = 0; st < steps; ++st) {
        {
            // the chain of this configuration, parked in LDS so that the link loop
            // below does not hold ~45 registers across the MFMA work
            float o[NDOF + 1][3], zx[NDOF][3];
            g3_chain<NDOF>(arm, q, o, zx);
            if (writer) {
#pragma unroll
                for (int i = 0; i <= NDOF; ++i)
#pragma unroll
                    for (int e = 0; e < 3; ++e) ko[3 * i + e] = o[i][e];
#pragma unroll
                for (int i = 0; i < NDOF; ++i)
#pragma unroll
                    for (int e = 0; e < 3; ++e) kz[3 * i + e] = zx[i][e];
            }
        }
        __syncthreads();
        float SG[3] = {0, 0, 0}, SM[3] = {0, 0, 0};
#pragma unroll 1
        for (int l = NDOF - 1; l >= 0; --l) {
            float p[3], ol[3];
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                ol[e] = ko[3 * l + e];
                p[e] = ol[e] + frac * (ko[3 * (l + 1) + e] - ol[e]);
            }
            float s, sx, sy, sz;
            g3_point<G0, G2, MORPH>(frag, ax, ay, az, kappa * p[0], kappa * p[1], kappa * p[2], s,
                                    sx, sy, sz);
            float c, sp;
            sigmoid_and_slope(s + beta, c, sp);
            if (MORPH) {
                const float f = own ? -sp * gscale : 0.0f;
                const float g0 = f * sx, g1 = f * sy, g2 = f * sz;
                SG[0] += sum8(g0);
                SG[1] += sum8(g1);
                SG[2] += sum8(g2);
                SM[0] += sum8(p[1] * g2 - p[2] * g1);
                SM[1] += sum8(p[2] * g0 - p[0] * g2);
                SM[2] += sum8(p[0] * g1 - p[1] * g0);
                // joint l moves links l..NDOF-1 about z_l through o_l
                const float v0 = SM[0] - (ol[1] * SG[2] - ol[2] * SG[1]);
                const float v1 = SM[1] - (ol[2] * SG[0] - ol[0] * SG[2]);
                const float v2 = SM[2] - (ol[0] * SG[1] - ol[1] * SG[0]);
                const float gq = kz[3 * l] * v0 + kz[3 * l + 1] * v1 + kz[3 * l + 2] * v2;
                if (writer) kg[l] = gq;
            } else if (own) {
                mc = fmaxf(mc, c);
            }
        }
        __syncthreads();
        if (MORPH) {
#pragma unroll
            for (int j = 0; j < NDOF; ++j) q[j] = q[j] - eta * kg[j];
        }
        __syncthreads();
    }
    if (!MORPH) {
        mc = fmaxf(mc, __shfl_xor(mc, 1, 64));
        mc = fmaxf(mc, __shfl_xor(mc, 2, 64));
        mc = fmaxf(mc, __shfl_xor(mc, 4, 64));
    }
    if (lane >= 32 || k != 0 || cfg >= n_eff) return;
    if (MORPH) {
#pragma unroll
        for (int j = 0; j < NDOF; ++j) q_out[(size_t)j * n + cfg] = q[j];
    } else {
        if (maxc_out) maxc_out[cfg] = mc;
        if (flag_out) flag_out[cfg] = mc > thresh ? 1 : 0;
    }
}

static bool g3_supported(const int *grid, int M) {
    return grid && grid[0] == 16 && grid[1] == kG3Y && grid[2] == 16 && M == 4096;
}

int32_t launch_grid3d_ws(int mode, const RbfArgs &a, const int *grid, hipStream_t st) {
    if (!g3_supported(grid, a.M) || (mode != kEval && mode != kGrad && mode != kMorph))
        return PDMP_EUNSUPPORTED;
    const dim3 g((unsigned)((a.n + 127) / 128)), b(256);
#define PDMP_G3(MODE)                                                                         \
    hipLaunchKernelGGL((k_grid3d_ws<16, 16, MODE>), g, b, 0, st, a.hinges, a.weights, a.kappa, \
                       a.gscale, a.x_in, a.n, a.T, a.eta, a.c_out, a.s_out, a.g_out, a.x_out)
    if (mode == kEval) PDMP_G3(kEval);
    else if (mode == kGrad) PDMP_G3(kGrad);
    else PDMP_G3(kMorph);
#undef PDMP_G3
    return check_launch("k_grid3d_ws");
}

int32_t launch_arm_grid3d(const pdmp_arm &arm, const float *h, const float *w, int M,
                          const int *grid, float kappa, float gscale, const float *qi, float *qo,
                          int64_t n, int T, float eta, const uint32_t *n_active, bool morph,
                          float thresh, float *maxc, uint8_t *flag, hipStream_t st) {
    if (!g3_supported(grid, M) || arm.pts_per_link > 8) return PDMP_EUNSUPPORTED;
    const dim3 g((unsigned)((n + 15) / 16)), b(256);
    switch (arm.n_dof) {
#define PDMP_CASE(N)                                                                            \
    case N:                                                                                     \
        if (morph)                                                                              \
            hipLaunchKernelGGL((k_arm_grid3d<N, 16, 16, true>), g, b, 0, st, arm, h, w, kappa,  \
                               gscale, qi, qo, n, T, eta, n_active, thresh, maxc, flag);        \
        else                                                                                    \
            hipLaunchKernelGGL((k_arm_grid3d<N, 16, 16, false>), g, b, 0, st, arm, h, w, kappa, \
                               gscale, qi, qo, n, T, eta, n_active, thresh, maxc, flag);        \
        return check_launch("k_arm_grid3d");
        PDMP_CASE(1) PDMP_CASE(2) PDMP_CASE(3) PDMP_CASE(4)
        PDMP_CASE(5) PDMP_CASE(6) PDMP_CASE(7) PDMP_CASE(8)
#undef PDMP_CASE
    }
    return PDMP_EUNSUPPORTED;
}

}  // namespace pdmp
