// grid3d.hip -- occupancy, joint-space morph and body-point check for hinges on a
// regular 3-D grid with 16 points on the y axis, as dense contractions on the matrix
// cores (FP16 or BF16 MFMA at FP32 accuracy, mfma_split.h).
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
// per wave go through the 32x32x16 MFMAs (A = W rows, B = [ex | ex dx] of the lane's
// own point, k = a, G0 = 16 in one k-step; two-part FP16 splits of both and three
// products per contraction, or three-way bf16 splits and six products when the
// operands' range needs FP32's exponent range); each 32-row tile holds two z-planes
// (c = 2t, 2t+1), so in the accumulator layout lane l owns the fixed y indices
// b = (8(v/4) + 4(l/32) + v%4) mod 16 and the y/z contractions need only per-lane
// tables of ey and ez.  The U terms are summed over z first (per y slot, the plane sums
// with ez and with ez (z - Z_c), then one y contraction after the tiles: 2 instead of 3
// multiply-adds per accumulator value and none per plane), the V term over y first.
// The two lanes of a point are summed by one xor-32 exchange (bit-identical).
//
// Arm mapping: a wave carries 4 configurations x 8 body points of one link at a
// time (lane = 8*config + point, mirrored in the upper 32 lanes), walks the links
// from the tip down, and keeps only the running suffix sums of the Eq. 3 pull-back.
#include "mfma_split.h"
#include "pdmp_common.h"

namespace pdmp {

constexpr int kG3Y = 16;  // points on the y axis (two z-planes per 32-row MFMA tile)
constexpr int kG3Block = 256;

// The x contraction runs on one of two split schemes (mfma_split.h): two-part FP16
// splits with three products where the operands' range allows, three-part BF16
// splits with six products otherwise.  The workspace morph and both arm kernels
// (morph and body-point check, each block running 7 links per configuration) test
// the range; a single workspace evaluation, whose blocks mostly stage W, skips the
// test and keeps the BF16 scheme.
static_assert(kG3Block == 64 * kSplitWaves, "the scheme test's block");

template <int G0, int G2>
struct G3 {
    static_assert(G0 == 16, "G0 = 16: one 16-wide k-step");
    static_assert(G2 % 2 == 0 && G2 <= 32, "G2 even, <= 32");
    static constexpr int TB = kG3Y * G2 / 32;  // 32-row tiles
    static constexpr int FRAG = 3 * TB * 64;   // 16-byte fragments: up to 3 parts x TB tiles
};

// Stage W fragments (frag[(p*TB + t)*64 + lane] = part p of W[32t + lane%32][8(lane/32)
// + j], j < 8: three bf16 parts, or two FP16 parts of 2^sw W) and the prescaled axes
// into LDS, choosing the scheme when allow16 (else the BF16 parts, no check).  All
// kG3Block threads call it; the caller synchronises before reading the fragments.
template <int G0, int G2>
__device__ __forceinline__ SplitScheme g3_stage(uint4 *fraw, float *ax, float *ay, float *az,
                                             SplitRange &rg, const float *__restrict__ hinges,
                                             const float *__restrict__ weights, float kappa,
                                             bool allow16) {
    using C = G3<G0, G2>;
    constexpr int M = G0 * kG3Y * G2;
    if (!allow16) {
        // BF16 parts straight from global memory, no range check
        bf16x8_t *frag = reinterpret_cast<bf16x8_t *>(fraw);
        for (int idx = threadIdx.x; idx < C::TB * 64; idx += kG3Block) {
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
        for (int i = threadIdx.x; i < G0; i += kG3Block) ax[i] = kappa * hinges[i];
        for (int i = threadIdx.x; i < kG3Y; i += kG3Block) ay[i] = kappa * hinges[M + G0 * i];
        for (int i = threadIdx.x; i < G2; i += kG3Block)
            az[i] = kappa * hinges[2 * M + G0 * kG3Y * i];
        return SplitScheme{0, 0, 0.0f, 0.0f};
    }
    constexpr int NI = (C::TB * 64 + kG3Block - 1) / kG3Block;
    float w8[NI][8];
    uint32_t mx = 0, mn = 0xffffffffu;
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = threadIdx.x + it * kG3Block;
        const int ln = idx & 63, r = 32 * (idx >> 6) + (ln & 31);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float w = idx < C::TB * 64 ? weights[8 * (ln >> 5) + j + G0 * r] : 0.0f;
            w8[it][j] = w;
            const uint32_t u = __float_as_uint(w) & 0x7fffffffu;
            mx = max(mx, u);
            if (u != 0) mn = min(mn, u);
        }
    }
    for (int i = threadIdx.x; i < G0; i += kG3Block) ax[i] = kappa * hinges[i];
    for (int i = threadIdx.x; i < kG3Y; i += kG3Block) ay[i] = kappa * hinges[M + G0 * i];
    for (int i = threadIdx.x; i < G2; i += kG3Block) az[i] = kappa * hinges[2 * M + G0 * kG3Y * i];
    const SplitScheme sc = split_decide(mx, mn, hinges, G0, kappa, rg);
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = threadIdx.x + it * kG3Block;
        if (idx >= C::TB * 64) break;
        const int ln = idx & 63, t = idx >> 6;
        if (sc.fp16) {
            f16x8_t *frag = reinterpret_cast<f16x8_t *>(fraw);
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = ldexpf(w8[it][j], sc.sw);
            f16x8_t p1, p2;
            split2h(v, p1, p2);
            frag[(0 * C::TB + t) * 64 + ln] = p1;
            frag[(1 * C::TB + t) * 64 + ln] = p2;
        } else {
            bf16x8_t *frag = reinterpret_cast<bf16x8_t *>(fraw);
            bf16x8_t p1, p2, p3;
            split3(w8[it], p1, p2, p3);
            frag[(0 * C::TB + t) * 64 + ln] = p1;
            frag[(1 * C::TB + t) * 64 + ln] = p2;
            frag[(2 * C::TB + t) * 64 + ln] = p3;
        }
    }
    return sc;
}

// s (without beta) and, with GRAD, the unscaled logit-gradient sums (sx, sy, sz) at the
// prescaled point (xs, ys, zs) this lane shares with its xor-32 partner, on the
// block's split scheme (F16 = sc.fp16).
template <int G0, int G2, bool GRAD, bool F16>
__device__ __forceinline__ void g3_point(const uint4 *fraw, const SplitScheme &sc, const float *ax,
                                         const float *ay, const float *az, float xs, float ys,
                                         float zs, float &s, float &sx, float &sy, float &sz) {
    using C = G3<G0, G2>;
    const int lane0 = threadIdx.x & 63, h = lane0 >> 5;
    // The weight fragments are the same at every call; an opaque copy of the lane
    // index keeps the compiler from hoisting their LDS reads out of the callers'
    // loops into registers.
    int lane = lane0;
    asm volatile("" : "+v"(lane));
    bf16x8_t e1, e2, e3, d1, d2, d3;
    f16x8_t h1, h2, k1, k2;
    int c = 0;  // FP16 scheme: this point's operand scale 2^c
    {
        float cf = 0.0f;
        if (F16) {
            c = split_scale_exp(xs, sc.gmin, sc.gmax);
            cf = (float)c;
        }
        float e[8], de[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float d = xs - ax[8 * h + j];
            e[j] = exp2_fast(F16 ? fmaf(-d, d, cf) : -d * d);
            de[j] = e[j] * d;
        }
        if (F16) {
            split2h(e, h1, h2);
            if (GRAD) split2h(de, k1, k2);
        } else {
            split3(e, e1, e2, e3);
            if (GRAD) split3(de, d1, d2, d3);
        }
    }
    // ey of the lane's 8 distinct y indices; the U terms z first (per y slot u the
    // plane sums q_u = sum_c ez_c U_(u,c) and qz_u with dez_c, contracted with ey and
    // ey dy after the tiles), the V term y first per plane
    float ey[8], q[8], qz[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int b = 8 * (u >> 2) + 4 * h + (u & 3);
        const float d = ys - ay[b];
        ey[u] = exp2_fast(-d * d);
        q[u] = qz[u] = 0.0f;
    }
    sx = 0.0f;
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
        f32x16_t U, V;
        if (F16) {
            const f16x8_t *frag = reinterpret_cast<const f16x8_t *>(fraw);
            const f16x8_t a1 = frag[(0 * C::TB + t) * 64 + lane];
            const f16x8_t a2 = frag[(1 * C::TB + t) * 64 + lane];
            U = mfma_h3(a1, a2, h1, h2, zero);
            if (GRAD) V = mfma_h3(a1, a2, k1, k2, zero);
        } else {
            const bf16x8_t *frag = reinterpret_cast<const bf16x8_t *>(fraw);
            const bf16x8_t a1 = frag[(0 * C::TB + t) * 64 + lane];
            const bf16x8_t a2 = frag[(1 * C::TB + t) * 64 + lane];
            const bf16x8_t a3 = frag[(2 * C::TB + t) * 64 + lane];
            U = mfma_x6(a1, a2, a3, e1, e2, e3, zero);
            if (GRAD) V = mfma_x6(a1, a2, a3, d1, d2, d3, zero);
        }
        // row i = 8(v/4) + 4h + v%4 of tile t: b = i mod 16 (y slot v%8), c = 2t + v/8,
        // so U[u] and U[u + 8] share slot u on the tile's two planes
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            q[u] = fmaf(ez[1], U[u + 8], fmaf(ez[0], U[u], q[u]));
            if (GRAD) qz[u] = fmaf(dez[1], U[u + 8], fmaf(dez[0], U[u], qz[u]));
        }
        if (GRAD) {
#pragma unroll
            for (int cz = 0; cz < 2; ++cz) {
                float pyx = 0.0f;
#pragma unroll
                for (int u = 0; u < 8; ++u) pyx = fmaf(ey[u], V[8 * cz + u], pyx);
                sx = fmaf(ez[cz], pyx, sx);
            }
        }
    }
    s = sy = sz = 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        s = fmaf(ey[u], q[u], s);
        if (GRAD) {
            const int b = 8 * (u >> 2) + 4 * h + (u & 3);
            sy = fmaf(ey[u] * (ys - ay[b]), q[u], sy);
            sz = fmaf(ey[u], qz[u], sz);
        }
    }
    s += __shfl_xor(s, 32, 64);
    if (GRAD) {
        sx += __shfl_xor(sx, 32, 64);
        sy += __shfl_xor(sy, 32, 64);
        sz += __shfl_xor(sz, 32, 64);
    }
    if (F16) {
        const int un = -(sc.sw + c);
        s = ldexpf(s, un);
        if (GRAD) {
            sx = ldexpf(sx, un);
            sy = ldexpf(sy, un);
            sz = ldexpf(sz, un);
        }
    }
}

// ---- workspace points [3][n]: eval / grad / morph, 32 points per wave ----
template <int G0, int G2, int MODE, bool F16>
__device__ __forceinline__ void g3_ws_body(const uint4 *fraw, const SplitScheme &sc, const float *ax,
                                           const float *ay, const float *az, float beta,
                                           float kappa, float gscale, const float *x_in,
                                           int64_t n, int T, float eta, float *c_out,
                                           float *s_out, float *g_out, float *x_out,
                                           const Traj &tr) {
    const int lane = threadIdx.x & 63;
    const int64_t i = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32 + (lane & 31);
    const int64_t ic = i < n ? i : n - 1;
    float x = x_in[ic], y = x_in[(size_t)n + ic], z = x_in[2 * (size_t)n + ic];
    float s, sx, sy, sz;
    const int steps = MODE == kMorph ? T : 1;
    int64_t tc;
    const bool rec = MODE == kMorph && (lane >> 5) == 0 && traj_col(tr, i, n, tc);
    for (int st = 0; st < steps; ++st) {
        if (rec) traj_put<3>(tr, st, tc, {x, y, z});
        g3_point<G0, G2, MODE != kEval, F16>(fraw, sc, ax, ay, az, kappa * x, kappa * y,
                                             kappa * z, s, sx, sy, sz);
        if (MODE == kMorph) {
            float c, sp;
            sigmoid_and_slope(s + beta, c, sp);
            const float step = eta * sp * gscale;
            x = fmaf(step, sx, x);
            y = fmaf(step, sy, y);
            z = fmaf(step, sz, z);
        }
    }
    if (rec) traj_put<3>(tr, steps, tc, {x, y, z});
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

template <int G0, int G2, int MODE>
__global__ void __launch_bounds__(kG3Block)
__attribute__((amdgpu_waves_per_eu(MODE == kMorph ? 3 : 1)))
k_grid3d_ws(const float *__restrict__ hinges, const float *__restrict__ weights, float kappa,
            float gscale, const float *x_in, int64_t n, int T, float eta, float *c_out,
            float *s_out, float *g_out, float *x_out, Traj tr) {
    using C = G3<G0, G2>;
    __shared__ uint4 fraw[C::FRAG];
    __shared__ float ax[G0], ay[kG3Y], az[G2];
    __shared__ SplitRange rg;
    // the range check pays off over a morph's steps; a single evaluation, whose blocks
    // mostly stage W, keeps the BF16 scheme without it
    const SplitScheme sc = g3_stage<G0, G2>(fraw, ax, ay, az, rg, hinges, weights, kappa,
                                         MODE == kMorph);
    __syncthreads();
    constexpr int M = G0 * kG3Y * G2;
    const float beta = weights[M];
    if (MODE == kMorph && sc.fp16)
        g3_ws_body<G0, G2, MODE, true>(fraw, sc, ax, ay, az, beta, kappa, gscale, x_in, n, T, eta,
                                       c_out, s_out, g_out, x_out, tr);
    else
        g3_ws_body<G0, G2, MODE, false>(fraw, sc, ax, ay, az, beta, kappa, gscale, x_in, n, T,
                                        eta, c_out, s_out, g_out, x_out, tr);
}

// Sum over the 8 lanes of a group (lanes 8g..8g+7), the same value in each: two
// quad exchanges and the half-row mirror, all DPP moves (the order of the pairwise
// sums is that of xor-1, xor-2, xor-4 exchanges).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL,
                                                              0xf, 0xf, true));
}
__device__ __forceinline__ float sum8(float v) {
    v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);  // row_half_mirror
    return v;
}

// The DH chain of one configuration by its 8 lanes: lane k = lane % 8 < NDOF forms link
// k's transform A_k (rotation Rz(theta0_k + q_k) Rx(alpha_k), translation (a_k cos,
// a_k sin, d_k) in frame k), and an inclusive scan composes them, P_k = A_0 ... A_k, in
// three rounds (lane k takes P from lane k - r by a DPP row shift and composes
// P <- P_{k-r} o P when k >= r, r = 1, 2, 4; lanes k >= NDOF carry the identity).  Lane
// k ends with frame k + 1: origin o_{k+1} = P_k's translation, axis z_{k+1} = the third
// column of its rotation.  lk: per link a, d, theta0, sin alpha, cos alpha (LDS).
template <int NDOF, int CTRL>
__device__ __forceinline__ void chain_round(int k, float (&R)[3][3], float (&t)[3]) {
    constexpr int r = CTRL & 15;
    float Rl[3][3], tl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        tl[a] = dpp_mov<CTRL>(t[a]);
#pragma unroll
        for (int b = 0; b < 3; ++b) Rl[a][b] = dpp_mov<CTRL>(R[a][b]);
    }
    if (k >= r) {
        float Rn[3][3], tn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            tn[a] = tl[a] + Rl[a][0] * t[0] + Rl[a][1] * t[1] + Rl[a][2] * t[2];
#pragma unroll
            for (int b = 0; b < 3; ++b)
                Rn[a][b] = Rl[a][0] * R[0][b] + Rl[a][1] * R[1][b] + Rl[a][2] * R[2][b];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            t[a] = tn[a];
#pragma unroll
            for (int b = 0; b < 3; ++b) R[a][b] = Rn[a][b];
        }
    }
}

template <int NDOF>
__device__ __forceinline__ void g3_chain_scan(const float *lk, const float (&q)[NDOF], int k,
                                              float (&R)[3][3], float (&t)[3]) {
    static_assert(NDOF <= 8, "one lane per link");
    float qk = q[0];
#pragma unroll
    for (int j = 1; j < NDOF; ++j) qk = k == j ? q[j] : qk;
    const bool act = k < NDOF;
    const float *p = lk + 5 * (act ? k : 0);
    const float a = p[0], d = p[1], sa = p[3], ca = p[4];
    float st, ct;
    sincosf(p[2] + qk, &st, &ct);
    if (act) {
        R[0][0] = ct, R[0][1] = -st * ca, R[0][2] = st * sa;
        R[1][0] = st, R[1][1] = ct * ca, R[1][2] = -ct * sa;
        R[2][0] = 0.0f, R[2][1] = sa, R[2][2] = ca;
        t[0] = a * ct, t[1] = a * st, t[2] = d;
    } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            t[i] = 0.0f;
#pragma unroll
            for (int j = 0; j < 3; ++j) R[i][j] = i == j ? 1.0f : 0.0f;
        }
    }
    chain_round<NDOF, 0x111>(k, R, t);  // row_shr:1
    chain_round<NDOF, 0x112>(k, R, t);  // row_shr:2
    chain_round<NDOF, 0x114>(k, R, t);  // row_shr:4
}

// The per-configuration records in LDS (chain, axes, joint gradient) are written and
// read by the lanes of one wave only, and a wave's LDS operations complete in issue
// order: ordering them needs a compiler barrier, not a block barrier.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- joint-space morph (MORPH) or largest body-point occupancy (check) ----
// 4 configurations per wave; lane%32 = 8*cfg + k, body point k of every link.
template <int NDOF, int G0, int G2, bool MORPH, bool F16>
__device__ __forceinline__ void arm_body(const pdmp_arm &arm, const uint4 *fraw,
                                         const SplitScheme &sc, const float *ax, const float *ay,
                                         const float *az, float *kin, const float *lk,
                                         float beta, float kappa,
                                         float gscale, const float *q_in, float *q_out, int64_t n,
                                         int64_t n_eff, int T, float eta, float thresh,
                                         float *maxc_out, uint8_t *flag_out, const Traj &tr) {
    constexpr int KIN = 3 * (NDOF + 1) + 3 * NDOF + NDOF;  // o, z, grad_q per configuration
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

    const int steps = MORPH ? T : 1;
    float mc = -1.0f;
    int64_t tc;
    const bool rec = MORPH && writer && traj_col(tr, cfg, n_eff, tc);
    for (int st = 0; st < steps; ++st) {
        if (rec) traj_put<NDOF>(tr, st, tc, q);
        {
            // the chain of this configuration (each lane of it one link, composed by a
            // scan), parked in LDS so that the link loop below does not hold ~45
            // registers across the MFMA work; the lower half-wave writes it
            float R[3][3], t[3];
            g3_chain_scan<NDOF>(lk, q, k, R, t);
            if (lane < 32) {
                if (k < NDOF) {
#pragma unroll
                    for (int e = 0; e < 3; ++e) ko[3 * (k + 1) + e] = t[e];
                }
                if (k + 1 < NDOF) {
#pragma unroll
                    for (int e = 0; e < 3; ++e) kz[3 * (k + 1) + e] = R[e][2];
                }
                if (k == 0) {
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        ko[e] = 0.0f;
                        kz[e] = e == 2 ? 1.0f : 0.0f;
                    }
                }
            }
        }
        wave_lds_sync();
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
            g3_point<G0, G2, MORPH, F16>(fraw, sc, ax, ay, az, kappa * p[0], kappa * p[1],
                                         kappa * p[2], s, sx, sy, sz);
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
        wave_lds_sync();
        if (MORPH) {
#pragma unroll
            for (int j = 0; j < NDOF; ++j) q[j] = q[j] - eta * kg[j];
        }
        wave_lds_sync();
    }
    if (rec) traj_put<NDOF>(tr, steps, tc, q);
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

template <int NDOF, int G0, int G2, bool MORPH>
__global__ void __launch_bounds__(kG3Block) __attribute__((amdgpu_waves_per_eu(3)))
k_arm_grid3d(pdmp_arm arm, const float *__restrict__ hinges, const float *__restrict__ weights,
             float kappa, float gscale, const float *q_in, float *q_out, int64_t n, int T,
             float eta, const uint32_t *__restrict__ n_active, float thresh, float *maxc_out,
             uint8_t *flag_out, Traj tr) {
    using C = G3<G0, G2>;
    constexpr int KIN = 3 * (NDOF + 1) + 3 * NDOF + NDOF;  // o, z, grad_q per configuration
    __shared__ uint4 fraw[C::FRAG];
    __shared__ float ax[G0], ay[kG3Y], az[G2];
    __shared__ float kin[16 * KIN];
    __shared__ float lk[5 * NDOF];  // per link: a, d, theta0, sin alpha, cos alpha
    __shared__ SplitRange rg;
    const int64_t n_eff = n_active ? min((int64_t)*n_active, n) : n;
    if ((int64_t)blockIdx.x * 16 >= n_eff) return;  // whole block idle (uniform)
    if (threadIdx.x < NDOF) {
        const int j = threadIdx.x;
        lk[5 * j] = arm.a[j];
        lk[5 * j + 1] = arm.d[j];
        lk[5 * j + 2] = arm.theta0[j];
        sincosf(arm.alpha[j], &lk[5 * j + 3], &lk[5 * j + 4]);
    }
    const SplitScheme sc = g3_stage<G0, G2>(fraw, ax, ay, az, rg, hinges, weights, kappa, true);
    __syncthreads();
    constexpr int M = G0 * kG3Y * G2;
    const float beta = weights[M];
    if (sc.fp16)
        arm_body<NDOF, G0, G2, MORPH, true>(arm, fraw, sc, ax, ay, az, kin, lk, beta, kappa, gscale,
                                            q_in, q_out, n, n_eff, T, eta, thresh, maxc_out,
                                            flag_out, tr);
    else
        arm_body<NDOF, G0, G2, MORPH, false>(arm, fraw, sc, ax, ay, az, kin, lk, beta, kappa, gscale,
                                             q_in, q_out, n, n_eff, T, eta, thresh, maxc_out,
                                             flag_out, tr);
}

static bool g3_supported(const int *grid, int M) {
    return grid && grid[0] == 16 && grid[1] == kG3Y && grid[2] == 16 && M == 4096;
}

// The split scheme the 3-D grid morphs (workspace and arm) take: one block runs their
// staging and writes 2 (two-part FP16 splits) or 1 (three-part BF16 splits).
__global__ void __launch_bounds__(kG3Block)
k_grid3d_scheme(const float *__restrict__ hinges, const float *__restrict__ weights, float kappa,
                int32_t *out) {
    using C = G3<16, 16>;
    __shared__ uint4 fraw[C::FRAG];
    __shared__ float ax[16], ay[kG3Y], az[16];
    __shared__ SplitRange rg;
    const SplitScheme sc = g3_stage<16, 16>(fraw, ax, ay, az, rg, hinges, weights, kappa, true);
    if (threadIdx.x == 0) *out = sc.fp16 ? 2 : 1;
}

int32_t launch_grid3d_scheme(const float *hinges, const float *weights, const int *grid, int M,
                             float kappa, int32_t *out, hipStream_t st) {
    if (!g3_supported(grid, M)) return PDMP_EUNSUPPORTED;
    hipLaunchKernelGGL(k_grid3d_scheme, dim3(1), dim3(kG3Block), 0, st, hinges, weights, kappa, out);
    return check_launch("k_grid3d_scheme");
}

int32_t launch_grid3d_ws(int mode, const RbfArgs &a, const int *grid, hipStream_t st) {
    if (!g3_supported(grid, a.M) || (mode != kEval && mode != kGrad && mode != kMorph))
        return PDMP_EUNSUPPORTED;
    if (int32_t e = grid_guard((a.n + 127) / 128, kG3Block, "k_grid3d_ws")) return e;
    const dim3 g((unsigned)((a.n + 127) / 128)), b(kG3Block);
#define PDMP_G3(MODE)                                                                         \
    hipLaunchKernelGGL((k_grid3d_ws<16, 16, MODE>), g, b, 0, st, a.hinges, a.weights, a.kappa, \
                       a.gscale, a.x_in, a.n, a.T, a.eta, a.c_out, a.s_out, a.g_out, a.x_out, \
                       a.traj)
    if (mode == kEval) PDMP_G3(kEval);
    else if (mode == kGrad) PDMP_G3(kGrad);
    else PDMP_G3(kMorph);
#undef PDMP_G3
    return check_launch("k_grid3d_ws");
}

int32_t launch_arm_grid3d(const pdmp_arm &arm, const float *h, const float *w, int M,
                          const int *grid, float kappa, float gscale, const float *qi, float *qo,
                          int64_t n, int T, float eta, const uint32_t *n_active, bool morph,
                          float thresh, float *maxc, uint8_t *flag, hipStream_t st,
                          const Traj &traj) {
    if (!g3_supported(grid, M) || arm.pts_per_link > 8) return PDMP_EUNSUPPORTED;
    if (int32_t e = grid_guard((n + 15) / 16, kG3Block, "k_arm_grid3d")) return e;
    const dim3 g((unsigned)((n + 15) / 16)), b(kG3Block);
    switch (arm.n_dof) {
#define PDMP_CASE(N)                                                                            \
    case N:                                                                                     \
        if (morph)                                                                              \
            hipLaunchKernelGGL((k_arm_grid3d<N, 16, 16, true>), g, b, 0, st, arm, h, w, kappa,  \
                               gscale, qi, qo, n, T, eta, n_active, thresh, maxc, flag, traj);  \
        else                                                                                    \
            hipLaunchKernelGGL((k_arm_grid3d<N, 16, 16, false>), g, b, 0, st, arm, h, w, kappa, \
                               gscale, qi, qo, n, T, eta, n_active, thresh, maxc, flag, traj);  \
        return check_launch("k_arm_grid3d");
        PDMP_CASE(1) PDMP_CASE(2) PDMP_CASE(3) PDMP_CASE(4)
        PDMP_CASE(5) PDMP_CASE(6) PDMP_CASE(7) PDMP_CASE(8)
#undef PDMP_CASE
    }
    return PDMP_EUNSUPPORTED;
}

}  // namespace pdmp
