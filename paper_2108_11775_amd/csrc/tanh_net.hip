// tanh_net.hip -- the paper's occupancy network (Sec. 3.1): a fully connected network
// with tanh between hidden layers and a sigmoid output, c(x) = sigma(s(x)), its input
// gradient by the chain rule, and the T-step Euler morph of Eq. 1 on top of it.
//
//   a_1 = tanh(W_0 x + b_0),  a_{l+1} = tanh(W_l a_l + b_l),  s = v . a_L + b_o
//   e_L = v * (1 - a_L^2),   e_l = (1 - a_l^2) * (W_l^T e_{l+1}),  grad s = W_0^T e_1
//
// One wave carries 16 points (four lanes per point) through the whole network.  The
// hidden-to-hidden products, forward (W_l a) and backward (W_l^T e), are FP32 MFMA
// (v_mfma_f32_16x16x4_f32) with the points as the 16 columns.  The accumulator of a
// 16-row tile t gives lane l the units 16t + 4(l/16) + v (v = 0..3) of point l%16;
// the contraction of the next product is ordered the same way (step (t, v) takes
// units 16t + 4k + v, k = 0..3), so each lane feeds its own accumulator entries back
// as the B operand -- activations never leave the registers.  The matching
// permutation is applied once to the weights when they are staged in LDS in
// fragment order (one conflict-free ds_read_b32 per MFMA).  The input layer
// (K = dim) and the output dot product are VALU work; the four lanes of a point are
// summed by xor-16 and xor-32 exchanges (the same sum in all four).  Widths up to 64
// run as 1, 2 or 4 tiles of 16, padded units having zero weights (tanh(0) = 0, so
// they add nothing).
#include "pdmp_common.h"

namespace pdmp {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_tn;

constexpr int kTnBlock = 256;   // 4 waves, 16 points each
constexpr int kTnPts = 16;      // points per wave

// tanh(z) and its slope 1 - tanh^2 from e = exp(-2|z|) in (0, 1]:
// tanh = sign(z) (1 - e)/(1 + e), slope = 4e/(1 + e)^2 (no cancellation near +-1).
__device__ __forceinline__ void tanh_slope(float z, float &a, float &d) {
    const float e = exp2_fast(-2.0f * kLog2e * fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    a = copysignf((1.0f - e) * r, z);
    d = 4.0f * e * (r * r);
}

template <int DIM, int NT, int L>
struct TnLds {
    static constexpr int HP = 16 * NT;
    static constexpr int NF = (L - 1) * NT * NT * 4 * 64;  // fragment floats per direction
    // fw[l-1][to][ti][v][lane] = W_l[16to + lane%16][16ti + 4(lane/16) + v]
    // bw[l-1][ti][to][v][lane] = W_l[16to + 4(lane/16) + v][16ti + lane%16]
    float fw[NF > 0 ? NF : 1];
    float bw[NF > 0 ? NF : 1];
    float w0t[DIM][HP];  // W_0 transposed
    float bias[L][HP];
    float vo[HP];
    float bo;
};

// Offset of W_l in the flat parameter vector (l = L gives v).
__device__ __forceinline__ int64_t tn_w_off(int l, int dim, int H) {
    return l == 0 ? 0 : (int64_t)H * dim + H + (int64_t)(l - 1) * (H * H + H);
}

template <int DIM, int NT, int L>
__device__ void tn_stage(TnLds<DIM, NT, L> &S, const float *__restrict__ P, int H) {
    using LD = TnLds<DIM, NT, L>;
    for (int idx = threadIdx.x; idx < LD::NF; idx += blockDim.x) {
        const int ln = idx & 63, v = (idx >> 6) & 3;
        const int q = idx >> 8;  // ((l-1) NT + first) NT + second
        const int second = q % NT, first = (q / NT) % NT, l = 1 + q / (NT * NT);
        const float *W = P + tn_w_off(l, DIM, H);
        {  // forward: first = to (row tile), second = ti (contraction tile)
            const int row = 16 * first + (ln & 15), col = 16 * second + 4 * (ln >> 4) + v;
            S.fw[idx] = (row < H && col < H) ? W[(int64_t)row * H + col] : 0.0f;
        }
        {  // backward: first = ti (row tile of W^T), second = to (contraction tile)
            const int row = 16 * second + 4 * (ln >> 4) + v, col = 16 * first + (ln & 15);
            S.bw[idx] = (row < H && col < H) ? W[(int64_t)row * H + col] : 0.0f;
        }
    }
    for (int idx = threadIdx.x; idx < LD::HP; idx += blockDim.x) {
        const bool ok = idx < H;
#pragma unroll
        for (int k = 0; k < DIM; ++k) S.w0t[k][idx] = ok ? P[(int64_t)idx * DIM + k] : 0.0f;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int64_t bo = tn_w_off(l, DIM, H) + (int64_t)H * (l == 0 ? DIM : H);
            S.bias[l][idx] = ok ? P[bo + idx] : 0.0f;
        }
        S.vo[idx] = ok ? P[tn_w_off(L, DIM, H) + idx] : 0.0f;
    }
    if (threadIdx.x == 0) S.bo = P[tn_w_off(L, DIM, H) + H];
}

__device__ __forceinline__ float4 tn_ld4(const float *p) {
    return *reinterpret_cast<const float4 *>(p);
}

// Sum over the four lanes of a point (the same value in all four).
__device__ __forceinline__ float tn_sum4(float p) {
    p = p + __shfl_xor(p, 16, 64);
    return p + __shfl_xor(p, 32, 64);
}

// s (all four lanes of the point) and, with GRAD, grad_x s at the point x.
template <int DIM, int NT, int L, bool GRAD>
__device__ __forceinline__ void tn_point(const TnLds<DIM, NT, L> &S, const float (&x)[DIM],
                                         float &s, float (&g)[DIM]) {
    const int lane0 = threadIdx.x & 63, u4 = 4 * (lane0 >> 4);
    // The weight fragments are the same on every call; an opaque copy of the lane
    // index keeps the compiler from hoisting their LDS reads out of the step loop
    // into registers (which would not fit).
    int lane = lane0;
    asm volatile("" : "+v"(lane));
    f32x4_tn a[NT];
    f32x4_tn d[L][NT];
    // input layer: z = b_0 + W_0 x
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int u0 = 16 * t + u4;
        const float4 bb = tn_ld4(&S.bias[0][u0]);
        float z[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const float4 w = tn_ld4(&S.w0t[k][u0]);
            z[0] = fmaf(w.x, x[k], z[0]);
            z[1] = fmaf(w.y, x[k], z[1]);
            z[2] = fmaf(w.z, x[k], z[2]);
            z[3] = fmaf(w.w, x[k], z[3]);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float av, dv;
            tanh_slope(z[v], av, dv);
            a[t][v] = av;
            d[0][t][v] = dv;
        }
    }
    // hidden layers: z = b_l + W_l a  (MFMA, the bias preloaded in the accumulator)
#pragma unroll
    for (int l = 1; l < L; ++l) {
        f32x4_tn z[NT];
#pragma unroll
        for (int to = 0; to < NT; ++to) {
            const float4 bb = tn_ld4(&S.bias[l][16 * to + u4]);
            z[to][0] = bb.x;
            z[to][1] = bb.y;
            z[to][2] = bb.z;
            z[to][3] = bb.w;
        }
        const float *fw = S.fw + (l - 1) * NT * NT * 256;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int to = 0; to < NT; ++to)
                    z[to] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                        fw[((to * NT + ti) * 4 + v) * 64 + lane], a[ti][v], z[to], 0, 0, 0);
#pragma unroll
        for (int to = 0; to < NT; ++to)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float av, dv;
                tanh_slope(z[to][v], av, dv);
                a[to][v] = av;
                d[l][to][v] = dv;
            }
    }
    // output: s = v . a_L + b_o
    float p = 0.0f;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const float4 vv = tn_ld4(&S.vo[16 * t + u4]);
        p = fmaf(vv.x, a[t][0], p);
        p = fmaf(vv.y, a[t][1], p);
        p = fmaf(vv.z, a[t][2], p);
        p = fmaf(vv.w, a[t][3], p);
    }
    s = tn_sum4(p) + S.bo;
    if (!GRAD) return;
    // reverse order: e_L = v * d_L, e_l = d_l * (W_l^T e_{l+1}), grad s = W_0^T e_1
    f32x4_tn e[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const float4 vv = tn_ld4(&S.vo[16 * t + u4]);
        e[t][0] = vv.x * d[L - 1][t][0];
        e[t][1] = vv.y * d[L - 1][t][1];
        e[t][2] = vv.z * d[L - 1][t][2];
        e[t][3] = vv.w * d[L - 1][t][3];
    }
#pragma unroll
    for (int l = L - 1; l >= 1; --l) {
        f32x4_tn G[NT];
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) G[ti][0] = G[ti][1] = G[ti][2] = G[ti][3] = 0.0f;
        const float *bw = S.bw + (l - 1) * NT * NT * 256;
#pragma unroll
        for (int to = 0; to < NT; ++to)
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int ti = 0; ti < NT; ++ti)
                    G[ti] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                        bw[((ti * NT + to) * 4 + v) * 64 + lane], e[to][v], G[ti], 0, 0, 0);
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int v = 0; v < 4; ++v) e[ti][v] = G[ti][v] * d[l - 1][ti][v];
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        float q = 0.0f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const float4 w = tn_ld4(&S.w0t[k][16 * t + u4]);
            q = fmaf(w.x, e[t][0], q);
            q = fmaf(w.y, e[t][1], q);
            q = fmaf(w.z, e[t][2], q);
            q = fmaf(w.w, e[t][3], q);
        }
        g[k] = tn_sum4(q);
    }
}

template <int DIM, int NT, int L, int MODE>
__global__ void __launch_bounds__(kTnBlock)
k_tanh_net(const float *__restrict__ P, int H, const float *x_in, int64_t n, int T, float eta,
           float *c_out, float *s_out, float *g_out, float *x_out) {
    __shared__ __attribute__((aligned(16))) TnLds<DIM, NT, L> S;
    tn_stage<DIM, NT, L>(S, P, H);
    __syncthreads();
    const int lane = threadIdx.x & 63, quad = lane >> 4;
    const int64_t tiles = (n + kTnPts - 1) / kTnPts;
    const int64_t wstride = (int64_t)gridDim.x * (kTnBlock / 64);
    for (int64_t tile = (int64_t)blockIdx.x * (kTnBlock / 64) + (threadIdx.x >> 6); tile < tiles;
         tile += wstride) {
        const int64_t i = tile * kTnPts + (lane & 15);
        const int64_t ic = i < n ? i : n - 1;
        float x[DIM], g[DIM], s = 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) x[k] = x_in[(size_t)k * n + ic];
        const int steps = MODE == kMorph ? T : 1;
        for (int st = 0; st < steps; ++st) {
            tn_point<DIM, NT, L, MODE != kEval>(S, x, s, g);
            if (MODE == kMorph) {
                float c, sp;
                sigmoid_and_slope(s, c, sp);
                const float step = eta * sp;
#pragma unroll
                for (int k = 0; k < DIM; ++k) x[k] = fmaf(-step, g[k], x[k]);
            }
        }
        if (quad != 0 || i >= n) continue;
        if (MODE == kMorph) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) x_out[(size_t)k * n + i] = x[k];
        } else {
            float c, sp;
            sigmoid_and_slope(s, c, sp);
            if (c_out) c_out[i] = c;
            if (MODE == kEval) {
                if (s_out) s_out[i] = s;
            } else {
#pragma unroll
                for (int k = 0; k < DIM; ++k) g_out[(size_t)k * n + i] = sp * g[k];
            }
        }
    }
}

template <int DIM, int NT, int L>
static void tn_launch(int mode, const pdmp_tanh_net &net, const float *x, int64_t n, int T,
                      float eta, float *c, float *s, float *g, float *xo, hipStream_t st) {
    const int64_t tiles = (n + kTnPts - 1) / kTnPts;
    int64_t blocks = (tiles + 3) / 4;
    if (blocks > 1024) blocks = 1024;
    const dim3 grid((unsigned)blocks), blk(kTnBlock);
    if (mode == kEval)
        hipLaunchKernelGGL((k_tanh_net<DIM, NT, L, kEval>), grid, blk, 0, st, net.params,
                           net.hidden, x, n, T, eta, c, s, g, xo);
    else if (mode == kGrad)
        hipLaunchKernelGGL((k_tanh_net<DIM, NT, L, kGrad>), grid, blk, 0, st, net.params,
                           net.hidden, x, n, T, eta, c, s, g, xo);
    else
        hipLaunchKernelGGL((k_tanh_net<DIM, NT, L, kMorph>), grid, blk, 0, st, net.params,
                           net.hidden, x, n, T, eta, c, s, g, xo);
}

template <int DIM, int NT>
static void tn_by_depth(int mode, const pdmp_tanh_net &net, const float *x, int64_t n, int T,
                        float eta, float *c, float *s, float *g, float *xo, hipStream_t st) {
    switch (net.n_hidden) {
        case 1: tn_launch<DIM, NT, 1>(mode, net, x, n, T, eta, c, s, g, xo, st); break;
        case 2: tn_launch<DIM, NT, 2>(mode, net, x, n, T, eta, c, s, g, xo, st); break;
        case 3: tn_launch<DIM, NT, 3>(mode, net, x, n, T, eta, c, s, g, xo, st); break;
        default: tn_launch<DIM, NT, 4>(mode, net, x, n, T, eta, c, s, g, xo, st); break;
    }
}

// The caller has validated net (dim 2 or 3, 1 <= hidden <= 64, 1 <= n_hidden <= 4)
// and n >= 1.
int32_t launch_tanh_net(const pdmp_tanh_net &net, int mode, const float *x, int64_t n, int T,
                        float eta, float *c_out, float *s_out, float *g_out, float *x_out,
                        hipStream_t st) {
    const int h = net.hidden;
#define PDMP_TN(D)                                                                          \
    if (h <= 16) tn_by_depth<D, 1>(mode, net, x, n, T, eta, c_out, s_out, g_out, x_out, st); \
    else if (h <= 32) tn_by_depth<D, 2>(mode, net, x, n, T, eta, c_out, s_out, g_out, x_out, st); \
    else tn_by_depth<D, 4>(mode, net, x, n, T, eta, c_out, s_out, g_out, x_out, st)
    if (net.dim == 2) {
        PDMP_TN(2);
    } else {
        PDMP_TN(3);
    }
#undef PDMP_TN
    return check_launch("k_tanh_net");
}

}  // namespace pdmp
