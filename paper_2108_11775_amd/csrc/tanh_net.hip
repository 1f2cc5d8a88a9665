// tanh_net.hip -- the paper's occupancy network (Sec. 3.1): a fully connected network
// with tanh between hidden layers and a sigmoid output, c(x) = sigma(s(x)), its input
// gradient by the chain rule, and the T-step Euler morph of Eq. 1 on top of it.
//
//   a_1 = tanh(W_0 x + b_0),  a_{l+1} = tanh(W_l a_l + b_l),  s = v . a_L + b_o
//   e_L = v * (1 - a_L^2),   e_l = (1 - a_l^2) * (W_l^T e_{l+1}),  grad s = W_0^T e_1
//
// One wave carries 16 points (four lanes per point) through the whole network.  The
// hidden-to-hidden products, forward (W_l a) and backward (W_l^T e), run on the matrix
// cores with the points as the 16 columns.  The accumulator of a 16-row tile t gives
// lane l the units 16t + 4(l/16) + v (v = 0..3) of point l%16; the contraction of the
// next product is ordered to match, so each lane feeds its own accumulator entries
// back as the B operand -- activations never leave the registers.  The matching
// permutation is applied once to the weights when they are staged in LDS in
// fragment order.  The morph, value and gradient kernel runs the products on BF16
// MFMA at FP32 accuracy (v_mfma_f32_16x16x32_bf16, three-way bf16 splits, six
// leading products: mfma_split.h); a 32-wide k-block takes tiles 2kb and 2kb + 1,
// lane l supplying units 16(2kb + j/4) + 4(l/16) + j%4, j < 8.  The fit kernels stay
// on FP32 MFMA (v_mfma_f32_16x16x4_f32, step (t, v) takes units 16t + 4k + v).  The input layer
// (K = dim) and the output dot product are VALU work; the four lanes of a point are
// summed by xor-16 and xor-32 exchanges (the same sum in all four).  Widths up to 64
// run as 1, 2 or 4 tiles of 16, padded units having zero weights (tanh(0) = 0, so
// they add nothing).
#include "mfma_split.h"
#include "pdmp_common.h"

namespace pdmp {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_tn;

constexpr int kTnBlock = 256;   // 4 waves, 16 points each (fit)
constexpr int kTnMorphBlock = 512;  // 8 waves share one LDS copy of the weights (morph)
constexpr int kTnPts = 16;      // points per wave

// tanh(z) and its slope 1 - tanh^2 from e = exp(-2|z|) in (0, 1]:
// tanh = sign(z) (1 - e)/(1 + e), slope = 4e/(1 + e)^2 (no cancellation near +-1).
__device__ __forceinline__ void tanh_slope(float z, float &a, float &d) {
    const float e = exp2_fast(-2.0f * kLog2e * fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    a = copysignf((1.0f - e) * r, z);
    d = 4.0f * e * (r * r);
}

// The same from a pre-activation held scaled by 2^zs, k = -2 log2(e) 2^-zs, returning
// as tanh (as a power of two): both scalings are exact, so a / as and d are the bits
// tanh_slope gives for z 2^-zs.
__device__ __forceinline__ void tanh_slope_sc(float z, float k, float as, float &a, float &d) {
    const float e = exp2_fast(k * fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    a = copysignf((1.0f - e) * (r * as), z);
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

// Called by blocks of kTnBlock threads.  The fragments are loaded in batches of
// eight per thread, every load unconditional (a padded entry reads W[0] and is
// replaced by zero), so that a batch's loads are in flight together before their LDS
// stores; a load per entry behind its own branch left their latency serialised.
template <int DIM, int NT, int L>
__device__ void tn_stage(TnLds<DIM, NT, L> &S, const float *__restrict__ P, int H) {
    using LD = TnLds<DIM, NT, L>;
    constexpr int NB = 8;
    for (int base = 0; base < LD::NF; base += kTnBlock * NB) {
        float fv[NB], bv[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int idx = base + u * kTnBlock + threadIdx.x;
            const int ln = idx & 63, v = (idx >> 6) & 3;
            const int q = idx >> 8;  // ((l-1) NT + first) NT + second
            const int second = q % NT, first = (q / NT) % NT, l = 1 + q / (NT * NT);
            const bool in = idx < LD::NF;  // then l < L (NF > 0 means L >= 2)
            const float *W = P + tn_w_off(in ? l : L - 1, DIM, H);
            // forward: first = to (row tile), second = ti (contraction tile)
            const int fr = 16 * first + (ln & 15), fc = 16 * second + 4 * (ln >> 4) + v;
            // backward: first = ti (row tile of W^T), second = to (contraction tile)
            const int br = 16 * second + 4 * (ln >> 4) + v, bc = 16 * first + (ln & 15);
            const bool fok = in && fr < H && fc < H, bok = in && br < H && bc < H;
            const float f = W[fok ? (int64_t)fr * H + fc : 0];
            const float b = W[bok ? (int64_t)br * H + bc : 0];
            fv[u] = fok ? f : 0.0f;
            bv[u] = bok ? b : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int idx = base + u * kTnBlock + threadIdx.x;
            if (idx < LD::NF) {
                S.fw[idx] = fv[u];
                S.bw[idx] = bv[u];
            }
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

// ---- BF16-MFMA form (morph, value, gradient) ----

// The forward hidden products' scheme (the block's choice from the weights, every
// block alike): FP16 parts when each hidden-to-hidden W_l is finite with every nonzero
// |w| at least 2^-19 of its largest -- then 2^fsw W_l, largest in [2^14, 2^15), has
// two FP16 parts of 11 bits each and three products carry a multiply-add at FP32
// accuracy (mfma_split.h) -- and the layer's scale 2^(fsw + kTnAct) lies in [1, 2^100]
// with the scaled bias at most 2^120 (the accumulator starts from it: nothing is lost
// or overflows in scaling); three-way BF16 splits and six products otherwise.  The
// backward products stay on BF16 parts: their vectors e_l have no bound to scale by.
struct TnFwd {
    int fwh;          // 1: FP16 forward products
    int fsw[4];       // per hidden-to-hidden layer l (index l - 1): the scale exponent
    uint32_t wmx[4], wmn[4], bmx[4];  // largest, smallest nonzero |w|; largest |b| (bits)
};

// Activations enter the FP16 forward products as 2^kTnAct a (|a| <= 1): FP16 keeps 11
// bits of every |a| >= 2^-28 and the products stay below 2^29 in the FP32 accumulator.
constexpr int kTnAct = 14;

// Every thread of the block calls it; it synchronises the block.
template <int L>
__device__ void tn_forward_scheme(TnFwd &F, const float *__restrict__ P, int dim, int H) {
    if (threadIdx.x < 4) {
        F.wmx[threadIdx.x] = 0u;
        F.wmn[threadIdx.x] = 0xffffffffu;
        F.bmx[threadIdx.x] = 0u;
    }
    __syncthreads();
    for (int l = 1; l < L; ++l) {
        const float *W = P + tn_w_off(l, dim, H);  // W_l (H x H), then b_l (H)
        uint32_t mx = 0u, mn = 0xffffffffu, bm = 0u;
        for (int e = threadIdx.x; e < H * H; e += blockDim.x) {
            const uint32_t u = __float_as_uint(W[e]) & 0x7fffffffu;
            mx = max(mx, u);
            if (u != 0u) mn = min(mn, u);
        }
        for (int e = threadIdx.x; e < H; e += blockDim.x)
            bm = max(bm, __float_as_uint(W[(int64_t)H * H + e]) & 0x7fffffffu);
        atomicMax(&F.wmx[l - 1], mx);
        atomicMin(&F.wmn[l - 1], mn);
        atomicMax(&F.bmx[l - 1], bm);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = L > 1;
        for (int l = 0; l < L - 1; ++l) {
            const uint32_t mx = F.wmx[l], mn = F.wmn[l], bm = F.bmx[l];
            int e = 0;
            if (mx >= 0x7f800000u || bm >= 0x7f800000u) {
                ok = 0;  // Inf or NaN
            } else if (mx != 0u) {
                frexpf(__uint_as_float(mx), &e);  // largest = m 2^e, m in [0.5, 1)
                if (__uint_as_float(mn) < ldexpf(__uint_as_float(mx), -19)) ok = 0;
            }
            const int fsw = mx != 0u ? 15 - e : 0;
            if (fsw + kTnAct < 0 || fsw + kTnAct > 100 ||
                ldexpf(__uint_as_float(bm), fsw + kTnAct) > 0x1p120f)
                ok = 0;
            F.fsw[l] = fsw;
        }
        F.fwh = ok;
    }
    __syncthreads();
}

template <int L>
__global__ void __launch_bounds__(256) k_tanh_scheme(const float *__restrict__ P, int dim, int H,
                                                     int32_t *out) {
    __shared__ TnFwd F;
    tn_forward_scheme<L>(F, P, dim, H);
    if (threadIdx.x == 0) *out = F.fwh ? 2 : 1;
}

// The forward scheme the morph, value and gradient kernel takes: 2 (FP16 parts) or 1.
int32_t launch_tanh_scheme(const pdmp_tanh_net &net, int32_t *out, hipStream_t st) {
#define PDMP_TS(L)                                                                         \
    hipLaunchKernelGGL(k_tanh_scheme<L>, dim3(1), dim3(256), 0, st, net.params, net.dim, \
                       net.hidden, out)
    switch (net.n_hidden) {
        case 1: PDMP_TS(1); break;
        case 2: PDMP_TS(2); break;
        case 3: PDMP_TS(3); break;
        default: PDMP_TS(4); break;
    }
#undef PDMP_TS
    return check_launch("k_tanh_scheme");
}

template <int DIM, int NT, int L>
struct TnLdsX6 {
    static constexpr int HP = 16 * NT;
    static constexpr int KB = (NT + 1) / 2;                      // 32-wide k-blocks
    static constexpr int NF = (L - 1) * NT * KB * 3 * 64;        // bf16x8 fragments per direction
    // fw[((l-1) NT + to) KB + kb][p][lane] = part p of W_l[16to + lane%16][unit(kb, lane, j)]
    // bw[((l-1) NT + ti) KB + kb][p][lane] = part p of W_l[unit(kb, lane, j)][16ti + lane%16]
    // with unit(kb, lane, j) = 16(2kb + j/4) + 4(lane/16) + j%4, j < 8
    bf16x8_t fw[NF > 0 ? NF : 1];
    bf16x8_t bw[NF > 0 ? NF : 1];
    float w0t[DIM][HP];  // W_0 transposed
    float bias[L][HP];
    float vo[HP];
    float bo;
    TnFwd F;  // the forward products' scheme
};

template <int DIM, int NT, int L>
__device__ void tn_stage_x6(TnLdsX6<DIM, NT, L> &S, const float *__restrict__ P, int H) {
    using LD = TnLdsX6<DIM, NT, L>;
    tn_forward_scheme<L>(S.F, P, DIM, H);
    const bool fh = S.F.fwh != 0;
    for (int idx = threadIdx.x; idx < LD::NF / 3; idx += blockDim.x) {
        const int ln = idx & 63, q = idx >> 6;  // q = ((l-1) NT + first) KB + kb
        const int kb = q % LD::KB, first = (q / LD::KB) % NT, l = 1 + q / (LD::KB * NT);
        const float *W = P + tn_w_off(l, DIM, H);
        float vf[8], vb[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int t = 2 * kb + j / 4;
            const int unit = 16 * t + 4 * (ln >> 4) + (j & 3);
            const int other = 16 * first + (ln & 15);
            const bool ok = t < NT && unit < H && other < H;
            vf[j] = ok ? W[(int64_t)other * H + unit] : 0.0f;  // forward: row other, col unit
            vb[j] = ok ? W[(int64_t)unit * H + other] : 0.0f;  // backward: W^T
        }
        bf16x8_t f1, f2, f3, b1, b2, b3;
        const int base = q * 3 * 64 + ln;
        if (fh) {
#pragma unroll
            for (int j = 0; j < 8; ++j) vf[j] = ldexpf(vf[j], S.F.fsw[l - 1]);
            f16x8_t h1, h2;
            split2h(vf, h1, h2);
            reinterpret_cast<f16x8_t *>(S.fw)[base] = h1;
            reinterpret_cast<f16x8_t *>(S.fw)[base + 64] = h2;
        } else {
            split3(vf, f1, f2, f3);
            S.fw[base] = f1;
            S.fw[base + 64] = f2;
            S.fw[base + 128] = f3;
        }
        split3(vb, b1, b2, b3);
        S.bw[base] = b1;
        S.bw[base + 64] = b2;
        S.bw[base + 128] = b3;
    }
    for (int idx = threadIdx.x; idx < LD::HP; idx += blockDim.x) {
        const bool ok = idx < H;
#pragma unroll
        for (int k = 0; k < DIM; ++k) S.w0t[k][idx] = ok ? P[(int64_t)idx * DIM + k] : 0.0f;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int64_t bo = tn_w_off(l, DIM, H) + (int64_t)H * (l == 0 ? DIM : H);
            // FP16 forward: the hidden biases enter the accumulator as 2^(fsw + kTnAct) b
            const float b = ok ? P[bo + idx] : 0.0f;
            S.bias[l][idx] = fh && l > 0 ? ldexpf(b, S.F.fsw[l - 1] + kTnAct) : b;
        }
        S.vo[idx] = ok ? P[tn_w_off(L, DIM, H) + idx] : 0.0f;
    }
    if (threadIdx.x == 0) S.bo = P[tn_w_off(L, DIM, H) + H];
}

// The lane's B operand of k-block kb from its accumulator-layout values v[t][0..3],
// split into three bf16 parts.
template <int NT>
__device__ __forceinline__ void tn_kblock(const f32x4_tn (&v)[NT], int kb, bf16x8_t &p1,
                                          bf16x8_t &p2, bf16x8_t &p3) {
    float b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int t = 2 * kb + j / 4;
        b[j] = t < NT ? v[t < NT ? t : 0][j & 3] : 0.0f;
    }
    split3(b, p1, p2, p3);
}

// s (all four lanes of the point) and, with GRAD, grad_x s at the point x; with FH
// the forward hidden products on the FP16 parts (the block's scheme, S.fwh).
template <int DIM, int NT, int L, bool GRAD, bool FH>
__device__ __forceinline__ void tn_point_x6(const TnLdsX6<DIM, NT, L> &S, const float (&x)[DIM],
                                            float &s, float (&g)[DIM]) {
    using LD = TnLdsX6<DIM, NT, L>;
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
            // FP16 forward: the activations feeding a hidden product are held as 2^kTnAct a
            tanh_slope_sc(z[v], -2.0f * kLog2e, FH ? (float)(1 << kTnAct) : 1.0f, av, dv);
            a[t][v] = av;
            d[0][t][v] = dv;
        }
    }
    // hidden layers: z = b_l + W_l a  (the bias preloaded in the accumulator)
#pragma unroll
    for (int l = 1; l < L; ++l) {
        f32x4_tn z[NT];
        // FP16 products accumulate 2^(fsw + kTnAct) (W a + b) from the bias staged at
        // that scale; the tanh below takes the unscaling in its exponent (exact)
        const float kz = FH ? ldexpf(-2.0f * kLog2e, -(S.F.fsw[l - 1] + kTnAct)) : -2.0f * kLog2e;
#pragma unroll
        for (int to = 0; to < NT; ++to) {
            const float4 bb = tn_ld4(&S.bias[l][16 * to + u4]);
            z[to][0] = bb.x;
            z[to][1] = bb.y;
            z[to][2] = bb.z;
            z[to][3] = bb.w;
        }
#pragma unroll
        for (int kb = 0; kb < LD::KB; ++kb) {
            if (FH) {
                float bv[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int t = 2 * kb + j / 4;
                    bv[j] = t < NT ? a[t < NT ? t : 0][j & 3] : 0.0f;  // 2^kTnAct a
                }
                f16x8_t h1, h2;
                split2h(bv, h1, h2);
#pragma unroll
                for (int to = 0; to < NT; ++to) {
                    const f16x8_t *f = reinterpret_cast<const f16x8_t *>(S.fw) +
                                       (((l - 1) * NT + to) * LD::KB + kb) * 3 * 64 + lane;
                    z[to] = mfma16_h3(f[0], f[64], h1, h2, z[to]);
                }
            } else {
                bf16x8_t b1, b2, b3;
                tn_kblock<NT>(a, kb, b1, b2, b3);
#pragma unroll
                for (int to = 0; to < NT; ++to) {
                    const bf16x8_t *f = S.fw + (((l - 1) * NT + to) * LD::KB + kb) * 3 * 64 + lane;
                    z[to] = mfma16_x6(f[0], f[64], f[128], b1, b2, b3, z[to]);
                }
            }
        }
#pragma unroll
        for (int to = 0; to < NT; ++to)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float av, dv;
                // scaled by 2^kTnAct again where the next hidden product takes it
                tanh_slope_sc(z[to][v], kz, FH && l + 1 < L ? (float)(1 << kTnAct) : 1.0f, av,
                              dv);
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
        const f32x4_tn zero = {};  // the first k-block starts from the zero accumulator
#pragma unroll
        for (int kb = 0; kb < LD::KB; ++kb) {
            bf16x8_t b1, b2, b3;
            tn_kblock<NT>(e, kb, b1, b2, b3);
#pragma unroll
            for (int ti = 0; ti < NT; ++ti) {
                const bf16x8_t *f = S.bw + (((l - 1) * NT + ti) * LD::KB + kb) * 3 * 64 + lane;
                G[ti] = mfma16_x6(f[0], f[64], f[128], b1, b2, b3, kb == 0 ? zero : G[ti]);
            }
        }
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
__global__ void __launch_bounds__(kTnMorphBlock)
k_tanh_net(const float *__restrict__ P, int H, const float *x_in, int64_t n, int T, float eta,
           float *c_out, float *s_out, float *g_out, float *x_out) {
    __shared__ __attribute__((aligned(16))) TnLdsX6<DIM, NT, L> S;
    tn_stage_x6<DIM, NT, L>(S, P, H);
    __syncthreads();
    const int lane = threadIdx.x & 63, quad = lane >> 4;
    const int64_t tiles = (n + kTnPts - 1) / kTnPts;
    const int64_t wstride = (int64_t)gridDim.x * (kTnMorphBlock / 64);
    for (int64_t tile = (int64_t)blockIdx.x * (kTnMorphBlock / 64) + (threadIdx.x >> 6); tile < tiles;
         tile += wstride) {
        const int64_t i = tile * kTnPts + (lane & 15);
        const int64_t ic = i < n ? i : n - 1;
        float x[DIM], g[DIM], s = 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) x[k] = x_in[(size_t)k * n + ic];
        const int steps = MODE == kMorph ? T : 1;
        for (int st = 0; st < steps; ++st) {
            if (S.F.fwh)
                tn_point_x6<DIM, NT, L, MODE != kEval, true>(S, x, s, g);
            else
                tn_point_x6<DIM, NT, L, MODE != kEval, false>(S, x, s, g);
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
    constexpr int wpb = kTnMorphBlock / 64;
    int64_t blocks = (tiles + wpb - 1) / wpb;
    if (blocks > 512) blocks = 512;
    const dim3 grid((unsigned)blocks), blk(kTnMorphBlock);
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


// ------------------------------------------------------------------ fit ---
//
// BCE fit of the network (Sec. 3.1), full batch over n labelled points.  One step:
//   k_tanh_fb      per point: forward, r = (sigma(s) - y)/n, the BCE (summed per block), and
//                  the reverse pass e_L = r v (1 - a_L^2), e_l = (1 - a_l^2) W_l^T e_{l+1};
//                  stores a_l and e_l ([layer][unit][point], coalesced per unit);
//   k_tanh_wgrad   dW_l = sum_i e_{l+1,i} [a_{l,i}; 1]^T (the bias as a column of ones;
//                  layer L: r against [a_L; 1]) on FP32 MFMA with the points as
//                  contraction index, one block per layer and range of points ->
//                  partial rows; the first range's row carries + l2 w on the weight
//                  entries (not the biases) and, when the loss is asked for, each
//                  layer's sum of w^2;
//   k_tanh_sum_adam fixed-order sum of the partial rows and the Adam step (fit), or
//   k_sum_rows     the sum alone (fit.hip; the loss and gradient query);
//   k_tanh_loss    the loss from the two kernels' partial sums (when asked for).

template <int DIM, int NT, int L>
__global__ void __launch_bounds__(kTnBlock)
k_tanh_fb(const float *__restrict__ P, int H, const float *__restrict__ x,
          const uint8_t *__restrict__ y, int64_t n, float inv_n, float *__restrict__ A,
          float *__restrict__ E, float *__restrict__ r_out, double *__restrict__ bce_part) {
    __shared__ __attribute__((aligned(16))) TnLds<DIM, NT, L> S;
    __shared__ double rb[kTnBlock];
    tn_stage<DIM, NT, L>(S, P, H);
    __syncthreads();
    const int lane = threadIdx.x & 63, quad = lane >> 4, u4 = 4 * quad;
    double bacc = 0.0;  // this lane's points' BCE (quad 0 lanes), in tile order
    const int64_t tiles = (n + kTnPts - 1) / kTnPts;
    const int64_t wstride = (int64_t)gridDim.x * (kTnBlock / 64);
    for (int64_t tile = (int64_t)blockIdx.x * (kTnBlock / 64) + (threadIdx.x >> 6); tile < tiles;
         tile += wstride) {
        const int64_t i = tile * kTnPts + (lane & 15);
        const bool ok = i < n;
        const int64_t ic = ok ? i : n - 1;
        // opaque per tile: keeps the fragment reads and the per-unit store offsets
        // inside the loop instead of hoisting them all into registers
        int lf = lane;
        asm volatile("" : "+v"(lf));
        size_t nn = (size_t)n;
        asm volatile("" : "+s"(nn));
        float xv[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) xv[k] = x[(size_t)k * n + ic];
        f32x4_tn a[NT];
        f32x4_tn d[L][NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int u0 = 16 * t + u4;
            const float4 bb = tn_ld4(&S.bias[0][u0]);
            float z[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const float4 w = tn_ld4(&S.w0t[k][u0]);
                z[0] = fmaf(w.x, xv[k], z[0]);
                z[1] = fmaf(w.y, xv[k], z[1]);
                z[2] = fmaf(w.z, xv[k], z[2]);
                z[3] = fmaf(w.w, xv[k], z[3]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float av, dv;
                tanh_slope(z[v], av, dv);
                a[t][v] = av;
                d[0][t][v] = dv;
                if (ok && u0 + v < H) A[(size_t)(u0 + v) * nn + i] = av;
            }
        }
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
                            fw[((to * NT + ti) * 4 + v) * 64 + lf], a[ti][v], z[to], 0, 0, 0);
#pragma unroll
            for (int to = 0; to < NT; ++to)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float av, dv;
                    tanh_slope(z[to][v], av, dv);
                    a[to][v] = av;
                    d[l][to][v] = dv;
                    const int u = 16 * to + u4 + v;
                    if (ok && u < H) A[((size_t)l * H + u) * nn + i] = av;
                }
        }
        float p = 0.0f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const float4 vv = tn_ld4(&S.vo[16 * t + u4]);
            p = fmaf(vv.x, a[t][0], p);
            p = fmaf(vv.y, a[t][1], p);
            p = fmaf(vv.z, a[t][2], p);
            p = fmaf(vv.w, a[t][3], p);
        }
        const float s = tn_sum4(p) + S.bo;
        const bool yes = ok && y[ic];
        const float yv = yes ? 1.0f : 0.0f;
        // dBCE/ds = sigma(s) - y as sigma(s) (y = 0) or -sigma(-s) (y = 1): full relative
        // accuracy also where sigma(s) rounds to y; e1 = exp(-|s|)
        const float e1 = exp2_fast(-fabsf(s) * kLog2e);
        const float inv = 1.0f / (1.0f + e1);
        const float sig_pos = s >= 0.0f ? inv : e1 * inv, sig_neg = s >= 0.0f ? e1 * inv : inv;
        const float r = ok ? (yes ? -sig_neg : sig_pos) * inv_n : 0.0f;
        if (ok && quad == 0) {
            r_out[i] = r;
            bacc += (double)(fmaxf(s, 0.0f) - yv * s + log1pf(e1));
        }
        f32x4_tn e[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const float4 vv = tn_ld4(&S.vo[16 * t + u4]);
            e[t][0] = r * vv.x * d[L - 1][t][0];
            e[t][1] = r * vv.y * d[L - 1][t][1];
            e[t][2] = r * vv.z * d[L - 1][t][2];
            e[t][3] = r * vv.w * d[L - 1][t][3];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int u = 16 * t + u4 + v;
                if (ok && u < H) E[((size_t)(L - 1) * H + u) * nn + i] = e[t][v];
            }
        }
#pragma unroll
        for (int l = L - 1; l >= 1; --l) {
            f32x4_tn G[NT];
            const f32x4_tn zero = {};
            const float *bw = S.bw + (l - 1) * NT * NT * 256;
#pragma unroll
            for (int to = 0; to < NT; ++to)
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int ti = 0; ti < NT; ++ti)
                        G[ti] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            bw[((ti * NT + to) * 4 + v) * 64 + lf], e[to][v],
                            (to == 0 && v == 0) ? zero : G[ti], 0, 0, 0);
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    e[ti][v] = G[ti][v] * d[l - 1][ti][v];
                    const int u = 16 * ti + u4 + v;
                    if (ok && u < H) E[((size_t)(l - 1) * H + u) * nn + i] = e[ti][v];
                }
        }
    }
    if (!bce_part) return;  // uniform over the block
    // the block's BCE sum, fixed order
    rb[threadIdx.x] = bacc;
    __syncthreads();
    for (unsigned s2 = kTnBlock / 2; s2 >= 1; s2 >>= 1) {
        if (threadIdx.x < s2) rb[threadIdx.x] += rb[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) bce_part[blockIdx.x] = rb[0];
}

// out = sa sum_{i < na} a[i] + sb sum_{i < nb} b[i], one block, fixed order (the loss
// from the BCE partials of k_tanh_fb and the w^2 partials of k_tanh_wgrad).
__global__ void __launch_bounds__(256)
k_tanh_loss(const double *__restrict__ a, int na, double sa, const double *__restrict__ b, int nb,
            double sb, float *out) {
    __shared__ double sh[2][256];
    double ta = 0.0, tb = 0.0;
    for (int i = threadIdx.x; i < na; i += 256) ta += a[i];
    for (int i = threadIdx.x; i < nb; i += 256) tb += b[i];
    sh[0][threadIdx.x] = ta;
    sh[1][threadIdx.x] = tb;
    __syncthreads();
    for (unsigned s2 = 128; s2 >= 1; s2 >>= 1) {
        if (threadIdx.x < s2) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s2];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s2];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)(sa * sh[0][0] + sb * sh[1][0]);
}

// Weight-gradient products, one block per (layer, split of the points).
constexpr int kTnWgChunk = 64;   // points staged per round
constexpr int kTnWgRS = kTnWgChunk + 1;  // LDS row stride: lanes of one MFMA hit 64 banks
constexpr int kTnWgRows = 64;    // rows of E (H <= 64)
constexpr int kTnWgCols = 80;    // columns [a; 1] padded to 16 (H + 1 <= 65)

// Partial rows of the loss gradient.  Block (l, split): layer l < L: dW_l = E_{l+1}
// [a_l; 1]^T (rows o of E (H), columns i of [a_l; 1], n_l + 1 of them, a_0 = x); layer
// L: the single row r against [a_L; 1]; over the points [split kps, min(n, (split +
// 1) kps)).  Each round stages 64 points of the rows and columns in LDS (coalesced row
// reads, issued a round ahead), then every 16 x 16 output tile of the layer, owned by
// one wave, takes 16 FP32 MFMAs (lane group q takes the points 16q + m, m < 16); each
// output sums its points in a fixed order.  The blocks of split 0 add the decay l2 w
// to the weight entries of their layer and, with wsq_part, write the layer's sum of
// w^2 (FP64, fixed order) to wsq_part[l].
__global__ void __launch_bounds__(256)
k_tanh_wgrad(int dim, int H, int L, const float *__restrict__ x, const float *__restrict__ A,
             const float *__restrict__ E, const float *__restrict__ r, int64_t n, int64_t kps,
             int64_t np, const float *__restrict__ P, float l2, float *__restrict__ part,
             double *__restrict__ wsq_part) {
    __shared__ float Xs[kTnWgRows * kTnWgRS];
    __shared__ float Ys[kTnWgCols * kTnWgRS];
    __shared__ double rw[256];
    const int l = blockIdx.x;
    const int rows = l < L ? H : 1;
    const int nl = l == 0 ? dim : H;  // columns before the ones column
    const int RT = (rows + 15) / 16, CT = (nl + 1 + 15) / 16, NTl = RT * CT;
    const float *X = l < L ? E + (size_t)l * H * n : r;
    const float *Y = l == 0 ? x : A + (size_t)(l - 1) * H * n;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, q = lane >> 4, c16 = lane & 15;
    const int64_t ks = (int64_t)blockIdx.y * kps;
    const int64_t ke = ks + kps < n ? ks + kps : n;
    f32x4_tn acc[5];  // this wave's tiles t = wv + 4 u (at most 20 per layer)
#pragma unroll
    for (int u = 0; u < 5; ++u) acc[u][0] = acc[u][1] = acc[u][2] = acc[u][3] = 0.0f;
    // this thread's staging values for one round: rows wv + 4u of X and of [Y; 1] at
    // point k0 + lane, loaded a round ahead so that their latency overlaps the MFMAs
    constexpr int XU = kTnWgRows / 4, YU = kTnWgCols / 4;
    float xv[XU], yv[YU];
    auto load_round = [&](int64_t k0) {
        const int64_t k = k0 + lane;
        const bool kin = k < ke;
#pragma unroll
        for (int u = 0; u < XU; ++u) {
            const int rr = wv + 4 * u;
            xv[u] = kin && rr < rows ? X[(size_t)rr * n + k] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < YU; ++u) {
            const int cc = wv + 4 * u;
            float v = 0.0f;
            if (cc < nl) v = kin ? Y[(size_t)cc * n + k] : 0.0f;
            else if (cc == nl) v = 1.0f;  // the bias column
            yv[u] = v;
        }
    };
    if (ks < ke) load_round(ks);
    for (int64_t k0 = ks; k0 < ke; k0 += kTnWgChunk) {
#pragma unroll
        for (int u = 0; u < XU; ++u)
            if (wv + 4 * u < 16 * RT) Xs[(wv + 4 * u) * kTnWgRS + lane] = xv[u];
#pragma unroll
        for (int u = 0; u < YU; ++u)
            if (wv + 4 * u < 16 * CT) Ys[(wv + 4 * u) * kTnWgRS + lane] = yv[u];
        __syncthreads();
        if (k0 + kTnWgChunk < ke) load_round(k0 + kTnWgChunk);
#pragma unroll
        for (int u = 0; u < 5; ++u) {
            const int t = wv + 4 * u;
            if (t >= NTl) break;  // uniform over the wave
            const int ro = t / CT, co = t % CT;
            const float *xa = Xs + (16 * ro + c16) * kTnWgRS + 16 * q;
            const float *yb = Ys + (16 * co + c16) * kTnWgRS + 16 * q;
#pragma unroll
            for (int m = 0; m < 16; ++m)
                acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[m], yb[m], acc[u], 0, 0, 0);
        }
        __syncthreads();
    }
    // entry v of lane (c16, q) in a tile is (row 4q + v, column c16)
    const int64_t off = (int64_t)(l == 0 ? 0 : (int64_t)H * dim + H + (int64_t)(l - 1) * (H * H + H));
    double wq = 0.0;  // this lane's w^2 over its weight entries (split 0)
#pragma unroll
    for (int u = 0; u < 5; ++u) {
        const int t = wv + 4 * u;
        if (t >= NTl) break;
        const int ro = t / CT, co = t % CT;
        const int i = 16 * co + c16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int o = 16 * ro + 4 * q + v;
            if (o >= rows || i > nl) continue;
            int64_t j;
            if (l < L) j = i < nl ? off + (int64_t)o * nl + i : off + (int64_t)H * nl + o;
            else j = off + i;  // v entries, then b_o at i == H
            float val = acc[u][v];
            if (blockIdx.y == 0 && i < nl) {  // a weight entry (i == nl: the bias)
                const float w = P[j];
                val = fmaf(l2, w, val);
                wq += (double)w * (double)w;
            }
            part[(size_t)blockIdx.y * np + j] = val;
        }
    }
    if (blockIdx.y != 0 || !wsq_part) return;  // uniform over the block
    rw[threadIdx.x] = wq;
    __syncthreads();
    for (unsigned s2 = 128; s2 >= 1; s2 >>= 1) {
        if (threadIdx.x < s2) rw[threadIdx.x] += rw[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) wsq_part[l] = rw[0];
}

// Points per split of the weight-gradient products: whole rounds of 64, about 128
// splits (at most as many as there are rounds).
static int tn_splits(int64_t n, int64_t &kps) {
    const int64_t rounds = (n + kTnWgChunk - 1) / kTnWgChunk;
    const int64_t per = (rounds + 127) / 128;
    kps = (per < 1 ? 1 : per) * kTnWgChunk;
    return (int)((n + kps - 1) / kps);
}

static size_t al256t(size_t b) { return (b + 255) & ~(size_t)255; }

size_t tanh_fit_ws_bytes(const pdmp_tanh_net &net, int64_t n) {
    const int64_t H = net.hidden, L = net.n_hidden;
    const int64_t np = H * net.dim + H + (L - 1) * (H * H + H) + H + 1;
    int64_t kps;
    const int S = tn_splits(n, kps);
    return 2 * al256t((size_t)(L * H * n) * 4) + al256t((size_t)n * 4) +
           al256t((size_t)S * np * 4) + al256t((size_t)np * 4) + al256t(1024 * 8) +
           al256t((size_t)(L + 1) * 8);
}

// Blocks of k_tanh_fb for n points: a wave per tile of 16 points, at most 1024 blocks.
static int tn_fb_blocks(int64_t n) {
    const int64_t tiles = (n + kTnPts - 1) / kTnPts;
    const int64_t blocks = (tiles + 3) / 4;
    return (int)(blocks < 1024 ? blocks : 1024);
}

template <int DIM, int NT, int L>
static void tn_fb_launch(const pdmp_tanh_net &net, const float *x, const uint8_t *y, int64_t n,
                         float *A, float *E, float *r, double *bce, hipStream_t st) {
    const int blocks = tn_fb_blocks(n);
    hipLaunchKernelGGL((k_tanh_fb<DIM, NT, L>), dim3((unsigned)blocks), dim3(kTnBlock), 0, st,
                       net.params, net.hidden, x, y, n, (float)(1.0 / (double)n), A, E, r, bce);
}

template <int DIM, int NT>
static void tn_fb_depth(const pdmp_tanh_net &net, const float *x, const uint8_t *y, int64_t n,
                        float *A, float *E, float *r, double *bce, hipStream_t st) {
    switch (net.n_hidden) {
        case 1: tn_fb_launch<DIM, NT, 1>(net, x, y, n, A, E, r, bce, st); break;
        case 2: tn_fb_launch<DIM, NT, 2>(net, x, y, n, A, E, r, bce, st); break;
        case 3: tn_fb_launch<DIM, NT, 3>(net, x, y, n, A, E, r, bce, st); break;
        default: tn_fb_launch<DIM, NT, 4>(net, x, y, n, A, E, r, bce, st); break;
    }
}

// One Adam step's state and coefficients (bc1 = 1/(1 - beta1^t), bc2 = 1/(1 - beta2^t)).
struct TnAdam {
    float *m, *v;
    float lr, b1, b2, eps, bc1, bc2;
};

// grad[j] = sum_{r < rows} part[r np + j] in the order of k_sum_rows (sixteen phases
// summing the rows r = ph mod 16 in increasing order, four loads at a time, the phases
// added in order), then the Adam step of parameter j on it (the update of k_adam).
constexpr int kTnSumPh = 16;
__global__ void __launch_bounds__(64 * kTnSumPh)
k_tanh_sum_adam(const float *__restrict__ part, int rows, int64_t np, float *__restrict__ grad,
                float *__restrict__ P, TnAdam ad) {
    __shared__ double sh[kTnSumPh][64];
    const int cl = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + cl;
    double acc = 0.0;
    if (j < np) {
        int r = ph;
        for (; r + 3 * kTnSumPh < rows; r += 4 * kTnSumPh) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = part[(size_t)(r + u * kTnSumPh) * np + j];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += v[u];
        }
        for (; r < rows; r += kTnSumPh) acc += part[(size_t)r * np + j];
    }
    sh[ph][cl] = acc;
    __syncthreads();
    if (ph != 0 || j >= np) return;
    double t = sh[0][cl];
#pragma unroll
    for (int q = 1; q < kTnSumPh; ++q) t += sh[q][cl];
    const float gk = (float)t;
    grad[j] = gk;
    const float mk = ad.b1 * ad.m[j] + (1.0f - ad.b1) * gk;
    const float vk = ad.b2 * ad.v[j] + (1.0f - ad.b2) * gk * gk;
    ad.m[j] = mk;
    ad.v[j] = vk;
    const float mh = mk * ad.bc1, vh = vk * ad.bc2;
    P[j] = P[j] - ad.lr * mh / (sqrtf(vh) + ad.eps);
}

// Loss (nullable, device [1]) and gradient (device [np]) of the fit objective at the
// current parameters, and with `ad` the Adam step on that gradient in the same pass
// over it.  `ws` holds tanh_fit_ws_bytes(net, n) bytes.
static int32_t tanh_loss_grad_step(const pdmp_tanh_net &net, const float *x, const uint8_t *y,
                                   int64_t n, float l2, float *loss, float *grad, void *ws,
                                   const TnAdam *ad, hipStream_t st) {
    const int dim = net.dim, H = net.hidden, L = net.n_hidden;
    const int64_t np = (int64_t)H * dim + H + (int64_t)(L - 1) * (H * H + H) + H + 1;
    int64_t kps;
    const int S = tn_splits(n, kps);
    char *p = (char *)ws;
    float *A = (float *)p;
    p += al256t((size_t)L * H * n * 4);
    float *E = (float *)p;
    p += al256t((size_t)L * H * n * 4);
    float *r = (float *)p;
    p += al256t((size_t)n * 4);
    float *part = (float *)p;
    p += al256t((size_t)S * np * 4);
    p += al256t((size_t)np * 4);  // spare (keeps the layout of the fit workspace)
    double *rparts = (double *)p;  // per k_tanh_fb block: the sum of its points' BCE
    p += al256t(1024 * 8);
    double *wsq = (double *)p;  // per layer: the sum of w^2 of its weight entries
    double *bce = loss ? rparts : nullptr;

#define PDMP_TNFB(D)                                                                 \
    if (H <= 16) tn_fb_depth<D, 1>(net, x, y, n, A, E, r, bce, st);                  \
    else if (H <= 32) tn_fb_depth<D, 2>(net, x, y, n, A, E, r, bce, st);             \
    else tn_fb_depth<D, 4>(net, x, y, n, A, E, r, bce, st)
    if (dim == 2) {
        PDMP_TNFB(2);
    } else {
        PDMP_TNFB(3);
    }
#undef PDMP_TNFB
    if (int32_t e = check_launch("k_tanh_fb")) return e;
    hipLaunchKernelGGL(k_tanh_wgrad, dim3((unsigned)(L + 1), (unsigned)S), dim3(256), 0, st, dim, H,
                       L, x, A, E, r, n, kps, np, net.params, l2, part, loss ? wsq : nullptr);
    if (int32_t e = check_launch("k_tanh_wgrad")) return e;
    if (ad) {
        hipLaunchKernelGGL(k_tanh_sum_adam, dim3((unsigned)((np + 63) / 64)), dim3(64 * kTnSumPh),
                           0, st, part, S, np, grad, (float *)net.params, *ad);
        if (int32_t e = check_launch("k_tanh_sum_adam")) return e;
    } else if (int32_t e = launch_sum_rows(part, S, np, 1.0, nullptr, 0.0f, grad, st)) {
        return e;
    }
    if (loss) {
        hipLaunchKernelGGL(k_tanh_loss, dim3(1), dim3(256), 0, st, rparts, tn_fb_blocks(n),
                           1.0 / (double)n, wsq, L + 1, 0.5 * (double)l2, loss);
        if (int32_t e = check_launch("k_tanh_loss")) return e;
    }
    return PDMP_OK;
}

int32_t launch_tanh_loss_grad(const pdmp_tanh_net &net, const float *x, const uint8_t *y,
                              int64_t n, float l2, float *loss, float *grad, void *ws,
                              hipStream_t st) {
    return tanh_loss_grad_step(net, x, y, n, l2, loss, grad, ws, nullptr, st);
}

// `steps` full-batch Adam steps on the fit objective; the parameters (net.params)
// are updated in place, m and v are the Adam state, the step counter continues from t0.
int32_t launch_tanh_fit(const pdmp_tanh_net &net, const float *x, const uint8_t *y, int64_t n,
                        int steps, float lr, float l2, float b1, float b2, float eps, float *m,
                        float *v, int t0, float *loss_out, void *ws, hipStream_t st) {
    const int dim = net.dim, H = net.hidden, L = net.n_hidden;
    const int64_t np = (int64_t)H * dim + H + (int64_t)(L - 1) * (H * H + H) + H + 1;
    int64_t kps;
    const int S = tn_splits(n, kps);
    char *p = (char *)ws;
    p += 2 * al256t((size_t)L * H * n * 4) + al256t((size_t)n * 4) + al256t((size_t)S * np * 4);
    float *grad = (float *)p;
    for (int t = 0; t < steps; ++t) {
        const int tt1 = t0 + t + 1;
        TnAdam ad;
        ad.m = m;
        ad.v = v;
        ad.lr = lr;
        ad.b1 = b1;
        ad.b2 = b2;
        ad.eps = eps;
        ad.bc1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)tt1)));
        ad.bc2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)tt1)));
        if (int32_t e = tanh_loss_grad_step(net, x, y, n, l2, loss_out ? loss_out + t : nullptr,
                                            grad, ws, &ad, st))
            return e;
    }
    return PDMP_OK;
}
}  // namespace pdmp
