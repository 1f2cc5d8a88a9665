// mlp.hip -- residual MLP of the amortised morph on BF16 MFMA with FP32 accumulation.
//
// q_hat = q + f(q),  f = W_L SiLU(... SiLU(W_1 q + b_1) ...) + b_L, trained by MSE
// against plain-morph targets.  Weights and activations are BF16, products are
// accumulated in FP32 (v_mfma_f32_32x32x16_bf16), biases, the residual and the
// optimiser state are FP32.
//
// Every layer product is one tiled GEMM  C[m][n] = sum_k A(m, k) B(n, k)  with
// general strides, so the same kernel serves
//   forward      Z[b][o]  = sum_i H[b][i] W[o][i]        (+ bias, SiLU epilogue)
//   data grad    dH[b][i] = sum_o dZ[b][o] W[o][i]        (x SiLU'(Z_prev) epilogue)
//   weight grad  dW[o][i] = sum_b dZ[b][o] H[b][i]        (split over b, fixed-order sum)
// Block tile 64 x 64, four waves each owning a 32 x 32 MFMA tile, K staged through
// LDS 32 at a time with rows padded so the fragment reads are conflict-light
// ds_read_b128.  Activations are sample-major [B][width].
#include "pdmp_common.h"

namespace pdmp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16_t;

__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    // round to nearest even; NaN stays NaN
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

__device__ __forceinline__ float silu_f(float z) {
    float c, sp;
    sigmoid_and_slope(z, c, sp);
    return z * c;
}

__device__ __forceinline__ float silu_grad_f(float z) {
    float c, sp;
    sigmoid_and_slope(z, c, sp);
    return c + z * sp;  // sigma (1 + z (1 - sigma))
}

enum GemmEpi { kEpiF32 = 0, kEpiHidden = 1, kEpiOut = 2, kEpiDSilu = 3 };

struct GemmArgs {
    int M = 0, N = 0, K = 0;
    const uint16_t *A = nullptr;
    int64_t a_sm = 0, a_sk = 0;
    const uint16_t *B = nullptr;
    int64_t b_sn = 0, b_sk = 0;
    int kps = 0;  // K per split (blockIdx.z)
    // epilogues
    float *c = nullptr;          // kEpiF32: c[z*M*N + m*N + n]
    const float *bias = nullptr; // kEpiHidden/kEpiOut: bias[n]
    float *zsave = nullptr;      // kEpiHidden: z[m*N + n] (nullable)
    uint16_t *hout = nullptr;    // kEpiHidden: bf16 silu(z)[m*N + n]; kEpiDSilu: bf16 out
    const float *qin = nullptr;  // kEpiOut: residual input [N][ldq] (SoA)
    float *qout = nullptr;       // kEpiOut: q + f, [N][ldq]
    int64_t ldq = 0;
    const float *zprev = nullptr; // kEpiDSilu: z of the layer below, [m*N + n]
};

constexpr int kGT = 64;      // block tile (M and N)
constexpr int kGK = 32;      // K per LDS stage
constexpr int kGPad = 8;     // row padding (bf16) against bank conflicts
constexpr int kGRow = kGK + kGPad;

// Stage a 64 x 32 (rows x k) tile of X(row, k) = X[row*s_row + k*s_k] into T[row][k]
// (row stride kGRow).  k-contiguous and row-contiguous operands use 16-byte loads
// when the whole tile is in range; anything else goes element by element.
__device__ __forceinline__ void stage_tile(const uint16_t *__restrict__ X, int64_t s_row,
                                           int64_t s_k, int rows, int r0, int k0, int ke,
                                           bool k_vec, bool r_vec, int lrow, int lseg, int kr,
                                           int rseg, uint16_t *T) {
    const bool full = r0 + kGT <= rows && k0 + kGK <= ke;
    if (full && k_vec) {
        const uint4 v = *reinterpret_cast<const uint4 *>(X + (int64_t)(r0 + lrow) * s_row + k0 + lseg);
        *reinterpret_cast<uint4 *>(&T[lrow * kGRow + lseg]) = v;
        return;
    }
    if (full && r_vec) {
        const uint4 v = *reinterpret_cast<const uint4 *>(X + (int64_t)(k0 + kr) * s_k + r0 + rseg);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            T[(rseg + 2 * j) * kGRow + kr] = (uint16_t)(w[j] & 0xffffu);
            T[(rseg + 2 * j + 1) * kGRow + kr] = (uint16_t)(w[j] >> 16);
        }
        return;
    }
    const int r = r0 + lrow;
    uint16_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = k0 + lseg + j;
        v[j] = (k < ke && r < rows) ? X[(int64_t)r * s_row + (int64_t)k * s_k] : (uint16_t)0;
    }
    uint4 p;
    p.x = v[0] | ((uint32_t)v[1] << 16);
    p.y = v[2] | ((uint32_t)v[3] << 16);
    p.z = v[4] | ((uint32_t)v[5] << 16);
    p.w = v[6] | ((uint32_t)v[7] << 16);
    *reinterpret_cast<uint4 *>(&T[lrow * kGRow + lseg]) = p;
}

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kGT * kGRow];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kGT * kGRow];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int m0 = blockIdx.x * kGT, n0 = blockIdx.y * kGT;
    const int kb = blockIdx.z * g.kps;
    const int ke = min(g.K, kb + g.kps);

    floatx16_t acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;

    const int lrow = tid >> 2;        // 0..63: tile row this thread stages
    const int lseg = (tid & 3) * 8;   // 8 consecutive k
    const int kr = tid >> 3;          // 0..31: k this thread stages (row-contiguous operands)
    const int rseg = (tid & 7) * 8;   // 8 consecutive rows
    // 16-byte loads when an operand is contiguous along k or along its rows
    const bool a_k = g.a_sk == 1 && (g.a_sm & 7) == 0 && ((uintptr_t)g.A & 15) == 0;
    const bool b_k = g.b_sk == 1 && (g.b_sn & 7) == 0 && ((uintptr_t)g.B & 15) == 0;
    const bool a_r = g.a_sm == 1 && (g.a_sk & 7) == 0 && ((uintptr_t)g.A & 15) == 0;
    const bool b_r = g.b_sn == 1 && (g.b_sk & 7) == 0 && ((uintptr_t)g.B & 15) == 0;
    for (int k0 = kb; k0 < ke; k0 += kGK) {
        stage_tile(g.A, g.a_sm, g.a_sk, g.M, m0, k0, ke, a_k, a_r, lrow, lseg, kr, rseg, As);
        stage_tile(g.B, g.b_sn, g.b_sk, g.N, n0, k0, ke, b_k, b_r, lrow, lseg, kr, rseg, Bs);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kGK; kk += 16) {
            const int ka = kk + 8 * (lane >> 5);
            const uint4 ra = *reinterpret_cast<const uint4 *>(&As[(wm * 32 + (lane & 31)) * kGRow + ka]);
            const uint4 rb = *reinterpret_cast<const uint4 *>(&Bs[(wn * 32 + (lane & 31)) * kGRow + ka]);
            bf16x8_t fa, fb;
            __builtin_memcpy(&fa, &ra, 16);
            __builtin_memcpy(&fb, &rb, 16);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb, acc, 0, 0, 0);
        }
        __syncthreads();
    }

    const int n = n0 + wn * 32 + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int m = m0 + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (m >= g.M || n >= g.N) continue;
        const float a = acc[v];
        const int64_t mn = (int64_t)m * g.N + n;
        if (EPI == kEpiF32) {
            g.c[(int64_t)blockIdx.z * g.M * g.N + mn] = a;
        } else if (EPI == kEpiHidden) {
            const float z = a + g.bias[n];
            if (g.zsave) g.zsave[mn] = z;
            g.hout[mn] = f32_to_bf16(silu_f(z));
        } else if (EPI == kEpiOut) {
            const int64_t o = (int64_t)n * g.ldq + m;  // SoA [n_out][B], m = sample
            g.qout[o] = g.qin[o] + (a + g.bias[n]);
        } else {
            g.hout[mn] = f32_to_bf16(a * silu_grad_f(g.zprev[mn]));
        }
    }
}

template <int EPI>
static int32_t launch_gemm(const GemmArgs &g, int splits, hipStream_t st) {
    if (int32_t e = grid_guard(((int64_t)g.M + kGT - 1) / kGT, 256, "k_gemm")) return e;
    dim3 grid((g.M + kGT - 1) / kGT, (g.N + kGT - 1) / kGT, splits);
    hipLaunchKernelGGL(k_gemm<EPI>, grid, dim3(256), 0, st, g);
    return check_launch("k_gemm");
}

// ---------------------------------------------------------- small kernels ---

// q [n_in][B] FP32 (SoA) -> H0 [B][n_in] BF16
__global__ void k_q_to_bf16(const float *__restrict__ q, int n_in, int64_t B, uint16_t *h0) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * n_in) return;
    const int64_t b = t / n_in;
    const int i = (int)(t - b * n_in);
    h0[t] = f32_to_bf16(q[(int64_t)i * B + b]);
}

__global__ void k_f32_to_bf16(const float *__restrict__ x, int64_t n, uint16_t *y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = f32_to_bf16(x[t]);
}

// MSE: dF[b][k] = bf16(2 u_b (q_hat - t) / (n_out B)), per-block sums of
// u_b (q_hat - t)^2, with sample weight u_b = hard_w where hard[b] != 0, else 1 (hard
// NULL: the plain MSE).
__global__ void __launch_bounds__(256)
k_mse(const float *__restrict__ qhat, const float *__restrict__ tgt, int n_out, int64_t B,
      float scale, const uint8_t *__restrict__ hard, float hard_w, uint16_t *dF, double *parts) {
    __shared__ double sh[256];
    const int64_t total = B * n_out;
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * per;
    const int64_t t1 = t0 + per < total ? t0 + per : total;
    double acc = 0.0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) {
        // t enumerates [b][k] (sample-major) so dF is written contiguously
        const int64_t b = t / n_out;
        const int k = (int)(t - b * n_out);
        const int64_t o = (int64_t)k * B + b;
        const float e = qhat[o] - tgt[o];
        const float u = (hard && hard[b]) ? hard_w : 1.0f;
        acc += (double)u * ((double)e * (double)e);
        dF[t] = f32_to_bf16(2.0f * scale * u * e);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (unsigned off = 128; off >= 1; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256)
k_final_scaled(const double *__restrict__ parts, int np, double scale, float *out) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) acc += parts[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (unsigned off = 128; off >= 1; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)(sh[0] * scale);
}

// out[j] = sum_{s < S} part[s * MN + j], fixed order; the loads go out eight at a
// time (the adds keep the order), so the sum is not a chain of dependent loads.
__global__ void k_sum_splits(const float *__restrict__ part, int S, int64_t MN, float *out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= MN) return;
    double acc = 0.0;
    int s = 0;
    for (; s + 8 <= S; s += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(s + u) * MN + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; s < S; ++s) acc += part[(int64_t)s * MN + j];
    out[j] = (float)acc;
}

// Column sums of a BF16 [B][N] matrix over the row range of blockIdx.y: 64 columns
// per block, four row phases per column combined in a fixed order; then
// k_sum_splits adds the range partials.  part[y * N + col].
__global__ void __launch_bounds__(256)
k_colsum_partial(const uint16_t *__restrict__ x, int64_t B, int N, int64_t rows_per, float *part) {
    __shared__ float sh[4][64];
    const int cl = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + cl;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per;
    const int64_t r1 = r0 + rows_per < B ? r0 + rows_per : B;
    float acc = 0.0f;
    if (col < N) {
        int64_t r = r0 + ph;
        for (; r + 28 < r1; r += 32) {  // eight loads in flight, added in row order
            uint16_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = x[(r + 4 * u) * N + col];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += bf16_to_f32(v[u]);
        }
        for (; r < r1; r += 4) acc += bf16_to_f32(x[r * N + col]);
    }
    sh[ph][cl] = acc;
    __syncthreads();
    if (ph == 0 && col < N)
        part[(int64_t)blockIdx.y * N + col] = ((sh[0][cl] + sh[1][cl]) + sh[2][cl]) + sh[3][cl];
}

// ------------------------------------------------- fused inference forward ---
//
// The inference forward of the whole network in one kernel: a block of four waves
// takes 128 samples through every layer, each wave its own 32, with the activations
// in registers.  A layer is C = W H^T on v_mfma_f32_32x32x16_bf16 (A = W rows, B =
// the samples' activations, k = input feature), so a wave's output tiles leave lane
// l holding features o = 32t + 8(v/4) + 4(l/32) + v%4 of sample l%32.  The next
// layer takes them as its B operand where they lie: its k-step s reads slot
// (s, l/32, j) as feature pi(16s + 8(l/32) + j) = 16s + 8(j/4) + 4(l/32) + j%4, which
// is accumulator value v = 8(s%2) + j of tile s/2, and its A operand reads W's
// columns in the same permuted order -- a permutation of the contraction index, so
// the sum is the same.  Every layer's BF16 weights are staged per block in LDS (rows
// padded against bank conflicts; a hidden layer of more than 4 tiles in two passes of
// output tiles, so that two blocks share a CU and one stages while the other
// computes).  Numerics as the layered path: BF16 inputs
// and activations, FP32 accumulation, bias, SiLU and residual in FP32.
constexpr int kMlpFB = 256;  // 4 waves, 128 samples; two blocks per CU

// Slot of column x (0..15) of a 16-column block in the A fragments: lane half h reads
// slots 8h .. 8h + 7, which must hold columns pi(8h + j) = 8(j/4) + 4h + j%4, so the
// block's quads (4 columns) sit in the order 0, 2, 1, 3.
__device__ __forceinline__ int mlp_slot(int x) { return ((x >> 2) & 1) * 8 + (x >> 3) * 4 + (x & 3); }

template <int TH>
__global__ void __launch_bounds__(kMlpFB) __attribute__((amdgpu_waves_per_eu(2)))
k_mlp_fused(const uint16_t *__restrict__ wbf, const float *__restrict__ par, int n_in, int L,
            const float *__restrict__ q, int64_t B, float *__restrict__ qhat) {
    constexpr int H = 32 * TH, KH = 2 * TH, LROW = H + 8;
    // hidden layers in passes of TP output tiles, so that two blocks fit in a CU's LDS
    constexpr int TP = TH > 4 ? (TH + 1) / 2 : TH;
    constexpr int WROWS = 32 * TP > 16 ? 32 * TP : 16;
    static_assert(WROWS * LROW >= 16 * H, "room for the first layer's weights");
    __shared__ __attribute__((aligned(16))) uint16_t Ws[WROWS * LROW];
    __shared__ __attribute__((aligned(16))) float bs[H];  // the layer's bias
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6, hh = lane >> 5, r = lane & 31;
    const int64_t n = (int64_t)blockIdx.x * (kMlpFB / 2) + wv * 32 + r;
    const bool live = n < B;
    // layout offsets (as the host's): layer 0 [H][n_in] + H, hidden [H][H] + H, last
    // [n_in][H] + n_in
    const int64_t w1 = (int64_t)H * n_in + H;
    auto woff = [&](int l) -> int64_t {
        return l == 0 ? 0 : w1 + (int64_t)(l - 1) * ((int64_t)H * H + H);
    };
    auto boff = [&](int l) -> int64_t {
        return woff(l) + (l == 0 ? (int64_t)H * n_in : (l == L - 1 ? (int64_t)n_in * H : (int64_t)H * H));
    };
    auto frag = [&](int row, int sk) {  // the A fragment of row, k-step sk, this lane's half
        bf16x8_t a;
        const uint4 w4 = *reinterpret_cast<const uint4 *>(&Ws[row * LROW + 16 * sk + 8 * hh]);
        __builtin_memcpy(&a, &w4, 16);
        return a;
    };
    // layer 0: W_0 [H][n_in] into rows of 16 (zero past n_in), k = column directly
    for (int e = tid; e < H * 16; e += kMlpFB) {
        const int row = e >> 4, c = e & 15;
        Ws[row * 16 + c] = c < n_in ? wbf[(int64_t)row * n_in + c] : (uint16_t)0;
    }
    for (int e = tid; e < H; e += kMlpFB) bs[e] = par[boff(0) + e];
    // its B operand: bf16(q[8hh + j][n]), zero past n_in
    bf16x8_t b0;
    {
        uint16_t u[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int f = 8 * hh + j;
            u[j] = (live && f < n_in) ? f32_to_bf16(q[(int64_t)f * B + n]) : (uint16_t)0;
        }
        __builtin_memcpy(&b0, u, 16);
    }
    __syncthreads();
    floatx16_t acc[TH];
#pragma unroll
    for (int t = 0; t < TH; ++t) {
        bf16x8_t a;
        const uint4 w4 = *reinterpret_cast<const uint4 *>(&Ws[(32 * t + r) * 16 + 8 * hh]);
        __builtin_memcpy(&a, &w4, 16);
        floatx16_t z = {};
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, z, 0, 0, 0);
    }
    bf16x8_t hb[KH];
    // bias (from bs) + SiLU, into the next layer's B operands (slot j of k-step
    // 2t + v/8 = v%8); biases o .. o + 3 of a quad are one 16-byte LDS read
    auto epilogue = [&]() {
#pragma unroll
        for (int t = 0; t < TH; ++t)
#pragma unroll
            for (int u8 = 0; u8 < 2; ++u8) {
                uint16_t u[8];
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    const int v0 = 8 * u8 + 4 * g;
                    const float4 b4 =
                        *reinterpret_cast<const float4 *>(&bs[32 * t + 8 * (v0 >> 2) + 4 * hh]);
                    const float bb[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        u[4 * g + i] = f32_to_bf16(silu_f(acc[t][v0 + i] + bb[i]));
                }
                __builtin_memcpy(&hb[2 * t + u8], u, 16);
            }
    };
    epilogue();
    // stage rows [0, rows) of a row-major [rows][H] weight matrix with each 16-column
    // block's quads in fragment order (8-byte moves)
    auto stage = [&](const uint16_t *__restrict__ W, int rows, const float *__restrict__ bias) {
        __syncthreads();  // every wave is done with the previous contents
        if (bias)
            for (int e = tid; e < H; e += kMlpFB) bs[e] = bias[e];
        const int nq = rows * (H / 4);
#pragma unroll 8
        for (int e = tid; e < nq; e += kMlpFB) {
            const int row = e / (H / 4), q4 = e - row * (H / 4);
            const int col = 4 * q4;
            const uint2 v = *reinterpret_cast<const uint2 *>(W + (int64_t)row * H + col);
            *reinterpret_cast<uint2 *>(&Ws[row * LROW + (col & ~15) + mlp_slot(col & 15)]) = v;
        }
        __syncthreads();
    };
    for (int l = 1; l < L - 1; ++l) {
#pragma unroll
        for (int t = 0; t < TH; ++t)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[t][v] = 0.0f;
#pragma unroll
        for (int t0 = 0; t0 < TH; t0 += TP) {
            const int nt = TH - t0 < TP ? TH - t0 : TP;
            stage(wbf + woff(l) + (int64_t)32 * t0 * H, 32 * nt, t0 == 0 ? par + boff(l) : nullptr);
#pragma unroll
            for (int sk = 0; sk < KH; ++sk)
#pragma unroll
                for (int t = t0; t < t0 + TP && t < TH; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        frag(32 * (t - t0) + r, sk), hb[sk], acc[t], 0, 0, 0);
        }
        epilogue();
    }
    // last layer: W_L [n_in][H] (rows past n_in read as zero)
    stage(wbf + woff(L - 1), n_in, nullptr);
    floatx16_t out = {};
    const bf16x8_t zero8 = {};
#pragma unroll
    for (int sk = 0; sk < KH; ++sk)
        out = __builtin_amdgcn_mfma_f32_32x32x16_bf16(r < n_in ? frag(r, sk) : zero8, hb[sk], out,
                                                      0, 0, 0);
    if (!live) return;
    const float *bL = par + boff(L - 1);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int f = 8 * (v >> 2) + 4 * hh + (v & 3);
        if (f < n_in) {
            const int64_t o = (int64_t)f * B + n;
            qhat[o] = q[o] + (out[v] + bL[f]);
        }
    }
}

// ------------------------------------------------------------------ host ---

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct MlpLayout {
    int L, n_in, H;
    int in(int l) const { return l == 0 ? n_in : H; }
    int out(int l) const { return l == L - 1 ? n_in : H; }
    int64_t woff(int l) const {
        int64_t o = 0;
        for (int k = 0; k < l; ++k) o += (int64_t)out(k) * in(k) + out(k);
        return o;
    }
    int64_t boff(int l) const { return woff(l) + (int64_t)out(l) * in(l); }
    int64_t nparams() const { return woff(L); }
};

static MlpLayout layout_of(const pdmp_mlp &m) { return MlpLayout{m.n_hidden + 1, m.n_in, m.hidden}; }

int64_t mlp_nparams(const pdmp_mlp &m) { return layout_of(m).nparams(); }

// Activations kept by a training forward: H0 bf16 [B][n_in]; for l < L-1:
// Z_l f32 [B][H] and H_l bf16 [B][H].
size_t mlp_acts_bytes(const pdmp_mlp &m, int64_t B) {
    const MlpLayout ly = layout_of(m);
    size_t b = al256((size_t)B * ly.n_in * 2);
    for (int l = 0; l < ly.L - 1; ++l) b += al256((size_t)B * ly.H * 4) + al256((size_t)B * ly.H * 2);
    return b;
}

struct ActPtrs {
    uint16_t *h0;
    float *z[8];
    uint16_t *h[8];
};

static ActPtrs act_ptrs(const MlpLayout &ly, void *acts, int64_t B) {
    ActPtrs p{};
    char *c = (char *)acts;
    p.h0 = (uint16_t *)c;
    c += al256((size_t)B * ly.n_in * 2);
    for (int l = 0; l < ly.L - 1; ++l) {
        p.z[l] = (float *)c;
        c += al256((size_t)B * ly.H * 4);
        p.h[l] = (uint16_t *)c;
        c += al256((size_t)B * ly.H * 2);
    }
    return p;
}

// Inference-only forward keeps two BF16 activation buffers.
size_t mlp_fwd_ws_bytes(const pdmp_mlp &m, int64_t B) {
    const MlpLayout ly = layout_of(m);
    return al256((size_t)B * ly.n_in * 2) + 2 * al256((size_t)B * ly.H * 2);
}

int32_t launch_mlp_forward(const pdmp_mlp &m, const float *q, int64_t B, float *qhat, void *acts,
                           void *ws, hipStream_t st) {
    const MlpLayout ly = layout_of(m);
    if (!acts && ly.H % 32 == 0 && ly.H <= 256 && ly.n_in <= 16 && ly.L >= 2 &&
        ((uintptr_t)m.params_bf16 & 15) == 0) {
        // inference only: the fused kernel (no workspace used)
        if (int32_t e = grid_guard((B + kMlpFB / 2 - 1) / (kMlpFB / 2), kMlpFB, "k_mlp_fused"))
            return e;
        const dim3 grid((unsigned)((B + kMlpFB / 2 - 1) / (kMlpFB / 2)));
        switch (ly.H / 32) {
#define PDMP_FUSED(TH)                                                                          \
    case TH:                                                                                    \
        hipLaunchKernelGGL(k_mlp_fused<TH>, grid, dim3(kMlpFB), 0, st, m.params_bf16, m.params, \
                           ly.n_in, ly.L, q, B, qhat);                                          \
        break;
            PDMP_FUSED(1) PDMP_FUSED(2) PDMP_FUSED(3) PDMP_FUSED(4)
            PDMP_FUSED(5) PDMP_FUSED(6) PDMP_FUSED(7) PDMP_FUSED(8)
#undef PDMP_FUSED
        }
        return check_launch("k_mlp_fused");
    }
    uint16_t *h0, *hb[2];
    float *zs[8] = {nullptr};
    uint16_t *hs[8] = {nullptr};
    if (acts) {
        ActPtrs p = act_ptrs(ly, acts, B);
        h0 = p.h0;
        for (int l = 0; l < ly.L - 1; ++l) {
            zs[l] = p.z[l];
            hs[l] = p.h[l];
        }
    } else {
        char *c = (char *)ws;
        h0 = (uint16_t *)c;
        c += al256((size_t)B * ly.n_in * 2);
        hb[0] = (uint16_t *)c;
        c += al256((size_t)B * ly.H * 2);
        hb[1] = (uint16_t *)c;
        for (int l = 0; l < ly.L - 1; ++l) hs[l] = hb[l & 1];
    }
    if (int32_t e = grid_guard((B * ly.n_in + 255) / 256, 256, "k_q_to_bf16")) return e;
    hipLaunchKernelGGL(k_q_to_bf16, dim3((unsigned)((B * ly.n_in + 255) / 256)), dim3(256), 0, st, q,
                       ly.n_in, B, h0);
    if (int32_t e = check_launch("k_q_to_bf16")) return e;
    const uint16_t *hin = h0;
    for (int l = 0; l < ly.L; ++l) {
        GemmArgs g;
        g.M = (int)B;
        g.N = ly.out(l);
        g.K = ly.in(l);
        g.A = hin;
        g.a_sm = ly.in(l);
        g.a_sk = 1;
        g.B = m.params_bf16 + ly.woff(l);
        g.b_sn = ly.in(l);
        g.b_sk = 1;
        g.kps = g.K;
        g.bias = m.params + ly.boff(l);
        int32_t e;
        if (l < ly.L - 1) {
            g.zsave = zs[l];
            g.hout = hs[l];
            e = launch_gemm<kEpiHidden>(g, 1, st);
            hin = hs[l];
        } else {
            g.qin = q;
            g.qout = qhat;
            g.ldq = B;
            e = launch_gemm<kEpiOut>(g, 1, st);
        }
        if (e) return e;
    }
    return PDMP_OK;
}

static int wgrad_splits(int64_t B) {
    int64_t s = B / 2048;
    if (s < 1) s = 1;
    if (s > 64) s = 64;
    return (int)s;
}

size_t mlp_bwd_ws_bytes(const pdmp_mlp &m, int64_t B) {
    const MlpLayout ly = layout_of(m);
    const int S = wgrad_splits(B);
    const int64_t rows_per = 256;
    const int64_t cs = (B + rows_per - 1) / rows_per;
    const int wmax = ly.H > ly.n_in ? ly.H : ly.n_in;
    return 2 * al256((size_t)B * wmax * 2) + al256((size_t)S * wmax * wmax * 4) +
           al256((size_t)cs * wmax * 4) + al256(1024 * sizeof(double));
}

// Backward of the MSE loss through the whole network from saved activations.
// grad: FP32 [nparams] in the flat layout; loss (nullable): device [1].
int32_t launch_mlp_backward(const pdmp_mlp &m, const float *qhat, const float *target, int64_t B,
                            void *acts, float *grad, float *loss, void *ws, hipStream_t st,
                            const uint8_t *hard, float hard_w) {
    const MlpLayout ly = layout_of(m);
    ActPtrs ap = act_ptrs(ly, acts, B);
    const int S = wgrad_splits(B);
    const int64_t rows_per = 256;
    const int cs = (int)((B + rows_per - 1) / rows_per);
    const int wmax = ly.H > ly.n_in ? ly.H : ly.n_in;
    char *c = (char *)ws;
    uint16_t *dz[2];
    dz[0] = (uint16_t *)c;
    c += al256((size_t)B * wmax * 2);
    dz[1] = (uint16_t *)c;
    c += al256((size_t)B * wmax * 2);
    float *part = (float *)c;
    c += al256((size_t)S * wmax * wmax * 4);
    float *cpart = (float *)c;
    c += al256((size_t)cs * wmax * 4);
    double *rparts = (double *)c;

    const int nb = 1024;
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, qhat, target, ly.n_in, B,
                       (float)(1.0 / ((double)ly.n_in * (double)B)), hard, hard_w, dz[0], rparts);
    if (loss)
        hipLaunchKernelGGL(k_final_scaled, dim3(1), dim3(256), 0, st, rparts, nb,
                           1.0 / ((double)ly.n_in * (double)B), loss);
    if (int32_t e = check_launch("k_mse")) return e;

    int cur = 0;
    for (int l = ly.L - 1; l >= 0; --l) {
        const int O = ly.out(l), I = ly.in(l);
        const uint16_t *hin = l == 0 ? ap.h0 : ap.h[l - 1];
        // dW_l[o][i] = sum_b dZ[b][o] H_{l-1}[b][i], split over b
        GemmArgs gw;
        gw.M = O;
        gw.N = I;
        gw.K = (int)B;
        gw.A = dz[cur];
        gw.a_sm = 1;
        gw.a_sk = O;
        gw.B = hin;
        gw.b_sn = 1;
        gw.b_sk = I;
        gw.kps = (int)(((B + S - 1) / S + kGK - 1) / kGK * kGK);
        const int splits = (int)((B + gw.kps - 1) / gw.kps);
        gw.c = part;
        if (int32_t e = launch_gemm<kEpiF32>(gw, splits, st)) return e;
        hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)(((int64_t)O * I + 255) / 256)), dim3(256), 0,
                           st, part, splits, (int64_t)O * I, grad + ly.woff(l));
        // db_l[o] = sum_b dZ[b][o]
        hipLaunchKernelGGL(k_colsum_partial, dim3((O + 63) / 64, cs), dim3(256), 0, st, dz[cur], B,
                           O, rows_per, cpart);
        hipLaunchKernelGGL(k_sum_splits, dim3((O + 255) / 256), dim3(256), 0, st, cpart, cs,
                           (int64_t)O, grad + ly.boff(l));
        if (int32_t e = check_launch("mlp wgrad")) return e;
        if (l == 0) break;
        // dZ_{l-1}[b][i] = (sum_o dZ[b][o] W_l[o][i]) * SiLU'(Z_{l-1}[b][i])
        GemmArgs gd;
        gd.M = (int)B;
        gd.N = I;
        gd.K = O;
        gd.A = dz[cur];
        gd.a_sm = O;
        gd.a_sk = 1;
        gd.B = m.params_bf16 + ly.woff(l);
        gd.b_sn = 1;
        gd.b_sk = I;
        gd.kps = O;
        gd.hout = dz[cur ^ 1];
        gd.zprev = ap.z[l - 1];
        if (int32_t e = launch_gemm<kEpiDSilu>(gd, 1, st)) return e;
        cur ^= 1;
    }
    return PDMP_OK;
}

int32_t launch_f32_to_bf16(const float *x, int64_t n, uint16_t *y, hipStream_t st) {
    if (int32_t e = grid_guard((n + 255) / 256, 256, "k_f32_to_bf16")) return e;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, y);
    return check_launch("k_f32_to_bf16");
}

}  // namespace pdmp
