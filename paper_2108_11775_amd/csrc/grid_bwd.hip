// grid_bwd.hip -- the weight gradient Phi^T g of the occupancy logit (Sec. 3.1: the
// gradient of the BCE fit, and the backward of s with respect to w) for hinges on a
// regular grid, as a dense FP32 MFMA product with the points as contraction index.
//
// With phi_m(x) = ex_a(x) ey_b(y) [ez_c(z)] for m = a + G0 (b + G1 c):
//   2-D:  grad[b][a]    = sum_i (g_i ey_b(y_i)) ex_a(x_i)
//         -- one G1 x G0 product, A = g ey (rows b, k = point), B = ex (k = point,
//            columns a), on v_mfma_f32_32x32x2_f32 (two points per instruction);
//   3-D:  grad[c][b][a] = sum_i (g_i ez_c(z_i) ey_b(y_i)) ex_a(x_i)
//         -- one 16 x 16 product per z-plane c on v_mfma_f32_16x16x4_f32 (four
//            points per instruction), all planes sharing the B operand.
// Per point that costs G0 + G1 (+ G2) exponentials instead of G0 G1 (G2).  A block
// stages 256 points per round in LDS (prescaled coordinates and g; in 3-D also the
// G2 products g ez_c); every lane then builds the operand entries of its own
// (point, row) and (point, column), so no exponential is evaluated twice.  Each
// block sums a contiguous range of rounds into one partial row (its four waves added
// in a fixed order through LDS); the rows are summed in a fixed order afterwards,
// so the result is deterministic.
#include "pdmp_common.h"

namespace pdmp {

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_wg;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_wg;

constexpr int kWgBlock = 256;      // threads per block = points per round
constexpr int kWgMaxRows = 512;    // partial rows (blocks) at most
constexpr int kWg3Planes = 16;     // z-planes of the 3-D kernel (G2)

// Blocks and rounds per block for n points: every block gets the same number of
// rounds (the last one fewer), and no block is empty.
__host__ __device__ inline void wgrad_split(int64_t n, int &blocks, int &rpb) {
    const int64_t R = (n + kWgBlock - 1) / kWgBlock;
    if (R == 0) {
        blocks = 1;
        rpb = 0;
        return;
    }
    const int64_t b = R < kWgMaxRows ? R : kWgMaxRows;
    const int64_t r = (R + b - 1) / b;
    rpb = (int)r;
    blocks = (int)((R + r - 1) / r);
}

size_t wgrad_rows_max(int64_t n) {
    int b, r;
    wgrad_split(n, b, r);
    return (size_t)b;
}

// Load point i (or a zero-weight dummy past the end).
template <int DIM>
__device__ __forceinline__ void wg_load(const float *__restrict__ x, const float *__restrict__ g,
                                        int64_t n, int64_t i, float &px, float &py, float &pz,
                                        float &pg) {
    if (i < n) {
        px = x[i];
        py = x[(size_t)n + i];
        pz = DIM == 3 ? x[2 * (size_t)n + i] : 0.0f;
        pg = g[i];
    } else {
        px = py = pz = pg = 0.0f;
    }
}

template <int TA, int TB>
__global__ void __launch_bounds__(kWgBlock)
k_wgrad2d(const float *__restrict__ hinges, int g0, int g1, float kappa,
          const float *__restrict__ x, const float *__restrict__ g, int64_t n, int rpb,
          float *__restrict__ part) {
    constexpr int RA = 32 * TA;  // padded row length of the block sum
    __shared__ float sx[2][kWgBlock], sy[2][kWgBlock], sg[2][kWgBlock];
    __shared__ float red[32 * TB * RA];
    const int tid = threadIdx.x, lane = tid & 63, half = lane >> 5, wv = tid >> 6;
    const int M = g0 * g1;

    float ax[TA], ay[TB];
    bool va[TA], vb[TB];
#pragma unroll
    for (int t = 0; t < TA; ++t) {
        const int a = 32 * t + (lane & 31);
        va[t] = a < g0;
        ax[t] = 0.0f;
        if (va[t]) ax[t] = kappa * hinges[a];
    }
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const int b = 32 * t + (lane & 31);
        vb[t] = b < g1;
        ay[t] = 0.0f;
        if (vb[t]) ay[t] = kappa * hinges[(size_t)M + (size_t)g0 * b];
    }

    f32x16_wg acc[TB][TA];
#pragma unroll
    for (int tb = 0; tb < TB; ++tb)
#pragma unroll
        for (int ta = 0; ta < TA; ++ta)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[tb][ta][v] = 0.0f;

    const int64_t R = (n + kWgBlock - 1) / kWgBlock;
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = r0 + rpb < R ? r0 + rpb : R;
    float px, py, pz, pg;
    wg_load<2>(x, g, n, r0 * kWgBlock + tid, px, py, pz, pg);
    int buf = 0;
    for (int64_t r = r0; r < r1; ++r, buf ^= 1) {
        sx[buf][tid] = kappa * px;
        sy[buf][tid] = kappa * py;
        sg[buf][tid] = pg;
        __syncthreads();
        if (r + 1 < r1) wg_load<2>(x, g, n, (r + 1) * kWgBlock + tid, px, py, pz, pg);
        const float *bx = sx[buf] + 64 * wv + half, *by = sy[buf] + 64 * wv + half,
                    *bg = sg[buf] + 64 * wv + half;
#pragma unroll 4
        for (int kk = 0; kk < 32; ++kk) {
            const float xs = bx[2 * kk], ys = by[2 * kk], gv = bg[2 * kk];
            float bv[TA], av[TB];
#pragma unroll
            for (int t = 0; t < TA; ++t) {
                const float d = xs - ax[t];
                bv[t] = va[t] ? exp2_fast(-d * d) : 0.0f;
            }
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const float d = ys - ay[t];
                av[t] = vb[t] ? gv * exp2_fast(-d * d) : 0.0f;
            }
#pragma unroll
            for (int tb = 0; tb < TB; ++tb)
#pragma unroll
                for (int ta = 0; ta < TA; ++ta)
                    acc[tb][ta] =
                        __builtin_amdgcn_mfma_f32_32x32x2f32(av[tb], bv[ta], acc[tb][ta], 0, 0, 0);
        }
    }

    // Block sum in wave order: red = ((w0 + w1) + w2) + w3.
    for (int w = 0; w < 4; ++w) {
        if (wv == w) {
#pragma unroll
            for (int tb = 0; tb < TB; ++tb)
#pragma unroll
                for (int ta = 0; ta < TA; ++ta)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int b = 32 * tb + 8 * (v >> 2) + 4 * half + (v & 3);
                        const int a = 32 * ta + (lane & 31);
                        float &dst = red[b * RA + a];
                        dst = w == 0 ? acc[tb][ta][v] : dst + acc[tb][ta][v];
                    }
        }
        __syncthreads();
    }
    float *out = part + (size_t)blockIdx.x * M;
    for (int m = tid; m < M; m += kWgBlock) out[m] = red[(m / g0) * RA + m % g0];
}

template <int NC>
__global__ void __launch_bounds__(kWgBlock)
k_wgrad3d(const float *__restrict__ hinges, int g0, int g1, int g2, float kappa,
          const float *__restrict__ x, const float *__restrict__ g, int64_t n, int rpb,
          float *__restrict__ part) {
    static_assert(NC % 4 == 0, "planes in groups of four");
    __shared__ float sx[2][kWgBlock], sy[2][kWgBlock];
    __shared__ float4 sz[2][kWgBlock][NC / 4];  // g ez_c of each staged point
    __shared__ float red[NC * 256];
    __shared__ float az[NC];
    const int tid = threadIdx.x, lane = tid & 63, q = lane >> 4, wv = tid >> 6;
    const int M = g0 * g1 * g2;
    if (tid < NC) {
        float v = 0.0f;
        if (tid < g2) v = kappa * hinges[2 * (size_t)M + (size_t)g0 * g1 * tid];
        az[tid] = v;
    }

    const int a = lane & 15, b = lane & 15;
    const bool va = a < g0, vb = b < g1;
    float ax = 0.0f, ay = 0.0f;
    if (va) ax = kappa * hinges[a];
    if (vb) ay = kappa * hinges[(size_t)M + (size_t)g0 * b];

    f32x4_wg acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[c][v] = 0.0f;

    const int64_t R = (n + kWgBlock - 1) / kWgBlock;
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = r0 + rpb < R ? r0 + rpb : R;
    float px, py, pz, pg;
    wg_load<3>(x, g, n, r0 * kWgBlock + tid, px, py, pz, pg);
    __syncthreads();  // az
    int buf = 0;
    for (int64_t r = r0; r < r1; ++r, buf ^= 1) {
        sx[buf][tid] = kappa * px;
        sy[buf][tid] = kappa * py;
        const float zs = kappa * pz;
#pragma unroll
        for (int c4 = 0; c4 < NC / 4; ++c4) {
            float e[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = 4 * c4 + u;
                const float d = zs - az[c];
                e[u] = c < g2 ? pg * exp2_fast(-d * d) : 0.0f;
            }
            sz[buf][tid][c4] = make_float4(e[0], e[1], e[2], e[3]);
        }
        __syncthreads();
        if (r + 1 < r1) wg_load<3>(x, g, n, (r + 1) * kWgBlock + tid, px, py, pz, pg);
#pragma unroll 2
        for (int kk = 0; kk < 16; ++kk) {
            const int p = 64 * wv + 4 * kk + q;
            const float dx = sx[buf][p] - ax, dy = sy[buf][p] - ay;
            const float bv = va ? exp2_fast(-dx * dx) : 0.0f;
            const float ey = vb ? exp2_fast(-dy * dy) : 0.0f;
#pragma unroll
            for (int c4 = 0; c4 < NC / 4; ++c4) {
                const float4 z4 = sz[buf][p][c4];
                acc[4 * c4 + 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(z4.x * ey, bv, acc[4 * c4 + 0], 0, 0, 0);
                acc[4 * c4 + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(z4.y * ey, bv, acc[4 * c4 + 1], 0, 0, 0);
                acc[4 * c4 + 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(z4.z * ey, bv, acc[4 * c4 + 2], 0, 0, 0);
                acc[4 * c4 + 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(z4.w * ey, bv, acc[4 * c4 + 3], 0, 0, 0);
            }
        }
    }

    // Accumulator layout of the 16 x 16 tile of plane c: lane l, entry v holds
    // row b = 4 (l/16) + v, column a = l % 16.  Block sum in wave order.
    for (int w = 0; w < 4; ++w) {
        if (wv == w) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float &dst = red[c * 256 + (4 * q + v) * 16 + a];
                    dst = w == 0 ? acc[c][v] : dst + acc[c][v];
                }
        }
        __syncthreads();
    }
    float *out = part + (size_t)blockIdx.x * M;
    for (int m = tid; m < M; m += kWgBlock) {
        const int ia = m % g0, ib = (m / g0) % g1, ic = m / (g0 * g1);
        out[m] = red[ic * 256 + ib * 16 + ia];
    }
}

// Partial rows of Phi^T g for hinges on `grid`; returns PDMP_EUNSUPPORTED (without
// launching) when the grid does not fit the kernels, else the number of rows.
int32_t launch_grid_wgrad(int dim, const float *hinges, int M, const int *grid, float kappa,
                          const float *x, int64_t n, const float *g, float *part, int *rows,
                          hipStream_t st) {
    if (!grid || grid[0] < 1 || grid[1] < 1) return PDMP_EUNSUPPORTED;
    int blocks, rpb;
    wgrad_split(n, blocks, rpb);
    const int g0 = grid[0], g1 = grid[1];
    if (dim == 2) {
        if (g0 > 64 || g1 > 64 || g0 * g1 != M) return PDMP_EUNSUPPORTED;
#define PDMP_WG2(TA, TB)                                                                      \
    hipLaunchKernelGGL((k_wgrad2d<TA, TB>), dim3(blocks), dim3(kWgBlock), 0, st, hinges, g0, g1, \
                       kappa, x, g, n, rpb, part)
        if (g0 <= 32 && g1 <= 32) PDMP_WG2(1, 1);
        else if (g0 <= 32) PDMP_WG2(1, 2);
        else if (g1 <= 32) PDMP_WG2(2, 1);
        else PDMP_WG2(2, 2);
#undef PDMP_WG2
    } else {
        const int g2 = grid[2];
        if (g0 > 16 || g1 > 16 || g2 < 1 || g2 > kWg3Planes || g0 * g1 * g2 != M)
            return PDMP_EUNSUPPORTED;
        hipLaunchKernelGGL((k_wgrad3d<kWg3Planes>), dim3(blocks), dim3(kWgBlock), 0, st, hinges, g0,
                           g1, g2, kappa, x, g, n, rpb, part);
    }
    *rows = blocks;
    return check_launch("k_wgrad");
}

}  // namespace pdmp
