// occupancy.hip -- RBF logistic occupancy (value, input gradient) and the fused
// T-step explicit-Euler workspace morph, for gfx950.
//
// Occupancy (Sec. 3.1, Hilbert-map form): s(x) = sum_j w_j exp(-|x-h_j|^2/(2 l^2)) + beta,
// c = sigma(s), grad c = sigma'(s) grad s, grad s = -(1/l^2) sum_j w_j phi_j (x - h_j).
// Morph (Sec. 3.2, Eq. 1 by Euler's method): x <- x - eta * grad c(x), T times.
//
// Mapping.  The work is FP32 VALU + v_exp_f32 bound (one exp and 3*DIM+2 VALU per
// sample-hinge pair), not HBM bound: samples stream in once and out once.
//   * Hinges live in LDS for the whole launch when they fit (64 KiB: 4096 3-D or
//     5460 2-D hinges), staged as chunks of four: DIM float4 rows of prescaled
//     coordinates kappa*h and one float4 of weights, so every ds_read_b128 is a
//     wave-wide broadcast that feeds four hinges.  Larger hinge sets are streamed
//     through LDS tile by tile inside each step.
//   * Coordinates are prescaled by kappa = sqrt(log2(e)/(2 l^2)) so that
//     phi = exp2(-|kappa x - kappa h|^2) needs no multiply before v_exp_f32.
//   * G lanes share one sample (G = 1 for large batches, 4 or 16 for small ones);
//     each lane sums a strided subset of hinge chunks and the G partial sums are
//     combined by an xor butterfly, which leaves bit-identical totals in all G
//     lanes, so their redundant copies of the state stay equal.
//   * With G = 1 each lane carries SPL samples for instruction-level parallelism.
//   * The T-step loop runs in registers; the state touches HBM only at the ends.
#include "pdmp_common.h"

namespace pdmp {

// Copy hinge chunks [c0, c0 + nc) into LDS, prescaled, zero-padded past M.
template <int DIM>
__device__ __forceinline__ void stage_chunks(float4 *lds, const float *__restrict__ hinges,
                                             const float *__restrict__ weights, int M,
                                             float kappa, int c0, int nc) {
    constexpr int R = DIM + 1;
    float *f = reinterpret_cast<float *>(lds);
    for (int idx = threadIdx.x; idx < nc * 4; idx += blockDim.x) {
        int c = idx >> 2, u = idx & 3;
        int j = (c0 + c) * 4 + u;
        bool ok = j < M;
        float *row = f + (size_t)c * R * 4;
#pragma unroll
        for (int k = 0; k < DIM; ++k) row[k * 4 + u] = ok ? kappa * hinges[(size_t)k * M + j] : 0.0f;
        row[DIM * 4 + u] = ok ? weights[j] : 0.0f;
    }
}

// Accumulate one chunk of four hinges into SPL samples' sums.
template <int DIM, int SPL>
__device__ __forceinline__ void chunk_accumulate(const float4 *__restrict__ ch,
                                                 const float (&xs)[SPL][DIM], float (&as)[SPL],
                                                 float (&ag)[SPL][DIM]) {
    float4 hc[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) hc[k] = ch[k];
    const float4 wv = ch[DIM];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            float d[DIM];
            d[0] = xs[s][0] - f4c(hc[0], u);
            float r2 = d[0] * d[0];
#pragma unroll
            for (int k = 1; k < DIM; ++k) {
                d[k] = xs[s][k] - f4c(hc[k], u);
                r2 = fmaf(d[k], d[k], r2);
            }
            const float wp = f4c(wv, u) * exp2_fast(-r2);
            as[s] += wp;
#pragma unroll
            for (int k = 0; k < DIM; ++k) ag[s][k] = fmaf(wp, d[k], ag[s][k]);
        }
    }
}

template <int G>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// MODE kEval   : c_out[n] (nullable), s_out[n] (nullable).  With gridDim.y > 1 the
//                hinge chunks are split into ranges of `cps` chunks, block row y sums
//                range y only and writes s_out[y*n + i] (partial sums, no bias).
// MODE kGrad   : c_out[n] (nullable), g_out[DIM][n] = sigma'(s) grad s
// MODE kGradBwd: g_out[DIM][n] = g_in[i] * (chain ? sigma'(s) : 1) * grad s
// MODE kMorph  : x_out[DIM][n] after T steps (x_out may equal x_in)
// The bias is *bias_ptr (nullable: no bias).
template <int DIM, int SPL, int G, int BLOCK, int MODE>
__global__ void __launch_bounds__(BLOCK)
k_rbf(const float *__restrict__ hinges, const float *__restrict__ weights, int M,
      const float *__restrict__ bias_ptr, float kappa, float gscale, const float *x_in, int64_t n,
      int T, float eta, float *c_out, float *s_out, float *g_out, float *x_out,
      const float *__restrict__ g_in, int chain, int cps, Traj tr) {
    static_assert(G == 1 || SPL == 1, "lane groups carry one sample");
    constexpr int R = DIM + 1;
    constexpr int TILE = tile_chunks<DIM>();
    extern __shared__ float4 lds[];

    const int nchunks_all = chunks_for(M);
    const int cbeg = (int)blockIdx.y * cps;                  // this block row's hinge chunks
    const int nchunks = min(cps, nchunks_all - cbeg);
    const int ntiles = (nchunks + TILE - 1) / TILE;
    const int lg = threadIdx.x % G;
    constexpr int GPB = BLOCK / G;  // sample groups per block
    const int64_t base = (int64_t)blockIdx.x * GPB * SPL + threadIdx.x / G;

    int64_t idx[SPL];
    float x[SPL][DIM];
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
        idx[s] = base + (int64_t)s * GPB;
        const int64_t i = idx[s] < n ? idx[s] : n - 1;  // tail lanes shadow a valid sample
#pragma unroll
        for (int k = 0; k < DIM; ++k) x[s][k] = x_in[(size_t)k * n + i];
    }
    const float beta = bias_ptr ? *bias_ptr : 0.0f;

    if (ntiles == 1) {
        stage_chunks<DIM>(lds, hinges, weights, M, kappa, cbeg, nchunks);
        __syncthreads();
    }

    const int steps = (MODE == kMorph) ? T : 1;
    int64_t tc[SPL];
    bool rec[SPL];
#pragma unroll
    for (int s = 0; s < SPL; ++s) rec[s] = MODE == kMorph && lg == 0 && traj_col(tr, idx[s], n, tc[s]);
    float as[SPL], ag[SPL][DIM];
    for (int t = 0; t < steps; ++t) {
#pragma unroll
        for (int s = 0; s < SPL; ++s)
            if (rec[s]) traj_put<DIM>(tr, t, tc[s], x[s]);
        float xs[SPL][DIM];
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            as[s] = 0.0f;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                xs[s][k] = kappa * x[s][k];
                ag[s][k] = 0.0f;
            }
        }
        for (int tile = 0; tile < ntiles; ++tile) {
            const int c0 = tile * TILE;
            const int nc = min(TILE, nchunks - c0);
            if (ntiles > 1) {
                __syncthreads();
                stage_chunks<DIM>(lds, hinges, weights, M, kappa, cbeg + c0, nc);
                __syncthreads();
            }
            for (int c = lg; c < nc; c += G) chunk_accumulate<DIM, SPL>(lds + (size_t)c * R, xs, as, ag);
        }
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            if (G > 1) {
                as[s] = group_sum<G>(as[s]);
#pragma unroll
                for (int k = 0; k < DIM; ++k) ag[s][k] = group_sum<G>(ag[s][k]);
            }
            if (MODE == kMorph) {
                float c, sp;
                sigmoid_and_slope(as[s] + beta, c, sp);
                // x - eta * sigma' * grad s,  grad s = -gscale * ag
                const float step = eta * sp * gscale;
#pragma unroll
                for (int k = 0; k < DIM; ++k) x[s][k] = fmaf(step, ag[s][k], x[s][k]);
            }
        }
    }

#pragma unroll
    for (int s = 0; s < SPL; ++s)
        if (rec[s]) traj_put<DIM>(tr, steps, tc[s], x[s]);
    if (lg != 0) return;
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
        if (idx[s] >= n) continue;
        const size_t i = (size_t)idx[s];
        if (MODE == kMorph) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) x_out[(size_t)k * n + i] = x[s][k];
        } else if (MODE == kEval) {
            const float sv = as[s] + beta;
            if (c_out) {
                float c, sp;
                sigmoid_and_slope(sv, c, sp);
                c_out[i] = c;
            }
            if (s_out) s_out[(size_t)blockIdx.y * n + i] = sv;
        } else {
            const float sv = as[s] + beta;
            float c, sp;
            sigmoid_and_slope(sv, c, sp);
            float f;
            if (MODE == kGrad) {
                if (c_out) c_out[i] = c;
                f = -sp * gscale;
            } else {
                f = -g_in[i] * (chain ? sp : 1.0f) * gscale;
            }
#pragma unroll
            for (int k = 0; k < DIM; ++k) g_out[(size_t)k * n + i] = f * ag[s][k];
        }
    }
}

// ---------------------------------------------------------------- launcher ---

template <int DIM, int SPL, int G, int BLOCK, int MODE>
static int32_t launch_rbf_v(const RbfArgs &a, hipStream_t st) {
    constexpr int TILE = tile_chunks<DIM>();
    const int nchunks = chunks_for(a.M);
    const int splits = a.splits > 1 ? a.splits : 1;
    const int cps = (nchunks + splits - 1) / splits;
    const int used = cps < TILE ? cps : TILE;
    const size_t lds = (size_t)used * ChunkLayout<DIM>::kBytes;
    const int64_t per_block = (int64_t)(BLOCK / G) * SPL;
    const int64_t blocks = (a.n + per_block - 1) / per_block;
    if (int32_t e = grid_guard(blocks, BLOCK, "k_rbf")) return e;
    hipLaunchKernelGGL((k_rbf<DIM, SPL, G, BLOCK, MODE>), dim3((unsigned)blocks, (unsigned)splits),
                       dim3(BLOCK), lds, st, a.hinges, a.weights, a.M, a.bias, a.kappa, a.gscale,
                       a.x_in, a.n, a.T, a.eta, a.c_out, a.s_out, a.g_out, a.x_out, a.g_in,
                       a.chain, cps, a.traj);
    return check_launch("k_rbf");
}

// Pick lanes-per-sample and samples-per-lane so that the launch fills gfx950's
// 1024 SIMDs with a few waves each.
template <int DIM, int MODE>
static int32_t launch_rbf_dim(const RbfArgs &a, hipStream_t st) {
    if (MODE == kEval && a.splits > 1) return launch_rbf_v<DIM, 1, 1, 256, MODE>(a, st);
    if (a.n >= (1 << 19)) return launch_rbf_v<DIM, 2, 1, 1024, MODE>(a, st);
    if (a.n >= (1 << 17)) return launch_rbf_v<DIM, 1, 1, 256, MODE>(a, st);
    if (a.n >= (1 << 15)) return launch_rbf_v<DIM, 1, 4, 256, MODE>(a, st);
    return launch_rbf_v<DIM, 1, 16, 256, MODE>(a, st);
}

template <int DIM>
static int32_t launch_rbf_mode(int mode, const RbfArgs &a, hipStream_t st) {
    switch (mode) {
        case kEval: return launch_rbf_dim<DIM, kEval>(a, st);
        case kGrad: return launch_rbf_dim<DIM, kGrad>(a, st);
        case kGradBwd: return launch_rbf_dim<DIM, kGradBwd>(a, st);
        default: return launch_rbf_dim<DIM, kMorph>(a, st);
    }
}

int32_t launch_rbf(int dim, int mode, const RbfArgs &a, hipStream_t st) {
    return dim == 2 ? launch_rbf_mode<2>(mode, a, st) : launch_rbf_mode<3>(mode, a, st);
}

int32_t launch_occ_any(int dim, int mode, const RbfArgs &a, const int *grid, hipStream_t st) {
    if (grid && grid[0] > 0 && a.splits <= 1) {
        const int32_t r = dim == 2 ? launch_grid2d(mode, a, grid[0], grid[1], st)
                                   : launch_grid3d_ws(mode, a, grid, st);
        if (r != PDMP_EUNSUPPORTED) return r;  // other grids take the pairwise sum
    }
    return launch_rbf(dim, mode, a, st);
}

}  // namespace pdmp
