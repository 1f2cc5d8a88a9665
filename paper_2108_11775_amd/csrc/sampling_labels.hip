// sampling_labels.hip -- batched prior samples (Philox4x32-10) and collision labels.
//
// Prior samples: the sampler of Sec. 3.3 draws large batches from the prior on the
// GPU.  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011) is counter based, so
// sample i's coordinates depend only on (seed, stream id, i) and not on the launch.
//
// Labels: a point is in collision iff it lies in a closed obstacle; a configuration
// iff any of its body points does (the "feasible" fraction of Table 1).  The test
// is taken in FP64 with contraction off and a fixed operation order, so the label
// of a given FP32 point is reproducible bit for bit.
#include "pdmp_common.h"

namespace pdmp {

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

struct Box16 {
    float lo[16], hi[16];
};

// One thread per (sample, block of four coordinates).
__global__ void __launch_bounds__(256)
k_uniform(uint32_t k0, uint32_t k1, uint32_t sid, Box16 box, int dim, int64_t n, float *out) {
#pragma clang fp contract(off)
    const int nb = (dim + 3) / 4;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    const int b = (int)(t / n);
    const int64_t i = t - (int64_t)b * n;
    uint32_t c[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)b, sid};
    philox4x32_10(c, k0, k1);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int k = b * 4 + w;
        if (k >= dim) break;
        const double u = (double)(c[w] >> 8) * (1.0 / 16777216.0);
        const double span = (double)box.hi[k] - (double)box.lo[k];
        const double v = (double)box.lo[k] + span * u;
        out[(size_t)k * n + i] = (float)v;
    }
}

int32_t launch_uniform(uint64_t seed, uint32_t sid, const float *lo, const float *hi, int dim,
                       int64_t n, float *out, hipStream_t st) {
    Box16 box;
    for (int k = 0; k < 16; ++k) {
        box.lo[k] = k < dim ? lo[k] : 0.0f;
        box.hi[k] = k < dim ? hi[k] : 0.0f;
    }
    const int64_t work = n * ((dim + 3) / 4);
    const int64_t blocks = (work + 255) / 256;
    if (int32_t e = grid_guard(blocks, 256, "k_uniform")) return e;
    hipLaunchKernelGGL(k_uniform, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t)seed,
                       (uint32_t)(seed >> 32), sid, box, dim, n, out);
    return check_launch("k_uniform");
}

// Epsilon mixture with the prior (Sec. 3.3): sample i keeps its prior value iff
// u_i < eps, u_i from word 0 of Philox at counter {i_lo, i_hi, 0xffffffff, sid} (a
// counter the coordinates never use), u = (word >> 8) 2^-24.
__global__ void __launch_bounds__(256)
k_mix_select(uint32_t k0, uint32_t k1, uint32_t sid, double eps, int dim, int64_t n,
             const float *__restrict__ x0, float *out, uint8_t *keep) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0xffffffffu, sid};
    philox4x32_10(c, k0, k1);
    const double u = (double)(c[0] >> 8) * (1.0 / 16777216.0);
    const bool k = u < eps;
    if (keep) keep[i] = (uint8_t)k;
    if (k)
        for (int d = 0; d < dim; ++d) out[(size_t)d * n + i] = x0[(size_t)d * n + i];
}

int32_t launch_mix_select(uint64_t seed, uint32_t sid, float eps, int dim, int64_t n,
                          const float *x0, float *out, uint8_t *keep, hipStream_t st) {
    if (int32_t e = grid_guard((n + 255) / 256, 256, "k_mix_select")) return e;
    hipLaunchKernelGGL(k_mix_select, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (uint32_t)seed, (uint32_t)(seed >> 32), sid, (double)eps, dim, n, x0, out,
                       keep);
    return check_launch("k_mix_select");
}

__global__ void k_zero_u64(uint64_t *p) {
    if (threadIdx.x == 0) *p = 0;
}

// Count of 1-labels: one integer atomic per wave (deterministic).
// Adds the block's hits (c per thread) with one global atomic per block: a single
// counter updated by every wave of a large launch serialises in L2 and had cost more
// than the labelling itself.  Every thread of the block calls it (uniform).
__device__ __forceinline__ void count_hits_block(int c, uint64_t *n_hit) {
    __shared__ unsigned int blk;
    if (!n_hit) return;
    if (threadIdx.x == 0) blk = 0;
    __syncthreads();
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&blk, (unsigned int)c);
    __syncthreads();
    if (threadIdx.x == 0 && blk) atomicAdd((unsigned long long *)n_hit, (unsigned long long)blk);
}

// Discs in tiles of kLabTile: each tile staged in LDS as FP64 (cx, cy, r^2) (r^2 of an
// FP32 radius is exact in FP64) and culled by a 16 x 16 cell grid over the tile's
// bounding box: cell (i, j) lists, as a bit mask, the discs whose box [c - R, c + R],
// R = |r| (1 + 2^-20), meets it, widened by 1/64 of a cell on each side; the outer
// cells reach to infinity (cell indices are clamped, for the discs' ranges and the
// points alike).  A point's FP64 test  (px - cx)^2 + (py - cy)^2 <= r^2  can hold only
// within R of the centre on each axis (the test's rounding is 2^-52 relative, the
// index arithmetic's a few FP32 ulps, both far inside the margins), so each point
// tests only its cell's discs and every decision is the one of the plain per-disc
// loop.  A tile with a non-finite disc, or a degenerate box, puts every disc in every
// cell.  Each thread carries kLabPts points (coalesced: point base + u * blockDim).
constexpr int kLabBlock = 1024;    // 4096 points share a block's cell masks
constexpr int kLabPts = 4;
constexpr int kLabTile = 128;      // discs per tile: 4 mask words per cell
constexpr int kLabCells = 16;      // per axis
constexpr int kLabWords = kLabTile / 32;

__global__ void __launch_bounds__(kLabBlock)
k_label_discs(const float *__restrict__ cen, const float *__restrict__ rad, int K,
              const float *__restrict__ x, int64_t n, uint8_t *out, uint64_t *n_hit) {
#pragma clang fp contract(off)
    __shared__ double sd[3][kLabTile];
    __shared__ uint32_t mask[kLabCells * kLabCells][kLabWords];
    __shared__ float red[5][kLabBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kLabBlock * kLabPts + threadIdx.x;
    float fx[kLabPts], fy[kLabPts];
    bool hit[kLabPts];
#pragma unroll
    for (int u = 0; u < kLabPts; ++u) {
        const int64_t i = base + (int64_t)u * kLabBlock;
        const int64_t ic = i < n ? i : n - 1;
        fx[u] = x[ic];
        fy[u] = x[(size_t)n + ic];
        hit[u] = false;
    }
    for (int k0 = 0; k0 < K; k0 += kLabTile) {
        const int kn = min(kLabTile, K - k0);
        __syncthreads();  // the previous tile's readers are done
        // stage the tile, its bounding box and whether every disc is finite
        float xlo = INFINITY, xhi = -INFINITY, ylo = INFINITY, yhi = -INFINITY, bad = 0.0f;
        float cx = 0.0f, cy = 0.0f, R = 0.0f;
        const int j = threadIdx.x;
        if (j < kn) {
            cx = cen[k0 + j];
            cy = cen[K + k0 + j];
            const float r = rad[k0 + j];
            sd[0][j] = (double)cx;
            sd[1][j] = (double)cy;
            sd[2][j] = (double)r * (double)r;
            R = fabsf(r) * (1.0f + 0x1p-20f);
            if (!__builtin_isfinite(cx) || !__builtin_isfinite(cy) || !__builtin_isfinite(R))
                bad = 1.0f;
            else {
                xlo = cx - R, xhi = cx + R, ylo = cy - R, yhi = cy + R;
            }
        }
        for (int c = threadIdx.x; c < kLabCells * kLabCells * kLabWords; c += kLabBlock)
            (&mask[0][0])[c] = 0u;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            xlo = fminf(xlo, __shfl_xor(xlo, off, 64));
            xhi = fmaxf(xhi, __shfl_xor(xhi, off, 64));
            ylo = fminf(ylo, __shfl_xor(ylo, off, 64));
            yhi = fmaxf(yhi, __shfl_xor(yhi, off, 64));
            bad = fmaxf(bad, __shfl_xor(bad, off, 64));
        }
        if (lane == 0) {
            red[0][wv] = xlo, red[1][wv] = xhi, red[2][wv] = ylo, red[3][wv] = yhi;
            red[4][wv] = bad;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kLabBlock / 64; ++w) {
            xlo = fminf(xlo, red[0][w]), xhi = fmaxf(xhi, red[1][w]);
            ylo = fminf(ylo, red[2][w]), yhi = fmaxf(yhi, red[3][w]);
            bad = fmaxf(bad, red[4][w]);
        }
        // cells per unit on each axis (0: no culling, every disc in every cell)
        const bool cull = bad == 0.0f && xhi > xlo && yhi > ylo &&
                          __builtin_isfinite(xhi - xlo) && __builtin_isfinite(yhi - ylo);
        const float sx = cull ? (float)kLabCells / (xhi - xlo) : 0.0f;
        const float sy = cull ? (float)kLabCells / (yhi - ylo) : 0.0f;
        auto cell_of = [](float v) {  // clamped, NaN to cell 0
            return (int)fminf(fmaxf(floorf(v), 0.0f), (float)(kLabCells - 1));
        };
        if (j < kn) {
            int i0 = 0, i1 = kLabCells - 1, j0 = 0, j1 = kLabCells - 1;
            if (cull) {
                constexpr float m = 1.0f / 64.0f;
                i0 = cell_of((cx - R - xlo) * sx - m), i1 = cell_of((cx + R - xlo) * sx + m);
                j0 = cell_of((cy - R - ylo) * sy - m), j1 = cell_of((cy + R - ylo) * sy + m);
            }
            const uint32_t bit = 1u << (j & 31);
            for (int cj = j0; cj <= j1; ++cj)
                for (int ci = i0; ci <= i1; ++ci)
                    atomicOr(&mask[cj * kLabCells + ci][j >> 5], bit);
        }
        __syncthreads();
        const int words = (kn + 31) >> 5;
        int cell[kLabPts];
#pragma unroll
        for (int u = 0; u < kLabPts; ++u)
            cell[u] = cull ? cell_of((fy[u] - ylo) * sy) * kLabCells + cell_of((fx[u] - xlo) * sx)
                           : 0;
        for (int q = 0; q < words; ++q) {
            // the lane's points walk their cells' discs side by side (independent tests
            // in flight together); a point stops at its first hit
            uint32_t mq[kLabPts];
#pragma unroll
            for (int u = 0; u < kLabPts; ++u) mq[u] = hit[u] ? 0u : mask[cell[u]][q];
            while (true) {
                uint32_t left = 0;
#pragma unroll
                for (int u = 0; u < kLabPts; ++u) left |= mq[u];
                if (!left) break;
#pragma unroll
                for (int u = 0; u < kLabPts; ++u) {
                    if (!mq[u]) continue;
                    const int k = 32 * q + __builtin_ctz(mq[u]);
                    mq[u] &= mq[u] - 1u;
                    const double dx = (double)fx[u] - sd[0][k];
                    const double dy = (double)fy[u] - sd[1][k];
                    const double a = dx * dx;
                    const double b = dy * dy;
                    const double d2 = a + b;
                    if (d2 <= sd[2][k]) {
                        hit[u] = true;
                        mq[u] = 0u;
                    }
                }
            }
        }
    }
    int c = 0;
#pragma unroll
    for (int u = 0; u < kLabPts; ++u) {
        const int64_t i = base + (int64_t)u * kLabBlock;
        const bool h = i < n && hit[u];
        if (i < n) out[i] = h ? 1 : 0;
        c += h ? 1 : 0;
    }
    count_hits_block(c, n_hit);
}

__device__ __forceinline__ bool in_any_box(const double p[3], const float *__restrict__ cen,
                                           const float *__restrict__ half, int K) {
#pragma clang fp contract(off)
    for (int k = 0; k < K; ++k) {
        bool in = true;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (!(fabs(p[a] - (double)cen[a * K + k]) <= (double)half[a * K + k])) in = false;
        if (in) return true;
    }
    return false;
}

__global__ void __launch_bounds__(256)
k_label_boxes(const float *__restrict__ cen, const float *__restrict__ half, int K,
              const float *__restrict__ x, int64_t n, uint8_t *out, uint64_t *n_hit) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool hit = false;
    if (i < n) {
        const double p[3] = {x[i], x[(size_t)n + i], x[2 * (size_t)n + i]};
        hit = in_any_box(p, cen, half, K);
        out[i] = hit ? 1 : 0;
    }
    count_hits_block(hit ? 1 : 0, n_hit);
}

// Standard-DH chain in FP64 for the label decision (same operation order as the
// plain definition: T_i = T_{i-1} A_i, each entry a k = 0..3 sum).
__global__ void __launch_bounds__(256)
k_label_configs(pdmp_arm arm, const float *__restrict__ cen, const float *__restrict__ half,
                int K, const float *__restrict__ q, int64_t n, uint8_t *out, uint64_t *n_hit) {
#pragma clang fp contract(off)
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool hit = false;
    if (s < n) {
        double T[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
        double op[3] = {0, 0, 0};
        const int P = arm.pts_per_link;
        for (int i = 0; i < arm.n_dof && !hit; ++i) {
            const double a = arm.a[i], d = arm.d[i], al = arm.alpha[i];
            const double th = (double)arm.theta0[i] + (double)q[(size_t)i * n + s];
            double st, ct, sa, ca;
            sincos(th, &st, &ct);
            sincos(al, &sa, &ca);
            const double A[4][4] = {{ct, -st * ca, st * sa, a * ct},
                                    {st, ct * ca, -ct * sa, a * st},
                                    {0.0, sa, ca, d},
                                    {0.0, 0.0, 0.0, 1.0}};
            double N[4][4];
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) {
                    double acc = 0.0;
                    for (int k = 0; k < 4; ++k) acc += T[r][k] * A[k][c];
                    N[r][c] = acc;
                }
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) T[r][c] = N[r][c];
            const double on[3] = {T[0][3], T[1][3], T[2][3]};
            for (int k = 0; k < P && !hit; ++k) {
                const double f = (double)(k + 1) / (double)P;
                double p[3];
                for (int e = 0; e < 3; ++e) p[e] = op[e] + f * (on[e] - op[e]);
                hit = in_any_box(p, cen, half, K);
            }
            for (int e = 0; e < 3; ++e) op[e] = on[e];
        }
        out[s] = hit ? 1 : 0;
    }
    count_hits_block(hit ? 1 : 0, n_hit);
}

int32_t launch_label_discs(const pdmp_discs &sc, const float *x, int64_t n, uint8_t *out,
                           uint64_t *n_hit, hipStream_t st) {
    if (n_hit) {
        // a fill kernel rather than a memset node, so the call can be graph-captured
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, n_hit);
        if (int32_t e = check_launch("k_zero_u64")) return e;
    }
    if (n == 0) return PDMP_OK;
    const int64_t per = (int64_t)kLabBlock * kLabPts;
    if (int32_t e = grid_guard((n + per - 1) / per, kLabBlock, "k_label_discs")) return e;
    hipLaunchKernelGGL(k_label_discs, dim3((unsigned)((n + per - 1) / per)), dim3(kLabBlock), 0,
                       st, sc.centres, sc.radii, sc.n, x, n, out, n_hit);
    return check_launch("k_label_discs");
}

int32_t launch_label_boxes(const pdmp_boxes &sc, const float *x, int64_t n, uint8_t *out,
                           uint64_t *n_hit, hipStream_t st) {
    if (n_hit) {
        // a fill kernel rather than a memset node, so the call can be graph-captured
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, n_hit);
        if (int32_t e = check_launch("k_zero_u64")) return e;
    }
    if (n == 0) return PDMP_OK;
    if (int32_t e = grid_guard((n + 255) / 256, 256, "k_label_boxes")) return e;
    hipLaunchKernelGGL(k_label_boxes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       sc.centres, sc.half, sc.n, x, n, out, n_hit);
    return check_launch("k_label_boxes");
}

int32_t launch_label_configs(const pdmp_arm &arm, const pdmp_boxes &sc, const float *q, int64_t n,
                             uint8_t *out, uint64_t *n_hit, hipStream_t st) {
    if (n_hit) {
        // a fill kernel rather than a memset node, so the call can be graph-captured
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, n_hit);
        if (int32_t e = check_launch("k_zero_u64")) return e;
    }
    if (n == 0) return PDMP_OK;
    if (int32_t e = grid_guard((n + 255) / 256, 256, "k_label_configs")) return e;
    hipLaunchKernelGGL(k_label_configs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, arm,
                       sc.centres, sc.half, sc.n, q, n, out, n_hit);
    return check_launch("k_label_configs");
}

}  // namespace pdmp
