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

// Discs staged in LDS as FP64 (cx, cy, r^2) tiles: r^2 of an FP32 radius is exact in
// FP64, so every decision is the one of the plain per-disc loop; each thread carries
// kLabPts points (coalesced: point base + u * blockDim).
constexpr int kLabBlock = 256;
constexpr int kLabPts = 4;
constexpr int kLabTile = 1024;

__global__ void __launch_bounds__(kLabBlock)
k_label_discs(const float *__restrict__ cen, const float *__restrict__ rad, int K,
              const float *__restrict__ x, int64_t n, uint8_t *out, uint64_t *n_hit) {
#pragma clang fp contract(off)
    __shared__ double sd[3][kLabTile];
    const int64_t base = (int64_t)blockIdx.x * kLabBlock * kLabPts + threadIdx.x;
    double px[kLabPts], py[kLabPts];
    bool hit[kLabPts];
#pragma unroll
    for (int u = 0; u < kLabPts; ++u) {
        const int64_t i = base + (int64_t)u * kLabBlock;
        const int64_t ic = i < n ? i : n - 1;
        px[u] = x[ic];
        py[u] = x[(size_t)n + ic];
        hit[u] = false;
    }
    for (int k0 = 0; k0 < K; k0 += kLabTile) {
        const int kn = min(kLabTile, K - k0);
        __syncthreads();
        for (int j = threadIdx.x; j < kn; j += kLabBlock) {
            sd[0][j] = (double)cen[k0 + j];
            sd[1][j] = (double)cen[K + k0 + j];
            const double r = rad[k0 + j];
            sd[2][j] = r * r;
        }
        __syncthreads();
        for (int k = 0; k < kn; ++k) {
            const double cx = sd[0][k], cy = sd[1][k], rr = sd[2][k];
#pragma unroll
            for (int u = 0; u < kLabPts; ++u) {
                const double dx = px[u] - cx;
                const double dy = py[u] - cy;
                const double a = dx * dx;
                const double b = dy * dy;
                const double d2 = a + b;
                hit[u] = hit[u] || d2 <= rr;
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
    hipLaunchKernelGGL(k_label_configs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, arm,
                       sc.centres, sc.half, sc.n, q, n, out, n_hit);
    return check_launch("k_label_configs");
}

}  // namespace pdmp
