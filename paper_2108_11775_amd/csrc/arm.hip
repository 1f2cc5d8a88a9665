// arm.hip -- forward kinematics of body points and the fused joint-space morph.
//
// Sec. 3.2: body points psi_p(q) on a serial arm, their FK Jacobians J_p, and the
// pull-back of Eq. 3 (read as grad_q C = sum_p J_p(q)^T grad_x c(psi_p(q)), with
// C the summed body-point occupancy), integrated by explicit Euler (Eq. 1).
//
// The Jacobian is never formed.  Body point p on link i is rigid in frame i, so
// column j of J_p is z_j x (p - o_j) for every joint j < i, and
//   dC/dq_j = z_j . ( sum_{p beyond j} p x g_p  -  o_j x sum_{p beyond j} g_p ),
// a suffix sum over links of the per-link totals G_i = sum g_p and Mo_i = sum p x g_p.
//
// Mapping: L = 8 lanes per configuration (pts_per_link <= L).  Lane k evaluates the
// DH chain itself (cheap next to the hinge loop) and owns body point k of every
// link, so the hinge loop has NDOF independent points per lane.  After the loop,
// the L lanes combine their (G_i, Mo_i) by an xor butterfly, which leaves
// bit-identical totals in every lane, and all lanes apply the same update.
#include "pdmp_common.h"

namespace pdmp {

template <int DIM, int SPL>
__device__ __forceinline__ void chunk_accumulate_arm(const float4 *__restrict__ ch,
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

template <int DIM>
__device__ __forceinline__ void stage_chunks_arm(float4 *lds, const float *__restrict__ hinges,
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

// FP32 DH chain: origins o[0..NDOF] and joint axes z[0..NDOF-1] (z_j of frame j).
template <int NDOF>
__device__ __forceinline__ void dh_chain_f32(const pdmp_arm &arm, const float (&q)[NDOF],
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
        // o_{i+1} = o_i + R (a ct, a st, d)
        const float lx = a * ct, ly = a * st;
#pragma unroll
        for (int r = 0; r < 3; ++r) o[i + 1][r] = o[i][r] + R[r][0] * lx + R[r][1] * ly + R[r][2] * d;
        // R <- R * Rot_i, Rot_i = [[ct, -st ca, st sa], [st, ct ca, -ct sa], [0, sa, ca]]
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

template <int L>
__device__ __forceinline__ float lane_group_sum(float v) {
#pragma unroll
    for (int off = L / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

constexpr int kArmLanes = 8;

template <int NDOF, int BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_morph_arm(pdmp_arm arm, const float *__restrict__ hinges, const float *__restrict__ weights,
            int M, float kappa, float gscale, const float *q_in, float *q_out, int64_t n, int T,
            float eta, const uint32_t *__restrict__ n_active, Traj tr) {
    constexpr int L = kArmLanes;
    constexpr int R = 4;  // 3-D chunk rows
    constexpr int TILE = tile_chunks<3>();
    extern __shared__ float4 lds[];
    const int nchunks = chunks_for(M);
    const int ntiles = (nchunks + TILE - 1) / TILE;
    // n is the row stride of q_in/q_out; with n_active only the first *n_active
    // configurations are morphed (the launch covers n).
    const int64_t n_eff = n_active ? min((int64_t)*n_active, n) : n;
    if ((int64_t)blockIdx.x * (BLOCK / L) >= n_eff) return;  // whole block idle
    const int k = threadIdx.x % L;                       // body point index on each link
    const int64_t cfg = (int64_t)blockIdx.x * (BLOCK / L) + threadIdx.x / L;
    const int64_t cs = cfg < n_eff ? cfg : n_eff - 1;
    const int P = arm.pts_per_link;
    const bool own = k < P;
    const float frac = own ? (float)(k + 1) / (float)P : 0.0f;

    float q[NDOF];
#pragma unroll
    for (int j = 0; j < NDOF; ++j) q[j] = q_in[(size_t)j * n + cs];
    const float beta = weights[M];

    if (ntiles == 1) {
        stage_chunks_arm<3>(lds, hinges, weights, M, kappa, 0, nchunks);
        __syncthreads();
    }

    int64_t tc;
    const bool rec = k == 0 && traj_col(tr, cfg, n_eff, tc);
    for (int t = 0; t < T; ++t) {
        if (rec) traj_put<NDOF>(tr, t, tc, q);
        float xs[NDOF][3], as[NDOF], ag[NDOF][3];
        {
            // only the prescaled points stay live through the hinge loop; the chain
            // is evaluated again afterwards instead of holding ~70 more registers
            float o[NDOF + 1][3], z[NDOF][3];
            dh_chain_f32<NDOF>(arm, q, o, z);
#pragma unroll
            for (int l = 0; l < NDOF; ++l) {
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    xs[l][e] = kappa * (o[l][e] + frac * (o[l + 1][e] - o[l][e]));
                    ag[l][e] = 0.0f;
                }
                as[l] = 0.0f;
            }
        }
        for (int tile = 0; tile < ntiles; ++tile) {
            const int c0 = tile * TILE;
            const int nc = min(TILE, nchunks - c0);
            if (ntiles > 1) {
                __syncthreads();
                stage_chunks_arm<3>(lds, hinges, weights, M, kappa, c0, nc);
                __syncthreads();
            }
            for (int c = 0; c < nc; ++c) chunk_accumulate_arm<3, NDOF>(lds + (size_t)c * R, xs, as, ag);
        }
        float o[NDOF + 1][3], z[NDOF][3], p[NDOF][3];
        dh_chain_f32<NDOF>(arm, q, o, z);
#pragma unroll
        for (int l = 0; l < NDOF; ++l)
#pragma unroll
            for (int e = 0; e < 3; ++e) p[l][e] = o[l][e] + frac * (o[l + 1][e] - o[l][e]);
        // per-link totals G_l = g_p and Mo_l = p x g_p of this lane's point
        float G[NDOF][3], Mo[NDOF][3];
#pragma unroll
        for (int l = 0; l < NDOF; ++l) {
            float c, sp;
            sigmoid_and_slope(as[l] + beta, c, sp);
            const float f = own ? -sp * gscale : 0.0f;  // grad c = sigma' * (-gscale * ag)
            const float g0 = f * ag[l][0], g1 = f * ag[l][1], g2 = f * ag[l][2];
            G[l][0] = g0;
            G[l][1] = g1;
            G[l][2] = g2;
            Mo[l][0] = p[l][1] * g2 - p[l][2] * g1;
            Mo[l][1] = p[l][2] * g0 - p[l][0] * g2;
            Mo[l][2] = p[l][0] * g1 - p[l][1] * g0;
        }
#pragma unroll
        for (int l = 0; l < NDOF; ++l)
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                G[l][e] = lane_group_sum<L>(G[l][e]);
                Mo[l][e] = lane_group_sum<L>(Mo[l][e]);
            }
        // suffix sums over links; joint j moves links j..NDOF-1 about z_j through o_j
        float SG[3] = {0, 0, 0}, SM[3] = {0, 0, 0};
#pragma unroll
        for (int j = NDOF - 1; j >= 0; --j) {
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                SG[e] += G[j][e];
                SM[e] += Mo[j][e];
            }
            const float v0 = SM[0] - (o[j][1] * SG[2] - o[j][2] * SG[1]);
            const float v1 = SM[1] - (o[j][2] * SG[0] - o[j][0] * SG[2]);
            const float v2 = SM[2] - (o[j][0] * SG[1] - o[j][1] * SG[0]);
            const float gq = z[j][0] * v0 + z[j][1] * v1 + z[j][2] * v2;
            q[j] = q[j] - eta * gq;
        }
    }
    if (rec) traj_put<NDOF>(tr, T, tc, q);
    if (k == 0 && cfg < n_eff) {
#pragma unroll
        for (int j = 0; j < NDOF; ++j) q_out[(size_t)j * n + cfg] = q[j];
    }
}

// Largest body-point occupancy of each configuration: max_p sigma(s(psi_p(q))),
// and flag = (max > thresh).  Same lane mapping as the morph, value only.
template <int NDOF, int BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_arm_max_occ(pdmp_arm arm, const float *__restrict__ hinges, const float *__restrict__ weights,
              int M, float kappa, const float *__restrict__ q_in, int64_t n, float thresh,
              float *maxc_out, uint8_t *flag_out) {
    constexpr int L = kArmLanes;
    constexpr int R = 4;
    constexpr int TILE = tile_chunks<3>();
    extern __shared__ float4 lds[];
    const int nchunks = chunks_for(M);
    const int ntiles = (nchunks + TILE - 1) / TILE;
    const int k = threadIdx.x % L;
    const int64_t cfg = (int64_t)blockIdx.x * (BLOCK / L) + threadIdx.x / L;
    const int64_t cs = cfg < n ? cfg : n - 1;
    const int P = arm.pts_per_link;
    const bool own = k < P;
    const float frac = own ? (float)(k + 1) / (float)P : 0.0f;
    float q[NDOF];
#pragma unroll
    for (int j = 0; j < NDOF; ++j) q[j] = q_in[(size_t)j * n + cs];
    const float beta = weights[M];
    float xs[NDOF][3], as[NDOF];
    {
        float o[NDOF + 1][3], z[NDOF][3];
        dh_chain_f32<NDOF>(arm, q, o, z);
#pragma unroll
        for (int l = 0; l < NDOF; ++l) {
#pragma unroll
            for (int e = 0; e < 3; ++e) xs[l][e] = kappa * (o[l][e] + frac * (o[l + 1][e] - o[l][e]));
            as[l] = 0.0f;
        }
    }
    for (int tile = 0; tile < ntiles; ++tile) {
        const int c0 = tile * TILE;
        const int nc = min(TILE, nchunks - c0);
        __syncthreads();
        stage_chunks_arm<3>(lds, hinges, weights, M, kappa, c0, nc);
        __syncthreads();
        for (int c = 0; c < nc; ++c) {
            const float4 *ch = lds + (size_t)c * R;
            const float4 h0 = ch[0], h1 = ch[1], h2 = ch[2], wv = ch[3];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int l = 0; l < NDOF; ++l) {
                    const float d0 = xs[l][0] - f4c(h0, u), d1 = xs[l][1] - f4c(h1, u),
                                d2 = xs[l][2] - f4c(h2, u);
                    const float r2 = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
                    as[l] = fmaf(f4c(wv, u), exp2_fast(-r2), as[l]);
                }
            }
        }
    }
    float mc = -1.0f;
#pragma unroll
    for (int l = 0; l < NDOF; ++l) {
        float c, sp;
        sigmoid_and_slope(as[l] + beta, c, sp);
        if (own) mc = fmaxf(mc, c);
    }
#pragma unroll
    for (int off = L / 2; off >= 1; off >>= 1) mc = fmaxf(mc, __shfl_xor(mc, off, 64));
    if (k == 0 && cfg < n) {
        if (maxc_out) maxc_out[cfg] = mc;
        if (flag_out) flag_out[cfg] = mc > thresh ? 1 : 0;
    }
}

// ---- compaction of flagged configurations (ascending index order) ----

// counts[b] = number of flags set in block b's range of 256 configurations
__global__ void __launch_bounds__(256) k_flag_count(const uint8_t *__restrict__ flag, int64_t n,
                                                    uint32_t *counts) {
    __shared__ uint32_t wc[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool f = i < n && flag[i];
    const uint64_t m = __ballot(f);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

// exclusive scan of counts[0..nb) into offs, total into *total (one block, fixed order)
__global__ void __launch_bounds__(256) k_scan_counts(const uint32_t *__restrict__ counts, int nb,
                                                     uint32_t *offs, uint32_t *total) {
    __shared__ uint32_t part[256];
    const int per = (nb + 255) / 256;
    const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    uint32_t s = 0;
    for (int b = b0; b < b1; ++b) s += counts[b];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int t = 0; t < 256; ++t) {
            const uint32_t v = part[t];
            part[t] = run;
            run += v;
        }
        *total = run;
    }
    __syncthreads();
    uint32_t run = part[threadIdx.x];
    for (int b = b0; b < b1; ++b) {
        offs[b] = run;
        run += counts[b];
    }
}

// idx[offs[block] + rank] = i for flagged i; gather their rows of q into qc
// (row stride n) so the compact batch keeps ascending order.
template <int NDOF>
__global__ void __launch_bounds__(256)
k_compact_gather(const uint8_t *__restrict__ flag, const uint32_t *__restrict__ offs,
                 const float *__restrict__ q, int64_t n, uint32_t *idx, float *qc) {
    __shared__ uint32_t wc[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool f = i < n && flag[i];
    const uint64_t m = __ballot(f);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) wc[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t base = offs[blockIdx.x];
    for (int k = 0; k < w; ++k) base += wc[k];
    const uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (f) {
        const uint32_t p = base + rank;
        idx[p] = (uint32_t)i;
#pragma unroll
        for (int j = 0; j < NDOF; ++j) qc[(size_t)j * n + p] = q[(size_t)j * n + i];
    }
}

template <int NDOF>
__global__ void __launch_bounds__(256)
k_scatter(const uint32_t *__restrict__ idx, const uint32_t *__restrict__ total,
          const float *__restrict__ qc, int64_t n, float *out) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)*total) return;
    const uint32_t i = idx[p];
#pragma unroll
    for (int j = 0; j < NDOF; ++j) out[(size_t)j * n + i] = qc[(size_t)j * n + p];
}

// One thread per configuration: FP32 body points [3][NDOF*P][n].
template <int NDOF>
__global__ void __launch_bounds__(256)
k_fk_points(pdmp_arm arm, const float *__restrict__ q_in, int64_t n, float *pts) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float q[NDOF];
#pragma unroll
    for (int j = 0; j < NDOF; ++j) q[j] = q_in[(size_t)j * n + s];
    float o[NDOF + 1][3], z[NDOF][3];
    dh_chain_f32<NDOF>(arm, q, o, z);
    const int P = arm.pts_per_link;
    const size_t nb = (size_t)NDOF * P;
#pragma unroll
    for (int l = 0; l < NDOF; ++l)
        for (int k = 0; k < P; ++k) {
            const float f = (float)(k + 1) / (float)P;
#pragma unroll
            for (int e = 0; e < 3; ++e)
                pts[((size_t)e * nb + (size_t)l * P + k) * n + s] = o[l][e] + f * (o[l + 1][e] - o[l][e]);
        }
}

template <int NDOF>
static int32_t launch_morph_arm_n(const pdmp_arm &arm, const float *h, const float *w, int M,
                                  float kappa, float gscale, const float *qi, float *qo, int64_t n,
                                  int T, float eta, const uint32_t *n_active, hipStream_t st,
                                  const Traj &traj) {
    constexpr int BLOCK = 512;
    constexpr int TILE = tile_chunks<3>();
    const int nchunks = chunks_for(M);
    const size_t lds = (size_t)(nchunks < TILE ? nchunks : TILE) * ChunkLayout<3>::kBytes;
    const int64_t blocks = (n + BLOCK / kArmLanes - 1) / (BLOCK / kArmLanes);
    if (int32_t e = grid_guard(blocks, BLOCK, "k_morph_arm")) return e;
    hipLaunchKernelGGL((k_morph_arm<NDOF, BLOCK>), dim3((unsigned)blocks), dim3(BLOCK), lds, st, arm,
                       h, w, M, kappa, gscale, qi, qo, n, T, eta, n_active, traj);
    return check_launch("k_morph_arm");
}

template <int NDOF>
static int32_t launch_arm_max_occ_n(const pdmp_arm &arm, const float *h, const float *w, int M,
                                    float kappa, const float *q, int64_t n, float thresh,
                                    float *maxc, uint8_t *flag, hipStream_t st) {
    constexpr int BLOCK = 512;
    constexpr int TILE = tile_chunks<3>();
    const int nchunks = chunks_for(M);
    const size_t lds = (size_t)(nchunks < TILE ? nchunks : TILE) * ChunkLayout<3>::kBytes;
    const int64_t blocks = (n + BLOCK / kArmLanes - 1) / (BLOCK / kArmLanes);
    if (int32_t e = grid_guard(blocks, BLOCK, "k_arm_max_occ")) return e;
    hipLaunchKernelGGL((k_arm_max_occ<NDOF, BLOCK>), dim3((unsigned)blocks), dim3(BLOCK), lds, st,
                       arm, h, w, M, kappa, q, n, thresh, maxc, flag);
    return check_launch("k_arm_max_occ");
}

int32_t launch_arm_max_occ(const pdmp_arm &arm, const float *h, const float *w, int M, float kappa,
                           const float *q, int64_t n, float thresh, float *maxc, uint8_t *flag,
                           hipStream_t st) {
    switch (arm.n_dof) {
#define PDMP_CASE(N) \
    case N: return launch_arm_max_occ_n<N>(arm, h, w, M, kappa, q, n, thresh, maxc, flag, st);
        PDMP_CASE(1) PDMP_CASE(2) PDMP_CASE(3) PDMP_CASE(4)
        PDMP_CASE(5) PDMP_CASE(6) PDMP_CASE(7) PDMP_CASE(8)
#undef PDMP_CASE
    }
    set_error("n_dof %d unsupported", arm.n_dof);
    return PDMP_EUNSUPPORTED;
}

// Gather the flagged configurations (ascending index) into qc, keep their indices
// in idx and their count in *total; all device-side, no host synchronisation.
int32_t launch_compact(const pdmp_arm &arm, const uint8_t *flag, const float *q, int64_t n,
                       uint32_t *counts, uint32_t *offs, uint32_t *total, uint32_t *idx, float *qc,
                       hipStream_t st) {
    if (int32_t e = grid_guard((n + 255) / 256, 256, "compact")) return e;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_flag_count, dim3(nb), dim3(256), 0, st, flag, n, counts);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(256), 0, st, counts, (int)nb, offs, total);
    switch (arm.n_dof) {
#define PDMP_CASE(N)                                                                          \
    case N:                                                                                   \
        hipLaunchKernelGGL(k_compact_gather<N>, dim3(nb), dim3(256), 0, st, flag, offs, q, n, idx, \
                           qc);                                                               \
        break;
        PDMP_CASE(1) PDMP_CASE(2) PDMP_CASE(3) PDMP_CASE(4)
        PDMP_CASE(5) PDMP_CASE(6) PDMP_CASE(7) PDMP_CASE(8)
#undef PDMP_CASE
    }
    return check_launch("compact");
}

int32_t launch_scatter(const pdmp_arm &arm, const uint32_t *idx, const uint32_t *total,
                       const float *qc, int64_t n, float *out, hipStream_t st) {
    if (int32_t e = grid_guard((n + 255) / 256, 256, "k_scatter")) return e;
    const unsigned nb = (unsigned)((n + 255) / 256);
    switch (arm.n_dof) {
#define PDMP_CASE(N)                                                                           \
    case N:                                                                                    \
        hipLaunchKernelGGL(k_scatter<N>, dim3(nb), dim3(256), 0, st, idx, total, qc, n, out); \
        break;
        PDMP_CASE(1) PDMP_CASE(2) PDMP_CASE(3) PDMP_CASE(4)
        PDMP_CASE(5) PDMP_CASE(6) PDMP_CASE(7) PDMP_CASE(8)
#undef PDMP_CASE
    }
    return check_launch("k_scatter");
}

int32_t launch_morph_arm(const pdmp_arm &arm, const float *h, const float *w, int M, float kappa,
                         float gscale, const float *qi, float *qo, int64_t n, int T, float eta,
                         const uint32_t *n_active, hipStream_t st, const Traj &traj) {
    switch (arm.n_dof) {
#define PDMP_CASE(N)                                                                            \
    case N:                                                                                     \
        return launch_morph_arm_n<N>(arm, h, w, M, kappa, gscale, qi, qo, n, T, eta, n_active, st, \
                                     traj);
        PDMP_CASE(1) PDMP_CASE(2) PDMP_CASE(3) PDMP_CASE(4)
        PDMP_CASE(5) PDMP_CASE(6) PDMP_CASE(7) PDMP_CASE(8)
#undef PDMP_CASE
    }
    set_error("n_dof %d unsupported", arm.n_dof);
    return PDMP_EUNSUPPORTED;
}

int32_t launch_fk_points(const pdmp_arm &arm, const float *q, int64_t n, float *pts,
                         hipStream_t st) {
    if (int32_t e = grid_guard((n + 255) / 256, 256, "k_fk_points")) return e;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    switch (arm.n_dof) {
#define PDMP_CASE(N)                                                                    \
    case N:                                                                             \
        hipLaunchKernelGGL(k_fk_points<N>, dim3(blocks), dim3(256), 0, st, arm, q, n, pts); \
        return check_launch("k_fk_points");
        PDMP_CASE(1) PDMP_CASE(2) PDMP_CASE(3) PDMP_CASE(4)
        PDMP_CASE(5) PDMP_CASE(6) PDMP_CASE(7) PDMP_CASE(8)
#undef PDMP_CASE
    }
    set_error("n_dof %d unsupported", arm.n_dof);
    return PDMP_EUNSUPPORTED;
}

}  // namespace pdmp
