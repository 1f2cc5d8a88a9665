// cull.hip -- compact-support hinge culling for the pairwise morph (a variant beyond
// the paper).  The RBF feature decays as exp(-r^2 / (2 l^2)); a point takes only the
// hinges of the 3^dim cells around its own cell (cells of side >= the cutoff r_c), so
// every hinge within r_c is kept and the dropped part of the logit is at most
// sum_j |w_j| exp(-r_c^2 / (2 l^2)).  A coordinate's cell is
// floor((v - lo) * inv_cell) in FP64 from the FP32 values, clamped to the grid, so the
// kept set is a property of the point alone.
//
// Layout: the hinges are sorted by cell once per call (counting sort; each cell's
// hinges in increasing index order, so sums are deterministic) and prescaled by
// kappa = sqrt(log2(e) / (2 l^2)), so that phi = exp2(-|kappa x - kappa h|^2) needs
// no multiply before v_exp_f32; cell_start[] gives each cell's range.  The samples are sorted by their starting cell so that a
// wave's points are close; at every step a wave takes the rectangle of cells covering
// its points' neighbourhoods, walks it cell by cell (wave-uniform bounds, hinge reads
// through the scalar unit), and each lane accumulates only the cells within one of
// its own.  A point visits its own cells in the same order whatever the rest of the
// wave, so its result does not depend on the batch.  The sample order only affects
// speed.
#include "pdmp_common.h"

#include <algorithm>

namespace pdmp {

constexpr int kCullBlock = 256;

struct CullGridDev {
    float lo[3];
    float inv_cell;
    int nc[3];
};

__host__ __device__ inline int cull_cell(float v, float lo, float inv_cell, int nc) {
    const double t = ((double)v - (double)lo) * (double)inv_cell;
    const double f = floor(t);
    if (f < 0.0) return 0;
    if (f > (double)(nc - 1)) return nc - 1;
    return (int)f;
}

template <int DIM>
__device__ __forceinline__ int cell_id(const CullGridDev &g, const float *x) {
    int c = 0, stride = 1;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        c += stride * cull_cell(x[k], g.lo[k], g.inv_cell, g.nc[k]);
        stride *= g.nc[k];
    }
    return c;
}

__global__ void k_fill_i32(int *p, int64_t n, int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// counts[cell(point i)] += 1 for n points x [DIM][n].
template <int DIM>
__global__ void __launch_bounds__(kCullBlock)
k_cull_count(CullGridDev g, const float *__restrict__ x, int64_t n, int *counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float p[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) p[k] = x[(size_t)k * n + i];
    atomicAdd(&counts[cell_id<DIM>(g, p)], 1);
}

// Exclusive scan of counts[0..m) into start[0..m], one block; cursor[c] = start[c].
__global__ void __launch_bounds__(1024)
k_cull_scan(const int *__restrict__ counts, int m, int *start, int *cursor) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int per = (m + 1023) / 1024;
    const int a = t * per, b = min(a + per, m);
    int s = 0;
    for (int c = a; c < b; ++c) s += counts[c];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
        const int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int c = a; c < b; ++c) {
        start[c] = run;
        cursor[c] = run;
        run += counts[c];
    }
    if (t == 1023) start[m] = part[1023];
}

// Block-privatised counting for the samples (grids of at most kCullLdsCells cells):
// block b takes samples [b chunk, (b + 1) chunk) and counts them per cell in LDS.
constexpr int kCullLdsCells = 8192;
constexpr int kCullSortBlocks = 256;

template <int DIM>
__global__ void __launch_bounds__(1024)
k_cull_bcount(CullGridDev g, const float *__restrict__ x, int64_t n, int m, int64_t chunk,
              int *bc) {
    __shared__ int hist[kCullLdsCells];
    for (int c = threadIdx.x; c < m; c += blockDim.x) hist[c] = 0;
    __syncthreads();
    const int64_t a = (int64_t)blockIdx.x * chunk, b = min(a + chunk, n);
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) {
        float p[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) p[k] = x[(size_t)k * n + i];
        atomicAdd(&hist[cell_id<DIM>(g, p)], 1);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < m; c += blockDim.x) bc[(size_t)blockIdx.x * m + c] = hist[c];
}

// Per cell: the total over blocks, and each block's offset within the cell (bc is
// overwritten by the exclusive prefix over blocks).
__global__ void __launch_bounds__(kCullBlock)
k_cull_bprefix(int *bc, int nblk, int m, int *total) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    int run = 0;
    for (int b = 0; b < nblk; ++b) {
        const int v = bc[(size_t)b * m + c];
        bc[(size_t)b * m + c] = run;
        run += v;
    }
    total[c] = run;
}

// order[start[cell] + block offset + rank within the block] = i (the rank is the
// arrival order of the block's LDS atomics; the sample order only affects speed)
template <int DIM>
__global__ void __launch_bounds__(1024)
k_cull_bscatter(CullGridDev g, const float *__restrict__ x, int64_t n, int m, int64_t chunk,
                const int *__restrict__ start, const int *__restrict__ boff, uint32_t *order) {
    __shared__ int cur[kCullLdsCells];
    for (int c = threadIdx.x; c < m; c += blockDim.x)
        cur[c] = start[c] + boff[(size_t)blockIdx.x * m + c];
    __syncthreads();
    const int64_t a = (int64_t)blockIdx.x * chunk, b = min(a + chunk, n);
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) {
        float p[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) p[k] = x[(size_t)k * n + i];
        const int pos = atomicAdd(&cur[cell_id<DIM>(g, p)], 1);
        order[pos] = (uint32_t)i;
    }
}

// pos = cursor[cell]++ ; order[pos] = i   (order within a cell: arrival order)
template <int DIM>
__global__ void __launch_bounds__(kCullBlock)
k_cull_scatter(CullGridDev g, const float *__restrict__ x, int64_t n, int *cursor,
               uint32_t *order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float p[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) p[k] = x[(size_t)k * n + i];
    const int pos = atomicAdd(&cursor[cell_id<DIM>(g, p)], 1);
    order[pos] = (uint32_t)i;
}

// Each cell's entries in increasing index order (insertion sort, one thread per cell).
__global__ void __launch_bounds__(kCullBlock)
k_cull_sort_cells(const int *__restrict__ start, int m, uint32_t *order) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    const int a = start[c], b = start[c + 1];
    for (int i = a + 1; i < b; ++i) {
        const uint32_t v = order[i];
        int j = i - 1;
        while (j >= a && order[j] > v) {
            order[j + 1] = order[j];
            --j;
        }
        order[j + 1] = v;
    }
}

// p[i] *= a for i < n.
__global__ void k_scale_f32(float *p, int64_t n, float a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = a * p[i];
}

// dst[k][pos] = src[k][order[pos]] for the rows k < rows of an SoA array [rows][n].
__global__ void __launch_bounds__(kCullBlock)
k_cull_gather(const float *__restrict__ src, int rows, int64_t n, const uint32_t *__restrict__ order,
              float *dst) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t i = order[p];
    for (int k = 0; k < rows; ++k) dst[(size_t)k * n + p] = src[(size_t)k * n + i];
}

template <int DIM>
__global__ void __launch_bounds__(kCullBlock)
k_cull_morph(CullGridDev g, const float *__restrict__ hs, const float *__restrict__ ws, int M,
             const float *__restrict__ bias, const int *__restrict__ cell_start, float kappa, float gscale,
             const float *__restrict__ xs, const uint32_t *__restrict__ order, int64_t n, int T,
             float eta, float *x_out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = p < n;
    const int64_t pc = live ? p : n - 1;
    const float beta = *bias;
    float x[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) x[k] = xs[(size_t)k * n + pc];
    for (int st = 0; st < T; ++st) {
        int my[DIM], lo[DIM], hi[DIM];
        float xk[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            xk[k] = kappa * x[k];
            my[k] = cull_cell(x[k], g.lo[k], g.inv_cell, g.nc[k]);
            int mn = my[k], mx = my[k];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                mn = min(mn, __shfl_xor(mn, off, 64));
                mx = max(mx, __shfl_xor(mx, off, 64));
            }
            lo[k] = __builtin_amdgcn_readfirstlane(max(mn - 1, 0));
            hi[k] = __builtin_amdgcn_readfirstlane(min(mx + 1, g.nc[k] - 1));
        }
        float s = 0.0f, gx[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) gx[k] = 0.0f;
        const int cz0 = DIM == 3 ? lo[2] : 0, cz1 = DIM == 3 ? hi[2] : 0;
        for (int cz = cz0; cz <= cz1; ++cz)
            for (int cy = lo[1]; cy <= hi[1]; ++cy)
                for (int cx = lo[0]; cx <= hi[0]; ++cx) {
                    bool near = cx >= my[0] - 1 && cx <= my[0] + 1 && cy >= my[1] - 1 &&
                                cy <= my[1] + 1;
                    if (DIM == 3) near = near && cz >= my[2] - 1 && cz <= my[2] + 1;
                    const int cid = cx + g.nc[0] * (cy + g.nc[1] * cz);
                    const int a = cell_start[cid], b = cell_start[cid + 1];
                    if (!near) continue;
                    // groups of 8 hinges: one batch of scalar loads per group, so the
                    // memory latency is paid once per 8 pairs
                    int j = a;
                    for (; j + 8 <= b; j += 8) {
                        float hv[DIM][8], wv[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
#pragma unroll
                            for (int k = 0; k < DIM; ++k) hv[k][u] = hs[(size_t)k * M + j + u];
                            wv[u] = ws[j + u];
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            float d[DIM], r2 = 0.0f;
#pragma unroll
                            for (int k = 0; k < DIM; ++k) {
                                d[k] = xk[k] - hv[k][u];
                                r2 = fmaf(d[k], d[k], r2);
                            }
                            const float wp = wv[u] * exp2_fast(-r2);
                            s += wp;
#pragma unroll
                            for (int k = 0; k < DIM; ++k) gx[k] = fmaf(wp, d[k], gx[k]);
                        }
                    }
                    for (; j < b; ++j) {
                        float d[DIM], r2 = 0.0f;
#pragma unroll
                        for (int k = 0; k < DIM; ++k) {
                            d[k] = xk[k] - hs[(size_t)k * M + j];
                            r2 = fmaf(d[k], d[k], r2);
                        }
                        const float wp = ws[j] * exp2_fast(-r2);
                        s += wp;
#pragma unroll
                        for (int k = 0; k < DIM; ++k) gx[k] = fmaf(wp, d[k], gx[k]);
                    }
                }
        float c, sp;
        sigmoid_and_slope(s + beta, c, sp);
        const float step = eta * sp * gscale;  // grad s = -gscale * sum w phi (kappa x - kappa h)
#pragma unroll
        for (int k = 0; k < DIM; ++k) x[k] = fmaf(step, gx[k], x[k]);
    }
    if (!live) return;
    const uint32_t i = order[p];
#pragma unroll
    for (int k = 0; k < DIM; ++k) x_out[(size_t)k * n + i] = x[k];
}

static size_t al256c(size_t b) { return (b + 255) & ~(size_t)255; }

static int64_t cull_cells(const pdmp_cull_grid &g) {
    int64_t m = 1;
    for (int k = 0; k < g.dim; ++k) m *= g.nc[k];
    return m;
}

// Per-block cell counts of the samples (LDS path only).
static int64_t cull_bc_ints(int64_t m) {
    return m <= kCullLdsCells ? (int64_t)kCullSortBlocks * m : 0;
}

size_t cull_ws_bytes(const pdmp_cull_grid &g, int M, int64_t n) {
    const int64_t m = cull_cells(g);
    return 2 * al256c((size_t)(g.dim + 1) * M * 4) + al256c((size_t)M * 4) +
           6 * al256c((size_t)(m + 1) * 4) + al256c((size_t)n * 4) + al256c((size_t)g.dim * n * 4) +
           al256c((size_t)cull_bc_ints(m) * 4);
}

int32_t launch_morph_culled(const pdmp_occupancy &occ, const pdmp_cull_grid &cg, const float *in,
                            float *out, int64_t n, int T, float eta, void *ws, hipStream_t st) {
    const int dim = occ.dim, M = occ.n_hinges;
    const int64_t m = cull_cells(cg);
    CullGridDev g;
    for (int k = 0; k < 3; ++k) {
        g.lo[k] = k < dim ? cg.lo[k] : 0.0f;
        g.nc[k] = k < dim ? cg.nc[k] : 1;
    }
    g.inv_cell = cg.inv_cell;
    char *p = (char *)ws;
    float *hw = (float *)p;  // [dim + 1][M]: hinges then weights, unsorted copy rows
    p += al256c((size_t)(dim + 1) * M * 4);
    float *hsw = (float *)p;  // sorted
    p += al256c((size_t)(dim + 1) * M * 4);
    uint32_t *horder = (uint32_t *)p;
    p += al256c((size_t)M * 4);
    int *hcount = (int *)p;
    p += al256c((size_t)(m + 1) * 4);
    int *hstart = (int *)p;
    p += al256c((size_t)(m + 1) * 4);
    int *hcur = (int *)p;
    p += al256c((size_t)(m + 1) * 4);
    int *scount = (int *)p;
    p += al256c((size_t)(m + 1) * 4);
    int *sstart = (int *)p;
    p += al256c((size_t)(m + 1) * 4);
    int *scur = (int *)p;
    p += al256c((size_t)(m + 1) * 4);
    uint32_t *sorder = (uint32_t *)p;
    p += al256c((size_t)n * 4);
    float *xs = (float *)p;
    p += al256c((size_t)dim * n * 4);
    int *bcnt = (int *)p;  // [kCullSortBlocks][m] (LDS path)
    const bool lds_sort = m <= kCullLdsCells;
    if (int32_t ge = grid_guard((n + kCullBlock - 1) / kCullBlock, kCullBlock, "k_cull_morph"))
        return ge;
    const int nblk = (int)std::min<int64_t>(kCullSortBlocks, (n + 1023) / 1024);
    const int64_t chunk = (n + nblk - 1) / nblk;

    auto fill = [&](int *q, int64_t cnt) {
        hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, q,
                           cnt, 0);
    };
    const dim3 bh((unsigned)((M + kCullBlock - 1) / kCullBlock)), bs((unsigned)((n + kCullBlock - 1) / kCullBlock));
    const dim3 bc((unsigned)((m + kCullBlock - 1) / kCullBlock)), blk(kCullBlock);
    // hinges (and weights as the last row) into one [dim + 1][M] array, sorted by cell
    hipError_t e = hipMemcpyAsync(hw, occ.hinges, (size_t)dim * M * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hw + (size_t)dim * M, occ.weights, (size_t)M * 4,
                           hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
        set_error("hipMemcpyAsync: %s", hipGetErrorString(e));
        return PDMP_EDEVICE;
    }
    fill(hcount, m);
    if (!lds_sort) fill(scount, m);
#define PDMP_CULL_D(D)                                                                          \
    hipLaunchKernelGGL((k_cull_count<D>), bh, blk, 0, st, g, occ.hinges, (int64_t)M, hcount);   \
    hipLaunchKernelGGL(k_cull_scan, dim3(1), dim3(1024), 0, st, hcount, (int)m, hstart, hcur);  \
    hipLaunchKernelGGL((k_cull_scatter<D>), bh, blk, 0, st, g, occ.hinges, (int64_t)M, hcur,    \
                       horder);                                                                 \
    hipLaunchKernelGGL(k_cull_sort_cells, bc, blk, 0, st, hstart, (int)m, horder);              \
    hipLaunchKernelGGL(k_cull_gather, bh, blk, 0, st, hw, D + 1, (int64_t)M, horder, hsw);      \
    if (lds_sort) {                                                                             \
        hipLaunchKernelGGL((k_cull_bcount<D>), dim3(nblk), dim3(1024), 0, st, g, in, n, (int)m, \
                           chunk, bcnt);                                                        \
        hipLaunchKernelGGL(k_cull_bprefix, bc, blk, 0, st, bcnt, nblk, (int)m, scount);         \
        hipLaunchKernelGGL(k_cull_scan, dim3(1), dim3(1024), 0, st, scount, (int)m, sstart,     \
                           scur);                                                               \
        hipLaunchKernelGGL((k_cull_bscatter<D>), dim3(nblk), dim3(1024), 0, st, g, in, n,       \
                           (int)m, chunk, sstart, bcnt, sorder);                                \
    } else {                                                                                    \
        hipLaunchKernelGGL((k_cull_count<D>), bs, blk, 0, st, g, in, n, scount);                \
        hipLaunchKernelGGL(k_cull_scan, dim3(1), dim3(1024), 0, st, scount, (int)m, sstart,     \
                           scur);                                                               \
        hipLaunchKernelGGL((k_cull_scatter<D>), bs, blk, 0, st, g, in, n, scur, sorder);        \
    }                                                                                           \
    hipLaunchKernelGGL(k_cull_gather, bs, blk, 0, st, in, D, n, sorder, xs)
    if (dim == 2) {
        PDMP_CULL_D(2);
    } else {
        PDMP_CULL_D(3);
    }
#undef PDMP_CULL_D
    if (int32_t r = check_launch("cull setup")) return r;
    float kappa, gscale;
    derive_scales(occ.lengthscale, kappa, gscale);
    hipLaunchKernelGGL(k_scale_f32, dim3((unsigned)((dim * M + kCullBlock - 1) / kCullBlock)), blk, 0,
                       st, hsw, (int64_t)dim * M, kappa);
    const float *bias = occ.weights + M;
    if (dim == 2)
        hipLaunchKernelGGL((k_cull_morph<2>), bs, blk, 0, st, g, hsw, hsw + (size_t)2 * M, M, bias,
                           hstart, kappa, gscale, xs, sorder, n, T, eta, out);
    else
        hipLaunchKernelGGL((k_cull_morph<3>), bs, blk, 0, st, g, hsw, hsw + (size_t)3 * M, M, bias,
                           hstart, kappa, gscale, xs, sorder, n, T, eta, out);
    return check_launch("k_cull_morph");
}

}  // namespace pdmp
