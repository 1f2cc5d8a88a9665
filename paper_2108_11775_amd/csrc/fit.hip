// fit.hip -- occupancy fit (Sec. 3.1: binary cross-entropy, gradient-descent and Adam
// optimisers) and the hand-written backward of the occupancy.
//
// Loss, full batch:  L(w, beta) = (1/n) sum_i BCE(sigma(s_i), y_i) + (l2/2) |w|^2.
// Gradient:          dL/dw_j = (1/n) sum_i r_i phi_ij + l2 w_j,  dL/dbeta = (1/n) sum_i r_i,
//                    r_i = sigma(s_i) - y_i.
// Backward of s(x; w, beta) for an upstream g:  grad_w = Phi^T g, grad_beta = sum g,
//                    grad_x_i = g_i grad s(x_i)   (with s_fwd: g_i sigma'(s_i) grad s(x_i)).
//
// Phi^T g is the same RBF sum as the forward with the roles of points and hinges
// exchanged (phi depends only on |x_i - h_j|), so it runs on the forward kernel:
// the data points become the LDS-staged weighted set, the hinges the lanes.  The
// point set is split into ranges of at most one LDS tile; each range writes a
// partial row and the rows are summed in a fixed order.  Every reduction here is
// fixed-order (block-range sums, then one block), so results are deterministic.
#include "pdmp_common.h"

namespace pdmp {

constexpr int kRedBlock = 256;
constexpr int kRedMaxBlocks = 1024;

__host__ __device__ inline int red_blocks(int64_t n) {
    int64_t b = (n + kRedBlock * 8 - 1) / (kRedBlock * 8);
    if (b < 1) b = 1;
    if (b > kRedMaxBlocks) b = kRedMaxBlocks;
    return (int)b;
}

// Fixed-order tree over the block's 256 partials in LDS.
__device__ __forceinline__ double block_tree_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (unsigned off = kRedBlock / 2; off >= 1; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    return sh[0];
}

// Per block: contiguous range, thread-strided sequential sums, tree.
// mode 0: sum x;  mode 1: sum x^2 over the first n entries.
__global__ void __launch_bounds__(kRedBlock)
k_sum_partial(const float *__restrict__ x, int64_t n, int mode, double *parts) {
    __shared__ double sh[kRedBlock];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = (int64_t)blockIdx.x * per;
    const int64_t b1 = b0 + per < n ? b0 + per : n;
    double acc = 0.0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kRedBlock) {
        const double v = x[i];
        acc += mode == 1 ? v * v : v;
    }
    const double t = block_tree_sum(acc, sh);
    if (threadIdx.x == 0) parts[blockIdx.x] = t;
}

// BCE on logits: g_i = (sigma(s_i) - y_i) * inv_n; per-block sum of
// max(s,0) - y s + log(1 + exp(-|s|)).
__global__ void __launch_bounds__(kRedBlock)
k_bce_partial(const float *__restrict__ s, const uint8_t *__restrict__ y, int64_t n, float inv_n,
              const float *__restrict__ g_scale, float *g_out, double *parts) {
    __shared__ double sh[kRedBlock];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = (int64_t)blockIdx.x * per;
    const int64_t b1 = b0 + per < n ? b0 + per : n;
    double acc = 0.0;
    const float gsc = g_scale ? *g_scale : 1.0f;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kRedBlock) {
        const float sv = s[i];
        const float yv = y[i] ? 1.0f : 0.0f;
        float c, sp;
        sigmoid_and_slope(sv, c, sp);
        if (g_out) g_out[i] = g_scale ? (c - yv) * inv_n * gsc : (c - yv) * inv_n;
        const float e = exp2_fast(-fabsf(sv) * kLog2e);
        acc += (double)(fmaxf(sv, 0.0f) - yv * sv) + (double)log1pf(e);
    }
    const double t = block_tree_sum(acc, sh);
    if (threadIdx.x == 0) parts[blockIdx.x] = t;
}

// out = sa * sum(a[0..na)) + sb * sum(b[0..nb)), fixed order, one block.
__global__ void __launch_bounds__(kRedBlock)
k_final(const double *__restrict__ a, int na, double sa, const double *__restrict__ b, int nb,
        double sb, float *out) {
    __shared__ double sh[kRedBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < na; i += kRedBlock) acc += a[i];
    const double ta = block_tree_sum(acc, sh);
    __syncthreads();
    acc = 0.0;
    if (b)
        for (int i = threadIdx.x; i < nb; i += kRedBlock) acc += b[i];
    const double tb = block_tree_sum(acc, sh);
    if (threadIdx.x == 0) *out = (float)(sa * ta + sb * tb);
}

// out[j] = scale * sum_{r < rows} part[r * m + j] (+ add[j] * add_scale).  A block
// owns 64 columns; its sixteen waves sum the rows r = ph (mod 16) in increasing order,
// issuing the loads four at a time (the adds keep the order), and the sixteen sums are
// added in a fixed order.  With few columns (4096 weights: 64 blocks) each thread's
// chain of loads is short.
constexpr int kSumPh = 16;

__global__ void __launch_bounds__(64 * kSumPh)
k_sum_rows(const float *__restrict__ part, int rows, int64_t m, double scale,
           const float *__restrict__ add, float add_scale, float *out) {
    __shared__ double sh[kSumPh][64];
    const int cl = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + cl;
    double acc = 0.0;
    if (j < m) {
        int r = ph;
        for (; r + 3 * kSumPh < rows; r += 4 * kSumPh) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = part[(size_t)(r + u * kSumPh) * m + j];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += v[u];
        }
        for (; r < rows; r += kSumPh) acc += part[(size_t)r * m + j];
    }
    sh[ph][cl] = acc;
    __syncthreads();
    if (ph != 0 || j >= m) return;
    double t = sh[0][cl];
#pragma unroll
    for (int q = 1; q < kSumPh; ++q) t += sh[q][cl];
    float v = (float)(t * scale);
    if (add) v = fmaf(add_scale, add[j], v);
    out[j] = v;
}

// g_eff[i] = g[i] * sigma'(s[i])
__global__ void __launch_bounds__(256)
k_chain_sigmoid(const float *__restrict__ g, const float *__restrict__ s, int64_t n, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float c, sp;
    sigmoid_and_slope(s[i], c, sp);
    out[i] = g[i] * sp;
}

// Gradient descent on [w (M), beta]: w -= lr (g + l2 w), beta -= lr_b g_beta.
__global__ void __launch_bounds__(256)
k_gd(float *w, const float *__restrict__ g, int M, float lr, float lr_b, float l2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < M) w[j] = w[j] - lr * fmaf(l2, w[j], g[j]);
    else if (j == M) w[M] = w[M] - lr_b * g[M];
}

// Adam (Kingma & Ba 2015, Algorithm 1); the first n_decay entries get l2 * p added to
// their gradient.  bc1 = 1/(1 - beta1^t), bc2 = 1/(1 - beta2^t).
__global__ void __launch_bounds__(256)
k_adam(float *p, const float *__restrict__ g, float *m, float *v, int64_t n, int64_t n_decay,
       float lr, float b1, float b2, float eps, float bc1, float bc2, float l2) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    float gk = g[k];
    if (k < n_decay) gk = fmaf(l2, p[k], gk);
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk * bc1, vh = vk * bc2;
    p[k] = p[k] - lr * mh / (sqrtf(vh) + eps);
}

// ------------------------------------------------------------------ host ---

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Splits of the point set for Phi^T g: at least enough block rows to fill the
// chip, and each range within one LDS tile.
static int bwd_splits(int dim, int M, int64_t n) {
    const int64_t nch = (n + 3) / 4;
    const int tile = dim == 2 ? tile_chunks<2>() : tile_chunks<3>();
    int64_t s = (nch + tile - 1) / tile;
    const int64_t hb = (M + 255) / 256;
    const int64_t want = (1024 + hb - 1) / hb;
    if (s < want) s = want;
    if (s > nch) s = nch;
    if (s < 1) s = 1;
    return (int)s;
}

// Partial rows: enough for the pairwise splits and for the grid kernels.
static size_t bwd_rows(int dim, int M, int64_t n) {
    const size_t a = (size_t)bwd_splits(dim, M, n), b = wgrad_rows_max(n);
    return a > b ? a : b;
}

size_t bwd_ws_bytes(int dim, int M, int64_t n) {
    return align256(bwd_rows(dim, M, n) * M * sizeof(float)) + align256((size_t)n * sizeof(float)) +
           align256(kRedMaxBlocks * sizeof(double));
}

// Phi^T g by the pairwise kernel with the roles exchanged: the data points are the
// weighted set and the hinges the lanes; S ranges of points give S partial rows.
static int32_t launch_pairwise_wgrad(int dim, const float *hinges, int M, float kappa,
                                     float gscale, const float *x, int64_t n, const float *gw,
                                     float *part, int S, hipStream_t st) {
    RbfArgs a;
    a.hinges = x;
    a.weights = gw;
    a.M = (int)n;
    a.bias = nullptr;
    a.kappa = kappa;
    a.gscale = gscale;
    a.x_in = hinges;
    a.n = M;
    a.s_out = part;
    a.splits = S;
    return launch_rbf(dim, kEval, a, st);
}

size_t bce_ws_bytes(int64_t) { return align256(kRedMaxBlocks * sizeof(double)); }

size_t fit_ws_bytes(int dim, int M, int64_t n) {
    return bwd_ws_bytes(dim, M, n) + 2 * align256((size_t)n * sizeof(float)) +
           align256((size_t)(M + 1) * sizeof(float)) + 2 * align256(kRedMaxBlocks * sizeof(double));
}

int32_t launch_sum(const float *x, int64_t n, int mode, double scale, float *out, double *parts,
                   hipStream_t st) {
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_sum_partial, dim3(nb), dim3(kRedBlock), 0, st, x, n, mode, parts);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedBlock), 0, st, parts, nb, scale,
                       (const double *)nullptr, 0, 0.0, out);
    return check_launch("k_sum");
}

int32_t launch_sum_rows(const float *part, int rows, int64_t m, double scale, const float *add,
                        float add_scale, float *out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_rows, dim3((unsigned)((m + 63) / 64)), dim3(64 * kSumPh), 0, st, part,
                       rows, m, scale, add, add_scale, out);
    return check_launch("k_sum_rows");
}

int32_t launch_sum_with(const float *x, int64_t n, double sa, const double *b, int nb, double sb,
                        float *out, double *parts, hipStream_t st) {
    const int nblk = red_blocks(n);
    hipLaunchKernelGGL(k_sum_partial, dim3(nblk), dim3(kRedBlock), 0, st, x, n, 0, parts);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedBlock), 0, st, parts, nblk, sa, b, nb, sb, out);
    return check_launch("k_sum_with");
}

// Backward of the logit: grad_w[0..M) = Phi^T g_eff, grad_w[M] = sum g_eff,
// grad_x = g (sigma'(s))? grad s.  `ws` holds partial rows, g_eff and reduce parts.
int32_t launch_logit_bwd(int dim, const float *hinges, const float *weights, int M,
                         const int *grid, float ell, const float *x, int64_t n, const float *g,
                         const float *s_fwd, float *grad_w, float *grad_x, float grad_scale,
                         const float *decay_w, float l2, void *ws, hipStream_t st) {
    float kappa, gscale;
    derive_scales(ell, kappa, gscale);
    char *p = (char *)ws;
    float *part = (float *)p;
    p += align256(bwd_rows(dim, M, n) * M * sizeof(float));
    float *geff = (float *)p;
    p += align256((size_t)n * sizeof(float));
    double *rparts = (double *)p;

    const float *gw = g;
    if (s_fwd) {
        if (int32_t e = grid_guard((n + 255) / 256, 256, "k_chain_sigmoid")) return e;
        hipLaunchKernelGGL(k_chain_sigmoid, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g,
                           s_fwd, n, geff);
        if (int32_t e = check_launch("k_chain_sigmoid")) return e;
        gw = geff;
    }
    if (grad_w) {
        int S = 0;
        int32_t e = launch_grid_wgrad(dim, hinges, M, grid, kappa, x, n, gw, part, &S, st);
        if (e == PDMP_EUNSUPPORTED) {
            S = bwd_splits(dim, M, n);
            e = launch_pairwise_wgrad(dim, hinges, M, kappa, gscale, x, n, gw, part, S, st);
        }
        if (e) return e;
        hipLaunchKernelGGL(k_sum_rows, dim3((unsigned)((M + 63) / 64)), dim3(64 * kSumPh), 0, st, part, S,
                           (int64_t)M, (double)grad_scale, decay_w, l2, grad_w);
        if (int32_t e2 = check_launch("k_sum_rows")) return e2;
        if (int32_t e2 = launch_sum(gw, n, 0, (double)grad_scale, grad_w + M, rparts, st)) return e2;
    }
    if (grad_x) {
        RbfArgs a;
        a.hinges = hinges;
        a.weights = weights;
        a.M = M;
        a.bias = weights + M;
        a.kappa = kappa;
        a.gscale = gscale;
        a.x_in = x;
        a.n = n;
        a.g_out = grad_x;
        a.g_in = g;
        a.chain = s_fwd ? 1 : 0;
        if (int32_t e = launch_rbf(dim, kGradBwd, a, st)) return e;
    }
    return PDMP_OK;
}

int32_t launch_bce(const float *s, const uint8_t *y, int64_t n, const float *g_scale, float *loss,
                   float *g_out, double *parts, hipStream_t st) {
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_bce_partial, dim3(nb), dim3(kRedBlock), 0, st, s, y, n,
                       (float)(1.0 / (double)n), g_scale, g_out, parts);
    if (loss)
        hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedBlock), 0, st, parts, nb, 1.0 / (double)n,
                           (const double *)nullptr, 0, 0.0, loss);
    return check_launch("k_bce");
}

int32_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, int64_t n_decay,
                    int t, float lr, float b1, float b2, float eps, float l2, hipStream_t st) {
    const double bc1 = 1.0 / (1.0 - std::pow((double)b1, (double)t));
    const double bc2 = 1.0 / (1.0 - std::pow((double)b2, (double)t));
    if (int32_t e = grid_guard((n + 255) / 256, 256, "k_adam")) return e;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n,
                       n_decay, lr, b1, b2, eps, (float)bc1, (float)bc2, l2);
    return check_launch("k_adam");
}

// One full-batch fit: `steps` iterations of forward, BCE, backward and update.
int32_t launch_fit(int dim, const float *hinges, int M, const int *grid, float ell, float *wb,
                   const float *pts, const uint8_t *y, int64_t n, const pdmp_fit_opts &o,
                   float *loss_out, void *ws, hipStream_t st) {
    float kappa, gscale;
    derive_scales(ell, kappa, gscale);
    char *p = (char *)ws;
    void *bwd_ws = p;
    p += bwd_ws_bytes(dim, M, n);
    float *s = (float *)p;
    p += align256((size_t)n * sizeof(float));
    float *g = (float *)p;
    p += align256((size_t)n * sizeof(float));
    float *grad = (float *)p;
    p += align256((size_t)(M + 1) * sizeof(float));
    double *bparts = (double *)p;
    p += align256(kRedMaxBlocks * sizeof(double));
    double *wparts = (double *)p;

    const int nb_n = red_blocks(n), nb_w = red_blocks(M);
    for (int t = 0; t < o.steps; ++t) {
        RbfArgs a;
        a.hinges = hinges;
        a.weights = wb;
        a.M = M;
        a.bias = wb + M;
        a.kappa = kappa;
        a.gscale = gscale;
        a.x_in = pts;
        a.n = n;
        a.s_out = s;
        if (int32_t e = launch_occ_any(dim, kEval, a, grid, st)) return e;
        hipLaunchKernelGGL(k_bce_partial, dim3(nb_n), dim3(kRedBlock), 0, st, s, y, n,
                           (float)(1.0 / (double)n), (const float *)nullptr, g, bparts);
        if (loss_out) {
            hipLaunchKernelGGL(k_sum_partial, dim3(nb_w), dim3(kRedBlock), 0, st, wb, (int64_t)M, 1,
                               wparts);
            hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedBlock), 0, st, bparts, nb_n,
                               1.0 / (double)n, wparts, nb_w, 0.5 * (double)o.l2, loss_out + t);
        }
        if (int32_t e = check_launch("fit step")) return e;
        // grad = Phi^T g + l2 w, grad_beta = sum g  (g already holds r_i / n)
        if (int32_t e = launch_logit_bwd(dim, hinges, wb, M, grid, ell, pts, n, g, nullptr, grad,
                                         nullptr, 1.0f, nullptr, 0.0f, bwd_ws, st))
            return e;
        if (o.optimizer == 0) {
            hipLaunchKernelGGL(k_gd, dim3((unsigned)((M + 1 + 255) / 256)), dim3(256), 0, st, wb, grad,
                               M, o.lr, o.lr_bias, o.l2);
            if (int32_t e = check_launch("k_gd")) return e;
        } else {
            if (int32_t e = launch_adam(wb, grad, o.adam_m, o.adam_v, M + 1, M, o.t0 + t + 1, o.lr,
                                        o.beta1, o.beta2, o.eps, o.l2, st))
                return e;
        }
    }
    return PDMP_OK;
}

}  // namespace pdmp
