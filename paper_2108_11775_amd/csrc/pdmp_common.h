// pdmp_common.h -- internal helpers shared by the HIP translation units of libpdmp.
// Not part of the public ABI (include/pdmp.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>

#include "pdmp.h"

namespace pdmp {

// Thread-local message of the last failure, returned by pdmp_last_error().
void set_error(const char *fmt, ...);
const char *last_error();

// Launch-status helper: returns PDMP_EDEVICE (with the HIP message) if the last
// launch on this thread failed.
int32_t check_launch(const char *what);

// One dispatch covers at most 2^32 - 1 work-items per grid dimension (the dispatch
// packet counts the grid in work-items, 32 bits): a larger grid would run truncated,
// without an error.  Launchers whose grid grows with the batch check it first and
// return PDMP_EINVAL (nothing launched for it).
inline int32_t grid_guard(int64_t blocks, int64_t threads, const char *what) {
    if (blocks >= 0 && threads >= 0 && blocks * threads <= 0xffffffffll) return 0;
    set_error("%s: %lld blocks of %lld threads exceed one dispatch (2^32 - 1 work-items); "
              "split the batch",
              what, (long long)blocks, (long long)threads);
    return PDMP_EINVAL;
}

// Argument check of an extern "C" entry point: on failure, record the message and
// return PDMP_EINVAL.
#define PDMP_REQUIRE(cond, ...)           \
    do {                                  \
        if (!(cond)) {                    \
            ::pdmp::set_error(__VA_ARGS__); \
            return PDMP_EINVAL;           \
        }                                 \
    } while (0)

// log2(e): exp(-r^2/(2 l^2)) = exp2(-(kappa*r)^2) with kappa^2 = log2(e)/(2 l^2).
constexpr float kLog2e = 1.4426950408889634f;

// Hinge staging in LDS: hinges are grouped in chunks of four; a chunk holds DIM
// float4 rows of prescaled coordinates (kappa*h) followed by one float4 of weights,
// so one ds_read_b128 feeds four hinges.  Chunks past M are padded with w = 0.
template <int DIM>
struct ChunkLayout {
    static constexpr int kRows = DIM + 1;             // float4 rows per chunk
    static constexpr int kBytes = 16 * kRows;         // bytes per chunk of 4 hinges
};

// Resident LDS budget per block for hinge chunks (bytes).  64 KiB keeps two
// 1024-thread blocks per CU within the 160 KiB of a gfx950 CU.
constexpr int kHingeLdsBytes = 64 * 1024;

__host__ __device__ inline int chunks_for(int M) { return (M + 3) / 4; }

// Number of hinge chunks one LDS tile holds.
template <int DIM>
__host__ __device__ constexpr int tile_chunks() { return kHingeLdsBytes / ChunkLayout<DIM>::kBytes; }

__device__ __forceinline__ float f4c(const float4 &v, int u) {
    return u == 0 ? v.x : (u == 1 ? v.y : (u == 2 ? v.z : v.w));
}

// v_exp_f32: 2^x with ~1 ulp error; flushes to 0 for very negative arguments.
__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// sigma(s) and sigma'(s) = sigma(1 - sigma) from e = exp(-|s|) in (0, 1], which keeps
// both to a few ulp relative even where sigma is within rounding of 0 or 1.  The
// reciprocal of 1 + e in [1, 2] is v_rcp_f32's (within 1 ulp; no range to guard).
__device__ __forceinline__ void sigmoid_and_slope(float s, float &c, float &sp) {
    float e = exp2_fast(-fabsf(s) * kLog2e);
    float inv = __builtin_amdgcn_rcpf(1.0f + e);
    c = s >= 0.0f ? inv : e * inv;
    sp = e * inv * inv;
}

// kappa^2 = log2(e) / (2 l^2):  exp(-r^2/(2 l^2)) = exp2(-(kappa r)^2).
// grad s = -(1/l^2) sum w phi (x - h) = -(1/(l^2 kappa)) sum w phi (kappa x - kappa h).
inline void derive_scales(float ell, float &kappa, float &gscale) {
    const double l = ell;
    const double k = std::sqrt(1.4426950408889634 / (2.0 * l * l));
    kappa = (float)k;
    gscale = (float)(1.0 / (l * l * k));
}

// Path recording of the morph kernels: state k (k = 0..T, state 0 the input) of every
// sample i with i % stride == 0 is written to p[(k rows + r) nt + i / stride], r over
// the sample's rows (dim, or n_dof for the arm).  p == nullptr records nothing; the
// arithmetic of the morph is the same either way.
struct Traj {
    float *p = nullptr;
    int64_t stride = 1, nt = 0;
};

// Whether sample i (of n) is recorded, and its column.
__device__ __forceinline__ bool traj_col(const Traj &tr, int64_t i, int64_t n, int64_t &col) {
    col = i / tr.stride;
    return tr.p != nullptr && i < n && i - col * tr.stride == 0;
}

// Record state k of a recorded sample (rows values).
template <int R>
__device__ __forceinline__ void traj_put(const Traj &tr, int k, int64_t col, const float (&v)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) tr.p[((size_t)k * R + r) * (size_t)tr.nt + (size_t)col] = v[r];
}

// ---- launchers (host side, one per kernel family) ----

enum RbfMode { kEval = 0, kGrad = 1, kMorph = 2, kGradBwd = 3, kLogdet = 4, kInverse = 5 };

// One RBF-sum launch: for every "sample" x_i (n of them) sum over the weighted
// "hinge" set (M of them).  The roles are symmetric: with hinges = data points,
// weights = upstream gradients and x_in = hinge positions, kEval computes Phi^T g.
struct RbfArgs {
    const float *hinges = nullptr, *weights = nullptr;
    int M = 0;
    const float *bias = nullptr;  // nullable
    float kappa = 0, gscale = 0;
    const float *x_in = nullptr;
    int64_t n = 0;
    int T = 1;
    float eta = 0;
    float *c_out = nullptr, *s_out = nullptr, *g_out = nullptr, *x_out = nullptr;
    const float *g_in = nullptr;  // kGradBwd upstream gradient
    int chain = 0;                // kGradBwd: multiply by sigma'(s)
    int splits = 1;               // kEval: hinge-range splits (partial sums)
    Traj traj;                    // kMorph: optional path recording
};

int32_t launch_rbf(int dim, int mode, const RbfArgs &a, hipStream_t st);
int32_t launch_grid2d(int mode, const RbfArgs &a, int g0, int g1, hipStream_t st);
// The morph of a large 2-D grid batch in spatial order (counting sort into `ws`, then
// the kernel that skips exact zeros); PDMP_EUNSUPPORTED when the batch takes another
// path, whose workspace size is then 0.
size_t grid2d_sorted_ws_bytes(int g0, int g1, int64_t n, int T);
int32_t launch_grid2d_sorted(const RbfArgs &a, int g0, int g1, void *ws, hipStream_t st);
// The counting sort alone (into a workspace of grid2d_sorted_ws_bytes): the
// permutation in ws and the samples per part.
int32_t launch_sort2d(const float *hinges, int g0, int g1, const float *x, int64_t n, void *ws,
                      hipStream_t st, const uint32_t **perm, int64_t *part);
int32_t launch_grid3d_ws(int mode, const RbfArgs &a, const int *grid, hipStream_t st);
int32_t launch_arm_grid3d(const pdmp_arm &arm, const float *h, const float *w, int M,
                          const int *grid, float kappa, float gscale, const float *qi, float *qo,
                          int64_t n, int T, float eta, const uint32_t *n_active, bool morph,
                          float thresh, float *maxc, uint8_t *flag, hipStream_t st,
                          const Traj &traj = Traj());
// The allocation-free entry point's static scratch: its size, and the current
// device's copy (device address, taken once per device).
size_t noalloc_scratch_bytes();
int32_t noalloc_scratch(void **ptr);
// Enqueue the device check that the hinges are the tensor grid `grid` states (a
// mismatch is reported by the next pdmp_sync on the device), and take that report.
int32_t launch_grid_check(int dim, const float *hinges, int M, const int *grid, hipStream_t st);
int32_t take_grid_mismatch(bool &mismatch);
// The split scheme of the grid morph kernels for these operands, written to out (device):
// 2 (FP16 parts) or 1 (BF16 parts); PDMP_EUNSUPPORTED when no grid kernel covers them.
int32_t launch_grid2d_scheme(const float *hinges, const float *weights, int g0, int g1,
                             float kappa, int32_t *out, hipStream_t st);
int32_t launch_grid3d_scheme(const float *hinges, const float *weights, const int *grid, int M,
                             float kappa, int32_t *out, hipStream_t st);
// The occupancy evaluation of one RBF launch, through the grid factorisation when
// `grid` describes one the grid kernels support, else the pairwise kernel.
int32_t launch_occ_any(int dim, int mode, const RbfArgs &a, const int *grid, hipStream_t st);
int32_t launch_uniform(uint64_t seed, uint32_t sid, const float *lo, const float *hi, int dim,
                       int64_t n, float *out, hipStream_t st);
int32_t launch_label_discs(const pdmp_discs &sc, const float *x, int64_t n, uint8_t *out,
                           uint64_t *n_hit, hipStream_t st);
int32_t launch_label_boxes(const pdmp_boxes &sc, const float *x, int64_t n, uint8_t *out,
                           uint64_t *n_hit, hipStream_t st);
int32_t launch_label_configs(const pdmp_arm &arm, const pdmp_boxes &sc, const float *q, int64_t n,
                             uint8_t *out, uint64_t *n_hit, hipStream_t st);
int32_t launch_morph_arm(const pdmp_arm &arm, const float *h, const float *w, int M, float kappa,
                         float gscale, const float *qi, float *qo, int64_t n, int T, float eta,
                         const uint32_t *n_active, hipStream_t st, const Traj &traj = Traj());
int32_t launch_arm_max_occ(const pdmp_arm &arm, const float *h, const float *w, int M, float kappa,
                           const float *q, int64_t n, float thresh, float *maxc, uint8_t *flag,
                           hipStream_t st);
int32_t launch_compact(const pdmp_arm &arm, const uint8_t *flag, const float *q, int64_t n,
                       uint32_t *counts, uint32_t *offs, uint32_t *total, uint32_t *idx, float *qc,
                       hipStream_t st);
int32_t launch_scatter(const pdmp_arm &arm, const uint32_t *idx, const uint32_t *total,
                       const float *qc, int64_t n, float *out, hipStream_t st);
int64_t mlp_nparams(const pdmp_mlp &m);
size_t mlp_acts_bytes(const pdmp_mlp &m, int64_t B);
size_t mlp_fwd_ws_bytes(const pdmp_mlp &m, int64_t B);
size_t mlp_bwd_ws_bytes(const pdmp_mlp &m, int64_t B);
int32_t launch_mlp_forward(const pdmp_mlp &m, const float *q, int64_t B, float *qhat, void *acts,
                           void *ws, hipStream_t st);
int32_t launch_mlp_backward(const pdmp_mlp &m, const float *qhat, const float *target, int64_t B,
                            void *acts, float *grad, float *loss, void *ws, hipStream_t st,
                            const uint8_t *hard = nullptr, float hard_w = 1.0f);
int32_t launch_f32_to_bf16(const float *x, int64_t n, uint16_t *y, hipStream_t st);
int32_t launch_fk_points(const pdmp_arm &arm, const float *q, int64_t n, float *pts,
                         hipStream_t st);
size_t bwd_ws_bytes(int dim, int M, int64_t n);
size_t bce_ws_bytes(int64_t n);
size_t fit_ws_bytes(int dim, int M, int64_t n);
// Backward of the logit; grad_w goes through the grid kernels when `grid` fits them.
int32_t launch_logit_bwd(int dim, const float *hinges, const float *weights, int M,
                         const int *grid, float ell, const float *x, int64_t n, const float *g,
                         const float *s_fwd, float *grad_w, float *grad_x, float grad_scale,
                         const float *decay_w, float l2, void *ws, hipStream_t st);
// Partial rows of Phi^T g on a hinge grid (PDMP_EUNSUPPORTED if it does not fit).
int32_t launch_grid_wgrad(int dim, const float *hinges, int M, const int *grid, float kappa,
                          const float *x, int64_t n, const float *g, float *part, int *rows,
                          hipStream_t st);
size_t wgrad_rows_max(int64_t n);
// Forward morph with log-determinant (kLogdet) or its inverse by fixed point (kInverse);
// with ws (grid2d_sorted_ws_bytes of the batch, nonzero) a large 2-D grid batch runs
// in spatial order, exact zeros skipped (the same bits).
int32_t launch_morph_inverse(int dim, int mode, const float *hinges, const float *weights, int M,
                             const int *grid, float ell, const float *x_in, int64_t n, int T,
                             float eta, int iters, float *x_out, float *logdet, float *resid,
                             hipStream_t st, void *ws = nullptr);
// Epsilon mixture: keep[i] = (u_i < eps) from Philox, out[:, i] = x0[:, i] where kept.
int32_t launch_mix_select(uint64_t seed, uint32_t sid, float eps, int dim, int64_t n,
                          const float *x0, float *out, uint8_t *keep, hipStream_t st);
size_t cull_ws_bytes(const pdmp_cull_grid &g, int M, int64_t n);
int32_t launch_morph_culled(const pdmp_occupancy &occ, const pdmp_cull_grid &cg, const float *in,
                            float *out, int64_t n, int T, float eta, void *ws, hipStream_t st);
// out[j] = scale * sum_r part[r m + j] (+ add_scale add[j]), fixed order.
int32_t launch_sum_rows(const float *part, int rows, int64_t m, double scale, const float *add,
                        float add_scale, float *out, hipStream_t st);
// out = sa * sum(x[0..n)) + sb * sum(b[0..nb)), fixed order; parts: 1024 doubles.
int32_t launch_sum_with(const float *x, int64_t n, double sa, const double *b, int nb, double sb,
                        float *out, double *parts, hipStream_t st);
size_t tanh_fit_ws_bytes(const pdmp_tanh_net &net, int64_t n);
int32_t launch_tanh_loss_grad(const pdmp_tanh_net &net, const float *x, const uint8_t *y,
                              int64_t n, float l2, float *loss, float *grad, void *ws,
                              hipStream_t st);
int32_t launch_tanh_fit(const pdmp_tanh_net &net, const float *x, const uint8_t *y, int64_t n,
                        int steps, float lr, float l2, float b1, float b2, float eps, float *m,
                        float *v, int t0, float *loss_out, void *ws, hipStream_t st);
// The tanh network's forward split scheme, as its kernels choose it: *out (device) = 2
// (FP16 parts) or 1 (BF16 parts).
int32_t launch_tanh_scheme(const pdmp_tanh_net &net, int32_t *out, hipStream_t st);
// The tanh occupancy network: kEval, kGrad or kMorph over n >= 1 points.
int32_t launch_tanh_net(const pdmp_tanh_net &net, int mode, const float *x, int64_t n, int T,
                        float eta, float *c_out, float *s_out, float *g_out, float *x_out,
                        hipStream_t st);
int32_t launch_bce(const float *s, const uint8_t *y, int64_t n, const float *g_scale, float *loss,
                   float *g_out, double *parts, hipStream_t st);
int32_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, int64_t n_decay,
                    int t, float lr, float b1, float b2, float eps, float l2, hipStream_t st);
int32_t launch_fit(int dim, const float *hinges, int M, const int *grid, float ell, float *wb,
                   const float *pts, const uint8_t *y, int64_t n, const pdmp_fit_opts &o,
                   float *loss_out, void *ws, hipStream_t st);

}  // namespace pdmp
