/*
 * pdmp.h -- C ABI of the MI355X (gfx950) library for the batched diffeomorphic
 * morph of planner samples (Lai, Zhi, Hermans, Ramos, "Parallelised
 * Diffeomorphic Sampling-based Motion Planning").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns a pdmp_status.  Arguments are validated on the host
 *   before anything is launched; an invalid argument returns PDMP_EINVAL and
 *   launches nothing.  The message of the last failure on the calling thread is
 *   available from pdmp_last_error().  No C++ exception crosses this boundary.
 * - Array arguments are DEVICE pointers owned by the caller (the library never
 *   frees them and keeps no reference after the call returns).  Floating-point
 *   arrays are FP32, structure-of-arrays: a batch of n vectors of dimension d is
 *   d contiguous rows of n values, element (k, i) at [k*n + i].  Labels are uint8.
 *   Pointers must be 4-byte aligned; 16-byte alignment is recommended.
 * - Structs (pdmp_occupancy, pdmp_arm, scenes, options) are HOST structs passed by
 *   pointer; the device arrays they point to follow the rules above.
 * - `stream` is a hipStream_t (NULL = the null stream).  Every call only enqueues
 *   work and returns; results are valid once the stream has been synchronised.
 *   pdmp_sync() synchronises and reports any deferred device error.
 * - Scratch memory, where an operation needs it, is a caller-provided device
 *   workspace whose size the matching *_workspace_size() query returns.
 * - NaN or Inf inputs propagate through the arithmetic and are not trapped; the
 *   occupancy is defined on all of R^d, so out-of-domain samples are legal.
 * - Results are deterministic: the same call on the same inputs gives the same
 *   bits (fixed-order reductions, no floating-point atomics).
 * - Batch sizes: one kernel dispatch covers at most 2^32 - 1 work-items, and each
 *   kernel whose grid grows with the batch is checked against that before its
 *   launch; a call that would exceed it returns PDMP_EINVAL instead of running a
 *   truncated grid (work already enqueued by the call, such as a sort into the
 *   workspace, may have run).  The 2-D and 3-D grid paths take up to 2^31 - 1024
 *   points (two threads per point), the grid arm kernel up to 2^28 - 16
 *   configurations (sixteen threads each).
 */
#ifndef PDMP_H
#define PDMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PDMP_ABI_VERSION 1

typedef enum {
    PDMP_OK = 0,
    PDMP_EINVAL = 1,        /* invalid argument (null pointer, bad size or dimension) */
    PDMP_EUNSUPPORTED = 2,  /* valid but not supported by this build (e.g. too many DOF) */
    PDMP_EDEVICE = 3,       /* a HIP call or kernel launch failed */
    PDMP_ENOMEM = 4         /* caller workspace too small */
} pdmp_status;

/* Continuous occupancy of Sec. 3.1 in the Hilbert-map (RBF logistic) form:
 *   c(x) = sigma(s(x)),  s(x) = sum_{j<M} w_j exp(-|x - h_j|^2 / (2 l^2)) + beta.
 * hinges  : device [dim][M] hinge coordinates.
 * weights : device [M+1]; weights[M] holds the bias beta, so a fitted model stays
 *           entirely on the device.
 * grid    : optional.  All zero: the hinges are arbitrary points.  Otherwise the
 *           caller states that the hinges are the tensor grid of grid[0] x grid[1]
 *           (x grid[2] in 3-D) points, x fastest: hinge j = i0 + g0 (i1 + g1 i2) has
 *           coordinates (X0[i0], X1[i1], X2[i2]) read from the hinge array itself.
 *           The library may then evaluate the same sums through the factorisation
 *           phi_j = prod_k exp(-(x_k - X_k[i_k])^2 / (2 l^2)) (equal up to rounding)
 *           as contractions on the matrix cores at FP32 accuracy: two-part FP16
 *           splits when every nonzero |w| is at least 2^-19 of the largest and no
 *           two consecutive X0 coordinates are more than 6 sqrt(2 ln 2) l apart
 *           (morphs only), three-part BF16 splits otherwise.
 *           Every call that takes the factorised path first checks the statement
 *           on the device (each hinge equal, by value, to its axis coordinates; a
 *           NaN coordinate fails).  Hinges that are not that grid give undefined
 *           results of that call, which still runs to completion, and the next
 *           pdmp_sync() returns PDMP_EINVAL (the flag is per device and cleared by
 *           that report).
 * dim must be 2 or 3, M >= 1, lengthscale > 0 and finite. */
typedef struct {
    int32_t dim;
    int32_t n_hinges;
    const float *hinges;
    const float *weights;
    float lengthscale;
    int32_t grid[3];
} pdmp_occupancy;

/* Serial arm with standard Denavit-Hartenberg links (Sec. 3.2, body points):
 *   A_i = Rz(theta0_i + q_i) Tz(d_i) Tx(a_i) Rx(alpha_i), base frame at the origin.
 * Link i runs from the origin o_{i-1} of frame i-1 to o_i; it carries
 * pts_per_link body points o_{i-1} + (k/P)(o_i - o_{i-1}), k = 1..P.
 * Body point index p = (i-1)*P + (k-1).  1 <= n_dof <= 8, 1 <= P <= 16. */
#define PDMP_MAX_DOF 8
#define PDMP_MAX_PTS_PER_LINK 16
typedef struct {
    int32_t n_dof;
    int32_t pts_per_link;
    float a[PDMP_MAX_DOF];
    float d[PDMP_MAX_DOF];
    float alpha[PDMP_MAX_DOF];
    float theta0[PDMP_MAX_DOF];
} pdmp_arm;

/* Closed discs (2-D) and closed axis-aligned boxes (3-D): device arrays
 * centres [2][n] / [3][n], radii [n], half-extents [3][n]. */
typedef struct {
    int32_t n;
    const float *centres;
    const float *radii;
} pdmp_discs;

typedef struct {
    int32_t n;
    const float *centres;
    const float *half;
} pdmp_boxes;

int32_t pdmp_abi_version(void);
const char *pdmp_last_error(void);

/* Wait for all work on `stream`, then return PDMP_EDEVICE if any earlier launch
 * on it failed asynchronously. */
int32_t pdmp_sync(void *stream);

/* ---- prior samples (Sec. 3.3: the sampler draws large prior batches on the GPU).
 * x ~ U[lo, hi)^dim, written to out [dim][n].  Sample i, coordinate k uses word
 * k%4 of Philox4x32-10 (Salmon et al., SC 2011) at counter {i_lo, i_hi, k/4,
 * stream_id} and key {seed_lo, seed_hi}: u = (word >> 8) * 2^-24 and
 * x = lo_k + (hi_k - lo_k) * u evaluated in FP64 and rounded once to FP32, so the
 * values do not depend on n, on the launch or on the device.
 * lo, hi: HOST arrays [dim]; 1 <= dim <= 16; n >= 0. */
int32_t pdmp_uniform_samples(uint64_t seed, uint32_t stream_id, const float *lo,
                             const float *hi, int32_t dim, int64_t n, float *out,
                             void *stream);

/* ---- collision labels (the "feasible" test behind Table 1).  The inside test is
 * taken in FP64 on the FP32 inputs with the operation order stated here and no
 * contraction, so it is bit-reproducible:
 *   disc:  (x - cx)^2 + (y - cy)^2 <= r^2   as  a = dx*dx; b = dy*dy; a + b <= r*r
 *   box:   |x_a - c_a| <= e_a for a = 0, 1, 2.
 * out[i] = 1 if point i lies in any obstacle, else 0.
 * n_hit (nullable, device): receives the number of points labelled 1. */
int32_t pdmp_label_points_discs(const pdmp_discs *scene, const float *x, int64_t n,
                                uint8_t *out, uint64_t *n_hit, void *stream);
int32_t pdmp_label_points_boxes(const pdmp_boxes *scene, const float *x, int64_t n,
                                uint8_t *out, uint64_t *n_hit, void *stream);

/* A configuration collides iff any of its body points lies in any box.  The body
 * points are computed in FP64 from the FP32 joint values for this decision.
 * q: [n_dof][n]. */
int32_t pdmp_label_configs(const pdmp_arm *arm, const pdmp_boxes *scene, const float *q,
                           int64_t n, uint8_t *out, uint64_t *n_hit, void *stream);

/* ---- occupancy (Sec. 3.1: batched queries of the occupancy and its input
 * derivative on the GPU).
 * occupancy_eval: c_out[n] = c(x_i); s_out (nullable) [n] = s(x_i).
 * occupancy_grad: grad_out[dim][n] = grad_x c(x_i) = sigma'(s) grad s;
 *                 c_out (nullable) [n]. */
int32_t pdmp_occupancy_eval(const pdmp_occupancy *occ, const float *x, int64_t n,
                            float *c_out, float *s_out, void *stream);
int32_t pdmp_occupancy_grad(const pdmp_occupancy *occ, const float *x, int64_t n,
                            float *c_out, float *grad_out, void *stream);

/* ---- the morph (Sec. 3.2, Eq. 1 solved by explicit Euler; Eq. 3 for the arm).
 * arm == NULL: workspace morph in R^dim,  x_{k+1} = x_k - eta * grad c(x_k).
 * arm != NULL: joint-space morph, occ->dim must be 3, with the summed body-point
 *              cost C(q) = sum_p c(psi_p(q)) and
 *              q_{k+1} = q_k - eta * sum_p J_p(q_k)^T grad c(psi_p(q_k)).
 * in, out: [dim or n_dof][n]; in == out (in place) is allowed, other overlap is
 * not.  T >= 0 steps with constant eta (finite).  No clipping, no angle wrapping. */
int32_t pdmp_morph_samples(const pdmp_occupancy *occ, const pdmp_arm *arm, const float *in,
                           float *out, int64_t n, int32_t T, float eta, void *stream);

/* The same morph with a caller workspace (pdmp_morph_workspace_size bytes: 32 KiB of
 * cell counters and 4 bytes per sample; 0 means the call needs none and ws is
 * ignored).  A large batch (2^17 <= n <= 2^31 - 1024, T >= 1) on a 2-D hinge grid of at most
 * 64 x 64 is first ordered by a counting sort into 32 x 32 cells over the hinge range,
 * each eighth of the batch on its own (it is then read and written from one XCD), so
 * that the samples of a wave lie close together; each step then skips, wave by wave,
 * the parts of the factorised sums that are exact zeros for all of the wave's samples
 * (16-hinge blocks whose FP16 operands underflow to zero, 8-row groups whose y
 * features underflow in FP32).  Every sample gets the same bits as from
 * pdmp_morph_samples.  PDMP_ENOMEM if ws is short; in == out allowed; calls that share
 * a workspace must not overlap. */
size_t pdmp_morph_workspace_size(const pdmp_occupancy *occ, const pdmp_arm *arm, int64_t n,
                                 int32_t T);
int32_t pdmp_morph_samples_ws(const pdmp_occupancy *occ, const pdmp_arm *arm, const float *in,
                              float *out, int64_t n, int32_t T, float eta, void *ws,
                              size_t ws_bytes, void *stream);

/* The same morph (Sec. 3.2, Eq. 1 and Eq. 3) with the explicit-Euler path of every
 * traj_stride-th sample written out, so that each step can be checked on its own:
 * traj (device, [(T+1)][rows][nt], rows = occ->dim or arm->n_dof,
 * nt = ceil(n / traj_stride)) receives state k (k = 0..T; state 0 the input, state T
 * the output) of sample i, for every i with i % traj_stride == 0, at
 * traj[(k rows + r) nt + i / traj_stride].  Same kernels, launch and arithmetic as
 * pdmp_morph_samples: out receives the same bits.  traj_stride >= 1; traj must not
 * overlap in or out. */
int32_t pdmp_morph_trajectory(const pdmp_occupancy *occ, const pdmp_arm *arm, const float *in,
                              float *out, int64_t n, int32_t T, float eta, float *traj,
                              int64_t traj_stride, void *stream);

/* The split scheme the grid morph kernels take for this occupancy (the grid field
 * above): *scheme = 2 for two-part FP16 splits (three products per FP32 multiply-add),
 * 1 for three-part BF16 splits (six products), 0 when the morph takes no grid kernel
 * (no grid, or a grid the grid kernels do not cover: the pairwise sum).  Decided on
 * the device by the morph kernels' own staging code from the same data.  scheme is a
 * HOST pointer; the call waits for `stream`. */
int32_t pdmp_split_scheme(const pdmp_occupancy *occ, int32_t *scheme, void *stream);

/* ---- the density of the morphed samples and the inverse map (Sec. 3.2: the flow's
 * inverse integrates the reversed field; the change of variables gives the
 * density p_z(z) = p_y(y) / |det D phi(y)|).  Workspace morph only (no arm);
 * 2-D hinges on a grid (occ->grid) take the matrix-core path (FP32-accurate split
 * contractions, as for the morph), any other hinge set (2-D or 3-D) a pairwise kernel.
 * pdmp_morph_logdet: the plain morph of in into out (as pdmp_morph_samples) and
 *   logdet [n] = sum_k log|det(I - eta Hc(x_k))| along each path (nullable).
 * pdmp_morph_inverse: y = phi^{-1}(z) for the T-step explicit-Euler map, each step
 *   inverted by fixed point in reverse order: x^(0) = x_{k+1},
 *   x^(j+1) = x_{k+1} + eta grad c(x^(j)) for j < iters (>= 1), x_k = x^(iters) --
 *   a contraction when eta Lip(grad c) < 1.  resid (nullable, [n]) gets the largest
 *   residual |x_k - x_{k+1} - eta grad c(x_k)|_inf over the steps, logdet (nullable)
 *   the forward log-determinant along the reconstructed path.
 * in/z, out/y: [dim][n]; in == out allowed. */
int32_t pdmp_morph_logdet(const pdmp_occupancy *occ, const float *in, float *out, int64_t n,
                          int32_t T, float eta, float *logdet, void *stream);
int32_t pdmp_morph_inverse(const pdmp_occupancy *occ, const float *z, float *y, int64_t n,
                           int32_t T, float eta, int32_t iters, float *logdet, float *resid,
                           void *stream);

/* The same two calls with a caller workspace (pdmp_morph_workspace_size(occ, NULL, n,
 * T) bytes; 0 means the call needs none and ws is ignored): a large batch on a 2-D
 * hinge grid (the cases pdmp_morph_samples_ws orders) is first ordered by its cell
 * (in, resp. z), and every evaluation then skips, wave by wave, the exact zeros of the
 * factorised sums, Hessian included (its third operand, ex dx^2, reaches further than
 * ex dx, so the Hessian's evaluations keep 16-hinge blocks out to dx^2 < c + 35
 * kappa units squared instead of c + 30).  out / y, logdet and resid receive the same
 * bits as from the calls above.
 * PDMP_ENOMEM if ws is short; in == out (z == y) allowed; calls that share a
 * workspace must not overlap. */
int32_t pdmp_morph_logdet_ws(const pdmp_occupancy *occ, const float *in, float *out, int64_t n,
                             int32_t T, float eta, float *logdet, void *ws, size_t ws_bytes,
                             void *stream);
int32_t pdmp_morph_inverse_ws(const pdmp_occupancy *occ, const float *z, float *y, int64_t n,
                              int32_t T, float eta, int32_t iters, float *logdet, float *resid,
                              void *ws, size_t ws_bytes, void *stream);

/* ---- epsilon mixture with the prior (Sec. 3.3: sampling with an epsilon bias toward
 * the base distribution keeps regions the morph stretches thin reachable).
 * Draws the prior batch x0 [dim][n] exactly as pdmp_uniform_samples(seed, stream_id,
 * lo, hi) (lo, hi: HOST arrays [occ->dim]), morphs it (as pdmp_morph_samples, T steps)
 * into out [dim][n], then keeps the prior value for every sample i with u_i < eps,
 * u_i = (word >> 8) 2^-24 from word 0 of Philox4x32-10 at counter
 * {i_lo, i_hi, 0xffffffff, stream_id}, key {seed_lo, seed_hi}.  keep (nullable) [n]
 * marks those samples.  0 <= eps <= 1. */
int32_t pdmp_mixture_samples(const pdmp_occupancy *occ, uint64_t seed, uint32_t stream_id,
                             const float *lo, const float *hi, int64_t n, float eps, int32_t T,
                             float eta, float *x0, float *out, uint8_t *keep, void *stream);

/* ---- compact-support hinge culling for the workspace morph (a variant beyond the
 * paper; the RBF feature decays as exp(-r^2/(2 l^2))).  A point takes only the hinges
 * of the 3^dim cells around its own: cells of side 1/inv_cell >= the cutoff r_c on the
 * box from lo with nc cells per axis, a coordinate's cell being
 * floor((v - lo) * inv_cell) in FP64 from the FP32 values, clamped to [0, nc - 1].  Every
 * hinge within r_c of the point is kept, so the dropped part of the logit is at most
 * sum_j |w_j| exp(-r_c^2 / (2 l^2)) at every step; the hinges should lie in the box.
 * pdmp_cull_grid_make (host): inv_cell = 1/cutoff rounded to FP32, lowered by ulps until
 *   1/inv_cell >= cutoff; nc[k] = floor((hi[k] - lo[k]) inv_cell) + 1 (FP64).
 * pdmp_morph_culled: the plain morph (as pdmp_morph_samples, arm == NULL) on the culled
 *   occupancy, the cells re-evaluated at every step; in == out allowed.  ws: device
 *   scratch of pdmp_morph_culled_workspace_size bytes.  Deterministic; a point's result
 *   does not depend on the rest of the batch. */
typedef struct {
    int32_t dim;
    float lo[3];
    float inv_cell;
    int32_t nc[3];
} pdmp_cull_grid;

int32_t pdmp_cull_grid_make(int32_t dim, const float *lo, const float *hi, float cutoff,
                            pdmp_cull_grid *g);
size_t pdmp_morph_culled_workspace_size(const pdmp_occupancy *occ, const pdmp_cull_grid *g,
                                        int64_t n);
int32_t pdmp_morph_culled(const pdmp_occupancy *occ, const pdmp_cull_grid *g, const float *in,
                          float *out, int64_t n, int32_t T, float eta, void *ws, size_t ws_bytes,
                          void *stream);

/* ---- forward kinematics (Sec. 3.2): body points of configurations q [n_dof][n]
 * in FP32, written to pts [3][n_dof*pts_per_link][n]. */
int32_t pdmp_fk_body_points(const pdmp_arm *arm, const float *q, int64_t n, float *pts,
                            void *stream);

/* ---- occupancy fit (Sec. 3.1: binary cross-entropy minimised by gradient-descent
 * optimisers), full batch over n labelled points:
 *   L(w, beta) = (1/n) sum_i BCE(sigma(s(x_i)), y_i) + (l2/2) sum_j w_j^2   (beta free)
 *   grad_w = (1/n) Phi^T r + l2 w,  grad_beta = (1/n) sum_i r_i,  r_i = sigma(s_i) - y_i.
 * optimizer 0 (gradient descent): w -= lr grad_w, beta -= lr_bias grad_beta.
 * optimizer 1 (Adam, Kingma & Ba 2015, Alg. 1, bias-corrected, eps added to
 *   sqrt(v_hat)): step lr on every parameter; adam_m, adam_v are device [M+1] state,
 *   in/out; the step counter continues from t0 (first step uses t0 + 1). */
typedef struct {
    int32_t optimizer;
    int32_t steps;
    float lr;
    float lr_bias;
    float l2;
    float beta1, beta2, eps;
    int32_t t0;
    float *adam_m;
    float *adam_v;
} pdmp_fit_opts;

/* Workspace bytes for pdmp_fit_occupancy / pdmp_occupancy_bwd / pdmp_bce_logits. */
size_t pdmp_fit_workspace_size(int32_t dim, int32_t n_hinges, int64_t n);
size_t pdmp_bwd_workspace_size(int32_t dim, int32_t n_hinges, int64_t n);
size_t pdmp_bce_workspace_size(int64_t n);

/* Fit the occupancy.  Hinges, dim and lengthscale come from `occ` (occ->weights is
 * not read); `weights` is the device [M+1] model (w, then beta), read as the
 * starting point and overwritten with the result.  pts: [dim][n] device; labels:
 * [n] device uint8 (nonzero = occupied).  loss_out (nullable): device [steps], the
 * loss at the start of each step.  Deterministic. */
int32_t pdmp_fit_occupancy(const pdmp_occupancy *occ, float *weights, const float *pts,
                           const uint8_t *labels, int64_t n, const pdmp_fit_opts *opts,
                           float *loss_out, void *ws, size_t ws_bytes, void *stream);

/* Hand-written backward of the occupancy at n points x [dim][n].
 * s_fwd == NULL: g is dL/ds (the logit);  s_fwd != NULL: g is dL/dc and s_fwd the
 * forward logits, so the chain through sigma'(s) is applied.  Outputs (each
 * nullable): grad_w [M+1] = (sum_i g_i ds_i/dw_j, sum_i g_i ds_i/dbeta) (chained),
 * grad_x [dim][n] = g_i ds_i/dx_i (chained). */
int32_t pdmp_occupancy_bwd(const pdmp_occupancy *occ, const float *x, int64_t n, const float *g,
                           const float *s_fwd, float *grad_w, float *grad_x, void *ws,
                           size_t ws_bytes, void *stream);

/* The same backward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops): identical arguments, results and kernels, but
 * the scratch comes from a static array of 32 MiB that the library keeps on each GPU it
 * runs on until the process ends, instead of a caller workspace.  A call whose
 * pdmp_bwd_workspace_size exceeds 32 MiB (about 4M points at 4096 hinges) returns
 * PDMP_ENOMEM before any launch.  Calls no hipMalloc, hipFree or allocating routine.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other host threads) race and must be ordered by the caller. */
int32_t pdmp_occupancy_bwd_noalloc(const pdmp_occupancy *occ, const float *x, int64_t n,
                                   const float *g, const float *s_fwd, float *grad_w,
                                   float *grad_x, void *stream);

/* Mean binary cross-entropy of sigma(s) against labels y (nonzero = 1), in the
 * overflow-free form max(s,0) - y s + log(1 + exp(-|s|)).  loss (nullable): device
 * [1]; g_s (nullable): device [n], dL/ds_i = (sigma(s_i) - y_i)/n, times g_scale[0]
 * when g_scale (nullable, device [1]: the upstream gradient of the loss) is given. */
int32_t pdmp_bce_logits(const float *s, const uint8_t *y, int64_t n, const float *g_scale,
                        float *loss, float *g_s, void *ws, size_t ws_bytes, void *stream);

/* One Adam update (Kingma & Ba 2015, Alg. 1) of n device parameters p with gradient
 * g and state m, v (all FP32, in place), at step t >= 1.  The first n_decay entries
 * get l2 * p added to their gradient (L2 regularisation). */
int32_t pdmp_adam_step(float *p, const float *g, float *m, float *v, int64_t n, int64_t n_decay,
                       int32_t t, float lr, float beta1, float beta2, float eps, float l2,
                       void *stream);

/* ---- amortised morph: residual MLP q_hat = q + f(q) with
 * f = W_L SiLU(... SiLU(W_1 q + b_1) ...) + b_L, n_hidden hidden layers of width
 * `hidden`, trained by MSE on (base, plain-morphed) pairs.  Products run on BF16
 * MFMA with FP32 accumulation; biases, the residual add and the optimiser are FP32.
 * params:      device FP32 master parameters, flat: for each layer W [out][in]
 *              row-major, then b [out] (layers in order).
 * params_bf16: device BF16 copy of params (same layout) from pdmp_mlp_pack; the
 *              matrix products read the weights from here. */
typedef struct {
    int32_t n_in;       /* input = output width, 1..16 */
    int32_t hidden;     /* 1..1024 */
    int32_t n_hidden;   /* 1..6 */
    const float *params;
    const uint16_t *params_bf16;
} pdmp_mlp;

int64_t pdmp_mlp_num_params(const pdmp_mlp *mlp);
/* Round params to BF16 (nearest even) into params_bf16 [num_params] (device). */
int32_t pdmp_mlp_pack(const pdmp_mlp *mlp, uint16_t *params_bf16, void *stream);
/* Bytes of saved activations for a training forward of B samples, and of the
 * scratch workspace that forward/backward need. */
size_t pdmp_mlp_acts_size(const pdmp_mlp *mlp, int64_t B);
size_t pdmp_mlp_workspace_size(const pdmp_mlp *mlp, int64_t B);
/* q_hat [n_in][B] = q + f(q) for q [n_in][B].  acts (nullable, device,
 * pdmp_mlp_acts_size bytes): keep the activations for pdmp_mlp_backward.  Without
 * acts, a network of hidden width a multiple of 32 up to 256 and n_in <= 16 runs
 * as one fused kernel (activations in registers, hidden weights staged in LDS; the
 * workspace is then unused); other shapes, and training forwards, run layer by
 * layer.  Both accumulate in FP32 from BF16 weights and activations. */
int32_t pdmp_mlp_forward(const pdmp_mlp *mlp, const float *q, int64_t B, float *q_hat, void *acts,
                         void *ws, size_t ws_bytes, void *stream);
/* MSE loss (1/(n_in B)) sum |q_hat - target|^2 (loss, nullable, device [1]) and its
 * gradient with respect to params (grad, device FP32 [num_params], overwritten),
 * from the activations of the matching forward. */
int32_t pdmp_mlp_backward(const pdmp_mlp *mlp, const float *q_hat, const float *target,
                          int64_t B, void *acts, float *grad, float *loss, void *ws,
                          size_t ws_bytes, void *stream);
/* The same with per-sample weights, for training that emphasises hard samples:
 * loss (1/(n_in B)) sum_b u_b |q_hat_b - target_b|^2 and its gradient, u_b = hard_weight
 * where hard[b] != 0 and 1 elsewhere (hard: device uint8 [B], nullable = all 1, e.g.
 * the flag of pdmp_arm_max_occupancy at q_hat).  hard_weight must be finite and >= 0
 * (else PDMP_EINVAL); the workspace is pdmp_mlp_backward's. */
int32_t pdmp_mlp_backward_weighted(const pdmp_mlp *mlp, const float *q_hat, const float *target,
                                   int64_t B, const uint8_t *hard, float hard_weight, void *acts,
                                   float *grad, float *loss, void *ws, size_t ws_bytes,
                                   void *stream);

/* Largest body-point occupancy of each configuration, max_p c(psi_p(q)) (maxc,
 * nullable, [n]) and flag = (max > thresh) (nullable, [n]).  FP32 kinematics. */
int32_t pdmp_arm_max_occupancy(const pdmp_occupancy *occ, const pdmp_arm *arm, const float *q,
                               int64_t n, float thresh, float *maxc, uint8_t *flag,
                               void *stream);

/* Amortised morph of configurations q [n_dof][n] into out [n_dof][n]:
 * q_hat = q + f(q); a configuration whose largest body-point occupancy at q_hat
 * exceeds `thresh` is re-morphed by the plain T-step joint-space morph from its base
 * q (the fallback), all others keep q_hat.  flag (nullable, [n]) marks the
 * fallbacks, n_fallback (nullable, device) receives their count.  No host
 * synchronisation inside; out must not alias q. */
size_t pdmp_amortised_workspace_size(const pdmp_mlp *mlp, const pdmp_arm *arm, int64_t n);
int32_t pdmp_amortised_morph(const pdmp_mlp *mlp, const pdmp_occupancy *occ, const pdmp_arm *arm,
                             const float *q, float *out, int64_t n, int32_t T, float eta,
                             float thresh, uint8_t *flag, uint32_t *n_fallback, void *ws,
                             size_t ws_bytes, void *stream);
/* The refining variant: a configuration whose q_hat is flagged takes T_refine plain
 * joint-space steps (Sec. 3.2, Eq. 1 and 3) from q_hat instead of the T steps from q,
 * so the plain morph repairs the network's output rather than replacing it (the
 * result then differs from the plain morph's for those configurations).  Arguments,
 * workspace and errors as pdmp_amortised_morph; T_refine = 0 returns q_hat. */
int32_t pdmp_amortised_morph_refine(const pdmp_mlp *mlp, const pdmp_occupancy *occ,
                                    const pdmp_arm *arm, const float *q, float *out, int64_t n,
                                    int32_t T_refine, float eta, float thresh, uint8_t *flag,
                                    uint32_t *n_fallback, void *ws, size_t ws_bytes,
                                    void *stream);

/* ---- the paper's occupancy network (Sec. 3.1): a fully connected network with
 * tanh activations between hidden layers and a sigmoid output, c(x) = sigma(s(x)),
 *   a_1 = tanh(W_0 x + b_0),  a_{l+1} = tanh(W_l a_l + b_l),  s = v . a_L + b_o,
 * and its input gradient by the chain rule.  params (device, FP32, read-only) is
 * flat: for l = 0..n_hidden-1 the matrix W_l [hidden][n_l] (row-major; n_0 = dim,
 * n_l = hidden after) and b_l [hidden]; then v [hidden] and b_o.  Supported:
 * dim 2 or 3, 1 <= hidden <= 64, 1 <= n_hidden <= 4 (else PDMP_EINVAL). */
typedef struct {
    int32_t dim;
    int32_t hidden;
    int32_t n_hidden;
    const float *params;
} pdmp_tanh_net;

/* Length of params: hidden*dim + hidden + (n_hidden-1)(hidden^2 + hidden) + hidden + 1,
 * or -1 for an unsupported shape. */
int64_t pdmp_tanh_num_params(const pdmp_tanh_net *net);
/* c_out (nullable) [n] = c(x_i), s_out (nullable) [n] = s(x_i); x [dim][n]. */
int32_t pdmp_tanh_occupancy_eval(const pdmp_tanh_net *net, const float *x, int64_t n,
                                 float *c_out, float *s_out, void *stream);
/* grad_out [dim][n] = grad_x c = sigma'(s) grad_x s; c_out (nullable) [n]. */
int32_t pdmp_tanh_occupancy_grad(const pdmp_tanh_net *net, const float *x, int64_t n,
                                 float *c_out, float *grad_out, void *stream);
/* The workspace morph of Sec. 3.2 (Eq. 1, explicit Euler) with the network's
 * occupancy: x_{k+1} = x_k - eta grad c(x_k), T >= 0 steps; in, out [dim][n],
 * in == out allowed, other overlap not. */
int32_t pdmp_tanh_morph_samples(const pdmp_tanh_net *net, const float *in, float *out, int64_t n,
                                int32_t T, float eta, void *stream);
/* The split scheme of the hidden-to-hidden products in the three calls above, as their
 * kernels decide it on the device from the weights: *scheme = 2 when the forward
 * products W_l a run on two FP16 parts of the power-of-two-scaled W_l and of 2^14 a
 * (three products per FP32-accurate multiply-add; every hidden W_l finite with each
 * nonzero |w| at least 2^-19 of its largest), 1 when they run on three-way BF16 splits
 * (six products).  The backward products W_l^T e always take the BF16 splits.  scheme is
 * a HOST pointer; the call waits for `stream`. */
int32_t pdmp_tanh_split_scheme(const pdmp_tanh_net *net, int32_t *scheme, void *stream);

/* Fit of the network (Sec. 3.1: binary cross-entropy minimised by a gradient-descent
 * optimiser), full batch over n >= 1 labelled points pts [dim][n], labels u8 [n]:
 *   L = (1/n) sum_i BCE(sigma(s(x_i)), y_i) + (l2/2) (sum_l |W_l|^2 + |v|^2)
 * (biases not decayed).  Parameter gradients by the chain rule through every layer
 * (reverse order), summed over the points in a fixed order (deterministic).
 * pdmp_tanh_loss_grad: loss (nullable, device [1]) and grad (device [num_params]).
 * pdmp_tanh_fit: opts->steps Adam steps (opts->optimizer must be 1; lr, l2, beta1,
 *   beta2, eps, adam_m, adam_v [num_params] in/out, t0 as for pdmp_fit_occupancy;
 *   lr_bias unused) updating net->params IN PLACE (it must point to writable device
 *   memory); loss_out (nullable, device [steps]) gets the loss before each step.
 * ws: device scratch of pdmp_tanh_fit_workspace_size bytes (PDMP_ENOMEM if short). */
size_t pdmp_tanh_fit_workspace_size(const pdmp_tanh_net *net, int64_t n);
int32_t pdmp_tanh_loss_grad(const pdmp_tanh_net *net, const float *pts, const uint8_t *labels,
                            int64_t n, float l2, float *loss, float *grad, void *ws,
                            size_t ws_bytes, void *stream);
int32_t pdmp_tanh_fit(const pdmp_tanh_net *net, const float *pts, const uint8_t *labels,
                      int64_t n, const pdmp_fit_opts *opts, float *loss_out, void *ws,
                      size_t ws_bytes, void *stream);

/* ---- diagnostics.  Measured issue costs on the current device, in shader-clock cycles
 * per wave64 instruction on one SIMD, from probe kernels of one instruction class each
 * (eight independent dependency chains per lane, eight waves per SIMD):
 *   out[0] v_fma_f32, out[1] v_exp_f32, out[2] v_cvt_pk_f16_f32, out[3] v_fma_mix_f32;
 *   out[4] one iteration of 4 v_exp_f32 and 4 v_fma_f32 in independent chains (4 out[1] +
 *          4 out[0] if the two classes add, less if they overlap);
 *   out[5] v_mfma_f32_32x32x16_f16 (four independent accumulators, four waves per SIMD);
 *   out[6] one iteration of 4 such MFMAs and 32 independent v_fma_f32 (four waves per
 *          SIMD: 4 out[5] + 32 out[0] if they add, the larger of the two if they overlap);
 *   out[7] the mean shader clock over the probes, GHz.
 * The first min(n_out, 8) figures are written to out (HOST).  Host-synchronous; allocates
 * and frees its own device memory.  The benchmark states its ceilings with these. */
int32_t pdmp_issue_rates(double *out, int32_t n_out);

/* ---- the producer/consumer of Sec. 3.3: a background diffeomorphic sampler keeps a
 * bounded concurrent bucket S filled with morphed samples; the planner's main thread
 * draws from S and never waits -- when S is empty it draws from the prior instead,
 * so a slow or failed GPU only reverts the planner to plain sampling.  Host memory;
 * all functions are host calls. */
typedef struct pdmp_bucket pdmp_bucket;
typedef struct pdmp_sampler pdmp_sampler;

/* Bucket: a single-producer single-consumer ring of `capacity` (a power of two)
 * samples of `dim` floats (1..16), each with a 64-bit index.  One thread may push and
 * one other thread may pop concurrently; neither call blocks.
 * push: samples [start, n) of the SoA batch x [dim][ld] (ld >= n) with indices
 *   base_index + j, as many as fit; returns the number pushed (-1 on bad arguments).
 * pop: one sample into x [dim] and its index (nullable); returns 1, or 0 if empty. */
int32_t pdmp_bucket_create(int32_t dim, int64_t capacity, pdmp_bucket **out);
int64_t pdmp_bucket_push(pdmp_bucket *b, const float *x, int64_t ld, int64_t start, int64_t n,
                         int64_t base_index);
int32_t pdmp_bucket_pop(pdmp_bucket *b, float *x, int64_t *index);
int64_t pdmp_bucket_size(const pdmp_bucket *b);
void pdmp_bucket_destroy(pdmp_bucket *b);

/* Sampler options.  Batch b of the producer is the Philox prior of stream
 * (stream_id + b) on the box [lo, hi)^dim (as pdmp_uniform_samples), morphed T steps
 * (as pdmp_morph_samples with arm == NULL); its sample i enters S with index
 * b * batch + i.  The k-th prior fallback draw is sample k of the prior of stream
 * prior_stream_id (same values as pdmp_uniform_samples) and gets index -1 - k. */
typedef struct {
    int32_t dim;              /* 2 or 3 */
    int32_t T;                /* >= 0 */
    float eta;
    int64_t batch;            /* samples per GPU batch, >= 1 */
    int64_t capacity;         /* bucket capacity in samples, a power of two */
    uint64_t seed;
    uint32_t stream_id;
    uint32_t prior_stream_id;
    float lo[3], hi[3];
} pdmp_sampler_opts;

typedef struct {
    int64_t batches;          /* GPU batches completed */
    int64_t produced;         /* samples pushed into S */
    int64_t popped_bucket;    /* samples the consumer took from S */
    int64_t popped_prior;     /* samples the consumer drew from the prior */
    int64_t bucket_size;
    int32_t status;           /* the producer's first failure (PDMP_OK if none) */
    int32_t running;
    double producer_busy_s;   /* producer wall time with a batch in flight */
    double elapsed_s;         /* since pdmp_sampler_start */
} pdmp_sampler_stats;

/* create: occ (nullable: a prior-only sampler) is copied; the device buffers it
 *   points to must outlive the sampler.  start: spawns the producer thread on the
 *   calling thread's current device (its own non-blocking HIP stream, default
 *   priority, device and pinned host buffers of a few batches); a producer that has
 *   stopped on a failure is not restarted (PDMP_EINVAL, the failure's message in
 *   pdmp_last_error()).  pause: the
 *   producer stops launching and pushing while paused != 0 (forces an empty S).
 *   pop: n samples into x [n][dim] (row per sample), index [n] and from_bucket [n]
 *   (both nullable); never waits.  Single consumer thread.  destroy: stops and
 *   joins the producer, frees everything, returns the producer's status.  When
 *   that status is not PDMP_OK, get_stats and destroy also leave the producer's
 *   message in the calling thread's pdmp_last_error(). */
int32_t pdmp_sampler_create(const pdmp_occupancy *occ, const pdmp_sampler_opts *opts,
                            pdmp_sampler **out);
int32_t pdmp_sampler_start(pdmp_sampler *s);
int32_t pdmp_sampler_pause(pdmp_sampler *s, int32_t paused);
int32_t pdmp_sampler_pop(pdmp_sampler *s, int64_t n, float *x, int64_t *index,
                         uint8_t *from_bucket);
int32_t pdmp_sampler_get_stats(const pdmp_sampler *s, pdmp_sampler_stats *st);
int32_t pdmp_sampler_destroy(pdmp_sampler *s);

/* The planner's main thread in its simplest form (an RRT in the plane, Sec. 3.3):
 * each iteration pops one sample from the sampler (dim 2), finds the nearest node
 * (squared distance in FP64, ties to the lowest index), steers at most `step` toward
 * the sample (FP64, stored as FP32), and adds the node if the edge misses every disc
 * (closed discs, FP64 segment distance); it stops when a new node within goal_tol of
 * the goal connects to it by a free edge (the goal becomes the last node), after
 * max_iters iterations, or when time_budget_s (> 0) has passed (goal_tol < 0: no
 * goal, the tree grows until one of the other two).
 * nodes [max_iters + 2][2], parent [max_iters + 2] (root -1); samples [max_iters][2],
 * from_bucket [max_iters] and t_sample [max_iters] (seconds since the start) record
 * each iteration's draw (all three nullable). */
typedef struct {
    int32_t max_iters;
    float step;
    float goal_tol;
    float start[2];
    float goal[2];
    double time_budget_s;
    int32_t n_discs;
    const double *disc_x, *disc_y, *disc_r;  /* host [n_discs] */
} pdmp_rrt_opts;

typedef struct {
    int32_t solved;
    int32_t iters;
    int32_t n_nodes;
    int64_t from_bucket;
    int64_t from_prior;
    double path_len;
    double elapsed_s;
} pdmp_rrt_result;

int32_t pdmp_rrt_run(pdmp_sampler *s, const pdmp_rrt_opts *o, float *nodes, int32_t *parent,
                     float *samples, uint8_t *from_bucket, double *t_sample,
                     pdmp_rrt_result *res);

#ifdef __cplusplus
}
#endif

#endif /* PDMP_H */
