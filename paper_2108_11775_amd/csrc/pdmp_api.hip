// pdmp_api.hip -- the extern "C" entry points of libpdmp: argument validation on the
// host, parameter derivation, and the launches.  See include/pdmp.h for the contract.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "pdmp_common.h"

namespace pdmp {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

const char *last_error() { return g_err; }

int32_t check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: %s", what, hipGetErrorString(e));
        return PDMP_EDEVICE;
    }
    return PDMP_OK;
}


// The grid field: all zero, or per-axis sizes >= 1 whose product is n_hinges.
static int32_t check_grid_field(const pdmp_occupancy *occ) {
    if (occ->grid[0] || occ->grid[1] || occ->grid[2]) {
        int64_t prod = 1;
        for (int k = 0; k < occ->dim; ++k) {
            PDMP_REQUIRE(occ->grid[k] >= 1, "grid[%d] = %d", k, occ->grid[k]);
            prod *= occ->grid[k];
        }
        PDMP_REQUIRE(occ->dim == 3 || occ->grid[2] == 0, "grid[2] must be 0 in 2-D");
        PDMP_REQUIRE(prod == occ->n_hinges, "grid product %lld != n_hinges %d", (long long)prod,
                     occ->n_hinges);
    }
    return PDMP_OK;
}

static int32_t check_occ(const pdmp_occupancy *occ) {
    PDMP_REQUIRE(occ != nullptr, "occupancy is NULL");
    PDMP_REQUIRE(occ->dim == 2 || occ->dim == 3, "occupancy dim %d not in {2,3}", occ->dim);
    PDMP_REQUIRE(occ->n_hinges >= 1, "n_hinges %d < 1", occ->n_hinges);
    PDMP_REQUIRE(occ->hinges != nullptr && occ->weights != nullptr, "hinges/weights NULL");
    PDMP_REQUIRE(std::isfinite(occ->lengthscale) && occ->lengthscale > 0.0f,
                 "lengthscale must be finite and > 0");
    return check_grid_field(occ);
}

static bool has_grid(const pdmp_occupancy *occ) { return occ->grid[0] > 0; }

// Before a launch that may take the grid factorisation: the device check of the
// stated grid (deferred report at pdmp_sync).
static int32_t grid_check(const pdmp_occupancy *occ, void *stream) {
    if (!has_grid(occ)) return PDMP_OK;
    return launch_grid_check(occ->dim, occ->hinges, occ->n_hinges, occ->grid, (hipStream_t)stream);
}

static int32_t check_arm(const pdmp_arm *arm, int max_ppl) {
    PDMP_REQUIRE(arm != nullptr, "arm is NULL");
    PDMP_REQUIRE(arm->n_dof >= 1 && arm->n_dof <= PDMP_MAX_DOF, "n_dof %d not in [1,%d]",
                 arm->n_dof, PDMP_MAX_DOF);
    PDMP_REQUIRE(arm->pts_per_link >= 1 && arm->pts_per_link <= PDMP_MAX_PTS_PER_LINK,
                 "pts_per_link %d not in [1,%d]", arm->pts_per_link, PDMP_MAX_PTS_PER_LINK);
    for (int i = 0; i < arm->n_dof; ++i)
        PDMP_REQUIRE(std::isfinite(arm->a[i]) && std::isfinite(arm->d[i]) &&
                         std::isfinite(arm->alpha[i]) && std::isfinite(arm->theta0[i]),
                     "non-finite DH parameter on joint %d", i);
    if (arm->pts_per_link > max_ppl) {
        set_error("pts_per_link %d > %d is not supported here", arm->pts_per_link, max_ppl);
        return PDMP_EUNSUPPORTED;
    }
    return PDMP_OK;
}

}  // namespace pdmp

using namespace pdmp;

extern "C" {

int32_t pdmp_abi_version(void) { return PDMP_ABI_VERSION; }

const char *pdmp_last_error(void) { return pdmp::last_error(); }

int32_t pdmp_sync(void *stream) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) {
        set_error("hipStreamSynchronize: %s", hipGetErrorString(e));
        return PDMP_EDEVICE;
    }
    bool mismatch = false;
    const int32_t st = take_grid_mismatch(mismatch);
    if (st) return st;
    if (mismatch) {
        set_error("an occupancy's hinges are not the tensor grid its grid field states "
                  "(results of that call are undefined)");
        return PDMP_EINVAL;
    }
    return PDMP_OK;
}

int32_t pdmp_uniform_samples(uint64_t seed, uint32_t stream_id, const float *lo, const float *hi,
                             int32_t dim, int64_t n, float *out, void *stream) {
    PDMP_REQUIRE(dim >= 1 && dim <= 16, "dim %d not in [1,16]", dim);
    PDMP_REQUIRE(n >= 0, "n < 0");
    PDMP_REQUIRE(lo != nullptr && hi != nullptr, "lo/hi NULL");
    for (int k = 0; k < dim; ++k)
        PDMP_REQUIRE(std::isfinite(lo[k]) && std::isfinite(hi[k]) && lo[k] <= hi[k],
                     "bad range on coordinate %d", k);
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(out != nullptr, "out NULL");
    return launch_uniform(seed, stream_id, lo, hi, dim, n, out, (hipStream_t)stream);
}

int32_t pdmp_label_points_discs(const pdmp_discs *scene, const float *x, int64_t n, uint8_t *out,
                                uint64_t *n_hit, void *stream) {
    PDMP_REQUIRE(scene != nullptr && scene->n >= 0, "bad disc scene");
    PDMP_REQUIRE(scene->n == 0 || (scene->centres && scene->radii), "disc arrays NULL");
    PDMP_REQUIRE(n >= 0, "n < 0");
    if (n == 0 && !n_hit) return PDMP_OK;
    PDMP_REQUIRE(n == 0 || (x && out), "x/out NULL");
    return launch_label_discs(*scene, x, n, out, n_hit, (hipStream_t)stream);
}

int32_t pdmp_label_points_boxes(const pdmp_boxes *scene, const float *x, int64_t n, uint8_t *out,
                                uint64_t *n_hit, void *stream) {
    PDMP_REQUIRE(scene != nullptr && scene->n >= 0, "bad box scene");
    PDMP_REQUIRE(scene->n == 0 || (scene->centres && scene->half), "box arrays NULL");
    PDMP_REQUIRE(n >= 0, "n < 0");
    if (n == 0 && !n_hit) return PDMP_OK;
    PDMP_REQUIRE(n == 0 || (x && out), "x/out NULL");
    return launch_label_boxes(*scene, x, n, out, n_hit, (hipStream_t)stream);
}

int32_t pdmp_label_configs(const pdmp_arm *arm, const pdmp_boxes *scene, const float *q,
                           int64_t n, uint8_t *out, uint64_t *n_hit, void *stream) {
    int32_t st = check_arm(arm, PDMP_MAX_PTS_PER_LINK);
    if (st) return st;
    PDMP_REQUIRE(scene != nullptr && scene->n >= 0, "bad box scene");
    PDMP_REQUIRE(scene->n == 0 || (scene->centres && scene->half), "box arrays NULL");
    PDMP_REQUIRE(n >= 0, "n < 0");
    if (n == 0 && !n_hit) return PDMP_OK;
    PDMP_REQUIRE(n == 0 || (q && out), "q/out NULL");
    return launch_label_configs(*arm, *scene, q, n, out, n_hit, (hipStream_t)stream);
}

static int32_t rbf_call(const pdmp_occupancy *occ, int mode, const float *x, int64_t n,
                        float *c_out, float *s_out, float *g_out, float *x_out, int32_t T,
                        float eta, void *stream, const Traj &traj = Traj()) {
    const int32_t gc = grid_check(occ, stream);
    if (gc) return gc;
    RbfArgs a;
    a.traj = traj;
    a.hinges = occ->hinges;
    a.weights = occ->weights;
    a.M = occ->n_hinges;
    a.bias = occ->weights + occ->n_hinges;
    derive_scales(occ->lengthscale, a.kappa, a.gscale);
    a.x_in = x;
    a.n = n;
    a.T = T;
    a.eta = eta;
    a.c_out = c_out;
    a.s_out = s_out;
    a.g_out = g_out;
    a.x_out = x_out;
    return launch_occ_any(occ->dim, mode, a, has_grid(occ) ? occ->grid : nullptr,
                          (hipStream_t)stream);
}

int32_t pdmp_occupancy_eval(const pdmp_occupancy *occ, const float *x, int64_t n, float *c_out,
                            float *s_out, void *stream) {
    int32_t st = check_occ(occ);
    if (st) return st;
    PDMP_REQUIRE(n >= 0, "n < 0");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(x && c_out, "x/c_out NULL");
    return rbf_call(occ, kEval, x, n, c_out, s_out, nullptr, nullptr, 1, 0.0f, stream);
}

int32_t pdmp_occupancy_grad(const pdmp_occupancy *occ, const float *x, int64_t n, float *c_out,
                            float *grad_out, void *stream) {
    int32_t st = check_occ(occ);
    if (st) return st;
    PDMP_REQUIRE(n >= 0, "n < 0");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(x && grad_out, "x/grad_out NULL");
    return rbf_call(occ, kGrad, x, n, c_out, nullptr, grad_out, nullptr, 1, 0.0f, stream);
}

// The morph of pdmp_morph_samples, recording the paths of traj's samples (if any);
// with a workspace, a large 2-D grid batch takes the spatially ordered kernel.
static int32_t morph_impl(const pdmp_occupancy *occ, const pdmp_arm *arm, const float *in,
                          float *out, int64_t n, int32_t T, float eta, const Traj &traj,
                          void *stream, void *ws = nullptr, size_t ws_bytes = 0) {
    int32_t st = check_occ(occ);
    if (st) return st;
    PDMP_REQUIRE(n >= 0, "n < 0");
    PDMP_REQUIRE(T >= 0, "T < 0");
    PDMP_REQUIRE(std::isfinite(eta), "eta not finite");
    if (arm) {
        st = check_arm(arm, 8);
        if (st) return st;
        PDMP_REQUIRE(occ->dim == 3, "the joint-space morph needs a 3-D occupancy");
    }
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(in && out, "in/out NULL");
    if (T == 0 && traj.p == nullptr) {
        if (in == out) return PDMP_OK;
        const size_t rows = arm ? (size_t)arm->n_dof : (size_t)occ->dim;
        hipError_t e = hipMemcpyAsync(out, in, rows * (size_t)n * sizeof(float),
                                      hipMemcpyDeviceToDevice, (hipStream_t)stream);
        if (e != hipSuccess) {
            set_error("hipMemcpyAsync: %s", hipGetErrorString(e));
            return PDMP_EDEVICE;
        }
        return PDMP_OK;
    }
    if (arm) {
        float kappa, gscale;
        derive_scales(occ->lengthscale, kappa, gscale);
        if (has_grid(occ)) {
            if ((st = grid_check(occ, stream))) return st;
            st = launch_arm_grid3d(*arm, occ->hinges, occ->weights, occ->n_hinges, occ->grid, kappa,
                                   gscale, in, out, n, T, eta, nullptr, true, 0.0f, nullptr,
                                   nullptr, (hipStream_t)stream, traj);
            if (st != PDMP_EUNSUPPORTED) return st;
        }
        return launch_morph_arm(*arm, occ->hinges, occ->weights, occ->n_hinges, kappa, gscale, in,
                                out, n, T, eta, nullptr, (hipStream_t)stream, traj);
    }
    if (ws && occ->dim == 2 && has_grid(occ)) {
        const size_t need = grid2d_sorted_ws_bytes(occ->grid[0], occ->grid[1], n, T);
        if (need && ws_bytes >= need) {
            if ((st = grid_check(occ, stream))) return st;
            RbfArgs a;
            a.traj = traj;
            a.hinges = occ->hinges;
            a.weights = occ->weights;
            a.M = occ->n_hinges;
            a.bias = occ->weights + occ->n_hinges;
            derive_scales(occ->lengthscale, a.kappa, a.gscale);
            a.x_in = in;
            a.n = n;
            a.T = T;
            a.eta = eta;
            a.x_out = out;
            st = launch_grid2d_sorted(a, occ->grid[0], occ->grid[1], ws, (hipStream_t)stream);
            if (st != PDMP_EUNSUPPORTED) return st;
        }
    }
    return rbf_call(occ, kMorph, in, n, nullptr, nullptr, nullptr, out, T, eta, stream, traj);
}

size_t pdmp_morph_workspace_size(const pdmp_occupancy *occ, const pdmp_arm *arm, int64_t n,
                                 int32_t T) {
    if (check_occ(occ) || arm || occ->dim != 2 || !has_grid(occ) || n < 1) return 0;
    return grid2d_sorted_ws_bytes(occ->grid[0], occ->grid[1], n, T);
}

int32_t pdmp_morph_samples_ws(const pdmp_occupancy *occ, const pdmp_arm *arm, const float *in,
                              float *out, int64_t n, int32_t T, float eta, void *ws,
                              size_t ws_bytes, void *stream) {
    const size_t need = pdmp_morph_workspace_size(occ, arm, n, T);
    if (need && (!ws || ws_bytes < need)) {
        set_error("workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        return PDMP_ENOMEM;
    }
    return morph_impl(occ, arm, in, out, n, T, eta, Traj(), stream, need ? ws : nullptr, ws_bytes);
}

int32_t pdmp_morph_samples(const pdmp_occupancy *occ, const pdmp_arm *arm, const float *in,
                           float *out, int64_t n, int32_t T, float eta, void *stream) {
    return morph_impl(occ, arm, in, out, n, T, eta, Traj(), stream);
}

int32_t pdmp_morph_trajectory(const pdmp_occupancy *occ, const pdmp_arm *arm, const float *in,
                              float *out, int64_t n, int32_t T, float eta, float *traj,
                              int64_t traj_stride, void *stream) {
    PDMP_REQUIRE(traj != nullptr, "traj NULL");
    PDMP_REQUIRE(traj_stride >= 1, "traj_stride %lld < 1", (long long)traj_stride);
    Traj tr;
    tr.p = traj;
    tr.stride = traj_stride;
    tr.nt = n > 0 ? (n + traj_stride - 1) / traj_stride : 0;
    return morph_impl(occ, arm, in, out, n, T, eta, tr, stream);
}

int32_t pdmp_split_scheme(const pdmp_occupancy *occ, int32_t *scheme, void *stream) {
    int32_t st = check_occ(occ);
    if (st) return st;
    PDMP_REQUIRE(scheme != nullptr, "scheme NULL");
    *scheme = 0;
    if (!has_grid(occ)) return PDMP_OK;
    float kappa, gscale;
    derive_scales(occ->lengthscale, kappa, gscale);
    hipStream_t s = (hipStream_t)stream;
    int32_t *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(int32_t));
    if (e != hipSuccess) {
        set_error("hipMalloc: %s", hipGetErrorString(e));
        return PDMP_EDEVICE;
    }
    st = occ->dim == 2 ? launch_grid2d_scheme(occ->hinges, occ->weights, occ->grid[0],
                                              occ->grid[1], kappa, d, s)
                       : launch_grid3d_scheme(occ->hinges, occ->weights, occ->grid,
                                              occ->n_hinges, kappa, d, s);
    int32_t v = 0;
    if (st == PDMP_OK) {
        e = hipMemcpyAsync(&v, d, sizeof(v), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            set_error("split scheme query: %s", hipGetErrorString(e));
            st = PDMP_EDEVICE;
        }
    }
    (void)hipFree(d);
    if (st == PDMP_EUNSUPPORTED) return PDMP_OK;  // the pairwise kernels: *scheme = 0
    if (st == PDMP_OK) *scheme = v;
    return st;
}

// The workspace a _ws call needs (0: none); PDMP_ENOMEM when ws is short.
static int32_t check_morph_ws(const pdmp_occupancy *occ, int64_t n, int32_t T, void *ws,
                              size_t ws_bytes, void **use) {
    const size_t need = pdmp_morph_workspace_size(occ, nullptr, n, T);
    if (need && (!ws || ws_bytes < need)) {
        set_error("workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        return PDMP_ENOMEM;
    }
    *use = need ? ws : nullptr;
    return PDMP_OK;
}

static int32_t logdet_impl(const pdmp_occupancy *occ, const float *in, float *out, int64_t n,
                           int32_t T, float eta, float *logdet, void *stream, bool with_ws,
                           void *ws, size_t ws_bytes) {
    int32_t st = check_occ(occ);
    if (st) return st;
    PDMP_REQUIRE(n >= 0, "n < 0");
    PDMP_REQUIRE(T >= 0, "T < 0");
    PDMP_REQUIRE(std::isfinite(eta), "eta not finite");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(in && out, "in/out NULL");
    void *use = nullptr;
    if (with_ws && (st = check_morph_ws(occ, n, T, ws, ws_bytes, &use))) return st;
    if ((st = grid_check(occ, stream))) return st;
    return launch_morph_inverse(occ->dim, kLogdet, occ->hinges, occ->weights, occ->n_hinges,
                                has_grid(occ) ? occ->grid : nullptr, occ->lengthscale, in, n, T,
                                eta, 0, out, logdet, nullptr, (hipStream_t)stream, use);
}

static int32_t inverse_impl(const pdmp_occupancy *occ, const float *z, float *y, int64_t n,
                            int32_t T, float eta, int32_t iters, float *logdet, float *resid,
                            void *stream, bool with_ws, void *ws, size_t ws_bytes) {
    int32_t st = check_occ(occ);
    if (st) return st;
    PDMP_REQUIRE(n >= 0, "n < 0");
    PDMP_REQUIRE(T >= 0, "T < 0");
    PDMP_REQUIRE(iters >= 1, "iters < 1");
    PDMP_REQUIRE(std::isfinite(eta), "eta not finite");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(z && y, "z/y NULL");
    void *use = nullptr;
    if (with_ws && (st = check_morph_ws(occ, n, T, ws, ws_bytes, &use))) return st;
    if ((st = grid_check(occ, stream))) return st;
    return launch_morph_inverse(occ->dim, kInverse, occ->hinges, occ->weights, occ->n_hinges,
                                has_grid(occ) ? occ->grid : nullptr, occ->lengthscale, z, n, T,
                                eta, iters, y, logdet, resid, (hipStream_t)stream, use);
}

int32_t pdmp_morph_logdet(const pdmp_occupancy *occ, const float *in, float *out, int64_t n,
                          int32_t T, float eta, float *logdet, void *stream) {
    return logdet_impl(occ, in, out, n, T, eta, logdet, stream, false, nullptr, 0);
}

int32_t pdmp_morph_logdet_ws(const pdmp_occupancy *occ, const float *in, float *out, int64_t n,
                             int32_t T, float eta, float *logdet, void *ws, size_t ws_bytes,
                             void *stream) {
    return logdet_impl(occ, in, out, n, T, eta, logdet, stream, true, ws, ws_bytes);
}

int32_t pdmp_morph_inverse(const pdmp_occupancy *occ, const float *z, float *y, int64_t n,
                           int32_t T, float eta, int32_t iters, float *logdet, float *resid,
                           void *stream) {
    return inverse_impl(occ, z, y, n, T, eta, iters, logdet, resid, stream, false, nullptr, 0);
}

int32_t pdmp_morph_inverse_ws(const pdmp_occupancy *occ, const float *z, float *y, int64_t n,
                              int32_t T, float eta, int32_t iters, float *logdet, float *resid,
                              void *ws, size_t ws_bytes, void *stream) {
    return inverse_impl(occ, z, y, n, T, eta, iters, logdet, resid, stream, true, ws, ws_bytes);
}

int32_t pdmp_mixture_samples(const pdmp_occupancy *occ, uint64_t seed, uint32_t stream_id,
                             const float *lo, const float *hi, int64_t n, float eps, int32_t T,
                             float eta, float *x0, float *out, uint8_t *keep, void *stream) {
    int32_t st = check_occ(occ);
    if (st) return st;
    PDMP_REQUIRE(n >= 0, "n < 0");
    PDMP_REQUIRE(T >= 0, "T < 0");
    PDMP_REQUIRE(std::isfinite(eta), "eta not finite");
    PDMP_REQUIRE(eps >= 0.0f && eps <= 1.0f, "eps not in [0, 1]");
    PDMP_REQUIRE(lo && hi, "lo/hi NULL");
    for (int k = 0; k < occ->dim; ++k)
        PDMP_REQUIRE(std::isfinite(lo[k]) && std::isfinite(hi[k]) && lo[k] <= hi[k],
                     "bad range on axis %d", k);
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(x0 && out && x0 != out, "x0/out NULL or aliased");
    hipStream_t s = (hipStream_t)stream;
    if ((st = launch_uniform(seed, stream_id, lo, hi, occ->dim, n, x0, s))) return st;
    if ((st = pdmp_morph_samples(occ, nullptr, x0, out, n, T, eta, stream))) return st;
    return launch_mix_select(seed, stream_id, eps, occ->dim, n, x0, out, keep, s);
}

int32_t pdmp_cull_grid_make(int32_t dim, const float *lo, const float *hi, float cutoff,
                            pdmp_cull_grid *g) {
    PDMP_REQUIRE(g && lo && hi, "NULL argument");
    PDMP_REQUIRE(dim == 2 || dim == 3, "dim must be 2 or 3");
    PDMP_REQUIRE(std::isfinite(cutoff) && cutoff > 0.0f, "cutoff must be finite and > 0");
    float inv = 1.0f / cutoff;
    while (1.0 / (double)inv < (double)cutoff) inv = std::nextafter(inv, 0.0f);
    std::memset(g, 0, sizeof(*g));
    g->dim = dim;
    g->inv_cell = inv;
    int64_t cells = 1;
    for (int k = 0; k < dim; ++k) {
        PDMP_REQUIRE(std::isfinite(lo[k]) && std::isfinite(hi[k]) && lo[k] <= hi[k],
                     "bad box on axis %d", k);
        const double c = std::floor(((double)hi[k] - (double)lo[k]) * (double)inv) + 1.0;
        PDMP_REQUIRE(c <= (double)(1 << 20), "too many cells on axis %d", k);
        g->lo[k] = lo[k];
        g->nc[k] = c < 1.0 ? 1 : (int32_t)c;
        cells *= g->nc[k];
    }
    PDMP_REQUIRE(cells <= (int64_t)1 << 24, "too many cells (%lld)", (long long)cells);
    return PDMP_OK;
}

static int32_t check_cull_grid(const pdmp_occupancy *occ, const pdmp_cull_grid *g) {
    PDMP_REQUIRE(g != nullptr, "grid NULL");
    PDMP_REQUIRE(g->dim == occ->dim, "grid dim %d differs from the occupancy's %d", g->dim,
                 occ->dim);
    PDMP_REQUIRE(std::isfinite(g->inv_cell) && g->inv_cell > 0.0f, "inv_cell invalid");
    int64_t cells = 1;
    for (int k = 0; k < g->dim; ++k) {
        PDMP_REQUIRE(g->nc[k] >= 1 && g->nc[k] <= (1 << 20), "nc out of range");
        cells *= g->nc[k];
    }
    PDMP_REQUIRE(cells <= (int64_t)1 << 24, "too many cells");
    return PDMP_OK;
}

size_t pdmp_morph_culled_workspace_size(const pdmp_occupancy *occ, const pdmp_cull_grid *g,
                                        int64_t n) {
    if (check_occ(occ) || check_cull_grid(occ, g) || n < 1) return 0;
    return cull_ws_bytes(*g, occ->n_hinges, n);
}

int32_t pdmp_morph_culled(const pdmp_occupancy *occ, const pdmp_cull_grid *g, const float *in,
                          float *out, int64_t n, int32_t T, float eta, void *ws, size_t ws_bytes,
                          void *stream) {
    int32_t st = check_occ(occ);
    if (st) return st;
    if ((st = check_cull_grid(occ, g))) return st;
    PDMP_REQUIRE(n >= 0 && n < ((int64_t)1 << 31), "n out of range");
    PDMP_REQUIRE(T >= 0, "T < 0");
    PDMP_REQUIRE(std::isfinite(eta), "eta not finite");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(in && out, "in/out NULL");
    const size_t need = cull_ws_bytes(*g, occ->n_hinges, n);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        return PDMP_ENOMEM;
    }
    return launch_morph_culled(*occ, *g, in, out, n, T, eta, ws, (hipStream_t)stream);
}

int32_t pdmp_fk_body_points(const pdmp_arm *arm, const float *q, int64_t n, float *pts,
                            void *stream) {
    int32_t st = check_arm(arm, PDMP_MAX_PTS_PER_LINK);
    if (st) return st;
    PDMP_REQUIRE(n >= 0, "n < 0");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(q && pts, "q/pts NULL");
    return launch_fk_points(*arm, q, n, pts, (hipStream_t)stream);
}

size_t pdmp_fit_workspace_size(int32_t dim, int32_t n_hinges, int64_t n) {
    if ((dim != 2 && dim != 3) || n_hinges < 1 || n < 1) return 0;
    return fit_ws_bytes(dim, n_hinges, n);
}

size_t pdmp_bwd_workspace_size(int32_t dim, int32_t n_hinges, int64_t n) {
    if ((dim != 2 && dim != 3) || n_hinges < 1 || n < 1) return 0;
    return bwd_ws_bytes(dim, n_hinges, n);
}

size_t pdmp_bce_workspace_size(int64_t n) { return n < 1 ? 0 : bce_ws_bytes(n); }

int32_t pdmp_fit_occupancy(const pdmp_occupancy *occ, float *weights, const float *pts,
                           const uint8_t *labels, int64_t n, const pdmp_fit_opts *opts,
                           float *loss_out, void *ws, size_t ws_bytes, void *stream) {
    PDMP_REQUIRE(occ != nullptr, "occupancy is NULL");
    PDMP_REQUIRE(occ->dim == 2 || occ->dim == 3, "occupancy dim %d not in {2,3}", occ->dim);
    PDMP_REQUIRE(occ->n_hinges >= 1 && occ->hinges, "bad hinges");
    PDMP_REQUIRE(std::isfinite(occ->lengthscale) && occ->lengthscale > 0.0f, "bad lengthscale");
    int32_t st = check_grid_field(occ);
    if (st) return st;
    PDMP_REQUIRE(weights && pts && labels && opts, "NULL argument");
    PDMP_REQUIRE(n >= 1, "n < 1");
    PDMP_REQUIRE(opts->optimizer == 0 || opts->optimizer == 1, "optimizer %d", opts->optimizer);
    PDMP_REQUIRE(opts->steps >= 0, "steps < 0");
    PDMP_REQUIRE(std::isfinite(opts->lr) && std::isfinite(opts->l2) && opts->l2 >= 0.0f,
                 "bad lr/l2");
    if (opts->optimizer == 1) {
        PDMP_REQUIRE(opts->adam_m && opts->adam_v, "Adam needs adam_m and adam_v");
        PDMP_REQUIRE(opts->beta1 >= 0 && opts->beta1 < 1 && opts->beta2 >= 0 && opts->beta2 < 1 &&
                         opts->eps > 0 && opts->t0 >= 0,
                     "bad Adam hyperparameters");
    } else {
        PDMP_REQUIRE(std::isfinite(opts->lr_bias), "bad lr_bias");
    }
    const size_t need = fit_ws_bytes(occ->dim, occ->n_hinges, n);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        return PDMP_ENOMEM;
    }
    if ((st = grid_check(occ, stream))) return st;
    return launch_fit(occ->dim, occ->hinges, occ->n_hinges, has_grid(occ) ? occ->grid : nullptr,
                      occ->lengthscale, weights, pts, labels, n, *opts, loss_out, ws,
                      (hipStream_t)stream);
}

// The backward's argument checks; *done = true when there is nothing to launch.
static int32_t check_bwd(const pdmp_occupancy *occ, const float *x, int64_t n, const float *g,
                         const float *grad_w, const float *grad_x, bool *done) {
    int32_t st = check_occ(occ);
    if (st) return st;
    PDMP_REQUIRE(n >= 0, "n < 0");
    *done = true;
    if (n == 0) {
        PDMP_REQUIRE(grad_w == nullptr, "grad_w of an empty batch: use n >= 1");
        return PDMP_OK;
    }
    PDMP_REQUIRE(x && g, "x/g NULL");
    *done = !grad_w && !grad_x;
    return PDMP_OK;
}

int32_t pdmp_occupancy_bwd_noalloc(const pdmp_occupancy *occ, const float *x, int64_t n,
                                   const float *g, const float *s_fwd, float *grad_w,
                                   float *grad_x, void *stream) {
    bool done = false;
    int32_t st = check_bwd(occ, x, n, g, grad_w, grad_x, &done);
    if (st || done) return st;
    const size_t need = bwd_ws_bytes(occ->dim, occ->n_hinges, n);
    if (need > noalloc_scratch_bytes()) {
        set_error("this backward needs %zu bytes of scratch; the static scratch holds %zu "
                  "(use pdmp_occupancy_bwd with a workspace)", need, noalloc_scratch_bytes());
        return PDMP_ENOMEM;
    }
    void *ws = nullptr;
    if ((st = noalloc_scratch(&ws))) return st;
    if ((st = grid_check(occ, stream))) return st;
    return launch_logit_bwd(occ->dim, occ->hinges, occ->weights, occ->n_hinges,
                            has_grid(occ) ? occ->grid : nullptr, occ->lengthscale, x, n, g, s_fwd,
                            grad_w, grad_x, 1.0f, nullptr, 0.0f, ws, (hipStream_t)stream);
}

int32_t pdmp_occupancy_bwd(const pdmp_occupancy *occ, const float *x, int64_t n, const float *g,
                           const float *s_fwd, float *grad_w, float *grad_x, void *ws,
                           size_t ws_bytes, void *stream) {
    bool done = false;
    int32_t st = check_bwd(occ, x, n, g, grad_w, grad_x, &done);
    if (st || done) return st;
    const size_t need = bwd_ws_bytes(occ->dim, occ->n_hinges, n);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        return PDMP_ENOMEM;
    }
    if ((st = grid_check(occ, stream))) return st;
    return launch_logit_bwd(occ->dim, occ->hinges, occ->weights, occ->n_hinges,
                            has_grid(occ) ? occ->grid : nullptr, occ->lengthscale, x, n, g, s_fwd,
                            grad_w, grad_x, 1.0f, nullptr, 0.0f, ws, (hipStream_t)stream);
}

int32_t pdmp_bce_logits(const float *s, const uint8_t *y, int64_t n, const float *g_scale,
                        float *loss, float *g_s, void *ws, size_t ws_bytes, void *stream) {
    PDMP_REQUIRE(n >= 1, "n < 1");
    PDMP_REQUIRE(s && y, "s/y NULL");
    const size_t need = bce_ws_bytes(n);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        return PDMP_ENOMEM;
    }
    return launch_bce(s, y, n, g_scale, loss, g_s, (double *)ws, (hipStream_t)stream);
}

int32_t pdmp_adam_step(float *p, const float *g, float *m, float *v, int64_t n, int64_t n_decay,
                       int32_t t, float lr, float beta1, float beta2, float eps, float l2,
                       void *stream) {
    PDMP_REQUIRE(n >= 0 && n_decay >= 0 && n_decay <= n, "bad sizes");
    PDMP_REQUIRE(t >= 1, "t < 1");
    PDMP_REQUIRE(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0 &&
                     std::isfinite(lr) && std::isfinite(l2),
                 "bad hyperparameters");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(p && g && m && v, "NULL argument");
    return launch_adam(p, g, m, v, n, n_decay, t, lr, beta1, beta2, eps, l2, (hipStream_t)stream);
}

static int32_t check_mlp(const pdmp_mlp *m, bool need_params) {
    PDMP_REQUIRE(m != nullptr, "mlp is NULL");
    PDMP_REQUIRE(m->n_in >= 1 && m->n_in <= 16, "mlp n_in %d not in [1,16]", m->n_in);
    PDMP_REQUIRE(m->hidden >= 1 && m->hidden <= 1024, "mlp hidden %d not in [1,1024]", m->hidden);
    PDMP_REQUIRE(m->n_hidden >= 1 && m->n_hidden <= 6, "mlp n_hidden %d not in [1,6]", m->n_hidden);
    if (need_params) PDMP_REQUIRE(m->params && m->params_bf16, "mlp params NULL");
    return PDMP_OK;
}

int64_t pdmp_mlp_num_params(const pdmp_mlp *mlp) {
    if (check_mlp(mlp, false)) return -1;
    return mlp_nparams(*mlp);
}

int32_t pdmp_mlp_pack(const pdmp_mlp *mlp, uint16_t *params_bf16, void *stream) {
    int32_t st = check_mlp(mlp, false);
    if (st) return st;
    PDMP_REQUIRE(mlp->params && params_bf16, "params/params_bf16 NULL");
    return launch_f32_to_bf16(mlp->params, mlp_nparams(*mlp), params_bf16, (hipStream_t)stream);
}

size_t pdmp_mlp_acts_size(const pdmp_mlp *mlp, int64_t B) {
    if (check_mlp(mlp, false) || B < 1) return 0;
    return mlp_acts_bytes(*mlp, B);
}

size_t pdmp_mlp_workspace_size(const pdmp_mlp *mlp, int64_t B) {
    if (check_mlp(mlp, false) || B < 1) return 0;
    const size_t a = mlp_fwd_ws_bytes(*mlp, B), b = mlp_bwd_ws_bytes(*mlp, B);
    return a > b ? a : b;
}

int32_t pdmp_mlp_forward(const pdmp_mlp *mlp, const float *q, int64_t B, float *q_hat, void *acts,
                         void *ws, size_t ws_bytes, void *stream) {
    int32_t st = check_mlp(mlp, true);
    if (st) return st;
    PDMP_REQUIRE(B >= 0, "B < 0");
    if (B == 0) return PDMP_OK;
    PDMP_REQUIRE(q && q_hat, "q/q_hat NULL");
    PDMP_REQUIRE(B <= 0x7fffffff, "B too large");
    if (!acts) {
        const size_t need = mlp_fwd_ws_bytes(*mlp, B);
        if (!ws || ws_bytes < need) {
            set_error("workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
            return PDMP_ENOMEM;
        }
    }
    return launch_mlp_forward(*mlp, q, B, q_hat, acts, ws, (hipStream_t)stream);
}

int32_t pdmp_mlp_backward(const pdmp_mlp *mlp, const float *q_hat, const float *target,
                          int64_t B, void *acts, float *grad, float *loss, void *ws,
                          size_t ws_bytes, void *stream) {
    int32_t st = check_mlp(mlp, true);
    if (st) return st;
    PDMP_REQUIRE(B >= 1 && B <= 0x7fffffff, "B out of range");
    PDMP_REQUIRE(q_hat && target && acts && grad, "NULL argument");
    const size_t need = mlp_bwd_ws_bytes(*mlp, B);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        return PDMP_ENOMEM;
    }
    return launch_mlp_backward(*mlp, q_hat, target, B, acts, grad, loss, ws, (hipStream_t)stream);
}

int32_t pdmp_mlp_backward_weighted(const pdmp_mlp *mlp, const float *q_hat, const float *target,
                                   int64_t B, const uint8_t *hard, float hard_weight, void *acts,
                                   float *grad, float *loss, void *ws, size_t ws_bytes,
                                   void *stream) {
    int32_t st = check_mlp(mlp, true);
    if (st) return st;
    PDMP_REQUIRE(B >= 1 && B <= 0x7fffffff, "B out of range");
    PDMP_REQUIRE(q_hat && target && acts && grad, "NULL argument");
    PDMP_REQUIRE(hard_weight >= 0.0f && hard_weight < INFINITY, "hard_weight not finite and >= 0");
    const size_t need = mlp_bwd_ws_bytes(*mlp, B);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        return PDMP_ENOMEM;
    }
    return launch_mlp_backward(*mlp, q_hat, target, B, acts, grad, loss, ws, (hipStream_t)stream,
                               hard, hard_weight);
}

int32_t pdmp_arm_max_occupancy(const pdmp_occupancy *occ, const pdmp_arm *arm, const float *q,
                               int64_t n, float thresh, float *maxc, uint8_t *flag,
                               void *stream) {
    int32_t st = check_occ(occ);
    if (st) return st;
    st = check_arm(arm, 8);
    if (st) return st;
    PDMP_REQUIRE(occ->dim == 3, "the body-point check needs a 3-D occupancy");
    PDMP_REQUIRE(n >= 0, "n < 0");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(q != nullptr, "q NULL");
    float kappa, gscale;
    derive_scales(occ->lengthscale, kappa, gscale);
    if (has_grid(occ)) {
        if ((st = grid_check(occ, stream))) return st;
        st = launch_arm_grid3d(*arm, occ->hinges, occ->weights, occ->n_hinges, occ->grid, kappa,
                               gscale, q, nullptr, n, 1, 0.0f, nullptr, false, thresh, maxc, flag,
                               (hipStream_t)stream);
        if (st != PDMP_EUNSUPPORTED) return st;
    }
    return launch_arm_max_occ(*arm, occ->hinges, occ->weights, occ->n_hinges, kappa, q, n, thresh,
                              maxc, flag, (hipStream_t)stream);
}

static size_t al256h(size_t b) { return (b + 255) & ~(size_t)255; }

size_t pdmp_amortised_workspace_size(const pdmp_mlp *mlp, const pdmp_arm *arm, int64_t n) {
    if (check_mlp(mlp, false) || !arm || n < 1) return 0;
    const size_t nb = (size_t)((n + 255) / 256);
    return mlp_fwd_ws_bytes(*mlp, n) + al256h((size_t)n) /* flags */ +
           2 * al256h(nb * 4) + al256h(8) + al256h((size_t)n * 4) /* idx */ +
           al256h((size_t)arm->n_dof * n * 4) /* compact batch */;
}

// from_qhat: the fallback gathers the flagged rows of q_hat (out) instead of q.
static int32_t amortised_impl(const pdmp_mlp *mlp, const pdmp_occupancy *occ, const pdmp_arm *arm,
                              const float *q, float *out, int64_t n, int32_t T, float eta,
                              float thresh, uint8_t *flag, uint32_t *n_fallback, void *ws,
                              size_t ws_bytes, void *stream, bool from_qhat) {
    int32_t st = check_mlp(mlp, true);
    if (st) return st;
    st = check_occ(occ);
    if (st) return st;
    st = check_arm(arm, 8);
    if (st) return st;
    PDMP_REQUIRE(occ->dim == 3, "the amortised arm morph needs a 3-D occupancy");
    PDMP_REQUIRE(mlp->n_in == arm->n_dof, "mlp width %d != n_dof %d", mlp->n_in, arm->n_dof);
    PDMP_REQUIRE(n >= 0 && n <= 0x7fffffff, "n out of range");
    PDMP_REQUIRE(T >= 0 && std::isfinite(eta) && std::isfinite(thresh), "bad T/eta/thresh");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(q && out && q != out, "q/out NULL or aliased");
    const size_t need = pdmp_amortised_workspace_size(mlp, arm, n);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        return PDMP_ENOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = (size_t)((n + 255) / 256);
    char *c = (char *)ws;
    void *mws = c;
    c += mlp_fwd_ws_bytes(*mlp, n);
    uint8_t *fl = flag ? flag : (uint8_t *)c;
    c += al256h((size_t)n);
    uint32_t *counts = (uint32_t *)c;
    c += al256h(nb * 4);
    uint32_t *offs = (uint32_t *)c;
    c += al256h(nb * 4);
    uint32_t *total = n_fallback ? n_fallback : (uint32_t *)c;
    c += al256h(8);
    uint32_t *idx = (uint32_t *)c;
    c += al256h((size_t)n * 4);
    float *qc = (float *)c;

    float kappa, gscale;
    derive_scales(occ->lengthscale, kappa, gscale);
    const int *grid = has_grid(occ) ? occ->grid : nullptr;
    if ((st = grid_check(occ, stream))) return st;
    if ((st = launch_mlp_forward(*mlp, q, n, out, nullptr, mws, s))) return st;
    st = PDMP_EUNSUPPORTED;
    if (grid)
        st = launch_arm_grid3d(*arm, occ->hinges, occ->weights, occ->n_hinges, grid, kappa, gscale,
                               out, nullptr, n, 1, 0.0f, nullptr, false, thresh, nullptr, fl, s);
    if (st == PDMP_EUNSUPPORTED)
        st = launch_arm_max_occ(*arm, occ->hinges, occ->weights, occ->n_hinges, kappa, out, n,
                                thresh, nullptr, fl, s);
    if (st) return st;
    if ((st = launch_compact(*arm, fl, from_qhat ? out : q, n, counts, offs, total, idx, qc, s)))
        return st;
    st = PDMP_EUNSUPPORTED;
    if (grid)
        st = launch_arm_grid3d(*arm, occ->hinges, occ->weights, occ->n_hinges, grid, kappa, gscale,
                               qc, qc, n, T, eta, total, true, 0.0f, nullptr, nullptr, s);
    if (st == PDMP_EUNSUPPORTED)
        st = launch_morph_arm(*arm, occ->hinges, occ->weights, occ->n_hinges, kappa, gscale, qc, qc,
                              n, T, eta, total, s);
    if (st) return st;
    return launch_scatter(*arm, idx, total, qc, n, out, s);
}

int32_t pdmp_amortised_morph(const pdmp_mlp *mlp, const pdmp_occupancy *occ, const pdmp_arm *arm,
                             const float *q, float *out, int64_t n, int32_t T, float eta,
                             float thresh, uint8_t *flag, uint32_t *n_fallback, void *ws,
                             size_t ws_bytes, void *stream) {
    return amortised_impl(mlp, occ, arm, q, out, n, T, eta, thresh, flag, n_fallback, ws,
                          ws_bytes, stream, false);
}

int32_t pdmp_amortised_morph_refine(const pdmp_mlp *mlp, const pdmp_occupancy *occ,
                                    const pdmp_arm *arm, const float *q, float *out, int64_t n,
                                    int32_t T_refine, float eta, float thresh, uint8_t *flag,
                                    uint32_t *n_fallback, void *ws, size_t ws_bytes,
                                    void *stream) {
    return amortised_impl(mlp, occ, arm, q, out, n, T_refine, eta, thresh, flag, n_fallback, ws,
                          ws_bytes, stream, true);
}

// ---- the tanh occupancy network ----

static int64_t tanh_nparams(const pdmp_tanh_net *net) {
    const int64_t H = net->hidden, D = net->dim, L = net->n_hidden;
    return H * D + H + (L - 1) * (H * H + H) + H + 1;
}

static int32_t check_tanh(const pdmp_tanh_net *net) {
    PDMP_REQUIRE(net != nullptr, "net is NULL");
    PDMP_REQUIRE(net->dim == 2 || net->dim == 3, "dim %d not 2 or 3", net->dim);
    PDMP_REQUIRE(net->hidden >= 1 && net->hidden <= 64, "hidden %d not in [1,64]", net->hidden);
    PDMP_REQUIRE(net->n_hidden >= 1 && net->n_hidden <= 4, "n_hidden %d not in [1,4]",
                 net->n_hidden);
    PDMP_REQUIRE(net->params != nullptr, "params NULL");
    return PDMP_OK;
}

int64_t pdmp_tanh_num_params(const pdmp_tanh_net *net) {
    if (!net || (net->dim != 2 && net->dim != 3) || net->hidden < 1 || net->hidden > 64 ||
        net->n_hidden < 1 || net->n_hidden > 4)
        return -1;
    return tanh_nparams(net);
}

int32_t pdmp_tanh_occupancy_eval(const pdmp_tanh_net *net, const float *x, int64_t n,
                                 float *c_out, float *s_out, void *stream) {
    int32_t st = check_tanh(net);
    if (st) return st;
    PDMP_REQUIRE(n >= 0, "n < 0");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(x != nullptr, "x NULL");
    PDMP_REQUIRE(c_out || s_out, "c_out and s_out both NULL");
    return launch_tanh_net(*net, kEval, x, n, 1, 0.0f, c_out, s_out, nullptr, nullptr,
                           (hipStream_t)stream);
}

int32_t pdmp_tanh_occupancy_grad(const pdmp_tanh_net *net, const float *x, int64_t n,
                                 float *c_out, float *grad_out, void *stream) {
    int32_t st = check_tanh(net);
    if (st) return st;
    PDMP_REQUIRE(n >= 0, "n < 0");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(x && grad_out, "x/grad_out NULL");
    return launch_tanh_net(*net, kGrad, x, n, 1, 0.0f, c_out, nullptr, grad_out, nullptr,
                           (hipStream_t)stream);
}

int32_t pdmp_tanh_split_scheme(const pdmp_tanh_net *net, int32_t *scheme, void *stream) {
    int32_t st = check_tanh(net);
    if (st) return st;
    PDMP_REQUIRE(scheme != nullptr, "scheme NULL");
    *scheme = 0;
    hipStream_t s = (hipStream_t)stream;
    int32_t *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(int32_t));
    if (e != hipSuccess) {
        set_error("hipMalloc: %s", hipGetErrorString(e));
        return PDMP_EDEVICE;
    }
    st = launch_tanh_scheme(*net, d, s);
    int32_t v = 0;
    if (st == PDMP_OK) {
        e = hipMemcpyAsync(&v, d, sizeof(v), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            set_error("tanh split scheme query: %s", hipGetErrorString(e));
            st = PDMP_EDEVICE;
        }
    }
    (void)hipFree(d);
    if (st == PDMP_OK) *scheme = v;
    return st;
}

int32_t pdmp_tanh_morph_samples(const pdmp_tanh_net *net, const float *in, float *out, int64_t n,
                                int32_t T, float eta, void *stream) {
    int32_t st = check_tanh(net);
    if (st) return st;
    PDMP_REQUIRE(n >= 0, "n < 0");
    PDMP_REQUIRE(T >= 0, "T < 0");
    PDMP_REQUIRE(std::isfinite(eta), "eta not finite");
    if (n == 0) return PDMP_OK;
    PDMP_REQUIRE(in && out, "in/out NULL");
    if (T == 0) {
        if (in == out) return PDMP_OK;
        hipError_t e = hipMemcpyAsync(out, in, (size_t)net->dim * (size_t)n * sizeof(float),
                                      hipMemcpyDeviceToDevice, (hipStream_t)stream);
        if (e != hipSuccess) {
            set_error("hipMemcpyAsync: %s", hipGetErrorString(e));
            return PDMP_EDEVICE;
        }
        return PDMP_OK;
    }
    return launch_tanh_net(*net, kMorph, in, n, T, eta, nullptr, nullptr, nullptr, out,
                           (hipStream_t)stream);
}

size_t pdmp_tanh_fit_workspace_size(const pdmp_tanh_net *net, int64_t n) {
    if (pdmp_tanh_num_params(net) < 0 || n < 1) return 0;
    return tanh_fit_ws_bytes(*net, n);
}

static int32_t check_tanh_fit_args(const pdmp_tanh_net *net, const float *pts,
                                   const uint8_t *labels, int64_t n, void *ws, size_t ws_bytes) {
    int32_t st = check_tanh(net);
    if (st) return st;
    PDMP_REQUIRE(n >= 1, "n < 1");
    PDMP_REQUIRE(pts && labels, "pts/labels NULL");
    const size_t need = tanh_fit_ws_bytes(*net, n);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        return PDMP_ENOMEM;
    }
    return PDMP_OK;
}

int32_t pdmp_tanh_loss_grad(const pdmp_tanh_net *net, const float *pts, const uint8_t *labels,
                            int64_t n, float l2, float *loss, float *grad, void *ws,
                            size_t ws_bytes, void *stream) {
    int32_t st = check_tanh_fit_args(net, pts, labels, n, ws, ws_bytes);
    if (st) return st;
    PDMP_REQUIRE(grad != nullptr, "grad NULL");
    PDMP_REQUIRE(std::isfinite(l2) && l2 >= 0.0f, "l2 must be finite and >= 0");
    return launch_tanh_loss_grad(*net, pts, labels, n, l2, loss, grad, ws, (hipStream_t)stream);
}

int32_t pdmp_tanh_fit(const pdmp_tanh_net *net, const float *pts, const uint8_t *labels,
                      int64_t n, const pdmp_fit_opts *opts, float *loss_out, void *ws,
                      size_t ws_bytes, void *stream) {
    int32_t st = check_tanh_fit_args(net, pts, labels, n, ws, ws_bytes);
    if (st) return st;
    PDMP_REQUIRE(opts != nullptr, "opts NULL");
    PDMP_REQUIRE(opts->optimizer == 1, "the network fit uses Adam (optimizer 1)");
    PDMP_REQUIRE(opts->steps >= 0, "steps < 0");
    PDMP_REQUIRE(opts->adam_m && opts->adam_v, "adam_m/adam_v NULL");
    PDMP_REQUIRE(std::isfinite(opts->lr) && std::isfinite(opts->l2) && opts->l2 >= 0.0f,
                 "lr/l2 invalid");
    PDMP_REQUIRE(opts->beta1 >= 0.0f && opts->beta1 < 1.0f && opts->beta2 >= 0.0f &&
                     opts->beta2 < 1.0f && opts->eps > 0.0f,
                 "Adam hyperparameters out of range");
    PDMP_REQUIRE(opts->t0 >= 0, "t0 < 0");
    return launch_tanh_fit(*net, pts, labels, n, opts->steps, opts->lr, opts->l2, opts->beta1,
                           opts->beta2, opts->eps, opts->adam_m, opts->adam_v, opts->t0, loss_out,
                           ws, (hipStream_t)stream);
}

}  // extern "C"
