/*
 * pdmp_oracle.c -- plain FP64 CPU oracle for the PDMP morph path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code, header,
 * table or constant with the HIP library; the product path never calls it.
 *
 * What it computes (Lai, Zhi, Hermans, Ramos, "Parallelised Diffeomorphic
 * Sampling-based Motion Planning"):
 *   - occupancy c(x) = sigma(s(x)), s(x) = sum_j w_j phi_j(x) + beta, with Gaussian
 *     RBF features phi_j(x) = exp(-|x-h_j|^2/(2 l^2)) on hinge points (the
 *     Hilbert-map form of the continuous occupancy of Sec. 3.1), its gradient and
 *     Hessian, written out from the definition;
 *   - the occupancy fit by binary cross-entropy with gradient descent or Adam
 *     (Sec. 3.1), full batch;
 *   - the morph: explicit Euler steps along the negative cost gradient, i.e. the
 *     integral curve of Eq. (1) solved by Euler's method (Sec. 3.2);
 *   - standard Denavit-Hartenberg forward kinematics of body points and the
 *     pull-back of the task-space gradient into joint space (Sec. 3.2, Eq. 3,
 *     read with the Jacobian transposed and each body point's own gradient);
 *   - collision labels of points and configurations (the "feasible" count of
 *     Table 1), decided in FP64;
 *   - Philox4x32-10 (Salmon et al., SC 2011) for the prior samples that the
 *     method draws in batches (Sec. 3.3);
 *   - the residual MLP of the amortised morph (forward, MSE backward, Adam).
 *
 * Every loop runs in the order the definition states: sums over hinges j = 0..M-1
 * and over points i = 0..n-1 in index order.  Build with -ffp-contract=off and no
 * fast-math.  OpenMP is used over independent samples only.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_DIM 3
#define ORC_MAX_DOF 8

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads the following parallel regions use (n >= 1). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011, Sec. 4 and Table 2).  */
/* ------------------------------------------------------------------------- */

static uint32_t mul_hi_lo(uint32_t a, uint32_t b, uint32_t *lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *lo = (uint32_t)p;
    return (uint32_t)(p >> 32);
}

/* Ten rounds; the key is bumped by the Weyl constants before every round after
 * the first.  Each round: two 32x32->64 multiplies of counter words 0 and 2, and
 * the high halves XOR-ed with the other counter words and the key. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t lo0, lo1;
        uint32_t hi0 = mul_hi_lo(0xD2511F53u, c0, &lo0);
        uint32_t hi1 = mul_hi_lo(0xCD9E8D57u, c2, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Prior samples x ~ U[lo, hi)^dim.  Sample i, coordinate k takes word k%4 of
 * Philox(counter = {i_lo, i_hi, k/4, stream}, key = {seed_lo, seed_hi});
 * u = (word >> 8) * 2^-24 in [0,1); x = lo + (hi - lo) * u in FP64, rounded
 * once to FP32. */
static float uniform_coord(uint64_t seed, uint32_t stream, const float *lo, const float *hi,
                           int k, int64_t i) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)(k / 4), stream};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    double u = (double)(r[k % 4] >> 8) * (1.0 / 16777216.0);
    double span = (double)hi[k] - (double)lo[k];
    double t = span * u;
    double x = (double)lo[k] + t;
    return (float)x;
}

void orc_uniform_samples(uint64_t seed, uint32_t stream, const float *lo, const float *hi,
                         int dim, int64_t n, float *out) {
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k)
            out[(int64_t)k * n + i] = uniform_coord(seed, stream, lo, hi, k, i);
}

/* The same batch at chosen sample indices (the counter holds the index, so a sample
 * needs no other): out[k m + j] = coordinate k of sample idx[j]. */
void orc_uniform_at(uint64_t seed, uint32_t stream, const float *lo, const float *hi, int dim,
                    const int64_t *idx, int64_t m, float *out) {
    for (int64_t j = 0; j < m; ++j)
        for (int k = 0; k < dim; ++k)
            out[(int64_t)k * m + j] = uniform_coord(seed, stream, lo, hi, k, idx[j]);
}

/* ------------------------------------------------------------------------- */
/* Collision labels (closed obstacles, FP64).                                */
/* ------------------------------------------------------------------------- */

/* Point (x, y) is inside disc k iff dx*dx + dy*dy <= r*r, dx = x - cx. */
void orc_label_discs(const double *cx, const double *cy, const double *r, int K,
                     const double *x, int64_t n, uint8_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int in = 0;
        for (int k = 0; k < K; ++k) {
            double dx = x[i] - cx[k];
            double dy = x[n + i] - cy[k];
            double a = dx * dx;
            double b = dy * dy;
            double d2 = a + b;
            double rr = r[k] * r[k];
            if (d2 <= rr) in = 1;
        }
        out[i] = (uint8_t)in;
    }
}

/* Point is inside axis-aligned box k iff |x_a - c_a| <= e_a for a = 0, 1, 2. */
static int in_any_box(const double p[3], const double *c, const double *e, int K) {
    for (int k = 0; k < K; ++k) {
        int in = 1;
        for (int a = 0; a < 3; ++a)
            if (!(fabs(p[a] - c[a * K + k]) <= e[a * K + k])) in = 0;
        if (in) return 1;
    }
    return 0;
}

void orc_label_boxes(const double *c, const double *e, int K, const double *x, int64_t n,
                     uint8_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double p[3] = {x[i], x[n + i], x[2 * n + i]};
        out[i] = (uint8_t)in_any_box(p, c, e, K);
    }
}

/* ------------------------------------------------------------------------- */
/* RBF occupancy: value, gradient, Hessian at one point.                     */
/* ------------------------------------------------------------------------- */

typedef struct {
    double s;               /* logit */
    double gs[ORC_MAX_DIM];  /* grad s */
    double Hs[ORC_MAX_DIM * ORC_MAX_DIM];
    double sabs;            /* |beta| + sum |w_j| phi_j */
    double graw;            /* l^-2 sum |w_j| phi_j |x - h_j| */
} rbf_val;

static void rbf_point(int dim, int M, const double *h, const double *w, double beta,
                      double ell, const double *x, int want_hess, rbf_val *v) {
    double il2 = 1.0 / (ell * ell);
    double i2l2 = 0.5 * il2;
    memset(v, 0, sizeof(*v));
    v->s = beta;
    v->sabs = fabs(beta);
    for (int j = 0; j < M; ++j) {
        double diff[ORC_MAX_DIM];
        double r2 = 0.0;
        for (int k = 0; k < dim; ++k) {
            diff[k] = x[k] - h[(int64_t)k * M + j];
            r2 += diff[k] * diff[k];
        }
        double phi = exp(-r2 * i2l2);
        double wp = w[j] * phi;
        v->s += wp;
        v->sabs += fabs(w[j]) * phi;
        v->graw += fabs(w[j]) * phi * sqrt(r2) * il2;
        for (int k = 0; k < dim; ++k) v->gs[k] += -il2 * wp * diff[k];
        if (want_hess)
            for (int a = 0; a < dim; ++a)
                for (int b = 0; b < dim; ++b)
                    v->Hs[a * dim + b] += wp * (diff[a] * diff[b] * il2 * il2 - (a == b ? il2 : 0.0));
    }
}

static double sigmoid(double s) { return 1.0 / (1.0 + exp(-s)); }

/* sigma'(s) = sigma(s)(1 - sigma(s)), written as e/(1 + e)^2 with e = exp(-|s|) so
 * that it keeps its relative accuracy where sigma(s) rounds to 0 or 1. */
static double sigmoid_slope(double s) {
    double e = exp(-fabs(s));
    return e / ((1.0 + e) * (1.0 + e));
}

/* c, grad c, Hessian of c and the gradient error scale G_abs from the logit. */
typedef struct {
    double c, dc;                       /* sigma(s), sigma'(s) */
    double g[ORC_MAX_DIM];              /* grad c */
    double H[ORC_MAX_DIM * ORC_MAX_DIM]; /* Hessian of c */
    double gabs;
} occ_val;

static void occ_point(int dim, int M, const double *h, const double *w, double beta, double ell,
                      const double *x, int want_hess, occ_val *o, rbf_val *rv) {
    rbf_val v;
    rbf_point(dim, M, h, w, beta, ell, x, want_hess, &v);
    double c = sigmoid(v.s);
    double d1 = sigmoid_slope(v.s);
    double d2 = d1 * (1.0 - 2.0 * c);
    o->c = c;
    o->dc = d1;
    double gn = 0.0;
    for (int k = 0; k < dim; ++k) {
        o->g[k] = d1 * v.gs[k];
        gn += v.gs[k] * v.gs[k];
    }
    o->gabs = d1 * v.graw + fabs(d2) * sqrt(gn) * v.sabs;
    if (want_hess)
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b)
                o->H[a * dim + b] = d1 * v.Hs[a * dim + b] + d2 * v.gs[a] * v.gs[b];
    if (rv) *rv = v;
}

/* Logit s, occupancy c and the logit error scale S_abs at n points. */
void orc_occ_eval(int dim, int M, const double *h, const double *w, double beta, double ell,
                  const double *x, int64_t n, double *s, double *c, double *sabs) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xi[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) xi[k] = x[(int64_t)k * n + i];
        rbf_val v;
        rbf_point(dim, M, h, w, beta, ell, xi, 0, &v);
        if (s) s[i] = v.s;
        if (c) c[i] = sigmoid(v.s);
        if (sabs) sabs[i] = v.sabs;
    }
}

/* grad c = sigma'(s) grad s, also grad s, the error scale G_abs and (graw) the
 * logit-gradient scale l^-2 sum_j |w_j| phi_j |x - h_j|. */
void orc_occ_grad(int dim, int M, const double *h, const double *w, double beta, double ell,
                  const double *x, int64_t n, double *c, double *gc, double *gs, double *gabs,
                  double *graw) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xi[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) xi[k] = x[(int64_t)k * n + i];
        occ_val o;
        rbf_val v;
        occ_point(dim, M, h, w, beta, ell, xi, 0, &o, &v);
        if (c) c[i] = o.c;
        for (int k = 0; k < dim; ++k) {
            if (gc) gc[(int64_t)k * n + i] = o.g[k];
            if (gs) gs[(int64_t)k * n + i] = v.gs[k];
        }
        if (gabs) gabs[i] = o.gabs;
        if (graw) graw[i] = v.graw;
    }
}

/* Hessian of c (row-major dim x dim per point, [dim*dim][n]) and of s. */
void orc_occ_hess(int dim, int M, const double *h, const double *w, double beta, double ell,
                  const double *x, int64_t n, double *Hc, double *Hs) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xi[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) xi[k] = x[(int64_t)k * n + i];
        occ_val o;
        rbf_val v;
        occ_point(dim, M, h, w, beta, ell, xi, 1, &o, &v);
        for (int a = 0; a < dim * dim; ++a) {
            if (Hc) Hc[(int64_t)a * n + i] = o.H[a];
            if (Hs) Hs[(int64_t)a * n + i] = v.Hs[a];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Symmetric eigenvalues by cyclic Jacobi rotations (Golub & Van Loan 8.5).  */
/* ------------------------------------------------------------------------- */

static void sym_eigvals(int n, double *A /* n*n, destroyed */, double *ev) {
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
        if (off < 1e-300) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) { /* columns p, q */
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = cs * akp - sn * akq;
                    A[k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) { /* rows p, q */
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = cs * apk - sn * aqk;
                    A[q * n + k] = sn * apk + cs * aqk;
                }
            }
    }
    for (int k = 0; k < n; ++k) ev[k] = A[k * n + k];
}

/* Spectral norm, determinant of the symmetric step Jacobian I - eta*H. */
static void step_jac_stats(int n, const double *H, double eta, double *norm2, double *det,
                           double *hnorm) {
    double A[ORC_MAX_DOF * ORC_MAX_DOF], B[ORC_MAX_DOF * ORC_MAX_DOF], ev[ORC_MAX_DOF];
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            A[a * n + b] = (a == b ? 1.0 : 0.0) - eta * 0.5 * (H[a * n + b] + H[b * n + a]);
            B[a * n + b] = 0.5 * (H[a * n + b] + H[b * n + a]);
        }
    sym_eigvals(n, A, ev);
    double nm = 0.0, d = 1.0;
    for (int k = 0; k < n; ++k) {
        if (fabs(ev[k]) > nm) nm = fabs(ev[k]);
        d *= ev[k];
    }
    *norm2 = nm;
    *det = d;
    sym_eigvals(n, B, ev);
    double hn = 0.0;
    for (int k = 0; k < n; ++k)
        if (fabs(ev[k]) > hn) hn = fabs(ev[k]);
    *hnorm = hn;
}

/* ------------------------------------------------------------------------- */
/* Plain workspace morph: x_{k+1} = x_k - eta * grad c(x_k), k = 0..T-1.      */
/* ------------------------------------------------------------------------- */

/* Optional diagnostics per sample (any pointer may be NULL):
 *   amp:     product over steps of |I - eta Hc(x_k)|_2 (FP64 error amplification),
 *   min_det: smallest det(I - eta Hc(x_k)) along the path,
 *   max_eh:  largest eta*|Hc(x_k)|_2 along the path,
 *   traj:    all states, [T+1][dim][n]. */
void orc_morph_ws(int dim, int M, const double *h, const double *w, double beta, double ell,
                  const double *xin, int64_t n, int T, double eta, double *xout, double *amp,
                  double *min_det, double *max_eh, double *traj) {
    int diag = (amp || min_det || max_eh);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) x[k] = xin[(int64_t)k * n + i];
        double A = 1.0, mdet = INFINITY, meh = 0.0;
        if (traj)
            for (int k = 0; k < dim; ++k) traj[(int64_t)k * n + i] = x[k];
        for (int t = 0; t < T; ++t) {
            occ_val o;
            occ_point(dim, M, h, w, beta, ell, x, diag, &o, NULL);
            if (diag) {
                double nm, det, hn;
                step_jac_stats(dim, o.H, eta, &nm, &det, &hn);
                A *= nm;
                if (det < mdet) mdet = det;
                if (eta * hn > meh) meh = eta * hn;
            }
            for (int k = 0; k < dim; ++k) x[k] = x[k] - eta * o.g[k];
            if (traj)
                for (int k = 0; k < dim; ++k)
                    traj[((int64_t)(t + 1) * dim + k) * n + i] = x[k];
        }
        for (int k = 0; k < dim; ++k) xout[(int64_t)k * n + i] = x[k];
        if (amp) amp[i] = A;
        if (min_det) min_det[i] = mdet;
        if (max_eh) max_eh[i] = meh;
    }
}

/* ------------------------------------------------------------------------- */
/* Occupancy fit: mean BCE on logits + (l2/2)|w|^2, beta unregularised.       */
/* ------------------------------------------------------------------------- */

/* Binary cross-entropy of sigma(s) against y in the overflow-free form
 * max(s,0) - y*s + log(1 + exp(-|s|)). */
static double bce_logit(double s, double y) {
    return (s > 0 ? s : 0.0) - y * s + log1p(exp(-fabs(s)));
}

/* Loss and gradient at wb = [w_0..w_{M-1}, beta]:
 *   grad_j = (1/n) sum_i r_i phi_ij + l2 w_j,  grad_M = (1/n) sum_i r_i,
 *   r_i = sigma(s_i) - y_i.
 * gscale (nullable) gets (1/n) sum_i |r_i| phi_ij + l2 |w_j| (and (1/n) sum |r_i|). */
double orc_fit_loss_grad(int dim, int M, const double *h, double ell, const double *wb,
                         const double *pts, const uint8_t *y, int64_t n, double l2,
                         double *grad, double *gscale) {
    double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *li = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double i2l2 = 0.5 / (ell * ell);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xi[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) xi[k] = pts[(int64_t)k * n + i];
        rbf_val v;
        rbf_point(dim, M, h, wb, wb[M], ell, xi, 0, &v);
        r[i] = sigmoid(v.s) - (double)y[i];
        li[i] = bce_logit(v.s, (double)y[i]);
    }
    double loss = 0.0;
    for (int64_t i = 0; i < n; ++i) loss += li[i];
    loss /= (double)n;
    double reg = 0.0;
    for (int j = 0; j < M; ++j) reg += wb[j] * wb[j];
    loss += 0.5 * l2 * reg;
    if (grad) {
#pragma omp parallel for schedule(static)
        for (int j = 0; j < M; ++j) {
            double acc = 0.0, aabs = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double r2 = 0.0;
                for (int k = 0; k < dim; ++k) {
                    double d = pts[(int64_t)k * n + i] - h[(int64_t)k * M + j];
                    r2 += d * d;
                }
                double phi = exp(-r2 * i2l2);
                acc += r[i] * phi;
                aabs += fabs(r[i]) * phi;
            }
            grad[j] = acc / (double)n + l2 * wb[j];
            if (gscale) gscale[j] = aabs / (double)n + l2 * fabs(wb[j]);
        }
        double acc = 0.0, aabs = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            acc += r[i];
            aabs += fabs(r[i]);
        }
        grad[M] = acc / (double)n;
        if (gscale) gscale[M] = aabs / (double)n;
    }
    free(r);
    free(li);
    return loss;
}

/* Adam (Kingma & Ba 2015, Algorithm 1), step t >= 1, on a flat parameter array. */
void orc_adam_step(double *p, const double *g, double *m, double *v, int64_t n, int t,
                   double lr, double b1, double b2, double eps) {
    double bc1 = 1.0 - pow(b1, (double)t);
    double bc2 = 1.0 - pow(b2, (double)t);
    for (int64_t k = 0; k < n; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * g[k];
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
        double mh = m[k] / bc1;
        double vh = v[k] / bc2;
        p[k] = p[k] - lr * mh / (sqrt(vh) + eps);
    }
}

/* Full-batch fit, `steps` iterations from the given wb (in/out, [M+1]).
 * optimizer 0: gradient descent, w <- w - lr * grad_w, beta <- beta - lr_bias * grad_beta;
 * optimizer 1: Adam with step lr on every parameter and state m, v ([M+1], in/out),
 *              whose step counter continues from t0.
 * loss[t] (nullable) is the loss at the start of step t. */
void orc_fit(int dim, int M, const double *h, double ell, const double *pts, const uint8_t *y,
             int64_t n, int optimizer, int steps, double lr, double lr_bias, double l2,
             double b1, double b2, double eps, double *wb, double *m, double *v, int t0,
             double *loss) {
    double *g = (double *)malloc(sizeof(double) * (size_t)(M + 1));
    for (int t = 0; t < steps; ++t) {
        double L = orc_fit_loss_grad(dim, M, h, ell, wb, pts, y, n, l2, g, NULL);
        if (loss) loss[t] = L;
        if (optimizer == 0) {
            for (int j = 0; j < M; ++j) wb[j] = wb[j] - lr * g[j];
            wb[M] = wb[M] - lr_bias * g[M];
        } else {
            orc_adam_step(wb, g, m, v, M + 1, t0 + t + 1, lr, b1, b2, eps);
        }
    }
    free(g);
}

/* Backward of the logit s(x; w, beta) for an upstream dL/ds = gs:
 *   grad_w_j = sum_i gs_i phi_ij, grad_beta = sum_i gs_i,
 *   grad_x_i = gs_i * grad s(x_i). */
void orc_logit_bwd(int dim, int M, const double *h, const double *w, double ell,
                   const double *x, int64_t n, const double *gsv, double *grad_w,
                   double *grad_x) {
    double i2l2 = 0.5 / (ell * ell);
    if (grad_w) {
#pragma omp parallel for schedule(static)
        for (int j = 0; j < M; ++j) {
            double acc = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double r2 = 0.0;
                for (int k = 0; k < dim; ++k) {
                    double d = x[(int64_t)k * n + i] - h[(int64_t)k * M + j];
                    r2 += d * d;
                }
                acc += gsv[i] * exp(-r2 * i2l2);
            }
            grad_w[j] = acc;
        }
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) acc += gsv[i];
        grad_w[M] = acc;
    }
    if (grad_x) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double xi[ORC_MAX_DIM];
            for (int k = 0; k < dim; ++k) xi[k] = x[(int64_t)k * n + i];
            rbf_val v;
            rbf_point(dim, M, h, w, 0.0, ell, xi, 0, &v);
            for (int k = 0; k < dim; ++k) grad_x[(int64_t)k * n + i] = gsv[i] * v.gs[k];
        }
    }
}

/* grad_w_j = sum_i gs_i phi_ij for the listed hinges js[0..nj) only (and, in
 * abs_out, sum_i |gs_i| phi_ij): the same sum as orc_logit_bwd, evaluated for a
 * subset so that large point sets stay cheap. */
void orc_logit_bwd_w_subset(int dim, int M, const double *h, double ell, const double *x,
                            int64_t n, const double *gsv, const int *js, int nj, double *out,
                            double *abs_out) {
    double i2l2 = 0.5 / (ell * ell);
#pragma omp parallel for schedule(static)
    for (int q = 0; q < nj; ++q) {
        int j = js[q];
        double acc = 0.0, aabs = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double r2 = 0.0;
            for (int k = 0; k < dim; ++k) {
                double d = x[(int64_t)k * n + i] - h[(int64_t)k * M + j];
                r2 += d * d;
            }
            double phi = exp(-r2 * i2l2);
            acc += gsv[i] * phi;
            aabs += fabs(gsv[i]) * phi;
        }
        out[q] = acc;
        if (abs_out) abs_out[q] = aabs;
    }
}

/* Mean BCE on logits and its gradient g_i = (sigma(s_i) - y_i)/n. */
double orc_bce_logits(const double *s, const uint8_t *y, int64_t n, double *g) {
    double loss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        loss += bce_logit(s[i], (double)y[i]);
        if (g) g[i] = (sigmoid(s[i]) - (double)y[i]) / (double)n;
    }
    return loss / (double)n;
}

/* ------------------------------------------------------------------------- */
/* Arm: standard DH chain, body points, cost gradient in joint space.        */
/* ------------------------------------------------------------------------- */

/* dh = [a(ndof), d(ndof), alpha(ndof), theta0(ndof)].
 * A_i = Rz(theta0_i + q_i) * Tz(d_i) * Tx(a_i) * Rx(alpha_i); T_0 = I; T_i = T_{i-1} A_i.
 * o[i], z[i] (i = 0..ndof) are the origin and z axis of T_i. */
static void dh_chain(int ndof, const double *dh, const double *q, double o[][3], double z[][3]) {
    double T[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    for (int a = 0; a < 3; ++a) {
        o[0][a] = T[a][3];
        z[0][a] = T[a][2];
    }
    for (int i = 0; i < ndof; ++i) {
        double a = dh[i], d = dh[ndof + i], al = dh[2 * ndof + i];
        double th = dh[3 * ndof + i] + q[i];
        double ct = cos(th), st = sin(th), ca = cos(al), sa = sin(al);
        double A[4][4] = {{ct, -st * ca, st * sa, a * ct},
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
        memcpy(T, N, sizeof(T));
        for (int r = 0; r < 3; ++r) {
            o[i + 1][r] = T[r][3];
            z[i + 1][r] = T[r][2];
        }
    }
}

/* Body point k (0-based) of link i (1-based): o_{i-1} + ((k+1)/ppl)(o_i - o_{i-1}). */
static void body_point(double o[][3], int i, int k, int ppl, double p[3]) {
    double f = (double)(k + 1) / (double)ppl;
    for (int a = 0; a < 3; ++a) p[a] = o[i - 1][a] + f * (o[i][a] - o[i - 1][a]);
}

/* pts: [3][ndof*ppl][n], body point index p = (i-1)*ppl + k. */
void orc_fk_points(int ndof, int ppl, const double *dh, const double *q, int64_t n, double *pts) {
    int nb = ndof * ppl;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        double qs[ORC_MAX_DOF], o[ORC_MAX_DOF + 1][3], z[ORC_MAX_DOF + 1][3];
        for (int j = 0; j < ndof; ++j) qs[j] = q[(int64_t)j * n + s];
        dh_chain(ndof, dh, qs, o, z);
        for (int i = 1; i <= ndof; ++i)
            for (int k = 0; k < ppl; ++k) {
                double p[3];
                body_point(o, i, k, ppl, p);
                for (int a = 0; a < 3; ++a) pts[((int64_t)a * nb + (i - 1) * ppl + k) * n + s] = p[a];
            }
    }
}

/* Positional Jacobian of body point p on link i, [3][ndof] row-major:
 * column j (0-based joint, rotating about z_j through o_j) is z_j x (p - o_j) for
 * j < i, zero otherwise. */
void orc_fk_jacobian(int ndof, int ppl, const double *dh, const double *q /*[ndof]*/, int body,
                     double *J) {
    double o[ORC_MAX_DOF + 1][3], z[ORC_MAX_DOF + 1][3], p[3];
    dh_chain(ndof, dh, q, o, z);
    int i = body / ppl + 1, k = body % ppl;
    body_point(o, i, k, ppl, p);
    for (int j = 0; j < ndof; ++j) {
        double col[3] = {0, 0, 0};
        if (j < i) {
            double r[3] = {p[0] - o[j][0], p[1] - o[j][1], p[2] - o[j][2]};
            col[0] = z[j][1] * r[2] - z[j][2] * r[1];
            col[1] = z[j][2] * r[0] - z[j][0] * r[2];
            col[2] = z[j][0] * r[1] - z[j][1] * r[0];
        }
        for (int a = 0; a < 3; ++a) J[a * ndof + j] = col[a];
    }
}

static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Cost c(q) = sum_p c(psi_p(q)) and its joint gradient at one configuration.
 * form 0: sum_p J_p^T grad_x c(p) with J_p column by column (brute force);
 * form 1: per-link sums G_i = sum g_p, Mo_i = sum p x g_p, suffix-summed over
 *         links, dc/dq_j = z_j . (SM_j - o_j x SG_j). */
static double arm_cost_grad1(int ndof, int ppl, const double *dh, int M, const double *h,
                             const double *w, double beta, double ell, const double *qs,
                             int form, double *gq) {
    double o[ORC_MAX_DOF + 1][3], z[ORC_MAX_DOF + 1][3];
    dh_chain(ndof, dh, qs, o, z);
    double cost = 0.0;
    double G[ORC_MAX_DOF + 1][3], Mo[ORC_MAX_DOF + 1][3];
    memset(G, 0, sizeof(G));
    memset(Mo, 0, sizeof(Mo));
    for (int j = 0; j < ndof; ++j) gq[j] = 0.0;
    for (int i = 1; i <= ndof; ++i)
        for (int k = 0; k < ppl; ++k) {
            double p[3];
            body_point(o, i, k, ppl, p);
            occ_val ov;
            occ_point(3, M, h, w, beta, ell, p, 0, &ov, NULL);
            cost += ov.c;
            if (form == 0) {
                for (int j = 0; j < i; ++j) {
                    double r[3] = {p[0] - o[j][0], p[1] - o[j][1], p[2] - o[j][2]}, col[3];
                    cross3(z[j], r, col);
                    gq[j] += col[0] * ov.g[0] + col[1] * ov.g[1] + col[2] * ov.g[2];
                }
            } else {
                double pg[3];
                cross3(p, ov.g, pg);
                for (int a = 0; a < 3; ++a) {
                    G[i][a] += ov.g[a];
                    Mo[i][a] += pg[a];
                }
            }
        }
    if (form == 1) {
        double SG[3] = {0, 0, 0}, SM[3] = {0, 0, 0};
        for (int i = ndof; i >= 1; --i) {
            for (int a = 0; a < 3; ++a) {
                SG[a] += G[i][a];
                SM[a] += Mo[i][a];
            }
            /* joint i-1 (0-based) rotates links i..ndof about z_{i-1} through o_{i-1} */
            double oxg[3];
            cross3(o[i - 1], SG, oxg);
            double v[3] = {SM[0] - oxg[0], SM[1] - oxg[1], SM[2] - oxg[2]};
            gq[i - 1] = z[i - 1][0] * v[0] + z[i - 1][1] * v[1] + z[i - 1][2] * v[2];
        }
    }
    return cost;
}

void orc_arm_cost_grad(int ndof, int ppl, const double *dh, int M, const double *h,
                       const double *w, double beta, double ell, const double *q, int64_t n,
                       int form, double *cost, double *grad) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        double qs[ORC_MAX_DOF], gq[ORC_MAX_DOF];
        for (int j = 0; j < ndof; ++j) qs[j] = q[(int64_t)j * n + s];
        double c = arm_cost_grad1(ndof, ppl, dh, M, h, w, beta, ell, qs, form, gq);
        if (cost) cost[s] = c;
        if (grad)
            for (int j = 0; j < ndof; ++j) grad[(int64_t)j * n + s] = gq[j];
    }
}

/* Joint-space morph q_{k+1} = q_k - eta * grad_q c(q_k) (brute-force pull-back).
 * amp (nullable): product of |I - eta H_q|_2 with H_q the central-difference
 * Jacobian (step fd_h) of the analytic gradient, symmetrised.  min_det likewise;
 * max_eh (nullable): the largest eta |H_q|_2 along the path. */
void orc_morph_arm(int ndof, int ppl, const double *dh, int M, const double *h, const double *w,
                   double beta, double ell, const double *qin, int64_t n, int T, double eta,
                   double *qout, double *amp, double *min_det, double *max_eh, double fd_h) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n; ++s) {
        double qs[ORC_MAX_DOF], gq[ORC_MAX_DOF];
        double A = 1.0, mdet = INFINITY, meh = 0.0;
        for (int j = 0; j < ndof; ++j) qs[j] = qin[(int64_t)j * n + s];
        for (int t = 0; t < T; ++t) {
            if (amp || min_det || max_eh) {
                double H[ORC_MAX_DOF * ORC_MAX_DOF];
                for (int b = 0; b < ndof; ++b) {
                    double qp[ORC_MAX_DOF], qm[ORC_MAX_DOF], gp[ORC_MAX_DOF], gm[ORC_MAX_DOF];
                    memcpy(qp, qs, sizeof(qp));
                    memcpy(qm, qs, sizeof(qm));
                    qp[b] += fd_h;
                    qm[b] -= fd_h;
                    arm_cost_grad1(ndof, ppl, dh, M, h, w, beta, ell, qp, 0, gp);
                    arm_cost_grad1(ndof, ppl, dh, M, h, w, beta, ell, qm, 0, gm);
                    for (int a = 0; a < ndof; ++a) H[a * ndof + b] = (gp[a] - gm[a]) / (2.0 * fd_h);
                }
                double nm, det, hn;
                step_jac_stats(ndof, H, eta, &nm, &det, &hn);
                A *= nm;
                if (det < mdet) mdet = det;
                if (eta * hn > meh) meh = eta * hn;
            }
            arm_cost_grad1(ndof, ppl, dh, M, h, w, beta, ell, qs, 0, gq);
            for (int j = 0; j < ndof; ++j) qs[j] = qs[j] - eta * gq[j];
        }
        for (int j = 0; j < ndof; ++j) qout[(int64_t)j * n + s] = qs[j];
        if (amp) amp[s] = A;
        if (min_det) min_det[s] = mdet;
        if (max_eh) max_eh[s] = meh;
    }
}

/* Error scale of one joint-space step's gradient: sum over body points p of
 * max_j |J_p[:, j]|_1 G_abs(p), J_p the positional Jacobian (columns z_j x (p - o_j)
 * for the joints before p's link) and G_abs(p) the workspace gradient's scale -- the
 * bound that FP32-class errors of each body point's grad c carry into grad_q. */
void orc_arm_step_scale(int ndof, int ppl, const double *dh, int M, const double *h,
                        const double *w, double beta, double ell, const double *q, int64_t n,
                        double *scale) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n; ++s) {
        double qs[ORC_MAX_DOF], o[ORC_MAX_DOF + 1][3], z[ORC_MAX_DOF + 1][3];
        for (int j = 0; j < ndof; ++j) qs[j] = q[(int64_t)j * n + s];
        dh_chain(ndof, dh, qs, o, z);
        double acc = 0.0;
        for (int i = 1; i <= ndof; ++i)
            for (int k = 0; k < ppl; ++k) {
                double p[3];
                body_point(o, i, k, ppl, p);
                double lever = 0.0;
                for (int j = 0; j < i; ++j) {
                    double r[3] = {p[0] - o[j][0], p[1] - o[j][1], p[2] - o[j][2]}, col[3];
                    cross3(z[j], r, col);
                    double l1 = fabs(col[0]) + fabs(col[1]) + fabs(col[2]);
                    if (l1 > lever) lever = l1;
                }
                occ_val ov;
                occ_point(3, M, h, w, beta, ell, p, 0, &ov, NULL);
                acc += lever * ov.gabs;
            }
        scale[s] = acc;
    }
}

/* A configuration collides iff any of its body points lies in any box. */
void orc_label_configs(int ndof, int ppl, const double *dh, const double *c, const double *e,
                       int K, const double *q, int64_t n, uint8_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        double qs[ORC_MAX_DOF], o[ORC_MAX_DOF + 1][3], z[ORC_MAX_DOF + 1][3];
        for (int j = 0; j < ndof; ++j) qs[j] = q[(int64_t)j * n + s];
        dh_chain(ndof, dh, qs, o, z);
        int hit = 0;
        for (int i = 1; i <= ndof && !hit; ++i)
            for (int k = 0; k < ppl && !hit; ++k) {
                double p[3];
                body_point(o, i, k, ppl, p);
                hit = in_any_box(p, c, e, K);
            }
        out[s] = (uint8_t)hit;
    }
}

/* Label margin of each configuration: min over body points p and boxes b of
 * |max_a (|p_a - c_a| - e_a)|.  The inside test of p in b flips only when that
 * maximum changes sign, and moving p by delta changes it by at most delta, so a
 * configuration whose margin exceeds delta keeps its label under any perturbation
 * of its body points smaller than delta. */
void orc_config_label_margin(int ndof, int ppl, const double *dh, const double *c,
                             const double *e, int K, const double *q, int64_t n, double *margin) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        double qs[ORC_MAX_DOF], o[ORC_MAX_DOF + 1][3], z[ORC_MAX_DOF + 1][3];
        for (int j = 0; j < ndof; ++j) qs[j] = q[(int64_t)j * n + s];
        dh_chain(ndof, dh, qs, o, z);
        double mg = INFINITY;
        for (int i = 1; i <= ndof; ++i)
            for (int k = 0; k < ppl; ++k) {
                double p[3];
                body_point(o, i, k, ppl, p);
                for (int b = 0; b < K; ++b) {
                    /* signed distance proxy: max_a (|p_a - c_a| - e_a) is <= 0 inside */
                    double dmax = -INFINITY;
                    for (int a = 0; a < 3; ++a) {
                        double d = fabs(p[a] - c[a * K + b]) - e[a * K + b];
                        if (d > dmax) dmax = d;
                    }
                    if (fabs(dmax) < mg) mg = fabs(dmax);
                }
            }
        margin[s] = mg;
    }
}

/* ------------------------------------------------------------------------- */
/* Residual MLP q_hat = q + f(q), f = W_L SiLU(... SiLU(W_1 q + b_1) ...) + b_L  */
/* ------------------------------------------------------------------------- */

/* Parameters are one flat array: for each layer l = 1..L, W_l [out][in] row-major
 * followed by b_l [out].  widths has L+1 entries. */
static int64_t mlp_nparams(int L, const int *widths) {
    int64_t np = 0;
    for (int l = 0; l < L; ++l) np += (int64_t)widths[l + 1] * widths[l] + widths[l + 1];
    return np;
}

int64_t orc_mlp_nparams(int L, const int *widths) { return mlp_nparams(L, widths); }

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double silu_d(double z) {
    double sg = 1.0 / (1.0 + exp(-z));
    return sg * (1.0 + z * (1.0 - sg));
}

#define ORC_MLP_MAXW 1024
#define ORC_MLP_MAXL 8

/* Forward for one sample; stores pre-activations z[l] and activations a[l]
 * (a[0] = input) when the buffers are given. */
static void mlp_fwd1(int L, const int *widths, const double *P, const double *in, double *out,
                     double *zbuf, double *abuf) {
    double a[ORC_MLP_MAXW], nx[ORC_MLP_MAXW];
    int w0 = widths[0];
    for (int k = 0; k < w0; ++k) a[k] = in[k];
    if (abuf) memcpy(abuf, a, sizeof(double) * (size_t)w0);
    const double *p = P;
    int64_t zoff = 0, aoff = w0;
    for (int l = 0; l < L; ++l) {
        int fi = widths[l], fo = widths[l + 1];
        const double *W = p, *b = p + (int64_t)fo * fi;
        for (int o = 0; o < fo; ++o) {
            double acc = 0.0;
            for (int k = 0; k < fi; ++k) acc += W[(int64_t)o * fi + k] * a[k];
            acc += b[o];
            nx[o] = acc;
        }
        if (zbuf) memcpy(zbuf + zoff, nx, sizeof(double) * (size_t)fo);
        zoff += fo;
        if (l < L - 1)
            for (int o = 0; o < fo; ++o) nx[o] = silu(nx[o]);
        memcpy(a, nx, sizeof(double) * (size_t)fo);
        if (abuf && l < L - 1) memcpy(abuf + aoff, a, sizeof(double) * (size_t)fo);
        if (l < L - 1) aoff += fo;
        p += (int64_t)fo * fi + fo;
    }
    for (int k = 0; k < widths[L]; ++k) out[k] = a[k];
}

/* q_hat = q + f(q) for [w0][B] inputs (SoA), residual requires widths[0]==widths[L].
 * fscale (nullable, [wL][B]): sum_k |W_L[o][k]| |a_{L-1,k}| + |b_L[o]|, the magnitude
 * scale the rounding of the last layer's inputs and weights acts on. */
void orc_mlp_forward(int L, const int *widths, const double *P, const double *q, int64_t B,
                     int residual, double *out, double *fscale) {
    int w0 = widths[0], wl = widths[L];
    int64_t zlen = 0, alen = w0, plast = 0;
    for (int l = 0; l < L; ++l) {
        zlen += widths[l + 1];
        if (l < L - 1) alen += widths[l + 1];
        if (l < L - 1) plast += (int64_t)widths[l + 1] * widths[l] + widths[l + 1];
    }
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < B; ++s) {
        double in[ORC_MLP_MAXW], f[ORC_MLP_MAXW];
        double *z = (double *)malloc(sizeof(double) * (size_t)zlen);
        double *a = (double *)malloc(sizeof(double) * (size_t)alen);
        for (int k = 0; k < w0; ++k) in[k] = q[(int64_t)k * B + s];
        mlp_fwd1(L, widths, P, in, f, z, a);
        for (int k = 0; k < wl; ++k) out[(int64_t)k * B + s] = (residual ? in[k] : 0.0) + f[k];
        if (fscale) {
            int fi = widths[L - 1];
            const double *W = P + plast, *b = P + plast + (int64_t)wl * fi;
            const double *alast = a + (alen - fi);
            for (int o = 0; o < wl; ++o) {
                double acc = fabs(b[o]);
                for (int k = 0; k < fi; ++k) acc += fabs(W[(int64_t)o * fi + k]) * fabs(alast[k]);
                fscale[(int64_t)o * B + s] = acc;
            }
        }
        free(z);
        free(a);
    }
}

/* MSE loss (1/(wL*B)) sum_s u_s |q_hat_s - target_s|^2 of the residual network and
 * its gradient with respect to every parameter (same flat layout as P), with sample
 * weight u_s = hard_w where hard[s] != 0 and 1 elsewhere (hard NULL: all 1, the
 * plain MSE). */
static double mlp_loss_grad(int L, const int *widths, const double *P, const double *q,
                            const double *target, int64_t B, const uint8_t *hard, double hard_w,
                            double *grad) {
    int w0 = widths[0], wl = widths[L];
    int64_t np = mlp_nparams(L, widths);
    int64_t zlen = 0, alen = w0;
    for (int l = 0; l < L; ++l) {
        zlen += widths[l + 1];
        if (l < L - 1) alen += widths[l + 1];
    }
    memset(grad, 0, sizeof(double) * (size_t)np);
    double loss = 0.0;
    double scale = 1.0 / ((double)wl * (double)B);
    double *z = (double *)malloc(sizeof(double) * (size_t)zlen);
    double *a = (double *)malloc(sizeof(double) * (size_t)alen);
    for (int64_t s = 0; s < B; ++s) {
        double in[ORC_MLP_MAXW], f[ORC_MLP_MAXW], d[ORC_MLP_MAXW], dn[ORC_MLP_MAXW];
        for (int k = 0; k < w0; ++k) in[k] = q[(int64_t)k * B + s];
        mlp_fwd1(L, widths, P, in, f, z, a);
        const double u = (hard && hard[s]) ? hard_w : 1.0;
        for (int k = 0; k < wl; ++k) {
            double e = in[k] + f[k] - target[(int64_t)k * B + s];
            loss += u * (e * e);
            d[k] = 2.0 * scale * u * e; /* dL/df = dL/dq_hat */
        }
        /* walk layers backwards; d holds dL/dz_l of the current layer */
        int64_t poff = np, zoff = zlen, aoff = alen;
        for (int l = L - 1; l >= 0; --l) {
            int fi = widths[l], fo = widths[l + 1];
            poff -= (int64_t)fo * fi + fo;
            zoff -= fo;
            aoff -= fi;
            const double *W = P + poff;
            double *gW = grad + poff, *gb = grad + poff + (int64_t)fo * fi;
            const double *ain = a + aoff; /* input activation of layer l */
            for (int o = 0; o < fo; ++o) {
                for (int k = 0; k < fi; ++k) gW[(int64_t)o * fi + k] += d[o] * ain[k];
                gb[o] += d[o];
            }
            if (l > 0) {
                const double *zin = z + zoff - fi; /* pre-activation feeding ain */
                for (int k = 0; k < fi; ++k) {
                    double acc = 0.0;
                    for (int o = 0; o < fo; ++o) acc += W[(int64_t)o * fi + k] * d[o];
                    dn[k] = acc * silu_d(zin[k]);
                }
                memcpy(d, dn, sizeof(double) * (size_t)fi);
            }
        }
    }
    free(z);
    free(a);
    return loss * scale;
}

double orc_mlp_loss_grad(int L, const int *widths, const double *P, const double *q,
                         const double *target, int64_t B, double *grad) {
    return mlp_loss_grad(L, widths, P, q, target, B, NULL, 1.0, grad);
}

double orc_mlp_loss_grad_weighted(int L, const int *widths, const double *P, const double *q,
                                  const double *target, int64_t B, const uint8_t *hard,
                                  double hard_w, double *grad) {
    return mlp_loss_grad(L, widths, P, q, target, B, hard, hard_w, grad);
}

/* ------------------------------------------------------------------------- */
/* Amortised morph: q_hat = q + f(q); a configuration whose largest body-point */
/* occupancy at q_hat exceeds `thresh` takes the plain morph from q instead.  */
/* ------------------------------------------------------------------------- */

/* With from_qhat the fallback starts from q_hat instead of q (the refining variant:
 * flagged configurations take T plain steps from the network's output). */
static void amortised_morph(int L, const int *widths, const double *P, int ndof, int ppl,
                            const double *dh, int M, const double *h, const double *w,
                            double beta, double ell, const double *q, int64_t n, int T,
                            double eta, double thresh, int from_qhat, double *qout,
                            uint8_t *flag, double *maxc) {
    double *qh = (double *)malloc(sizeof(double) * (size_t)ndof * (size_t)(n > 0 ? n : 1));
    orc_mlp_forward(L, widths, P, q, n, 1, qh, NULL);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n; ++s) {
        double qs[ORC_MAX_DOF], o[ORC_MAX_DOF + 1][3], z[ORC_MAX_DOF + 1][3];
        for (int j = 0; j < ndof; ++j) qs[j] = qh[(int64_t)j * n + s];
        dh_chain(ndof, dh, qs, o, z);
        double mc = -INFINITY;
        for (int i = 1; i <= ndof; ++i)
            for (int k = 0; k < ppl; ++k) {
                double p[3];
                body_point(o, i, k, ppl, p);
                occ_val ov;
                occ_point(3, M, h, w, beta, ell, p, 0, &ov, NULL);
                if (ov.c > mc) mc = ov.c;
            }
        int fb = mc > thresh;
        if (maxc) maxc[s] = mc;
        if (flag) flag[s] = (uint8_t)fb;
        if (fb) {
            double gq[ORC_MAX_DOF];
            if (!from_qhat)
                for (int j = 0; j < ndof; ++j) qs[j] = q[(int64_t)j * n + s];
            for (int t = 0; t < T; ++t) {
                arm_cost_grad1(ndof, ppl, dh, M, h, w, beta, ell, qs, 0, gq);
                for (int j = 0; j < ndof; ++j) qs[j] = qs[j] - eta * gq[j];
            }
        }
        for (int j = 0; j < ndof; ++j) qout[(int64_t)j * n + s] = qs[j];
    }
    free(qh);
}

void orc_amortised_morph(int L, const int *widths, const double *P, int ndof, int ppl,
                         const double *dh, int M, const double *h, const double *w, double beta,
                         double ell, const double *q, int64_t n, int T, double eta,
                         double thresh, double *qout, uint8_t *flag, double *maxc) {
    amortised_morph(L, widths, P, ndof, ppl, dh, M, h, w, beta, ell, q, n, T, eta, thresh, 0, qout,
                    flag, maxc);
}

void orc_amortised_morph_refine(int L, const int *widths, const double *P, int ndof, int ppl,
                                const double *dh, int M, const double *h, const double *w,
                                double beta, double ell, const double *q, int64_t n, int T,
                                double eta, double thresh, double *qout, uint8_t *flag,
                                double *maxc) {
    amortised_morph(L, widths, P, ndof, ppl, dh, M, h, w, beta, ell, q, n, T, eta, thresh, 1, qout,
                    flag, maxc);
}

/* ------------------------------------------------------------------------- */
/* The paper's occupancy network (Sec. 3.1): a fully connected network with    */
/* tanh activations between hidden layers and a sigmoid at the output,         */
/* c(x) = sigma(s(x)), trained with binary cross-entropy.                      */
/*                                                                             */
/* L hidden layers of width H.  Flat parameters: for l = 0..L-1 the matrix     */
/* W_l [H][n_l] (row-major; n_0 = dim, n_l = H after) and the bias b_l [H];    */
/* then the output weights v [H] and the output bias b_o:                      */
/*   a_0 = x,  a_{l+1} = tanh(W_l a_l + b_l),  s = v . a_L + b_o.              */
/* Reverse mode (chain rule) for the input gradient:                           */
/*   d_l = 1 - a_l^2 (l >= 1),  e_L = v * d_L,                                 */
/*   e_l = d_l * (W_l^T e_{l+1})  (l = L-1..1),  grad_x s = W_0^T e_1.         */
/* ------------------------------------------------------------------------- */

#define ORC_TANH_MAXH 256
#define ORC_TANH_MAXL 6

int64_t orc_tanh_nparams(int dim, int H, int L) {
    return (int64_t)H * dim + H + (int64_t)(L - 1) * (H * H + H) + H + 1;
}

typedef struct {
    double a[ORC_TANH_MAXL + 1][ORC_TANH_MAXH];  /* a[l] for l >= 1 (a[0] unused) */
    double zs[ORC_TANH_MAXL + 1][ORC_TANH_MAXH]; /* error scale of each pre-activation */
    double s, sabs;
} tanh_fwd;

/* Forward pass.  Error scales: a pre-activation z = b + sum W a' gets
 * |b| + sum |W| A', where A' = |a'| + (1 - a'^2) Z' is the scale of an input a'
 * = tanh(z') including the rounding carried from z' (scale Z'); for the inputs
 * A' = |x|.  sabs is the same sum for s. */
static void tanh_forward(int dim, int H, int L, const double *P, const double *x, tanh_fwd *f) {
    const double *p = P;
    double in[ORC_TANH_MAXH], inabs[ORC_TANH_MAXH];
    int nin = dim;
    for (int k = 0; k < dim; ++k) {
        in[k] = x[k];
        inabs[k] = fabs(x[k]);
    }
    for (int l = 0; l < L; ++l) {
        const double *W = p, *b = p + (int64_t)H * nin;
        p = b + H;
        for (int u = 0; u < H; ++u) {
            double z = b[u], za = fabs(b[u]);
            for (int k = 0; k < nin; ++k) {
                z += W[(int64_t)u * nin + k] * in[k];
                za += fabs(W[(int64_t)u * nin + k]) * inabs[k];
            }
            f->a[l + 1][u] = tanh(z);
            f->zs[l + 1][u] = za;
        }
        for (int u = 0; u < H; ++u) {
            double a = f->a[l + 1][u];
            in[u] = a;
            inabs[u] = fabs(a) + (1.0 - a * a) * f->zs[l + 1][u];
        }
        nin = H;
    }
    const double *v = p, bo = p[H];
    double s = bo, sa = fabs(bo);
    for (int u = 0; u < H; ++u) {
        s += v[u] * in[u];
        sa += fabs(v[u]) * inabs[u];
    }
    f->s = s;
    f->sabs = sa;
}

/* Input gradient of s by the chain rule (reverse order).  gabs (nullable) gets
 * the error scale of the largest component: the same recursion on absolute
 * values, each layer's derivative d widened by (1 + 2|a| Z) for the rounding of
 * the forward value it is computed from. */
static void tanh_backward_x(int dim, int H, int L, const double *P, const tanh_fwd *f,
                            double *g, double *gabs) {
    int64_t off[ORC_TANH_MAXL + 1];
    int64_t o = 0;
    for (int l = 0; l < L; ++l) {
        off[l] = o;
        int nin = l == 0 ? dim : H;
        o += (int64_t)H * nin + H;
    }
    const double *v = P + o;
    double e[ORC_TANH_MAXH], ea[ORC_TANH_MAXH], t[ORC_TANH_MAXH], ta[ORC_TANH_MAXH];
    for (int u = 0; u < H; ++u) {
        double a = f->a[L][u], d = 1.0 - a * a;
        e[u] = v[u] * d;
        ea[u] = fabs(v[u]) * d * (1.0 + 2.0 * fabs(a) * f->zs[L][u]);
    }
    for (int l = L - 1; l >= 1; --l) {
        const double *W = P + off[l]; /* W_l: [H][H], maps a_l -> z_{l+1} */
        for (int i = 0; i < H; ++i) {
            double acc = 0.0, acca = 0.0;
            for (int u = 0; u < H; ++u) {
                acc += W[(int64_t)u * H + i] * e[u];
                acca += fabs(W[(int64_t)u * H + i]) * ea[u];
            }
            double a = f->a[l][i], d = 1.0 - a * a;
            t[i] = d * acc;
            ta[i] = d * (1.0 + 2.0 * fabs(a) * f->zs[l][i]) * acca;
        }
        for (int i = 0; i < H; ++i) {
            e[i] = t[i];
            ea[i] = ta[i];
        }
    }
    const double *W0 = P; /* [H][dim] */
    double gm = 0.0;
    for (int k = 0; k < dim; ++k) {
        double acc = 0.0, acca = 0.0;
        for (int u = 0; u < H; ++u) {
            acc += W0[(int64_t)u * dim + k] * e[u];
            acca += fabs(W0[(int64_t)u * dim + k]) * ea[u];
        }
        g[k] = acc;
        if (acca > gm) gm = acca;
    }
    if (gabs) *gabs = gm;
}

/* s, c = sigma(s) and the error scale of s at each point; x is [dim][n]. */
void orc_tanh_eval(int dim, int H, int L, const double *P, const double *x, int64_t n, double *s,
                   double *c, double *sabs) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xi[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) xi[k] = x[(int64_t)k * n + i];
        tanh_fwd f;
        tanh_forward(dim, H, L, P, xi, &f);
        if (s) s[i] = f.s;
        if (c) c[i] = sigmoid(f.s);
        if (sabs) sabs[i] = f.sabs;
    }
}

/* grad_x s ([dim][n]) and grad_x c = sigma'(s) grad_x s, with the error scales of
 * s and of grad_x s. */
void orc_tanh_grad(int dim, int H, int L, const double *P, const double *x, int64_t n, double *s,
                   double *gs, double *gc, double *sabs, double *gabs) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xi[ORC_MAX_DIM], g[ORC_MAX_DIM], ga;
        for (int k = 0; k < dim; ++k) xi[k] = x[(int64_t)k * n + i];
        tanh_fwd f;
        tanh_forward(dim, H, L, P, xi, &f);
        tanh_backward_x(dim, H, L, P, &f, g, &ga);
        double sp = sigmoid_slope(f.s);
        for (int k = 0; k < dim; ++k) {
            if (gs) gs[(int64_t)k * n + i] = g[k];
            if (gc) gc[(int64_t)k * n + i] = sp * g[k];
        }
        if (s) s[i] = f.s;
        if (sabs) sabs[i] = f.sabs;
        if (gabs) gabs[i] = ga;
    }
}

static void tanh_grad_c(int dim, int H, int L, const double *P, const double *x, double *gc) {
    tanh_fwd f;
    double g[ORC_MAX_DIM];
    tanh_forward(dim, H, L, P, x, &f);
    tanh_backward_x(dim, H, L, P, &f, g, NULL);
    double sp = sigmoid_slope(f.s);
    for (int k = 0; k < dim; ++k) gc[k] = sp * g[k];
}

/* Plain morph with the network's occupancy (Eq. 1 with explicit Euler steps):
 * x_{k+1} = x_k - eta grad c(x_k), T steps.  amp (nullable) gets the product over
 * steps of |I - eta Hc|_2, with Hc from central differences of grad c (FP64,
 * step 1e-5 max(1, |x|)); it only sizes the FP32 tolerance. */
void orc_tanh_morph(int dim, int H, int L, const double *P, const double *xin, int64_t n, int T,
                    double eta, double *xout, double *amp) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x[ORC_MAX_DIM], g[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) x[k] = xin[(int64_t)k * n + i];
        double A = 1.0;
        for (int t = 0; t < T; ++t) {
            if (amp) {
                double Hm[ORC_MAX_DIM * ORC_MAX_DIM];
                for (int j = 0; j < dim; ++j) {
                    double xp[ORC_MAX_DIM], xm[ORC_MAX_DIM], gp[ORC_MAX_DIM], gm[ORC_MAX_DIM];
                    double hstep = 1e-5 * (fabs(x[j]) > 1.0 ? fabs(x[j]) : 1.0);
                    for (int k = 0; k < dim; ++k) xp[k] = xm[k] = x[k];
                    xp[j] += hstep;
                    xm[j] -= hstep;
                    tanh_grad_c(dim, H, L, P, xp, gp);
                    tanh_grad_c(dim, H, L, P, xm, gm);
                    for (int k = 0; k < dim; ++k) Hm[k * dim + j] = (gp[k] - gm[k]) / (2.0 * hstep);
                }
                double nm, det, hn;
                step_jac_stats(dim, Hm, eta, &nm, &det, &hn);
                A *= nm;
            }
            tanh_grad_c(dim, H, L, P, x, g);
            for (int k = 0; k < dim; ++k) x[k] = x[k] - eta * g[k];
        }
        for (int k = 0; k < dim; ++k) xout[(int64_t)k * n + i] = x[k];
        if (amp) amp[i] = A;
    }
}

/* Fit objective of the network (Sec. 3.1): mean BCE of sigma(s(x_i)) against
 * y_i plus (l2/2) times the squared weights (the matrices W_l and v, not the
 * biases).  Returns the loss; grad ([nparams]) gets its gradient by the chain
 * rule through every layer (reverse order).  gscale (nullable, [nparams]) gets
 * the error scale of each gradient entry: the same sums over absolute values, with
 * r = sigma(s) - y widened by sigma'(s) S_abs and every layer's forward value and
 * slope widened as in the input-gradient scale, plus l2 |w|. */
double orc_tanh_loss_grad(int dim, int H, int L, const double *P, const double *pts,
                          const uint8_t *y, int64_t n, double l2, double *grad, double *gscale) {
    const int64_t np = orc_tanh_nparams(dim, H, L);
    int64_t off[ORC_TANH_MAXL + 1];
    int64_t o = 0;
    for (int l = 0; l < L; ++l) {
        off[l] = o;
        o += (int64_t)H * (l == 0 ? dim : H) + H;
    }
    off[L] = o; /* v, then b_o */
    int nt = orc_num_threads();
    int want_s = gscale != NULL;
    double *acc = (double *)calloc((size_t)nt * (size_t)np, sizeof(double));
    double *acca = want_s ? (double *)calloc((size_t)nt * (size_t)np, sizeof(double)) : NULL;
    double *lsum = (double *)calloc((size_t)nt, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *G = acc + (int64_t)tid * np;
        double *GA = want_s ? acca + (int64_t)tid * np : NULL;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double xi[ORC_MAX_DIM];
            for (int k = 0; k < dim; ++k) xi[k] = pts[(int64_t)k * n + i];
            tanh_fwd f;
            tanh_forward(dim, H, L, P, xi, &f);
            double yi = (double)y[i];
            lsum[tid] += bce_logit(f.s, yi);
            /* dBCE/ds = sigma(s) - y, formed as sigma(s) (y = 0) or -sigma(-s) (y = 1) so
             * that it keeps its relative accuracy where sigma(s) is within rounding of y */
            double r = y[i] ? -sigmoid(-f.s) : sigmoid(f.s);
            double ra = fabs(r) + sigmoid_slope(f.s) * f.sabs;
            const double *v = P + off[L];
            double aa[ORC_TANH_MAXH]; /* forward scale of the layer input */
            for (int u = 0; u < H; ++u) {
                double a = f.a[L][u];
                G[off[L] + u] += r * a;
                if (GA) GA[off[L] + u] += ra * (fabs(a) + (1.0 - a * a) * f.zs[L][u]);
            }
            G[off[L] + H] += r;
            if (GA) GA[off[L] + H] += ra;
            double e[ORC_TANH_MAXH], t[ORC_TANH_MAXH], ea[ORC_TANH_MAXH], ta[ORC_TANH_MAXH];
            for (int u = 0; u < H; ++u) {
                double a = f.a[L][u], d = 1.0 - a * a;
                e[u] = r * v[u] * d;
                ea[u] = ra * fabs(v[u]) * d * (1.0 + 2.0 * fabs(a) * f.zs[L][u]);
            }
            for (int l = L - 1; l >= 0; --l) {
                int nin = l == 0 ? dim : H;
                const double *ain = l == 0 ? xi : f.a[l];
                for (int k = 0; k < nin; ++k)
                    aa[k] = l == 0 ? fabs(xi[k])
                                   : fabs(ain[k]) + (1.0 - ain[k] * ain[k]) * f.zs[l][k];
                double *GW = G + off[l], *Gb = G + off[l] + (int64_t)H * nin;
                for (int u = 0; u < H; ++u) {
                    for (int k = 0; k < nin; ++k) GW[(int64_t)u * nin + k] += e[u] * ain[k];
                    Gb[u] += e[u];
                }
                if (GA) {
                    double *GAW = GA + off[l], *GAb = GA + off[l] + (int64_t)H * nin;
                    for (int u = 0; u < H; ++u) {
                        for (int k = 0; k < nin; ++k) GAW[(int64_t)u * nin + k] += ea[u] * aa[k];
                        GAb[u] += ea[u];
                    }
                }
                if (l == 0) break;
                const double *W = P + off[l];
                for (int k = 0; k < H; ++k) {
                    double s2 = 0.0, s2a = 0.0;
                    for (int u = 0; u < H; ++u) {
                        s2 += W[(int64_t)u * H + k] * e[u];
                        s2a += fabs(W[(int64_t)u * H + k]) * ea[u];
                    }
                    double a = f.a[l][k], d = 1.0 - a * a;
                    t[k] = s2 * d;
                    ta[k] = s2a * d * (1.0 + 2.0 * fabs(a) * f.zs[l][k]);
                }
                for (int k = 0; k < H; ++k) {
                    e[k] = t[k];
                    ea[k] = ta[k];
                }
            }
        }
    }
    double loss = 0.0;
    for (int t = 0; t < nt; ++t) loss += lsum[t];
    loss /= (double)n;
    for (int64_t j = 0; j < np; ++j) {
        double s2 = 0.0, s2a = 0.0;
        for (int t = 0; t < nt; ++t) {
            s2 += acc[(int64_t)t * np + j];
            if (want_s) s2a += acca[(int64_t)t * np + j];
        }
        grad[j] = s2 / (double)n;
        if (want_s) gscale[j] = s2a / (double)n;
    }
    /* weight decay on the matrices and v */
    double wsq = 0.0;
    for (int l = 0; l <= L; ++l) {
        int64_t cnt = l < L ? (int64_t)H * (l == 0 ? dim : H) : H;
        for (int64_t j = 0; j < cnt; ++j) {
            double w = P[off[l] + j];
            grad[off[l] + j] += l2 * w;
            if (want_s) gscale[off[l] + j] += l2 * fabs(w);
            wsq += w * w;
        }
    }
    free(acc);
    free(acca);
    free(lsum);
    return loss + 0.5 * l2 * wsq;
}

/* ------------------------------------------------------------------------- */
/* The inverse of the morph and the log-determinant of its Jacobian (Sec. 3.2: */
/* the flow phi has the inverse obtained by integrating the reversed field;    */
/* for the explicit-Euler map the exact inverse of one step                    */
/* x_{k+1} = x_k - eta grad c(x_k) is the fixed point x_k = x_{k+1} + eta      */
/* grad c(x_k), a contraction when eta Lip(grad c) < 1), and the epsilon       */
/* mixture with the prior (Sec. 3.3).                                          */
/* ------------------------------------------------------------------------- */

/* det of a dim x dim matrix (dim <= 3), row-major. */
static double det_small(int dim, const double *A) {
    if (dim == 1) return A[0];
    if (dim == 2) return A[0] * A[3] - A[1] * A[2];
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* log|det(I - eta Hc(x))| at one point and the error scale of that term for an FP32
 * evaluation: the Hessian entries carry the scale
 *   Habs = sigma' Hs_abs + |sigma''| (S_abs |Hs|_max + 2 |grad s| G_raw + |grad s|^2)
 *          + |sigma'''| S_abs |grad s|^2,
 * Hs_abs = l^-2 sum |w| phi (|x - h|^2 / l^2 + 1), and a perturbation dH of the entries
 * moves det by at most eta |dH| dim (1 + eta |H|_max dim)^(dim-1). */
static double step_logdet(int dim, int M, const double *h, const double *w, double beta,
                          double ell, const double *x, double eta, double *scale) {
    occ_val o;
    rbf_val v;
    occ_point(dim, M, h, w, beta, ell, x, 1, &o, &v);
    double A[ORC_MAX_DIM * ORC_MAX_DIM] = {0};
    double hmax = 0.0, hsmax = 0.0;
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) {
            A[a * dim + b] = (a == b ? 1.0 : 0.0) - eta * o.H[a * dim + b];
            if (fabs(o.H[a * dim + b]) > hmax) hmax = fabs(o.H[a * dim + b]);
            if (fabs(v.Hs[a * dim + b]) > hsmax) hsmax = fabs(v.Hs[a * dim + b]);
        }
    double det = det_small(dim, A);
    if (scale) {
        double il2 = 1.0 / (ell * ell), habs = 0.0;
        for (int j = 0; j < M; ++j) {
            double r2 = 0.0;
            for (int k = 0; k < dim; ++k) {
                double d = x[k] - h[(int64_t)k * M + j];
                r2 += d * d;
            }
            habs += fabs(w[j]) * exp(-0.5 * r2 * il2) * il2 * (r2 * il2 + 1.0);
        }
        double c = o.c, d1 = o.dc, d2 = d1 * (1.0 - 2.0 * c), d3 = d1 * (1.0 - 6.0 * d1);
        double gn = 0.0;
        for (int k = 0; k < dim; ++k) gn += v.gs[k] * v.gs[k];
        double Habs = d1 * habs + fabs(d2) * (v.sabs * hsmax + 2.0 * sqrt(gn) * v.graw + gn) +
                      fabs(d3) * v.sabs * gn;
        double grow = pow(1.0 + eta * hmax * dim, dim - 1);
        *scale = eta * Habs * dim * grow / fabs(det);
    }
    return log(fabs(det));
}

/* Forward morph with the log-determinant of its Jacobian,
 *   logdet = sum_k log|det(I - eta Hc(x_k))|  (so p_z(z) = p_y(y) exp(-logdet)),
 * and ldscale = the sum of the per-step error scales (both nullable). */
void orc_morph_logdet(int dim, int M, const double *h, const double *w, double beta, double ell,
                      const double *xin, int64_t n, int T, double eta, double *xout,
                      double *logdet, double *ldscale) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) x[k] = xin[(int64_t)k * n + i];
        double ld = 0.0, sc = 0.0;
        for (int t = 0; t < T; ++t) {
            double s1;
            ld += step_logdet(dim, M, h, w, beta, ell, x, eta, &s1);
            sc += s1;
            occ_val o;
            occ_point(dim, M, h, w, beta, ell, x, 0, &o, NULL);
            for (int k = 0; k < dim; ++k) x[k] = x[k] - eta * o.g[k];
        }
        for (int k = 0; k < dim; ++k) xout[(int64_t)k * n + i] = x[k];
        if (logdet) logdet[i] = ld;
        if (ldscale) ldscale[i] = sc;
    }
}

/* Inverse of the T-step morph by fixed point, step by step in reverse: from
 * z = x_T, for each step x^(0) = x_{k+1}, x^(j+1) = x_{k+1} + eta grad c(x^(j)) for
 * j < iters, and x_k = x^(iters).  resid (nullable) gets the largest fixed-point
 * residual |x_k - x_{k+1} - eta grad c(x_k)|_inf over the steps; logdet and ldscale
 * (nullable) the forward log-determinant along the reconstructed path, evaluated at
 * each x_k. */
void orc_morph_inverse(int dim, int M, const double *h, const double *w, double beta, double ell,
                       const double *zin, int64_t n, int T, double eta, int iters, double *yout,
                       double *logdet, double *ldscale, double *resid) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x[ORC_MAX_DIM], zt[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) x[k] = zin[(int64_t)k * n + i];
        double ld = 0.0, sc = 0.0, rmax = 0.0;
        for (int t = 0; t < T; ++t) {
            for (int k = 0; k < dim; ++k) zt[k] = x[k];
            for (int j = 0; j < iters; ++j) {
                occ_val o;
                occ_point(dim, M, h, w, beta, ell, x, 0, &o, NULL);
                for (int k = 0; k < dim; ++k) x[k] = zt[k] + eta * o.g[k];
            }
            occ_val o;
            occ_point(dim, M, h, w, beta, ell, x, 0, &o, NULL);
            for (int k = 0; k < dim; ++k) {
                double r = fabs(x[k] - zt[k] - eta * o.g[k]);
                if (r > rmax) rmax = r;
            }
            if (logdet || ldscale) {
                double s1;
                ld += step_logdet(dim, M, h, w, beta, ell, x, eta, &s1);
                sc += s1;
            }
        }
        for (int k = 0; k < dim; ++k) yout[(int64_t)k * n + i] = x[k];
        if (logdet) logdet[i] = ld;
        if (ldscale) ldscale[i] = sc;
        if (resid) resid[i] = rmax;
    }
}

/* Epsilon mixture with the prior: sample i keeps its prior value iff u_i < eps, with
 * u_i from word 0 of Philox4x32-10 at counter {i_lo, i_hi, 0xffffffff, stream} and
 * key {seed_lo, seed_hi}, u = (word >> 8) 2^-24 (a counter the coordinates never use). */
void orc_mixture_coins(uint64_t seed, uint32_t stream, int64_t n, double eps, uint8_t *keep) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < n; ++i) {
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0xffffffffu, stream};
        uint32_t r[4];
        orc_philox4x32_10(ctr, key, r);
        double u = (double)(r[0] >> 8) * (1.0 / 16777216.0);
        keep[i] = (uint8_t)(u < eps);
    }
}

/* ------------------------------------------------------------------------- */
/* Compact-support culling (a variant beyond the paper): a point takes only   */
/* the hinges whose cell lies in the 3^dim block of cells around its own.     */
/* Cells have side `cell` >= the cutoff r_c on the box [lo, lo + nc cell);    */
/* a coordinate's cell is floor((v - lo) * inv_cell) in double precision from */
/* the single-precision v, lo and inv_cell, clamped to [0, nc - 1].  Every    */
/* hinge within r_c of the point is then included, so the dropped part of the */
/* logit is at most sum_j |w_j| exp(-r_c^2 / (2 l^2)).                        */
/* ------------------------------------------------------------------------- */

static int cull_cell(float v, float lo, float inv_cell, int nc) {
    double t = ((double)v - (double)lo) * (double)inv_cell;
    double f = floor(t);
    if (f < 0.0) return 0;
    if (f > (double)(nc - 1)) return nc - 1;
    return (int)f;
}

/* Logit, gradient of c over the culled hinge set at one point. */
static void cull_point(int dim, int M, const double *h, const double *w, double beta, double ell,
                       const float *lo, float inv_cell, const int *nc, const double *x,
                       double *s_out, double *gc) {
    int cx[ORC_MAX_DIM];
    for (int k = 0; k < dim; ++k) cx[k] = cull_cell((float)x[k], lo[k], inv_cell, nc[k]);
    double il2 = 1.0 / (ell * ell), i2l2 = 0.5 * il2;
    double s = beta, gs[ORC_MAX_DIM] = {0};
    for (int j = 0; j < M; ++j) {
        int near = 1;
        for (int k = 0; k < dim; ++k) {
            int hc = cull_cell((float)h[(int64_t)k * M + j], lo[k], inv_cell, nc[k]);
            if (hc < cx[k] - 1 || hc > cx[k] + 1) near = 0;
        }
        if (!near) continue;
        double r2 = 0.0, d[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) {
            d[k] = x[k] - h[(int64_t)k * M + j];
            r2 += d[k] * d[k];
        }
        double wp = w[j] * exp(-r2 * i2l2);
        s += wp;
        for (int k = 0; k < dim; ++k) gs[k] += -il2 * wp * d[k];
    }
    double sp = sigmoid_slope(s);
    if (s_out) *s_out = s;
    if (gc)
        for (int k = 0; k < dim; ++k) gc[k] = sp * gs[k];
}

/* s and grad c of the culled occupancy at n points. */
void orc_cull_eval(int dim, int M, const double *h, const double *w, double beta, double ell,
                   const float *lo, float inv_cell, const int *nc, const double *x, int64_t n,
                   double *s, double *gc) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xi[ORC_MAX_DIM], g[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) xi[k] = x[(int64_t)k * n + i];
        cull_point(dim, M, h, w, beta, ell, lo, inv_cell, nc, xi, s ? &s[i] : NULL, g);
        if (gc)
            for (int k = 0; k < dim; ++k) gc[(int64_t)k * n + i] = g[k];
    }
}

/* The plain morph (Eq. 1, explicit Euler) on the culled occupancy; the cells are
 * re-evaluated at every step from the current point. */
void orc_morph_culled(int dim, int M, const double *h, const double *w, double beta, double ell,
                      const float *lo, float inv_cell, const int *nc, const double *xin,
                      int64_t n, int T, double eta, double *xout) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x[ORC_MAX_DIM], g[ORC_MAX_DIM];
        for (int k = 0; k < dim; ++k) x[k] = xin[(int64_t)k * n + i];
        for (int t = 0; t < T; ++t) {
            cull_point(dim, M, h, w, beta, ell, lo, inv_cell, nc, x, NULL, g);
            for (int k = 0; k < dim; ++k) x[k] = x[k] - eta * g[k];
        }
        for (int k = 0; k < dim; ++k) xout[(int64_t)k * n + i] = x[k];
    }
}
