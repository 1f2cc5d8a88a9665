"""FP64 CPU oracle for the PDMP morph path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, `__graft_entry__.smoke()` and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the HIP library and
the product path never calls it.

Thin ctypes marshalling over `pdmp_oracle.c` (plain C, FP64, -ffp-contract=off):
arrays go in as FP64 copies of the caller's values (an exact upcast of FP32
inputs) and come back as numpy arrays.  Each function names the passage of the
paper it follows; the arithmetic itself lives in the C source.

Pins (tests/test_oracle_*.py) tie every function here to something other than
itself: published known-answer vectors, closed forms, finite differences,
textbook reductions, library integrators and optimisers, and brute force.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpdmp_oracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_u8p = C.POINTER(C.c_uint8)
_u32p = C.POINTER(C.c_uint32)
_ip = C.POINTER(C.c_int)
_i64 = C.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    sig = {
        "orc_num_threads": (C.c_int, []),
        "orc_set_num_threads": (None, [C.c_int]),
        "orc_philox4x32_10": (None, [_u32p, _u32p, _u32p]),
        "orc_uniform_samples": (None, [C.c_uint64, C.c_uint32, _fp, _fp, C.c_int, _i64, _fp]),
        "orc_uniform_at": (None, [C.c_uint64, C.c_uint32, _fp, _fp, C.c_int,
                                  C.POINTER(C.c_int64), _i64, _fp]),
        "orc_label_discs": (None, [_dp, _dp, _dp, C.c_int, _dp, _i64, _u8p]),
        "orc_label_boxes": (None, [_dp, _dp, C.c_int, _dp, _i64, _u8p]),
        "orc_occ_eval": (None, [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double, _dp, _i64,
                                _dp, _dp, _dp]),
        "orc_occ_grad": (None, [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double, _dp, _i64,
                                _dp, _dp, _dp, _dp, _dp]),
        "orc_logit_bwd_w_subset": (None, [C.c_int, C.c_int, _dp, C.c_double, _dp, _i64, _dp, _ip,
                                          C.c_int, _dp, _dp]),
        "orc_occ_hess": (None, [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double, _dp, _i64,
                                _dp, _dp]),
        "orc_morph_ws": (None, [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double, _dp, _i64,
                                C.c_int, C.c_double, _dp, _dp, _dp, _dp, _dp]),
        "orc_fit_loss_grad": (C.c_double, [C.c_int, C.c_int, _dp, C.c_double, _dp, _dp, _u8p,
                                           _i64, C.c_double, _dp, _dp]),
        "orc_adam_step": (None, [_dp, _dp, _dp, _dp, _i64, C.c_int, C.c_double, C.c_double,
                                 C.c_double, C.c_double]),
        "orc_fit": (None, [C.c_int, C.c_int, _dp, C.c_double, _dp, _u8p, _i64, C.c_int, C.c_int,
                           C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                           C.c_double, _dp, _dp, _dp, C.c_int, _dp]),
        "orc_logit_bwd": (None, [C.c_int, C.c_int, _dp, _dp, C.c_double, _dp, _i64, _dp, _dp,
                                 _dp]),
        "orc_bce_logits": (C.c_double, [_dp, _u8p, _i64, _dp]),
        "orc_fk_points": (None, [C.c_int, C.c_int, _dp, _dp, _i64, _dp]),
        "orc_fk_jacobian": (None, [C.c_int, C.c_int, _dp, _dp, C.c_int, _dp]),
        "orc_arm_cost_grad": (None, [C.c_int, C.c_int, _dp, C.c_int, _dp, _dp, C.c_double,
                                     C.c_double, _dp, _i64, C.c_int, _dp, _dp]),
        "orc_morph_arm": (None, [C.c_int, C.c_int, _dp, C.c_int, _dp, _dp, C.c_double,
                                 C.c_double, _dp, _i64, C.c_int, C.c_double, _dp, _dp, _dp,
                                 _dp, C.c_double]),
        "orc_arm_step_scale": (None, [C.c_int, C.c_int, _dp, C.c_int, _dp, _dp, C.c_double,
                                      C.c_double, _dp, _i64, _dp]),
        "orc_label_configs": (None, [C.c_int, C.c_int, _dp, _dp, _dp, C.c_int, _dp, _i64, _u8p]),
        "orc_config_label_margin": (None, [C.c_int, C.c_int, _dp, _dp, _dp, C.c_int, _dp, _i64,
                                           _dp]),
        "orc_mlp_nparams": (C.c_int64, [C.c_int, _ip]),
        "orc_mlp_forward": (None, [C.c_int, _ip, _dp, _dp, _i64, C.c_int, _dp, _dp]),
        "orc_mlp_loss_grad": (C.c_double, [C.c_int, _ip, _dp, _dp, _dp, _i64, _dp]),
        "orc_mlp_loss_grad_weighted": (C.c_double, [C.c_int, _ip, _dp, _dp, _dp, _i64, _u8p,
                                                    C.c_double, _dp]),
        "orc_amortised_morph": (None, [C.c_int, _ip, _dp, C.c_int, C.c_int, _dp, C.c_int, _dp,
                                       _dp, C.c_double, C.c_double, _dp, _i64, C.c_int,
                                       C.c_double, C.c_double, _dp, _u8p, _dp]),
        "orc_amortised_morph_refine": (None, [C.c_int, _ip, _dp, C.c_int, C.c_int, _dp, C.c_int,
                                              _dp, _dp, C.c_double, C.c_double, _dp, _i64,
                                              C.c_int, C.c_double, C.c_double, _dp, _u8p, _dp]),
        "orc_tanh_nparams": (C.c_int64, [C.c_int, C.c_int, C.c_int]),
        "orc_tanh_eval": (None, [C.c_int, C.c_int, C.c_int, _dp, _dp, _i64, _dp, _dp, _dp]),
        "orc_tanh_grad": (None, [C.c_int, C.c_int, C.c_int, _dp, _dp, _i64, _dp, _dp, _dp, _dp,
                                 _dp]),
        "orc_tanh_morph": (None, [C.c_int, C.c_int, C.c_int, _dp, _dp, _i64, C.c_int,
                                  C.c_double, _dp, _dp]),
        "orc_tanh_loss_grad": (C.c_double, [C.c_int, C.c_int, C.c_int, _dp, _dp, _u8p, _i64,
                                            C.c_double, _dp, _dp]),
        "orc_morph_logdet": (None, [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double, _dp,
                                    _i64, C.c_int, C.c_double, _dp, _dp, _dp]),
        "orc_morph_inverse": (None, [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double, _dp,
                                     _i64, C.c_int, C.c_double, C.c_int, _dp, _dp, _dp, _dp]),
        "orc_mixture_coins": (None, [C.c_uint64, C.c_uint32, _i64, C.c_double, _u8p]),
        "orc_cull_eval": (None, [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double, _fp,
                                 C.c_float, _ip, _dp, _i64, _dp, _dp]),
        "orc_morph_culled": (None, [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double, _fp,
                                    C.c_float, _ip, _dp, _i64, C.c_int, C.c_double, _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def num_threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS, else all host cores)."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads the oracle's parallel loops use from now on."""
    _load().orc_set_num_threads(int(n))


def _d(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _P(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


def _zeros(*shape):
    return np.zeros(shape, dtype=np.float64)


@dataclass
class Occupancy:
    """Occupancy model c(x) = sigma(sum_j w_j phi_j(x) + beta) (Sec. 3.1)."""
    hinges: np.ndarray   # [dim][M]
    weights: np.ndarray  # [M]
    beta: float
    lengthscale: float

    @property
    def dim(self):
        return int(np.asarray(self.hinges).shape[0])

    @property
    def M(self):
        return int(np.asarray(self.hinges).shape[1])

    def args(self):
        # FP64 copies are kept on the object so the pointers outlive the call.
        self._h64 = _d(self.hinges)
        self._w64 = _d(self.weights)
        return (self.dim, self.M, _P(self._h64), _P(self._w64), float(self.beta),
                float(self.lengthscale))


# ---------------------------------------------------------------- sampling ---

def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block (Salmon et al. 2011)."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    o = np.zeros(4, np.uint32)
    _load().orc_philox4x32_10(_P(c, _u32p), _P(k, _u32p), _P(o, _u32p))
    return o


def uniform_samples(seed: int, stream: int, lo, hi, n: int) -> np.ndarray:
    """Prior samples U[lo,hi)^dim, [dim][n] float32 (batched prior draw, Sec. 3.3)."""
    lo = np.ascontiguousarray(np.asarray(lo, dtype=np.float32).reshape(-1))
    hi = np.ascontiguousarray(np.asarray(hi, dtype=np.float32).reshape(-1))
    dim = lo.size
    out = np.zeros((dim, n), np.float32)
    _load().orc_uniform_samples(C.c_uint64(seed), C.c_uint32(stream), _P(lo, _fp), _P(hi, _fp),
                                dim, n, _P(out, _fp))
    return out


# ------------------------------------------------------------------ labels ---

def uniform_at(seed: int, stream: int, lo, hi, idx) -> np.ndarray:
    """Samples idx (any int64 indices) of the prior batch uniform_samples(seed, stream,
    lo, hi, n) for any n above them: [dim][len(idx)] float32."""
    lo = np.ascontiguousarray(np.asarray(lo, dtype=np.float32).reshape(-1))
    hi = np.ascontiguousarray(np.asarray(hi, dtype=np.float32).reshape(-1))
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).reshape(-1))
    out = np.zeros((lo.size, idx.size), np.float32)
    _load().orc_uniform_at(C.c_uint64(seed), C.c_uint32(stream), _P(lo, _fp), _P(hi, _fp),
                           lo.size, idx.ctypes.data_as(C.POINTER(C.c_int64)), idx.size,
                           _P(out, _fp))
    return out


def label_discs(centres, radii, x) -> np.ndarray:
    """1 where a 2-D point lies in any closed disc (the Table 1 feasibility test)."""
    c = _d(centres)
    r = _d(radii)
    x = _d(x)
    n = x.shape[1]
    out = np.zeros(n, np.uint8)
    _load().orc_label_discs(_P(_d(c[0])), _P(_d(c[1])), _P(r), r.size, _P(x), n, _P(out, _u8p))
    return out


def label_boxes(centres, half, x) -> np.ndarray:
    """1 where a 3-D point lies in any closed axis-aligned box."""
    c, e, x = _d(centres), _d(half), _d(x)
    n = x.shape[1]
    out = np.zeros(n, np.uint8)
    _load().orc_label_boxes(_P(c), _P(e), c.shape[1], _P(x), n, _P(out, _u8p))
    return out


# --------------------------------------------------------------- occupancy ---

def occ_eval(occ: Occupancy, x):
    """(s, c, S_abs) at [dim][n] points: logit, occupancy and logit error scale."""
    x = _d(x)
    n = x.shape[1]
    s, c, sa = _zeros(n), _zeros(n), _zeros(n)
    _load().orc_occ_eval(*occ.args(), _P(x), n, _P(s), _P(c), _P(sa))
    return s, c, sa


def occ_grad(occ: Occupancy, x, with_raw: bool = False):
    """(c, grad c, grad s, G_abs[, l^-2 sum |w| phi |x-h|]) at [dim][n] points."""
    x = _d(x)
    dim, n = x.shape
    c, gc, gs, ga, gr = _zeros(n), _zeros(dim, n), _zeros(dim, n), _zeros(n), _zeros(n)
    _load().orc_occ_grad(*occ.args(), _P(x), n, _P(c), _P(gc), _P(gs), _P(ga), _P(gr))
    return (c, gc, gs, ga, gr) if with_raw else (c, gc, gs, ga)


def occ_hess(occ: Occupancy, x):
    """(Hessian of c, Hessian of s), each [dim][dim][n]."""
    x = _d(x)
    dim, n = x.shape
    hc, hs = _zeros(dim * dim, n), _zeros(dim * dim, n)
    _load().orc_occ_hess(*occ.args(), _P(x), n, _P(hc), _P(hs))
    return hc.reshape(dim, dim, n), hs.reshape(dim, dim, n)


def morph_ws(occ: Occupancy, x, T: int, eta: float, diag: bool = False, traj: bool = False):
    """Explicit-Euler morph of workspace points (Eq. 1 solved by Euler's method).

    Returns x_T [dim][n]; with diag also (amplification, min det, max eta|H|) per
    sample; with traj also all states [T+1][dim][n].
    """
    x = _d(x)
    dim, n = x.shape
    out = _zeros(dim, n)
    amp = _zeros(n) if diag else None
    mdet = _zeros(n) if diag else None
    meh = _zeros(n) if diag else None
    tr = _zeros(T + 1, dim, n) if traj else None
    _load().orc_morph_ws(*occ.args(), _P(x), n, int(T), float(eta), _P(out), _P(amp), _P(mdet),
                         _P(meh), _P(tr))
    res = [out]
    if diag:
        res += [amp, mdet, meh]
    if traj:
        res += [tr]
    return res[0] if len(res) == 1 else tuple(res)


def morph_logdet(occ: Occupancy, x, T: int, eta: float):
    """(x_T, logdet, ldscale): the forward morph with sum_k log|det(I - eta Hc(x_k))|
    and the FP32 error scale of that sum."""
    x = _d(x)
    dim, n = x.shape
    out, ld, sc = _zeros(dim, n), _zeros(n), _zeros(n)
    _load().orc_morph_logdet(*occ.args(), _P(x), n, int(T), float(eta), _P(out), _P(ld), _P(sc))
    return out, ld, sc


def morph_inverse(occ: Occupancy, z, T: int, eta: float, iters: int):
    """(y, logdet, ldscale, resid): the inverse of the T-step morph by fixed point
    (iters iterations per step, in reverse step order), the forward log-determinant
    along the reconstructed path and the largest fixed-point residual."""
    z = _d(z)
    dim, n = z.shape
    y, ld, sc, r = _zeros(dim, n), _zeros(n), _zeros(n), _zeros(n)
    _load().orc_morph_inverse(*occ.args(), _P(z), n, int(T), float(eta), int(iters), _P(y),
                              _P(ld), _P(sc), _P(r))
    return y, ld, sc, r


def mixture_coins(seed: int, stream: int, n: int, eps: float) -> np.ndarray:
    """keep[i] = 1 where sample i stays at its prior value in the epsilon mixture."""
    out = np.zeros(n, dtype=np.uint8)
    _load().orc_mixture_coins(int(seed), int(stream), int(n), float(eps), _P(out, _u8p))
    return out


# --------------------------------------------------------------------- fit ---

def fit_loss_grad(hinges, ell, wb, pts, y, l2):
    """(loss, grad [M+1], grad scale [M+1]) of mean BCE + (l2/2)|w|^2 (Sec. 3.1)."""
    h, wb, pts = _d(hinges), _d(wb), _d(pts)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    dim, M = h.shape
    g, gsc = _zeros(M + 1), _zeros(M + 1)
    L = _load().orc_fit_loss_grad(dim, M, _P(h), float(ell), _P(wb), _P(pts), _P(y, _u8p),
                                  pts.shape[1], float(l2), _P(g), _P(gsc))
    return L, g, gsc


def adam_step(p, g, m, v, t, lr, b1, b2, eps):
    """One Adam update in place (Kingma & Ba 2015, Algorithm 1)."""
    _load().orc_adam_step(_P(p), _P(_d(g)), _P(m), _P(v), p.size, int(t), float(lr), float(b1),
                          float(b2), float(eps))


def fit(hinges, ell, pts, y, optimizer, steps, lr, l2, lr_bias=None, b1=0.9, b2=0.999,
        eps=1e-8, wb0=None, m=None, v=None, t0=0):
    """Full-batch occupancy fit (Sec. 3.1); returns (wb, m, v, loss per step).

    optimizer 0 is gradient descent (step lr on w, lr_bias on beta, default lr);
    optimizer 1 is Adam with step lr.
    """
    lr_bias = lr if lr_bias is None else lr_bias
    h, pts = _d(hinges), _d(pts)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    dim, M = h.shape
    wb = _zeros(M + 1) if wb0 is None else _d(wb0).copy()
    m = _zeros(M + 1) if m is None else _d(m).copy()
    v = _zeros(M + 1) if v is None else _d(v).copy()
    loss = _zeros(max(steps, 1))
    _load().orc_fit(dim, M, _P(h), float(ell), _P(pts), _P(y, _u8p), pts.shape[1],
                    int(optimizer), int(steps), float(lr), float(lr_bias), float(l2),
                    float(b1), float(b2),
                    float(eps), _P(wb), _P(m), _P(v), int(t0), _P(loss))
    return wb, m, v, loss[:steps]


def logit_bwd(hinges, w, ell, x, g_s, want_w=True, want_x=True):
    """(grad_w [M+1], grad_x [dim][n]) of sum_i g_i s(x_i) (the backward of the logit)."""
    h, w, x, g = _d(hinges), _d(w), _d(x), _d(g_s)
    dim, M = h.shape
    n = x.shape[1]
    gw = _zeros(M + 1) if want_w else None
    gx = _zeros(dim, n) if want_x else None
    _load().orc_logit_bwd(dim, M, _P(h), _P(w), float(ell), _P(x), n, _P(g), _P(gw), _P(gx))
    return gw, gx


def logit_bwd_w_subset(hinges, ell, x, g_s, js):
    """(sum_i g_i phi_ij, sum_i |g_i| phi_ij) for the hinges listed in js only."""
    h, x, g = _d(hinges), _d(x), _d(g_s)
    js = np.ascontiguousarray(np.asarray(js, dtype=np.intc))
    dim, M = h.shape
    out, ab = _zeros(js.size), _zeros(js.size)
    _load().orc_logit_bwd_w_subset(dim, M, _P(h), float(ell), _P(x), x.shape[1], _P(g),
                                   _P(js, _ip), js.size, _P(out), _P(ab))
    return out, ab


def bce_logits(s, y):
    """(mean BCE of sigma(s) vs y, dL/ds)."""
    s = _d(s)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    g = _zeros(s.size)
    L = _load().orc_bce_logits(_P(s), _P(y, _u8p), s.size, _P(g))
    return L, g


# --------------------------------------------------------------------- arm ---

@dataclass
class Arm:
    """Standard-DH serial arm with `ppl` body points per link (Sec. 3.2)."""
    a: np.ndarray
    d: np.ndarray
    alpha: np.ndarray
    theta0: np.ndarray
    ppl: int = 8

    @property
    def ndof(self):
        return int(np.asarray(self.a).size)

    def dh(self):
        return _d(np.concatenate([np.asarray(self.a, np.float64), np.asarray(self.d, np.float64),
                                  np.asarray(self.alpha, np.float64),
                                  np.asarray(self.theta0, np.float64)]))


def fk_points(arm: Arm, q):
    """Body points [3][ndof*ppl][n] of configurations q [ndof][n]."""
    q = _d(q)
    n = q.shape[1]
    nb = arm.ndof * arm.ppl
    out = _zeros(3, nb, n)
    _load().orc_fk_points(arm.ndof, arm.ppl, _P(arm.dh()), _P(q), n, _P(out))
    return out


def fk_jacobian(arm: Arm, q1, body: int):
    """Positional Jacobian [3][ndof] of one body point at one configuration."""
    q1 = _d(np.asarray(q1).reshape(-1))
    J = _zeros(3, arm.ndof)
    _load().orc_fk_jacobian(arm.ndof, arm.ppl, _P(arm.dh()), _P(q1), int(body), _P(J))
    return J


def arm_cost_grad(arm: Arm, occ: Occupancy, q, form: int = 0):
    """(cost [n], grad_q [ndof][n]) of the summed body-point occupancy (Eq. 3).

    form 0 sums J_p^T grad c(p) column by column; form 1 uses per-link suffix sums.
    """
    q = _d(q)
    n = q.shape[1]
    cost, g = _zeros(n), _zeros(arm.ndof, n)
    _, M, h, w, beta, ell = occ.args()
    _load().orc_arm_cost_grad(arm.ndof, arm.ppl, _P(arm.dh()), M, h, w, beta, ell, _P(q),
                              n, int(form), _P(cost), _P(g))
    return cost, g


def morph_arm(arm: Arm, occ: Occupancy, q, T: int, eta: float, diag: bool = False,
              fd_h: float = 1e-5, with_eh: bool = False):
    """Joint-space explicit-Euler morph; with diag also (amplification, min det), and
    with with_eh also the largest eta |H_q|_2 along each path."""
    q = _d(q)
    n = q.shape[1]
    out = _zeros(arm.ndof, n)
    amp = _zeros(n) if diag else None
    mdet = _zeros(n) if diag else None
    meh = _zeros(n) if diag and with_eh else None
    _, M, h, w, beta, ell = occ.args()
    _load().orc_morph_arm(arm.ndof, arm.ppl, _P(arm.dh()), M, h, w, beta, ell, _P(q), n,
                          int(T), float(eta), _P(out), _P(amp), _P(mdet), _P(meh), float(fd_h))
    if not diag:
        return out
    return (out, amp, mdet, meh) if with_eh else (out, amp, mdet)


def arm_step_scale(arm: Arm, occ: Occupancy, q):
    """Per configuration: sum over body points of max_j |J_p[:, j]|_1 G_abs(p), the
    scale FP32-class errors of the body-point gradients carry into grad_q."""
    q = _d(q)
    n = q.shape[1]
    out = _zeros(n)
    _, M, h, w, beta, ell = occ.args()
    _load().orc_arm_step_scale(arm.ndof, arm.ppl, _P(arm.dh()), M, h, w, beta, ell, _P(q), n,
                               _P(out))
    return out


def label_configs(arm: Arm, centres, half, q):
    """1 where any body point of a configuration lies in any box."""
    c, e, q = _d(centres), _d(half), _d(q)
    n = q.shape[1]
    out = np.zeros(n, np.uint8)
    _load().orc_label_configs(arm.ndof, arm.ppl, _P(arm.dh()), _P(c), _P(e), c.shape[1], _P(q), n,
                              _P(out, _u8p))
    return out


def config_label_margin(arm: Arm, centres, half, q):
    """Per configuration, how far its body points are from flipping any box test."""
    c, e, q = _d(centres), _d(half), _d(q)
    n = q.shape[1]
    out = _zeros(n)
    _load().orc_config_label_margin(arm.ndof, arm.ppl, _P(arm.dh()), _P(c), _P(e), c.shape[1],
                                    _P(q), n, _P(out))
    return out


# --------------------------------------------------------------------- MLP ---

def mlp_pack(layers) -> np.ndarray:
    """Flatten [(W [out][in], b [out]), ...] into one FP64 vector (W then b per layer)."""
    return _d(np.concatenate([np.concatenate([np.asarray(W, np.float64).reshape(-1),
                                              np.asarray(b, np.float64).reshape(-1)])
                              for W, b in layers]))


def mlp_unpack(P, widths):
    out, off = [], 0
    for li in range(len(widths) - 1):
        fi, fo = widths[li], widths[li + 1]
        W = P[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        b = P[off:off + fo]
        off += fo
        out.append((W, b))
    return out


def _widths(widths):
    return np.ascontiguousarray(np.asarray(widths, dtype=np.int32)).astype(np.intc)


def mlp_forward(widths, P, q, residual: bool = True, with_scale: bool = False):
    """q + f(q) (or f(q)) for [w0][B] inputs; f is the SiLU MLP.  with_scale also
    returns sum_k |W_L| |a_{L-1}| + |b_L| per output."""
    wd = _widths(widths)
    q = _d(q)
    B = q.shape[1]
    out = _zeros(int(wd[-1]), B)
    sc = _zeros(int(wd[-1]), B) if with_scale else None
    _load().orc_mlp_forward(wd.size - 1, _P(wd, _ip), _P(_d(P)), _P(q), B, int(residual), _P(out),
                            _P(sc))
    return (out, sc) if with_scale else out


def mlp_loss_grad(widths, P, q, target):
    """(MSE of q + f(q) against target, gradient in the flat parameter layout)."""
    wd = _widths(widths)
    q, t, P = _d(q), _d(target), _d(P)
    g = np.zeros_like(P)
    L = _load().orc_mlp_loss_grad(wd.size - 1, _P(wd, _ip), _P(P), _P(q), _P(t), q.shape[1],
                                  _P(g))
    return L, g


def mlp_loss_grad_weighted(widths, P, q, target, hard, hard_weight):
    """The MSE with sample weight hard_weight where hard[s] != 0 (1 elsewhere), still
    normalised by n_out B, and its gradient."""
    wd = _widths(widths)
    q, t, P = _d(q), _d(target), _d(P)
    hard = np.ascontiguousarray(np.asarray(hard, np.uint8))
    assert hard.shape == (q.shape[1],)
    g = np.zeros_like(P)
    L = _load().orc_mlp_loss_grad_weighted(wd.size - 1, _P(wd, _ip), _P(P), _P(q), _P(t),
                                           q.shape[1], _P(hard, _u8p), float(hard_weight), _P(g))
    return L, g


def amortised_morph(widths, P, arm: Arm, occ: Occupancy, q, T, eta, thresh=0.5,
                    refine: bool = False):
    """(q_out, flag, max body-point occupancy at q_hat) of the amortised morph; with
    refine, flagged configurations take the T plain steps from q_hat instead of q."""
    wd = _widths(widths)
    q = _d(q)
    n = q.shape[1]
    out = _zeros(arm.ndof, n)
    flag = np.zeros(n, np.uint8)
    maxc = _zeros(n)
    _, M, h, w, beta, ell = occ.args()
    fn = _load().orc_amortised_morph_refine if refine else _load().orc_amortised_morph
    fn(wd.size - 1, _P(wd, _ip), _P(_d(P)), arm.ndof, arm.ppl, _P(arm.dh()), M, h, w, beta, ell,
       _P(q), n, int(T), float(eta), float(thresh), _P(out), _P(flag, _u8p), _P(maxc))
    return out, flag, maxc


# ---------------------------------------------- the paper's tanh network ---

@dataclass
class TanhNet:
    """The paper's occupancy network (Sec. 3.1): L hidden tanh layers of width H,
    sigmoid output.  P is flat: W_l [H][n_l], b_l [H] for each layer, then v [H], b_o."""
    dim: int
    H: int
    L: int
    P: np.ndarray

    def args(self):
        self._p64 = _d(self.P)
        assert self._p64.size == tanh_nparams(self.dim, self.H, self.L)
        return (int(self.dim), int(self.H), int(self.L), _P(self._p64))


def tanh_nparams(dim: int, H: int, L: int) -> int:
    return int(_load().orc_tanh_nparams(int(dim), int(H), int(L)))


def tanh_layers(net: TanhNet):
    """[(W_l, b_l)] for the hidden layers and (v, b_o), as views of net.P."""
    P = np.asarray(net.P)
    out, o, nin = [], 0, net.dim
    for _ in range(net.L):
        W = P[o:o + net.H * nin].reshape(net.H, nin)
        o += net.H * nin
        out.append((W, P[o:o + net.H]))
        o += net.H
        nin = net.H
    return out, (P[o:o + net.H], P[o + net.H])


def tanh_eval(net: TanhNet, x):
    """(s, c, S_abs) at [dim][n] points."""
    x = _d(x)
    n = x.shape[1]
    s, c, sa = _zeros(n), _zeros(n), _zeros(n)
    _load().orc_tanh_eval(*net.args(), _P(x), n, _P(s), _P(c), _P(sa))
    return s, c, sa


def tanh_grad(net: TanhNet, x):
    """(s, grad s, grad c, S_abs, G_abs) at [dim][n] points (chain rule, reverse order)."""
    x = _d(x)
    dim, n = x.shape
    s, gs, gc, sa, ga = _zeros(n), _zeros(dim, n), _zeros(dim, n), _zeros(n), _zeros(n)
    _load().orc_tanh_grad(*net.args(), _P(x), n, _P(s), _P(gs), _P(gc), _P(sa), _P(ga))
    return s, gs, gc, sa, ga


def tanh_morph(net: TanhNet, x, T: int, eta: float, diag: bool = False):
    """Explicit-Euler morph (Eq. 1) with the network's occupancy; with diag also the
    per-sample product of |I - eta Hc|_2 along the path."""
    x = _d(x)
    dim, n = x.shape
    out = _zeros(dim, n)
    amp = _zeros(n) if diag else None
    _load().orc_tanh_morph(*net.args(), _P(x), n, int(T), float(eta), _P(out), _P(amp))
    return (out, amp) if diag else out


def tanh_loss_grad(net: TanhNet, pts, y, l2: float, with_scale: bool = False):
    """(loss, grad [nparams][, grad error scale]) of mean BCE + (l2/2) |weights|^2
    (biases not decayed)."""
    pts = _d(pts)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    g = _zeros(tanh_nparams(net.dim, net.H, net.L))
    gs = _zeros(g.size) if with_scale else None
    L = _load().orc_tanh_loss_grad(*net.args(), _P(pts), _P(y, _u8p), pts.shape[1], float(l2),
                                   _P(g), _P(gs))
    return (L, g, gs) if with_scale else (L, g)


def tanh_fit(net: TanhNet, pts, y, steps: int, lr: float, l2: float, b1=0.9, b2=0.999,
             eps=1e-8):
    """Full-batch Adam on the BCE objective (Sec. 3.1); returns (P, loss per step)."""
    P = _d(net.P).copy()
    m, v = np.zeros_like(P), np.zeros_like(P)
    losses = np.zeros(steps)
    cur = TanhNet(net.dim, net.H, net.L, P)
    for t in range(steps):
        losses[t], g = tanh_loss_grad(cur, pts, y, l2)
        adam_step(P, g, m, v, t + 1, lr, b1, b2, eps)
    return P, losses


# ----------------------------------------------- compact-support culling ---

@dataclass
class CullGrid:
    """Cells of side `cell` (>= the cutoff) on the box starting at `lo`, nc per axis;
    inv_cell = 1/cell rounded to single precision, as the GPU uses it."""
    lo: np.ndarray
    inv_cell: float
    nc: np.ndarray

    @staticmethod
    def make(lo, hi, cutoff):
        lo = np.asarray(lo, np.float32)
        hi = np.asarray(hi, np.float32)
        cutoff = np.float32(cutoff)
        inv = np.float32(1.0) / cutoff
        # cell side from the rounded inverse, so that a cell is never below the cutoff
        while 1.0 / float(inv) < float(cutoff):
            inv = np.nextafter(inv, np.float32(0))
        nc = np.maximum(1, np.floor((hi.astype(np.float64) - lo) * float(inv)).astype(np.int64) + 1)
        return CullGrid(lo, float(inv), nc.astype(np.intc))

    def args(self):
        self._lo = np.ascontiguousarray(self.lo, np.float32)
        self._nc = np.ascontiguousarray(self.nc, np.intc)
        return (_P(self._lo, _fp), float(self.inv_cell), _P(self._nc, _ip))


def cull_eval(occ: Occupancy, grid: CullGrid, x):
    """(s, grad c) of the culled occupancy at [dim][n] points."""
    x = _d(x)
    dim, n = x.shape
    s, gc = _zeros(n), _zeros(dim, n)
    _load().orc_cull_eval(*occ.args(), *grid.args(), _P(x), n, _P(s), _P(gc))
    return s, gc


def morph_culled(occ: Occupancy, grid: CullGrid, x, T: int, eta: float):
    """The plain morph (Eq. 1) on the culled occupancy."""
    x = _d(x)
    dim, n = x.shape
    out = _zeros(dim, n)
    _load().orc_morph_culled(*occ.args(), *grid.args(), _P(x), n, int(T), float(eta), _P(out))
    return out
