"""MI355X (gfx950) batched diffeomorphic morph of planner samples.

Python binding over libpdmp.so (include/pdmp.h).  Every step of the path runs in
the library's HIP kernels; this module only marshals torch device tensors (used
for device memory and streams) into the C ABI.  There is no CPU fallback: a call
without the built library, or with CPU tensors, raises.

Method: Lai, Zhi, Hermans, Ramos, "Parallelised Diffeomorphic Sampling-based
Motion Planning" -- occupancy learning (Sec. 3.1), cost-informed diffeomorphism
by Euler integration of Eq. 1 and its joint-space pull-back (Sec. 3.2, Eq. 3),
batched GPU sampling (Sec. 3.3).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional, Sequence

from . import _lib
from ._lib import PdmpError

__all__ = ["Occupancy", "Arm", "PdmpError", "abi_version", "uniform_samples",
           "label_points_discs", "label_points_boxes", "label_configs", "occupancy_eval",
           "occupancy_grad", "morph_samples", "morph_samples_ws", "morph_workspace",
           "morph_trajectory", "split_scheme", "issue_rates",
           "fk_body_points", "sync",
           "occupancy_bwd", "occupancy_bwd_noalloc", "bce_logits", "adam_step", "fit_occupancy", "Mlp", "arm_max_occupancy",
           "amortised_morph", "TanhNet", "tanh_occupancy_eval", "tanh_occupancy_grad",
           "tanh_morph_samples", "tanh_split_scheme", "tanh_loss_grad", "tanh_fit", "morph_logdet", "morph_inverse",
           "mixture_samples", "Bucket", "Sampler", "rrt_run", "cull_grid", "morph_culled"]


def _torch():
    import torch
    return torch


def _stream(device=None):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev(t, name, dtype=None, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor; there is no CPU path")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def abi_version() -> int:
    return int(_lib.load().pdmp_abi_version())


def sync(device=None):
    _lib.call("pdmp_sync", _stream(device))


@dataclass
class Occupancy:
    """c(x) = sigma(sum_j w_j exp(-|x-h_j|^2/(2 l^2)) + beta) (Sec. 3.1).

    hinges: [dim][M] float32 device tensor; weights: [M+1] float32 device tensor
    whose last entry is the bias beta.
    """
    hinges: "object"
    weights: "object"
    lengthscale: float
    grid: Optional[tuple] = None  # points per axis when the hinges are a tensor grid

    @property
    def dim(self) -> int:
        return int(self.hinges.shape[0])

    @property
    def n_hinges(self) -> int:
        return int(self.hinges.shape[1])

    def c_struct(self) -> _lib.pdmp_occupancy:
        torch = _torch()
        _dev(self.hinges, "hinges", torch.float32)
        _dev(self.weights, "weights", torch.float32, (self.n_hinges + 1,))
        g = (0, 0, 0)
        if self.grid:
            g = tuple(int(v) for v in self.grid) + (0,) * (3 - len(self.grid))
        return _lib.pdmp_occupancy(self.dim, self.n_hinges, self.hinges.data_ptr(),
                                   self.weights.data_ptr(), float(self.lengthscale),
                                   (C.c_int32 * 3)(*g))


@dataclass
class Arm:
    """Standard-DH serial arm, pts_per_link body points per link (Sec. 3.2)."""
    a: Sequence[float]
    d: Sequence[float]
    alpha: Sequence[float]
    theta0: Sequence[float]
    pts_per_link: int = 8

    @property
    def n_dof(self) -> int:
        return len(self.a)

    @property
    def n_body(self) -> int:
        return self.n_dof * self.pts_per_link

    def c_struct(self) -> _lib.pdmp_arm:
        s = _lib.pdmp_arm()
        s.n_dof = self.n_dof
        s.pts_per_link = int(self.pts_per_link)
        n = min(self.n_dof, _lib.MAX_DOF)
        for i in range(n):
            s.a[i] = float(self.a[i])
            s.d[i] = float(self.d[i])
            s.alpha[i] = float(self.alpha[i])
            s.theta0[i] = float(self.theta0[i])
        return s


def uniform_samples(seed: int, stream_id: int, lo, hi, n: int, device="cuda", out=None):
    """Prior batch x ~ U[lo, hi)^dim as a [dim][n] float32 device tensor (Sec. 3.3)."""
    torch = _torch()
    lo = [float(v) for v in lo]
    hi = [float(v) for v in hi]
    dim = len(lo)
    if out is None:
        out = torch.empty((dim, n), dtype=torch.float32, device=device)
    _dev(out, "out", torch.float32, (dim, n))
    lo_a = (C.c_float * dim)(*lo)
    hi_a = (C.c_float * dim)(*hi)
    _lib.call("pdmp_uniform_samples", C.c_uint64(seed & (2**64 - 1)), C.c_uint32(stream_id),
              lo_a, hi_a, dim, n, _dev(out, "out") if n else None, _stream(out.device))
    return out


def _labels_out(n, device, count, out=None, hit=None):
    torch = _torch()
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=device)
    if count and hit is None:
        hit = torch.empty(1, dtype=torch.int64, device=device)
    return out, hit


def label_points_discs(centres, radii, x, count: bool = False, out=None, hit=None):
    """1 where a 2-D point lies in any closed disc; optionally the count of 1s."""
    torch = _torch()
    n = int(x.shape[1])
    sc = _lib.pdmp_discs(int(radii.shape[0]), _dev(centres, "centres", torch.float32).value,
                         _dev(radii, "radii", torch.float32).value)
    out, hit = _labels_out(n, x.device, count, out, hit)
    _lib.call("pdmp_label_points_discs", C.byref(sc), _dev(x, "x", torch.float32, (2, n)), n,
              _dev(out, "out"), _dev(hit, "n_hit") if count else None, _stream(x.device))
    return (out, hit) if count else out


def label_points_boxes(centres, half, x, count: bool = False, out=None, hit=None):
    """1 where a 3-D point lies in any closed axis-aligned box."""
    torch = _torch()
    n = int(x.shape[1])
    sc = _lib.pdmp_boxes(int(centres.shape[1]), _dev(centres, "centres", torch.float32).value,
                         _dev(half, "half", torch.float32).value)
    out, hit = _labels_out(n, x.device, count, out, hit)
    _lib.call("pdmp_label_points_boxes", C.byref(sc), _dev(x, "x", torch.float32, (3, n)), n,
              _dev(out, "out"), _dev(hit, "n_hit") if count else None, _stream(x.device))
    return (out, hit) if count else out


def label_configs(arm: Arm, centres, half, q, count: bool = False, out=None, hit=None):
    """1 where any body point of a configuration lies in any box."""
    torch = _torch()
    n = int(q.shape[1])
    sc = _lib.pdmp_boxes(int(centres.shape[1]), _dev(centres, "centres", torch.float32).value,
                         _dev(half, "half", torch.float32).value)
    a = arm.c_struct()
    out, hit = _labels_out(n, q.device, count, out, hit)
    _lib.call("pdmp_label_configs", C.byref(a), C.byref(sc),
              _dev(q, "q", torch.float32, (arm.n_dof, n)), n, _dev(out, "out"),
              _dev(hit, "n_hit") if count else None, _stream(q.device))
    return (out, hit) if count else out


def occupancy_eval(occ: Occupancy, x):
    """(c, s) at [dim][n] points."""
    torch = _torch()
    n = int(x.shape[1])
    c = torch.empty(n, dtype=torch.float32, device=x.device)
    s = torch.empty(n, dtype=torch.float32, device=x.device)
    o = occ.c_struct()
    _lib.call("pdmp_occupancy_eval", C.byref(o), _dev(x, "x", torch.float32, (occ.dim, n)), n,
              _dev(c, "c"), _dev(s, "s"), _stream(x.device))
    return c, s


def occupancy_grad(occ: Occupancy, x):
    """(c, grad_x c) at [dim][n] points."""
    torch = _torch()
    n = int(x.shape[1])
    c = torch.empty(n, dtype=torch.float32, device=x.device)
    g = torch.empty((occ.dim, n), dtype=torch.float32, device=x.device)
    o = occ.c_struct()
    _lib.call("pdmp_occupancy_grad", C.byref(o), _dev(x, "x", torch.float32, (occ.dim, n)), n,
              _dev(c, "c"), _dev(g, "grad"), _stream(x.device))
    return c, g


def morph_samples(occ: Occupancy, x, T: int, eta: float, arm: Optional[Arm] = None,
                  out=None):
    """Explicit-Euler morph of base samples (Eq. 1; Eq. 3 when `arm` is given).

    x: [dim][n] workspace points, or [n_dof][n] joint configurations with an arm.
    Returns `out` (a new tensor unless given; out may be x for in-place).
    """
    torch = _torch()
    n = int(x.shape[1])
    rows = arm.n_dof if arm is not None else occ.dim
    _dev(x, "x", torch.float32, (rows, n))
    if out is None:
        out = torch.empty_like(x)
    o = occ.c_struct()
    a = C.byref(arm.c_struct()) if arm is not None else None
    _lib.call("pdmp_morph_samples", C.byref(o), a, C.c_void_p(x.data_ptr()),
              _dev(out, "out", torch.float32, (rows, n)), n, int(T), float(eta),
              _stream(x.device))
    return out


SPLIT_SCHEMES = {0: ("pairwise", None), 1: ("bf16", 6), 2: ("fp16", 3)}


def split_scheme(occ: Occupancy):
    """(name, products per FP32 multiply-add) of the split scheme the grid morph
    kernels take for this occupancy, as the library decides it: ("fp16", 3),
    ("bf16", 6), or ("pairwise", None) when the morph takes no grid kernel."""
    torch = _torch()
    v = C.c_int32(-1)
    _lib.call("pdmp_split_scheme", C.byref(occ.c_struct()), C.byref(v),
              _stream(occ.hinges.device if isinstance(occ.hinges, torch.Tensor) else None))
    return SPLIT_SCHEMES[int(v.value)]


ISSUE_RATE_KEYS = ("v_fma_f32", "v_exp_f32", "v_cvt_pk_f16_f32", "v_fma_mix_f32",
                   "iter_4exp_4fma", "v_mfma_f32_32x32x16_f16", "iter_4mfma_32fma", "clock_ghz")


def issue_rates() -> dict:
    """Measured issue costs on the current device (cycles per wave64 instruction on one
    SIMD; the two mixed entries are cycles per iteration) and the probes' clock."""
    out = (C.c_double * len(ISSUE_RATE_KEYS))()
    _lib.call("pdmp_issue_rates", out, len(ISSUE_RATE_KEYS))
    return dict(zip(ISSUE_RATE_KEYS, [float(v) for v in out]))


def morph_workspace(occ: Occupancy, n: int, T: int, arm: Optional[Arm] = None):
    """A device workspace for morph_samples_ws of n samples over T steps (None if the
    call needs none)."""
    lib = _lib.load()
    a = C.byref(arm.c_struct()) if arm is not None else None
    nb = int(lib.pdmp_morph_workspace_size(C.byref(occ.c_struct()), a, int(n), int(T)))
    return _workspace(nb, occ.hinges.device) if nb else None


def morph_samples_ws(occ: Occupancy, x, T: int, eta: float, arm: Optional[Arm] = None,
                     out=None, ws=None):
    """morph_samples with a workspace: a large 2-D grid batch is ordered spatially and
    each wave skips the exact zeros of the sums (the same bits).  ws from
    morph_workspace (allocated here if None)."""
    torch = _torch()
    n = int(x.shape[1])
    rows = arm.n_dof if arm is not None else occ.dim
    _dev(x, "x", torch.float32, (rows, n))
    if out is None:
        out = torch.empty_like(x)
    if ws is None:
        ws = morph_workspace(occ, n, T, arm)
    o = occ.c_struct()
    a = C.byref(arm.c_struct()) if arm is not None else None
    _lib.call("pdmp_morph_samples_ws", C.byref(o), a, C.c_void_p(x.data_ptr()),
              _dev(out, "out", torch.float32, (rows, n)), n, int(T), float(eta),
              _dev(ws, "ws") if ws is not None else None, ws.numel() if ws is not None else 0,
              _stream(x.device))
    return out


def morph_trajectory(occ: Occupancy, x, T: int, eta: float, stride: int = 1,
                     arm: Optional[Arm] = None, out=None):
    """(x_T, traj): the morph of morph_samples with the path of every stride-th sample,
    traj [T+1][rows][ceil(n/stride)] (state 0 the input, state T the output)."""
    torch = _torch()
    n = int(x.shape[1])
    rows = arm.n_dof if arm is not None else occ.dim
    _dev(x, "x", torch.float32, (rows, n))
    if out is None:
        out = torch.empty_like(x)
    nt = (n + int(stride) - 1) // int(stride) if n > 0 else 0
    traj = torch.empty((int(T) + 1, rows, nt), dtype=torch.float32, device=x.device)
    o = occ.c_struct()
    a = C.byref(arm.c_struct()) if arm is not None else None
    _lib.call("pdmp_morph_trajectory", C.byref(o), a, C.c_void_p(x.data_ptr()),
              _dev(out, "out", torch.float32, (rows, n)), n, int(T), float(eta),
              C.c_void_p(traj.data_ptr()), int(stride), _stream(x.device))
    return out, traj


def _ws_args(ws):
    return (_dev(ws, "ws") if ws is not None else None, ws.numel() if ws is not None else 0)


def morph_logdet(occ: Occupancy, x, T: int, eta: float, out=None, ordered: bool = False,
                 ws=None):
    """(x_T, logdet): the workspace morph of x [dim][n] and, per sample,
    sum_k log|det(I - eta Hc(x_k))| (the log-Jacobian of the map, Sec. 3.2).  With
    ordered, pdmp_morph_logdet_ws (a large 2-D grid batch in spatial order, exact zeros
    skipped, the same bits; ws from morph_workspace, allocated here if None)."""
    torch = _torch()
    n = int(x.shape[1])
    _dev(x, "x", torch.float32, (occ.dim, n))
    if out is None:
        out = torch.empty_like(x)
    ld = torch.empty(n, dtype=torch.float32, device=x.device)
    o = occ.c_struct()
    args = (C.byref(o), C.c_void_p(x.data_ptr()), _dev(out, "out", torch.float32, (occ.dim, n)),
            n, int(T), float(eta), _dev(ld, "logdet"))
    if ordered:
        if ws is None:
            ws = morph_workspace(occ, n, T)
        _lib.call("pdmp_morph_logdet_ws", *args, *_ws_args(ws), _stream(x.device))
    else:
        _lib.call("pdmp_morph_logdet", *args, _stream(x.device))
    return out, ld


def morph_inverse(occ: Occupancy, z, T: int, eta: float, iters: int = 30,
                  ordered: bool = False, ws=None):
    """(y, logdet, resid): the inverse of the T-step morph at z [dim][n] by fixed point
    (iters iterations per step), the forward log-determinant along the reconstructed
    path and the largest fixed-point residual per sample.  With ordered,
    pdmp_morph_inverse_ws (as in morph_logdet)."""
    torch = _torch()
    n = int(z.shape[1])
    _dev(z, "z", torch.float32, (occ.dim, n))
    y = torch.empty_like(z)
    ld = torch.empty(n, dtype=torch.float32, device=z.device)
    r = torch.empty(n, dtype=torch.float32, device=z.device)
    o = occ.c_struct()
    args = (C.byref(o), C.c_void_p(z.data_ptr()), _dev(y, "y"), n, int(T), float(eta),
            int(iters), _dev(ld, "logdet"), _dev(r, "resid"))
    if ordered:
        if ws is None:
            ws = morph_workspace(occ, n, T)
        _lib.call("pdmp_morph_inverse_ws", *args, *_ws_args(ws), _stream(z.device))
    else:
        _lib.call("pdmp_morph_inverse", *args, _stream(z.device))
    return y, ld, r


def mixture_samples(occ: Occupancy, seed: int, stream_id: int, lo, hi, n: int, eps: float,
                    T: int, eta: float, device="cuda"):
    """(x0, out, keep): a Philox prior batch, its morph, and the epsilon mixture that
    keeps the prior value of each sample with probability eps (Sec. 3.3)."""
    torch = _torch()
    lo_a = (C.c_float * occ.dim)(*[float(v) for v in lo])
    hi_a = (C.c_float * occ.dim)(*[float(v) for v in hi])
    x0 = torch.empty((occ.dim, n), dtype=torch.float32, device=device)
    out = torch.empty_like(x0)
    keep = torch.empty(n, dtype=torch.uint8, device=device)
    o = occ.c_struct()
    _lib.call("pdmp_mixture_samples", C.byref(o), int(seed), int(stream_id), lo_a, hi_a, n,
              float(eps), int(T), float(eta), _dev(x0, "x0"), _dev(out, "out"), _dev(keep, "keep"),
              _stream(x0.device))
    return x0, out, keep


def fk_body_points(arm: Arm, q):
    """Body points [3][n_dof*pts_per_link][n] of configurations q [n_dof][n]."""
    torch = _torch()
    n = int(q.shape[1])
    pts = torch.empty((3, arm.n_body, n), dtype=torch.float32, device=q.device)
    a = arm.c_struct()
    _lib.call("pdmp_fk_body_points", C.byref(a), _dev(q, "q", torch.float32, (arm.n_dof, n)), n,
              _dev(pts, "pts"), _stream(q.device))
    return pts


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def occupancy_bwd(occ: Occupancy, x, g, s_fwd=None, want_w: bool = True, want_x: bool = True):
    """Hand-written backward of the occupancy at points x [dim][n].

    g is dL/ds (s_fwd None) or dL/dc (s_fwd = forward logits).  Returns
    (grad_w [M+1] or None, grad_x [dim][n] or None).
    """
    torch = _torch()
    lib = _lib.load()
    n = int(x.shape[1])
    gw = torch.empty(occ.n_hinges + 1, dtype=torch.float32, device=x.device) if want_w else None
    gx = torch.empty((occ.dim, n), dtype=torch.float32, device=x.device) if want_x else None
    wsb = lib.pdmp_bwd_workspace_size(occ.dim, occ.n_hinges, n)
    ws = _workspace(wsb, x.device)
    o = occ.c_struct()
    _lib.call("pdmp_occupancy_bwd", C.byref(o), _dev(x, "x", torch.float32, (occ.dim, n)), n,
              _dev(g, "g", torch.float32, (n,)),
              _dev(s_fwd, "s_fwd", torch.float32, (n,)) if s_fwd is not None else None,
              _dev(gw, "grad_w") if want_w else None, _dev(gx, "grad_x") if want_x else None,
              _dev(ws, "ws"), ws.numel(), _stream(x.device))
    return gw, gx


def occupancy_bwd_noalloc(occ: Occupancy, x, g, s_fwd=None, grad_w=None, grad_x=None):
    """The backward of occupancy_bwd through the allocation-free entry point: the
    library's static per-GPU scratch instead of a workspace.  The caller passes the
    outputs it wants (grad_w [M+1], grad_x [dim][n], device FP32, written in place) so
    that the call itself allocates nothing; returns them."""
    torch = _torch()
    n = int(x.shape[1])
    o = occ.c_struct()
    _lib.call("pdmp_occupancy_bwd_noalloc", C.byref(o),
              _dev(x, "x", torch.float32, (occ.dim, n)), n, _dev(g, "g", torch.float32, (n,)),
              _dev(s_fwd, "s_fwd", torch.float32, (n,)) if s_fwd is not None else None,
              _dev(grad_w, "grad_w", torch.float32, (occ.n_hinges + 1,))
              if grad_w is not None else None,
              _dev(grad_x, "grad_x", torch.float32, (occ.dim, n)) if grad_x is not None else None,
              _stream(x.device))
    return grad_w, grad_x


def bce_logits(s, y, g_scale=None, want_loss: bool = True, want_grad: bool = True):
    """(mean BCE loss [1], dL/ds [n]) of logits s against uint8 labels y; the gradient
    is multiplied by g_scale (a device tensor of one element) when given.  Outputs not
    wanted are returned as None."""
    torch = _torch()
    lib = _lib.load()
    n = int(s.shape[0])
    loss = torch.empty(1, dtype=torch.float32, device=s.device) if want_loss else None
    g = torch.empty(n, dtype=torch.float32, device=s.device) if want_grad else None
    sc = None
    if g_scale is not None:
        sc = _dev(g_scale.reshape(1), "g_scale", torch.float32, (1,))
    ws = _workspace(lib.pdmp_bce_workspace_size(n), s.device)
    _lib.call("pdmp_bce_logits", _dev(s, "s", torch.float32), _dev(y, "y", torch.uint8, (n,)), n,
              sc, _dev(loss, "loss") if want_loss else None, _dev(g, "g") if want_grad else None,
              _dev(ws, "ws"), ws.numel(), _stream(s.device))
    return loss, g


def adam_step(p, g, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, l2=0.0,
              n_decay=None):
    """One in-place Adam update of flat FP32 device tensors (Kingma & Ba 2015, Alg. 1)."""
    torch = _torch()
    n = int(p.numel())
    nd = n if n_decay is None else int(n_decay)
    _lib.call("pdmp_adam_step", _dev(p, "p", torch.float32), _dev(g, "g", torch.float32, p.shape),
              _dev(m, "m", torch.float32, p.shape), _dev(v, "v", torch.float32, p.shape), n, nd,
              int(t), float(lr), float(beta1), float(beta2), float(eps), float(l2),
              _stream(p.device))


def fit_occupancy(hinges, lengthscale: float, weights, pts, labels, steps: int, lr: float,
                  l2: float, optimizer: str = "gd", lr_bias=None, beta1=0.9, beta2=0.999,
                  eps=1e-8, adam_m=None, adam_v=None, t0: int = 0, record_loss: bool = True,
                  grid=None):
    """Full-batch occupancy fit on the GPU (Sec. 3.1); updates `weights` in place.

    Returns the per-step loss tensor [steps] (device) or None.
    """
    torch = _torch()
    lib = _lib.load()
    dim, M = int(hinges.shape[0]), int(hinges.shape[1])
    n = int(pts.shape[1])
    occ = Occupancy(hinges, weights, lengthscale, grid=grid)
    o = occ.c_struct()
    opt = _lib.pdmp_fit_opts()
    opt.optimizer = 0 if optimizer == "gd" else 1
    opt.steps = int(steps)
    opt.lr = float(lr)
    opt.lr_bias = float(lr if lr_bias is None else lr_bias)
    opt.l2 = float(l2)
    opt.beta1, opt.beta2, opt.eps = float(beta1), float(beta2), float(eps)
    opt.t0 = int(t0)
    if opt.optimizer == 1:
        if adam_m is None or adam_v is None:
            raise ValueError("Adam needs adam_m and adam_v state tensors [M+1]")
        opt.adam_m = _dev(adam_m, "adam_m", torch.float32, (M + 1,)).value
        opt.adam_v = _dev(adam_v, "adam_v", torch.float32, (M + 1,)).value
    loss = torch.empty(max(steps, 1), dtype=torch.float32, device=pts.device) if record_loss else None
    ws = _workspace(lib.pdmp_fit_workspace_size(dim, M, n), pts.device)
    _lib.call("pdmp_fit_occupancy", C.byref(o), _dev(weights, "weights", torch.float32, (M + 1,)),
              _dev(pts, "pts", torch.float32, (dim, n)), _dev(labels, "labels", torch.uint8, (n,)),
              n, C.byref(opt), _dev(loss, "loss") if record_loss else None, _dev(ws, "ws"),
              ws.numel(), _stream(pts.device))
    return loss[:steps] if record_loss else None


class Mlp:
    """Residual MLP q_hat = q + f(q) on BF16 MFMA (the amortised morph's network).

    Holds FP32 master parameters (flat, per layer W [out][in] then b [out]) and
    their BF16 copy; `widths` = (n_in, hidden, ..., hidden, n_in).
    """

    def __init__(self, widths, params=None, device="cuda"):
        torch = _torch()
        widths = tuple(int(w) for w in widths)
        if len(widths) < 3 or widths[0] != widths[-1] or len(set(widths[1:-1])) != 1:
            raise ValueError("widths must be (n, h, ..., h, n)")
        self.widths = widths
        self.n_in, self.hidden, self.n_hidden = widths[0], widths[1], len(widths) - 2
        n = sum(widths[l + 1] * widths[l] + widths[l + 1] for l in range(len(widths) - 1))
        self.params = (torch.zeros(n, dtype=torch.float32, device=device) if params is None
                       else params.to(device=device, dtype=torch.float32).contiguous())
        if self.params.numel() != n:
            raise ValueError(f"expected {n} parameters, got {self.params.numel()}")
        self.params_bf16 = torch.empty(n, dtype=torch.int16, device=device)
        self.pack()

    @classmethod
    def from_layers(cls, layers, device="cuda"):
        import numpy as np
        torch = _torch()
        widths = [layers[0][0].shape[1]] + [W.shape[0] for W, _ in layers]
        flat = np.concatenate([np.concatenate([np.asarray(W, np.float32).reshape(-1),
                                               np.asarray(b, np.float32).reshape(-1)])
                               for W, b in layers])
        return cls(widths, torch.from_numpy(flat), device)

    @property
    def num_params(self):
        return int(self.params.numel())

    def c_struct(self) -> _lib.pdmp_mlp:
        return _lib.pdmp_mlp(self.n_in, self.hidden, self.n_hidden, self.params.data_ptr(),
                             self.params_bf16.data_ptr())

    def pack(self):
        """Refresh the BF16 copy from the FP32 master parameters."""
        m = self.c_struct()
        _lib.call("pdmp_mlp_pack", C.byref(m), C.c_void_p(self.params_bf16.data_ptr()),
                  _stream(self.params.device))

    def forward(self, q, acts=None, out=None):
        """q_hat = q + f(q) for q [n_in][B]; `acts` (from acts_buffer) keeps activations."""
        torch = _torch()
        lib = _lib.load()
        B = int(q.shape[1])
        m = self.c_struct()
        if out is None:
            out = torch.empty_like(q)
        ws = None
        if acts is None:
            ws = _workspace(lib.pdmp_mlp_workspace_size(C.byref(m), B), q.device)
        _lib.call("pdmp_mlp_forward", C.byref(m), _dev(q, "q", torch.float32, (self.n_in, B)), B,
                  _dev(out, "q_hat", torch.float32, (self.n_in, B)),
                  _dev(acts, "acts") if acts is not None else None,
                  _dev(ws, "ws") if ws is not None else None, ws.numel() if ws is not None else 0,
                  _stream(q.device))
        return out

    def acts_buffer(self, B, device="cuda"):
        lib = _lib.load()
        m = self.c_struct()
        return _workspace(lib.pdmp_mlp_acts_size(C.byref(m), int(B)), device)

    def backward(self, q_hat, target, acts, grad=None, loss=None, ws=None, hard=None,
                 hard_weight: float = 1.0):
        """MSE loss and its parameter gradient (FP32 flat) from saved activations; with
        hard (uint8 [B]) the samples it marks weigh hard_weight in the loss."""
        torch = _torch()
        lib = _lib.load()
        B = int(q_hat.shape[1])
        m = self.c_struct()
        if grad is None:
            grad = torch.empty_like(self.params)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=q_hat.device)
        if ws is None:
            ws = _workspace(lib.pdmp_mlp_workspace_size(C.byref(m), B), q_hat.device)
        args = (_dev(acts, "acts"), _dev(grad, "grad", torch.float32, (self.num_params,)),
                _dev(loss, "loss"), _dev(ws, "ws"), ws.numel(), _stream(q_hat.device))
        qh = _dev(q_hat, "q_hat", torch.float32)
        tg = _dev(target, "target", torch.float32, tuple(q_hat.shape))
        if hard is None:
            _lib.call("pdmp_mlp_backward", C.byref(m), qh, tg, B, *args)
        else:
            _lib.call("pdmp_mlp_backward_weighted", C.byref(m), qh, tg, B,
                      _dev(hard, "hard", torch.uint8, (B,)), float(hard_weight), *args)
        return loss, grad


def arm_max_occupancy(occ: Occupancy, arm: Arm, q, thresh: float = 0.5):
    """(max body-point occupancy [n], flag [n]) of configurations q [n_dof][n]."""
    torch = _torch()
    n = int(q.shape[1])
    maxc = torch.empty(n, dtype=torch.float32, device=q.device)
    flag = torch.empty(n, dtype=torch.uint8, device=q.device)
    o, a = occ.c_struct(), arm.c_struct()
    _lib.call("pdmp_arm_max_occupancy", C.byref(o), C.byref(a),
              _dev(q, "q", torch.float32, (arm.n_dof, n)), n, float(thresh), _dev(maxc, "maxc"),
              _dev(flag, "flag"), _stream(q.device))
    return maxc, flag


def amortised_morph(mlp: Mlp, occ: Occupancy, arm: Arm, q, T: int, eta: float,
                    thresh: float = 0.5, out=None, flag=None, n_fallback=None, ws=None,
                    refine: bool = False):
    """Amortised morph: q + f(q), plain-morph fallback where max occupancy > thresh
    (T steps from q; with refine, T steps from q + f(q)).

    Returns (out [n_dof][n], flag [n] uint8, n_fallback [1] int32 device).
    """
    torch = _torch()
    lib = _lib.load()
    n = int(q.shape[1])
    m, o, a = mlp.c_struct(), occ.c_struct(), arm.c_struct()
    if out is None:
        out = torch.empty_like(q)
    if flag is None:
        flag = torch.empty(n, dtype=torch.uint8, device=q.device)
    if n_fallback is None:
        n_fallback = torch.zeros(1, dtype=torch.int32, device=q.device)
    if ws is None:
        ws = _workspace(lib.pdmp_amortised_workspace_size(C.byref(m), C.byref(a), n), q.device)
    _lib.call("pdmp_amortised_morph_refine" if refine else "pdmp_amortised_morph", C.byref(m),
              C.byref(o), C.byref(a),
              _dev(q, "q", torch.float32, (arm.n_dof, n)), _dev(out, "out", torch.float32, (arm.n_dof, n)),
              n, int(T), float(eta), float(thresh), _dev(flag, "flag", torch.uint8, (n,)),
              _dev(n_fallback, "n_fallback"), _dev(ws, "ws"), ws.numel(), _stream(q.device))
    return out, flag, n_fallback


# ------------------------------------------- the paper's tanh occupancy ---

class TanhNet:
    """The paper's occupancy network (Sec. 3.1): n_hidden tanh layers of width
    `hidden`, sigmoid output.  params: flat FP32 device tensor, per layer W_l
    [hidden][n_l] then b_l [hidden], and last v [hidden], b_o."""

    def __init__(self, dim: int, hidden: int, n_hidden: int, params):
        self.dim, self.hidden, self.n_hidden = int(dim), int(hidden), int(n_hidden)
        s = _lib.pdmp_tanh_net(self.dim, self.hidden, self.n_hidden, None)
        n = _lib.load().pdmp_tanh_num_params(C.byref(s))
        if n < 0:
            raise ValueError(f"unsupported network shape dim={dim} hidden={hidden} "
                             f"n_hidden={n_hidden}")
        self.params = params
        _dev(params, "params", _torch().float32, (n,))

    def c_struct(self):
        return _lib.pdmp_tanh_net(self.dim, self.hidden, self.n_hidden,
                                  C.c_void_p(self.params.data_ptr()))


def tanh_occupancy_eval(net: TanhNet, x):
    """(c, s) of the network at [dim][n] points."""
    torch = _torch()
    n = int(x.shape[1])
    c = torch.empty(n, dtype=torch.float32, device=x.device)
    s = torch.empty(n, dtype=torch.float32, device=x.device)
    o = net.c_struct()
    _lib.call("pdmp_tanh_occupancy_eval", C.byref(o), _dev(x, "x", torch.float32, (net.dim, n)),
              n, _dev(c, "c"), _dev(s, "s"), _stream(x.device))
    return c, s


def tanh_occupancy_grad(net: TanhNet, x):
    """(c, grad_x c) of the network at [dim][n] points."""
    torch = _torch()
    n = int(x.shape[1])
    c = torch.empty(n, dtype=torch.float32, device=x.device)
    g = torch.empty((net.dim, n), dtype=torch.float32, device=x.device)
    o = net.c_struct()
    _lib.call("pdmp_tanh_occupancy_grad", C.byref(o), _dev(x, "x", torch.float32, (net.dim, n)),
              n, _dev(c, "c"), _dev(g, "grad"), _stream(x.device))
    return c, g


def tanh_split_scheme(net: TanhNet):
    """(name, products per FP32 multiply-add) of the forward hidden-to-hidden products
    in the network's eval, gradient and morph kernels, as the library decides it from
    the weights: ("fp16", 3) or ("bf16", 6).  The backward products take ("bf16", 6)."""
    v = C.c_int32(-1)
    o = net.c_struct()
    _lib.call("pdmp_tanh_split_scheme", C.byref(o), C.byref(v), _stream(net.params.device))
    return SPLIT_SCHEMES[int(v.value)]


def tanh_morph_samples(net: TanhNet, x, T: int, eta: float, out=None):
    """Explicit-Euler morph (Eq. 1) of [dim][n] points with the network's occupancy."""
    torch = _torch()
    n = int(x.shape[1])
    _dev(x, "x", torch.float32, (net.dim, n))
    if out is None:
        out = torch.empty_like(x)
    o = net.c_struct()
    _lib.call("pdmp_tanh_morph_samples", C.byref(o), C.c_void_p(x.data_ptr()),
              _dev(out, "out", torch.float32, (net.dim, n)), n, int(T), float(eta),
              _stream(x.device))
    return out


def _tanh_ws(net: TanhNet, n: int, device):
    lib = _lib.load()
    o = net.c_struct()
    return _workspace(lib.pdmp_tanh_fit_workspace_size(C.byref(o), n), device)


def tanh_loss_grad(net: TanhNet, pts, labels, l2: float):
    """(loss [1], grad [num_params]) of the network's fit objective (Sec. 3.1):
    mean BCE over the labelled points + (l2/2) |weights|^2 (biases not decayed)."""
    torch = _torch()
    n = int(pts.shape[1])
    loss = torch.empty(1, dtype=torch.float32, device=pts.device)
    grad = torch.empty_like(net.params)
    ws = _tanh_ws(net, n, pts.device)
    o = net.c_struct()
    _lib.call("pdmp_tanh_loss_grad", C.byref(o), _dev(pts, "pts", torch.float32, (net.dim, n)),
              _dev(labels, "labels", torch.uint8, (n,)), n, float(l2), _dev(loss, "loss"),
              _dev(grad, "grad"), _dev(ws, "ws"), ws.numel(), _stream(pts.device))
    return loss, grad


def tanh_fit(net: TanhNet, pts, labels, steps: int, lr: float, l2: float, beta1=0.9,
             beta2=0.999, eps=1e-8, adam_m=None, adam_v=None, t0: int = 0,
             record_loss: bool = True):
    """Full-batch Adam fit of the network on the GPU (Sec. 3.1); updates net.params in
    place and returns the per-step loss tensor [steps] (device) or None."""
    torch = _torch()
    n = int(pts.shape[1])
    m = adam_m if adam_m is not None else torch.zeros_like(net.params)
    v = adam_v if adam_v is not None else torch.zeros_like(net.params)
    loss = torch.empty(max(steps, 1), dtype=torch.float32, device=pts.device) if record_loss \
        else None
    ws = _tanh_ws(net, n, pts.device)
    opts = _lib.pdmp_fit_opts(1, int(steps), float(lr), 0.0, float(l2), float(beta1),
                              float(beta2), float(eps), int(t0), _dev(m, "adam_m"),
                              _dev(v, "adam_v"))
    o = net.c_struct()
    _lib.call("pdmp_tanh_fit", C.byref(o), _dev(pts, "pts", torch.float32, (net.dim, n)),
              _dev(labels, "labels", torch.uint8, (n,)), n, C.byref(opts),
              _dev(loss, "loss") if loss is not None else None, _dev(ws, "ws"), ws.numel(),
              _stream(pts.device))
    return loss[:steps] if loss is not None else None


# ------------------------------------------ producer / consumer (Sec. 3.3) ---

class Bucket:
    """Host SPSC ring of samples (the concurrent bucket S); push/pop never block."""

    def __init__(self, dim: int, capacity: int):
        lib = _lib.load()
        self.dim = int(dim)
        h = C.c_void_p()
        _lib.call("pdmp_bucket_create", int(dim), int(capacity), C.byref(h))
        self._h = h
        self._lib = lib

    def push(self, x, start: int = 0, base_index: int = 0) -> int:
        """Push samples [start, n) of a contiguous float32 numpy array x [dim][n]."""
        import numpy as np
        x = np.ascontiguousarray(x, dtype=np.float32)
        n = x.shape[1]
        r = self._lib.pdmp_bucket_push(self._h, x.ctypes.data, n, int(start), n, int(base_index))
        if r < 0:
            raise ValueError("bad push arguments")
        return int(r)

    def pop(self):
        """(x [dim] float32, index) or None when empty."""
        import numpy as np
        x = np.zeros(self.dim, np.float32)
        idx = C.c_int64()
        r = self._lib.pdmp_bucket_pop(self._h, x.ctypes.data, C.byref(idx))
        return (x, idx.value) if r == 1 else None

    def size(self) -> int:
        return int(self._lib.pdmp_bucket_size(self._h))

    def close(self):
        if self._h:
            self._lib.pdmp_bucket_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sampler:
    """The background diffeomorphic sampler of Sec. 3.3: a producer thread keeps the
    bucket filled with morphed Philox prior batches; pop() never waits and falls back
    to the prior when the bucket is empty.  occ None gives a prior-only sampler."""

    def __init__(self, occ, dim: int, lo, hi, T: int, eta: float, batch: int, capacity: int,
                 seed: int, stream_id: int = 0, prior_stream_id: int = 0xFFFF):
        lib = _lib.load()
        o = _lib.pdmp_sampler_opts()
        o.dim, o.T, o.eta, o.batch, o.capacity = int(dim), int(T), float(eta), int(batch), \
            int(capacity)
        o.seed, o.stream_id, o.prior_stream_id = int(seed), int(stream_id), int(prior_stream_id)
        for k in range(int(dim)):
            o.lo[k], o.hi[k] = float(lo[k]), float(hi[k])
        self.dim = int(dim)
        self.occ = occ  # keeps the device buffers alive
        self._occ_struct = occ.c_struct() if occ is not None else None
        h = C.c_void_p()
        _lib.call("pdmp_sampler_create",
                  C.byref(self._occ_struct) if occ is not None else None, C.byref(o), C.byref(h))
        self._h = h
        self._lib = lib

    def start(self):
        _lib.call("pdmp_sampler_start", self._h)

    def pause(self, paused: bool = True):
        _lib.call("pdmp_sampler_pause", self._h, 1 if paused else 0)

    def pop(self, n: int):
        """(x [n][dim] float32, index [n] int64, from_bucket [n] uint8)."""
        import numpy as np
        x = np.zeros((n, self.dim), np.float32)
        idx = np.zeros(n, np.int64)
        fb = np.zeros(n, np.uint8)
        _lib.call("pdmp_sampler_pop", self._h, int(n), x.ctypes.data, idx.ctypes.data,
                  fb.ctypes.data)
        return x, idx, fb

    def stats(self) -> dict:
        """Counters of pdmp_sampler_stats; "error" holds the producer's message once
        its status is not PDMP_OK."""
        st = _lib.pdmp_sampler_stats()
        _lib.call("pdmp_sampler_get_stats", self._h, C.byref(st))
        out = {f: getattr(st, f) for f, _ in st._fields_}
        msg = self._lib.pdmp_last_error() if st.status != _lib.PDMP_OK else None
        out["error"] = msg.decode() if msg else ""
        return out

    def close(self) -> int:
        """Stop and join the producer; returns its status."""
        if not self._h:
            return 0
        r = self._lib.pdmp_sampler_destroy(self._h)
        self._h = None
        return int(r)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rrt_run(sampler: Sampler, start, goal, step: float, goal_tol: float, discs,
            max_iters: int, time_budget_s: float = 0.0):
    """The planner's main thread (a plane RRT, Sec. 3.3) drawing from `sampler`.

    discs: (centres [2][K] or [K][2], radii [K]) host arrays.  Returns a dict with the
    result fields and the arrays nodes, parent, samples, sample_from_bucket, t_sample."""
    import numpy as np
    cen, rad = discs
    cen = np.asarray(cen, np.float64)
    if cen.shape[0] != 2:
        cen = cen.T
    dx = np.ascontiguousarray(cen[0], np.float64)
    dy = np.ascontiguousarray(cen[1], np.float64)
    dr = np.ascontiguousarray(rad, np.float64)
    o = _lib.pdmp_rrt_opts()
    o.max_iters, o.step, o.goal_tol = int(max_iters), float(step), float(goal_tol)
    o.start[0], o.start[1] = float(start[0]), float(start[1])
    o.goal[0], o.goal[1] = float(goal[0]), float(goal[1])
    o.time_budget_s = float(time_budget_s)
    o.n_discs = int(dr.size)
    o.disc_x, o.disc_y, o.disc_r = dx.ctypes.data, dy.ctypes.data, dr.ctypes.data
    nodes = np.zeros((max_iters + 2, 2), np.float32)
    parent = np.zeros(max_iters + 2, np.int32)
    samples = np.zeros((max_iters, 2), np.float32)
    fb = np.zeros(max_iters, np.uint8)
    ts = np.zeros(max_iters, np.float64)
    res = _lib.pdmp_rrt_result()
    _lib.call("pdmp_rrt_run", sampler._h, C.byref(o), nodes.ctypes.data, parent.ctypes.data,
              samples.ctypes.data, fb.ctypes.data, ts.ctypes.data, C.byref(res))
    out = {f: getattr(res, f) for f, _ in res._fields_}
    k, m = res.iters, res.n_nodes
    out.update(nodes=nodes[:m], parent=parent[:m], samples=samples[:k], sample_from_bucket=fb[:k],
               t_sample=ts[:k])
    return out


# ----------------------------------------------- compact-support culling ---

def cull_grid(dim: int, lo, hi, cutoff: float):
    """The cell grid of the culled morph (cells of side >= cutoff on the box [lo, hi])."""
    g = _lib.pdmp_cull_grid()
    lo_a = (C.c_float * dim)(*[float(v) for v in lo])
    hi_a = (C.c_float * dim)(*[float(v) for v in hi])
    _lib.call("pdmp_cull_grid_make", int(dim), lo_a, hi_a, float(cutoff), C.byref(g))
    return g


def morph_culled(occ: Occupancy, grid, x, T: int, eta: float, out=None):
    """The workspace morph with compact-support hinge culling (3^dim cells per point)."""
    torch = _torch()
    lib = _lib.load()
    n = int(x.shape[1])
    _dev(x, "x", torch.float32, (occ.dim, n))
    if out is None:
        out = torch.empty_like(x)
    o = occ.c_struct()
    ws = _workspace(lib.pdmp_morph_culled_workspace_size(C.byref(o), C.byref(grid), n), x.device)
    _lib.call("pdmp_morph_culled", C.byref(o), C.byref(grid), C.c_void_p(x.data_ptr()),
              _dev(out, "out", torch.float32, (occ.dim, n)), n, int(T), float(eta), _dev(ws, "ws"),
              ws.numel(), _stream(x.device))
    return out
