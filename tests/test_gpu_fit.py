"""GPU parity: the hand-written occupancy backward, BCE, Adam and the fit (Sec. 3.1).

Tolerances (FP32 against FP64 on identical inputs):
  grad_w_j  |.| <= 1e-5 * sum_i |g_i| phi_ij            (the scale its rounding acts on)
  grad_x_i  |.|_inf <= 1e-5 * |g_i| l^-2 sum_j |w_j| phi_ij |x_i - h_j|  (+ the sigma''
            term of G_abs when chained through the occupancy)
  one fit step from identical state: |w' - w'_ref| <= 1e-5 * (lr * gscale + |w'|)
  (gradient descent); for Adam, the gradient's tolerance carried through the moments
  and the normalised step m_hat / (sqrt(v_hat) + eps) with their FP32 roundings
and the backward is also checked against central finite differences of the FP64
forward (h = 1e-3, Richardson-extrapolated, 1e-4 relative).
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import paper_2108_11775_amd as P
from paper_2108_11775_amd import configs as K, inputs as I

from helpers import arm_scene, dev, gpu_occ, host, oracle_occ, require_gpu, ws_scene

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _bwd_case(h, wb, ell, x, g, chain, grid=None, want_x=True):
    go, oo = gpu_occ(h, wb, ell, grid=grid), oracle_occ(h, wb, ell)
    M = h.shape[1]
    s_fwd = None
    if chain:
        _, s_d = P.occupancy_eval(go, dev(x))
        s_fwd = s_d
    gw, gx = P.occupancy_bwd(go, dev(x), dev(g), s_fwd=s_fwd, want_x=want_x)
    gw = host(gw)
    gx = host(gx) if want_x else None
    s_r, c_r, _ = O.occ_eval(oo, x)
    sp = c_r * (1 - c_r) if chain else np.ones_like(c_r)
    geff = g.astype(np.float64) * sp
    ref_w, ref_x = O.logit_bwd(h, wb[:-1], ell, x, geff)
    scale_w, _ = O.logit_bwd(h, wb[:-1], ell, x, np.abs(geff), want_x=False)
    # chaining also carries the FP32 error of s into sigma'(s): |sigma''| S_abs per point
    _, _, _, gabs, graw = O.occ_grad(oo, x, with_raw=True)
    _, _, sabs = O.occ_eval(oo, x)
    if chain:
        d2 = np.abs(c_r * (1 - c_r) * (1 - 2 * c_r))
        scale_w = scale_w + O.logit_bwd(h, wb[:-1], ell, x, np.abs(g) * d2 * sabs, want_x=False)[0]
        scale_x = np.abs(g) * gabs
    else:
        scale_x = np.abs(g) * graw
    assert np.all(np.abs(gw - ref_w) <= TOL * scale_w + 1e-30), np.max(np.abs(gw - ref_w) / scale_w)
    if not want_x:
        return gw, None
    err_x = np.abs(gx - ref_x).max(axis=0)
    assert np.all(err_x <= TOL * scale_x + 1e-30), np.max(err_x / scale_x)
    return gw, gx


@pytest.mark.parametrize("on_grid", [False, True])
@pytest.mark.parametrize("chain", [False, True])
def test_backward_2d(chain, on_grid):
    require_gpu()
    sc = ws_scene(K.C1)
    x = I.uniform_points(1, K.STREAM_EVAL, 2, 3001, -10, 10)
    g = I.rng(1, 9).normal(size=3001).astype(np.float32)
    grid = (K.C1.grid, K.C1.grid) if on_grid else None
    _bwd_case(sc["h"], sc["wb"], sc["ell"], x, g, chain, grid=grid)


@pytest.mark.parametrize("on_grid", [False, True])
@pytest.mark.parametrize("chain", [False, True])
def test_backward_3d(chain, on_grid):
    require_gpu()
    sc = arm_scene()
    x = I.uniform_points(4, K.STREAM_EVAL, 3, 5001, -1, 1)
    g = I.rng(4, 9).normal(size=5001).astype(np.float32)
    grid = (K.C3.grid,) * 3 if on_grid else None
    _bwd_case(sc["h"], sc["wb"], sc["ell"], x, g, chain, grid=grid)


def _ragged_grid(shape, seed):
    """Hinges on a tensor grid with unequal, unevenly spaced axes (x fastest)."""
    rng = np.random.default_rng(seed)
    axes = [np.sort(rng.uniform(-1.5, 1.5, k)) for k in shape]
    j = np.arange(int(np.prod(shape)))
    idx, stride = [], 1
    for k in shape:
        idx.append((j // stride) % k)
        stride *= k
    h = np.stack([axes[d][idx[d]] for d in range(len(shape))]).astype(np.float32)
    wb = rng.normal(0, 1.0, h.shape[1] + 1).astype(np.float32)
    return h, wb, rng


# grids that fill and that pad the MFMA tiles; n spans one partial round, several
# rounds per block (n > 512 * 256) and ragged tails
@pytest.mark.parametrize("shape,n", [((64, 64), 140001), ((37, 50), 70001), ((5, 3), 1),
                                     ((33, 20), 257), ((16, 16, 16), 140001), ((5, 7, 3), 255),
                                     ((16, 9, 11), 3001), ((1, 16, 16), 512)])
def test_grid_weight_gradient_shapes(shape, n):
    require_gpu()
    h, wb, rng = _ragged_grid(shape, 31 * n + len(shape))
    x = rng.uniform(-1.8, 1.8, (len(shape), n)).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    _bwd_case(h, wb, 0.3, x, g, False, grid=shape, want_x=False)


def test_grid_weight_gradient_deterministic():
    require_gpu()
    sc = arm_scene()
    x = I.uniform_points(4, K.STREAM_EVAL, 3, 200003, -1, 1)
    g = I.rng(4, 13).normal(size=200003).astype(np.float32)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"], grid=(16, 16, 16))
    a, _ = P.occupancy_bwd(go, dev(x), dev(g), want_x=False)
    b, _ = P.occupancy_bwd(go, dev(x), dev(g), want_x=False)
    assert np.array_equal(host(a), host(b))


def test_backward_against_finite_differences():
    require_gpu()
    sc = arm_scene()
    h, wb, ell = sc["h"], sc["wb"], sc["ell"]
    M = h.shape[1]
    x = I.uniform_points(4, K.STREAM_EVAL, 3, 64, -0.8, 0.8)
    g = I.rng(4, 10).normal(size=64).astype(np.float32)
    gw, gx = P.occupancy_bwd(gpu_occ(h, wb, ell), dev(x), dev(g))
    gw, gx = host(gw), host(gx)
    f = lambda xx: float(g.astype(np.float64) @ O.occ_eval(oracle_occ(h, wb, ell), xx)[0])
    # d/dx: per point, central differences of the FP64 forward, h = 1e-3, Richardson
    for i in (0, 17, 63):
        for k in range(3):
            def F(d):
                xx = x.astype(np.float64).copy()
                xx[k, i] += d
                return f(xx)
            d1 = (F(2e-3) - F(-2e-3)) / 4e-3
            d2 = (F(1e-3) - F(-1e-3)) / 2e-3
            fd = (4 * d2 - d1) / 3
            assert abs(gx[k, i] - fd) <= 1e-4 * max(abs(fd), np.abs(gx[:, i]).max()) + 1e-6
    # d/dw: the logit is linear in w, so a difference quotient is exact up to rounding
    for j in (0, 1234, M - 1, M):
        def W(d):
            w2 = wb.astype(np.float64).copy()
            w2[j] += d
            return float(g.astype(np.float64) @ O.occ_eval(O.Occupancy(h, w2[:-1], w2[-1], ell), x)[0])
        fd = (W(1e-3) - W(-1e-3)) / 2e-3
        assert abs(gw[j] - fd) <= 1e-4 * max(abs(fd), 1e-3)


@pytest.mark.parametrize("on_grid", [False, True])
def test_backward_full_size_sampled(on_grid):
    """d/dw at the 2^20-point, 4096-hinge size of the 3-D fit, on sampled hinges."""
    require_gpu()
    sc = arm_scene()
    h, wb, ell = sc["h"], sc["wb"], sc["ell"]
    n = K.C4.n_points
    x = I.uniform_points(K.C4.cfg_id, K.STREAM_FIT, 3, n, -1, 1)
    g = (I.rng(4, 11).normal(size=n) / n).astype(np.float32)
    grid = (16, 16, 16) if on_grid else None
    gw, _ = P.occupancy_bwd(gpu_occ(h, wb, ell, grid=grid), dev(x), dev(g), want_x=False)
    gw = host(gw)
    js = np.r_[0, 1, 777, 2048, 4095]
    ref, scale = O.logit_bwd_w_subset(h, ell, x, g, js)
    assert np.all(np.abs(gw[js] - ref) <= TOL * scale), np.max(np.abs(gw[js] - ref) / scale)
    assert abs(gw[-1] - g.astype(np.float64).sum()) <= TOL * np.abs(g).sum()


def test_bce_and_adam():
    require_gpu()
    rng = I.rng(9, 1)
    s = rng.normal(0, 4, 100003).astype(np.float32)
    s[:3] = [0.0, 60.0, -60.0]
    y = (rng.uniform(size=s.size) < 0.3).astype(np.uint8)
    loss, g = P.bce_logits(dev(s), dev(y))
    L, gr = O.bce_logits(s, y)
    assert abs(host(loss)[0] - L) <= 1e-6 * abs(L)
    assert np.abs(host(g) - gr).max() <= 1e-6 / s.size
    # an upstream gradient scales dL/ds inside the kernel: one more FP32 rounding
    sc = np.float32(-2.7182817)
    _, g2 = P.bce_logits(dev(s), dev(y), g_scale=dev(np.array([sc], np.float32)),
                         want_loss=False)
    assert np.array_equal(host(g2), host(g) * sc)
    p0 = rng.normal(size=5000).astype(np.float32)
    gg = rng.normal(size=5000).astype(np.float32)
    m0 = rng.normal(0, 0.1, 5000).astype(np.float32)
    v0 = rng.uniform(0, 0.1, 5000).astype(np.float32)
    # the kernel receives FP32 hyperparameters; the oracle gets the same values
    lr, b1, b2, eps, l2 = (float(np.float32(v)) for v in (1e-2, 0.9, 0.999, 1e-8, 1e-3))
    p, m, v = dev(p0), dev(m0), dev(v0)
    P.adam_step(p, dev(gg), m, v, 7, lr, b1, b2, eps, l2=l2, n_decay=4000)
    pr, mr, vr = p0.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64)
    ge = gg.astype(np.float64)
    ge[:4000] += l2 * pr[:4000]
    O.adam_step(pr, ge, mr, vr, 7, lr, b1, b2, eps)
    e32 = 2.0 ** -23
    assert np.all(np.abs(host(m) - mr) <= 4 * e32 * (b1 * np.abs(m0) + (1 - b1) * np.abs(ge)))
    assert np.all(np.abs(host(v) - vr) <= 4 * e32 * (b2 * np.abs(v0) + (1 - b2) * ge * ge))
    assert np.all(np.abs(host(p) - pr) <= 4 * e32 * np.abs(pr) + 1e-5 * lr)


def _fit_problem_2d():
    cfg = K.C1
    sc = ws_scene(cfg)
    pts = I.uniform_points(cfg.cfg_id, K.STREAM_FIT, 2, cfg.fit_points, cfg.lo, cfg.hi)
    dc, dr = sc["discs"]
    y = O.label_discs(dc, dr, pts)
    return cfg, sc, pts, y


@pytest.mark.parametrize("on_grid", [False, True])
def test_fit_one_step_from_identical_state(on_grid):
    require_gpu()
    cfg, sc, pts, y = _fit_problem_2d()
    wb = sc["wb"]
    M = wb.size - 1
    w_d = dev(wb.copy())
    loss = P.fit_occupancy(dev(sc["h"]), sc["ell"], w_d, dev(pts), dev(y), 1, cfg.fit_lr,
                           cfg.fit_l2, "gd", lr_bias=cfg.fit_lr_bias,
                           grid=(cfg.grid, cfg.grid) if on_grid else None)
    L, g, gsc = O.fit_loss_grad(sc["h"], sc["ell"], wb, pts, y, cfg.fit_l2)
    ref = wb.astype(np.float64).copy()
    ref[:M] -= cfg.fit_lr * g[:M]
    ref[M] -= cfg.fit_lr_bias * g[M]
    lr = np.full(M + 1, cfg.fit_lr)
    lr[M] = cfg.fit_lr_bias
    got = host(w_d)
    assert np.all(np.abs(got - ref) <= TOL * (lr * gsc + np.abs(ref))), \
        np.max(np.abs(got - ref) / (lr * gsc + np.abs(ref)))
    assert abs(host(loss)[0] - L) <= 1e-6 * L


@pytest.mark.parametrize("on_grid", [False, True])
def test_fit_adam_one_step_from_identical_state(on_grid):
    require_gpu()
    sc = arm_scene()
    c4 = K.C4
    pts = I.uniform_points(c4.cfg_id, K.STREAM_FIT, 3, 20000, -1, 1)
    bc, be = sc["boxes"]
    y = O.label_boxes(bc, be, pts)
    wb = sc["wb"]
    M = wb.size - 1
    rng = I.rng(4, 12)
    m0 = (rng.normal(size=M + 1) * 1e-3).astype(np.float32)
    v0 = (rng.uniform(size=M + 1) * 1e-5).astype(np.float32)
    w_d, m_d, v_d = dev(wb.copy()), dev(m0), dev(v0)
    # the kernels receive FP32 hyperparameters; the oracle gets the same values
    lr, l2, b1, b2, eps = (float(np.float32(v)) for v in (c4.lr, c4.l2, 0.9, 0.999, 1e-8))
    P.fit_occupancy(dev(sc["h"]), sc["ell"], w_d, dev(pts), dev(y), 1, lr, l2, "adam",
                    beta1=b1, beta2=b2, eps=eps, adam_m=m_d, adam_v=v_d, t0=9,
                    grid=(16, 16, 16) if on_grid else None)
    ref, mr, vr, _ = O.fit(sc["h"], sc["ell"], pts, y, 1, 1, lr, l2, b1=b1, b2=b2, eps=eps,
                           wb0=wb, m=m0, v=v0, t0=9)
    _, g, gsc = O.fit_loss_grad(sc["h"], sc["ell"], wb, pts, y, l2)
    assert np.all(np.abs(host(m_d) - mr) <= TOL * (0.1 * gsc + np.abs(mr)) + 1e-12)
    bound = _adam_step_bound(g, gsc, m0, v0, wb, 10, lr, b1, b2, eps)
    err = np.abs(host(w_d) - ref)
    assert np.all(err <= bound), float(np.max(err / bound))


def _adam_step_bound(g, gsc, m0, v0, w, t, lr, b1, b2, eps, tol=TOL):
    """Per parameter: how far one Adam update (Kingma & Ba, Alg. 1) from identical
    state may move on the GPU from the FP64 oracle's, given the gradient's tolerance
    tol * gsc.  The gradient error passes through the moments m and v (with a few FP32
    roundings of each) into r = m_hat / (sqrt(v_hat) + eps); the step is lr r, added
    to w with one more rounding.  A factor 2 covers the bound's own first-order terms."""
    u = 2.0 ** -24
    g, gsc = np.asarray(g, np.float64), np.asarray(gsc, np.float64)
    m0, v0, w = (np.asarray(a, np.float64) for a in (m0, v0, w))
    bc1, bc2 = 1.0 / (1.0 - b1 ** t), 1.0 / (1.0 - b2 ** t)
    dg = tol * gsc
    m1 = b1 * m0 + (1 - b1) * g
    v1 = b2 * v0 + (1 - b2) * g * g
    mh, vh = m1 * bc1, v1 * bc2
    dm = ((1 - b1) * dg + 4 * u * (b1 * np.abs(m0) + (1 - b1) * np.abs(g))) * bc1 + 2 * u * np.abs(mh)
    dv = ((1 - b2) * (2 * np.abs(g) * dg + dg * dg) + 4 * u * (b2 * v0 + (1 - b2) * g * g)) * bc2 \
        + 2 * u * vh
    sv = np.sqrt(vh)
    dsv = np.where(sv > 0, np.minimum(dv / np.maximum(2 * sv, 1e-300), np.sqrt(dv)), np.sqrt(dv))
    den = sv + eps
    r = np.abs(mh) / den
    dr = dm / den + np.abs(mh) * dsv / (den * (den - dsv).clip(min=eps)) + 6 * u * r
    return 2.0 * (lr * dr + 2 * u * (np.abs(w) + lr * r))


def test_fit_gd_trajectory_config1():
    require_gpu()
    cfg, sc, pts, y = _fit_problem_2d()
    M = sc["h"].shape[1]
    w_d = dev(np.zeros(M + 1, np.float32))
    loss = host(P.fit_occupancy(dev(sc["h"]), sc["ell"], w_d, dev(pts), dev(y), cfg.fit_steps,
                                cfg.fit_lr, cfg.fit_l2, "gd", lr_bias=cfg.fit_lr_bias))
    ref = np.load(__import__("os").path.join(__import__("helpers").GOLDEN, "ws2d_4096.npy"))
    _, _, _, lref = O.fit(sc["h"], sc["ell"], pts, y, 0, 20, cfg.fit_lr, cfg.fit_l2,
                          lr_bias=cfg.fit_lr_bias)
    np.testing.assert_allclose(loss[:20], lref, rtol=1e-4)
    got = host(w_d)
    # end-to-end drift over 200 steps: report-level agreement with the FP64 fit
    assert np.abs(got - ref).max() <= 1e-2 * np.abs(ref).max()
    assert loss[-1] < 0.5 * loss[0]


def test_autograd_drives_the_fit_gradient():
    require_gpu()
    import torch
    from paper_2108_11775_amd.autograd import OccupancyLogit, Occupancy as OccC, BCEWithLogits
    cfg, sc, pts, y = _fit_problem_2d()
    M = sc["h"].shape[1]
    wb = sc["wb"]
    w = dev(wb.copy()).requires_grad_(True)
    h_d, x_d, y_d = dev(sc["h"]), dev(pts), dev(y)
    s = OccupancyLogit.apply(x_d, w, h_d, sc["ell"])
    loss = BCEWithLogits.apply(s, y_d) + 0.5 * cfg.fit_l2 * (w[:M] ** 2).sum()
    loss.backward()
    L, g, gsc = O.fit_loss_grad(sc["h"], sc["ell"], wb, pts, y, cfg.fit_l2)
    assert abs(loss.item() - L) <= 1e-6 * L
    assert np.all(np.abs(host(w.grad) - g) <= TOL * gsc + 1e-12)
    # occupancy form: d/dx of sum c through the chained kernel
    x2 = dev(pts[:, :500].copy()).requires_grad_(True)
    c = OccC.apply(x2, w.detach(), h_d, sc["ell"])
    c.sum().backward()
    oo = oracle_occ(sc["h"], wb, sc["ell"])
    _, gc, _, gabs = O.occ_grad(oo, pts[:, :500])
    assert np.all(np.abs(host(x2.grad) - gc).max(axis=0) <= TOL * gabs)


def test_fit3d_reduced_trajectory():
    """The 3-D fit of config 4 reduced to 65,536 points (Sec. 3.1): all 500 Adam steps on
    the GPU's 16^3 grid path, from w = 0, against the oracle's FP64 fit of the same
    inputs (tests/golden/fit3d_65536.npz, written by make_fit3d_reduced.py).  The loss
    before every step agrees to 1e-5 relative; the final weights' drift
    max|w_gpu - w|/max|w| is reported (no a-priori bound: where a gradient is near zero,
    Adam's normalised step is ill-conditioned and FP32 errors may change its sign)."""
    require_gpu()
    import sys
    from helpers import GOLDEN
    sys.path.insert(0, GOLDEN)
    import make_fit3d_reduced as MF
    h, ell, pts, y = MF.problem()
    hp = MF.hyper()
    ref = np.load(os.path.join(GOLDEN, "fit3d_65536.npz"))
    M = h.shape[1]
    w_d = dev(np.zeros(M + 1, np.float32))
    m_d, v_d = dev(np.zeros(M + 1, np.float32)), dev(np.zeros(M + 1, np.float32))
    loss = host(P.fit_occupancy(dev(h.astype(np.float32)), ell, w_d, dev(pts.astype(np.float32)),
                                dev(y), K.C4.steps, hp["lr"], hp["l2"], "adam", beta1=hp["b1"],
                                beta2=hp["b2"], eps=hp["eps"], adam_m=m_d, adam_v=v_d,
                                grid=(16, 16, 16)))
    rel = np.abs(loss - ref["loss"]) / ref["loss"]
    drift = float(np.abs(host(w_d) - ref["wb"]).max() / np.abs(ref["wb"]).max())
    print(f"\n[fit3d reduced] loss {ref['loss'][0]:.6f} -> {ref['loss'][-1]:.6f}; "
          f"max rel loss diff {rel.max():.3e} (step {int(rel.argmax())}); "
          f"weight drift max|dw|/max|w| {drift:.3e}", flush=True)
    assert rel.max() <= 1e-5, (float(rel.max()), int(rel.argmax()))
    assert drift <= 1e-2
