"""Pins of the oracle's tanh-network occupancy (Sec. 3.1) to closed forms, finite
differences, symmetry and the BCE definition -- nothing here re-calls the oracle's
own chain-rule code to check itself."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2108_11775_amd import configs as K, inputs as I


def _net(dim, H, L, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    n = O.tanh_nparams(dim, H, L)
    return O.TanhNet(dim, H, L, rng.normal(0, scale, n))


def test_nparams_and_layout():
    assert O.tanh_nparams(2, 64, 3) == 64 * 2 + 64 + 2 * (64 * 64 + 64) + 64 + 1
    net = _net(3, 5, 2, 0)
    layers, (v, bo) = O.tanh_layers(net)
    assert [W.shape for W, _ in layers] == [(5, 3), (5, 5)]
    assert v.shape == (5,) and np.ndim(bo) == 0
    assert I.tanh_init(1, 2, 64, 3, 10.0).size == O.tanh_nparams(2, 64, 3)


def test_one_unit_closed_form():
    # s = v tanh(a.x + b) + b_o, grad s = v (1 - tanh^2) a
    a1, a2, b, v, bo = 0.7, -1.3, 0.2, 2.5, -0.4
    net = O.TanhNet(2, 1, 1, np.array([a1, a2, b, v, bo]))
    x = np.array([[0.3, -1.0, 2.0], [0.5, 0.25, -0.75]])
    s, gs, gc, _, _ = O.tanh_grad(net, x)
    for i in range(3):
        t = math.tanh(a1 * x[0, i] + a2 * x[1, i] + b)
        assert abs(s[i] - (v * t + bo)) <= 1e-15
        assert abs(gs[0, i] - v * (1 - t * t) * a1) <= 1e-15
        assert abs(gs[1, i] - v * (1 - t * t) * a2) <= 1e-15
        c = 1 / (1 + math.exp(-(v * t + bo)))
        assert abs(gc[0, i] - c * (1 - c) * v * (1 - t * t) * a1) <= 1e-15


def test_two_layers_one_unit_closed_form():
    # s = v tanh(w tanh(a.x + b0) + b1) + b_o
    a, b0, w, b1, v, bo = (0.4, -0.9, 0.1), 0.3, -1.7, 0.05, 1.1, 0.2
    net = O.TanhNet(3, 1, 2, np.array([*a, b0, w, b1, v, bo]))
    x = np.array([[0.5], [-0.2], [1.5]])
    s, gs, _, _, _ = O.tanh_grad(net, x)
    z1 = sum(ai * xi for ai, xi in zip(a, x[:, 0])) + b0
    t1 = math.tanh(z1)
    t2 = math.tanh(w * t1 + b1)
    assert abs(s[0] - (v * t2 + bo)) <= 1e-15
    for k in range(3):
        assert abs(gs[k, 0] - v * (1 - t2 * t2) * w * (1 - t1 * t1) * a[k]) <= 1e-15


@pytest.mark.parametrize("dim,H,L", [(2, 16, 3), (3, 8, 4), (2, 7, 1)])
def test_gradient_matches_finite_differences(dim, H, L):
    net = _net(dim, H, L, 10 * dim + L, scale=0.8)
    x = np.random.default_rng(1).uniform(-1.5, 1.5, (dim, 20))
    _, gs, _, _, _ = O.tanh_grad(net, x)
    for k in range(dim):
        def S(d):
            xx = x.copy()
            xx[k] += d
            return O.tanh_eval(net, xx)[0]
        d1 = (S(2e-4) - S(-2e-4)) / 4e-4
        d2 = (S(1e-4) - S(-1e-4)) / 2e-4
        fd = (4 * d2 - d1) / 3
        assert np.all(np.abs(gs[k] - fd) <= 1e-8 * (1 + np.abs(fd)))


def test_zero_network_is_constant_and_morph_is_identity():
    net = O.TanhNet(2, 6, 2, np.zeros(O.tanh_nparams(2, 6, 2)))
    net.P[-1] = 0.8
    x = np.random.default_rng(2).uniform(-3, 3, (2, 50))
    s, gs, gc, _, _ = O.tanh_grad(net, x)
    assert np.all(s == 0.8) and np.all(gs == 0) and np.all(gc == 0)
    assert np.array_equal(O.tanh_morph(net, x, 10, 0.1), x)


def test_odd_symmetry_without_biases():
    net = _net(2, 9, 3, 5)
    layers, (v, bo) = O.tanh_layers(net)
    for _, b in layers:
        b[:] = 0
    x = np.random.default_rng(3).uniform(-2, 2, (2, 40))
    s_p, g_p, _, _, _ = O.tanh_grad(net, x)
    s_m, g_m, _, _, _ = O.tanh_grad(net, -x)
    assert np.allclose(s_p - bo, -(s_m - bo), rtol=0, atol=1e-14)
    assert np.allclose(g_p, g_m, rtol=0, atol=1e-14)


def test_morph_one_dimensional_recursion():
    # W_0 = (a, 0): the y coordinate never moves and x follows a scalar recursion.
    a, b, v, bo, eta, T = 1.2, -0.3, 3.0, -1.0, 0.05, 25
    net = O.TanhNet(2, 1, 1, np.array([a, 0.0, b, v, bo]))
    x0 = np.array([[-1.0, 0.1, 0.6, 2.0], [0.3, -0.7, 5.0, 0.0]])
    out = O.tanh_morph(net, x0, T, eta)
    for i in range(x0.shape[1]):
        x = x0[0, i]
        for _ in range(T):
            t = math.tanh(a * x + b)
            c = 1 / (1 + math.exp(-(v * t + bo)))
            x = x - eta * c * (1 - c) * v * (1 - t * t) * a
        assert abs(out[0, i] - x) <= 1e-13
        assert out[1, i] == x0[1, i]


def test_morph_diag_amplification_is_one_for_flat_cost():
    net = O.TanhNet(2, 3, 1, np.zeros(O.tanh_nparams(2, 3, 1)))
    _, amp = O.tanh_morph(net, np.zeros((2, 4)), 5, 0.1, diag=True)
    assert np.allclose(amp, 1.0)


def test_loss_is_the_bce_definition():
    net = _net(2, 5, 2, 7)
    rng = np.random.default_rng(8)
    pts = rng.uniform(-2, 2, (2, 300))
    y = (rng.uniform(size=300) < 0.4).astype(np.uint8)
    l2 = 0.03
    loss, _ = O.tanh_loss_grad(net, pts, y, l2)
    _, c, _ = O.tanh_eval(net, pts)
    bce = -np.mean(y * np.log(c) + (1 - y) * np.log(1 - c))
    layers, (v, _) = O.tanh_layers(net)
    wsq = sum(float(np.sum(W * W)) for W, _ in layers) + float(np.sum(v * v))
    assert abs(loss - (bce + 0.5 * l2 * wsq)) <= 1e-12 * loss


@pytest.mark.parametrize("dim,H,L", [(2, 5, 2), (3, 4, 3)])
def test_loss_gradient_matches_finite_differences(dim, H, L):
    net = _net(dim, H, L, 11 + L)
    rng = np.random.default_rng(12)
    pts = rng.uniform(-2, 2, (dim, 60))
    y = (rng.uniform(size=60) < 0.5).astype(np.uint8)
    l2 = 0.01
    _, g = O.tanh_loss_grad(net, pts, y, l2)
    P = net.P.copy()
    for j in range(P.size):
        def F(d):
            Q = P.copy()
            Q[j] += d
            return O.tanh_loss_grad(O.TanhNet(dim, H, L, Q), pts, y, l2)[0]
        d1 = (F(2e-5) - F(-2e-5)) / 4e-5
        d2 = (F(1e-5) - F(-1e-5)) / 2e-5
        fd = (4 * d2 - d1) / 3
        assert abs(g[j] - fd) <= 1e-7 * (1 + abs(fd)), j


def test_fit_reduces_the_loss():
    cfg = K.C1
    dc, dr = I.discs(cfg.cfg_id, cfg.n_discs, cfg.lo, cfg.hi, cfg.r_min, cfg.r_max)
    pts = I.uniform_points(cfg.cfg_id, K.STREAM_FIT, 2, 2000, cfg.lo, cfg.hi)
    y = O.label_discs(dc, dr, pts)
    net = O.TanhNet(2, 8, 2, I.tanh_init(1, 2, 8, 2, cfg.hi).astype(np.float64))
    _, losses = O.tanh_fit(net, pts, y, 40, 1e-2, 1e-5)
    assert losses[-1] < 0.8 * losses[0]


def test_error_scale_bounds_a_float32_evaluation():
    """A plain float32 evaluation stays within 1e-5 S_abs and 1e-5 G_abs of FP64."""
    net = _net(2, 32, 3, 21, scale=0.5)
    x = np.random.default_rng(22).uniform(-3, 3, (2, 500))
    s64, g64, _, sabs, gabs = O.tanh_grad(net, x)
    layers, (v, bo) = O.tanh_layers(net)
    f32 = np.float32
    a = x.astype(f32)
    acts, ds = [], []
    for W, b in layers:
        a = np.tanh(W.astype(f32) @ a + b.astype(f32)[:, None]).astype(f32)
        acts.append(a)
        ds.append((1 - a * a).astype(f32))
    s32 = v.astype(f32) @ a + f32(bo)
    assert np.all(np.abs(s32 - s64) <= 1e-5 * sabs)
    e = (v.astype(f32)[:, None] * ds[-1]).astype(f32)
    for li in range(len(layers) - 1, 0, -1):
        e = ((layers[li][0].astype(f32).T @ e) * ds[li - 1]).astype(f32)
    g32 = layers[0][0].astype(f32).T @ e
    assert np.all(np.abs(g32 - g64).max(axis=0) <= 1e-5 * gabs)


def test_gradient_error_scale_bounds_a_float32_evaluation():
    """A plain float32 loss gradient stays within 1e-5 of the oracle's gradient error
    scale, entry by entry."""
    net = _net(2, 24, 3, 31, scale=0.4)
    rng = np.random.default_rng(32)
    pts = rng.uniform(-3, 3, (2, 800))
    y = (rng.uniform(size=800) < 0.3).astype(np.uint8)
    l2 = 1e-3
    _, g64, gsc = O.tanh_loss_grad(net, pts, y, l2, with_scale=True)
    layers, (v, bo) = O.tanh_layers(net)
    f32 = np.float32
    n = pts.shape[1]
    a = pts.astype(f32)
    ins, ds = [a], []
    for W, b in layers:
        a = np.tanh(W.astype(f32) @ a + b.astype(f32)[:, None]).astype(f32)
        ins.append(a)
        ds.append((1 - a * a).astype(f32))
    s = v.astype(f32) @ a + f32(bo)
    r = np.where(y == 1, -1 / (1 + np.exp(s)), 1 / (1 + np.exp(-s))).astype(f32) / f32(n)
    grads = []
    e = (v.astype(f32)[:, None] * ds[-1] * r[None, :]).astype(f32)
    for li in range(len(layers) - 1, -1, -1):
        W = layers[li][0].astype(f32)
        grads.append(((e @ ins[li].T) + f32(l2) * W, e.sum(axis=1)))
        if li > 0:
            e = ((W.T @ e) * ds[li - 1]).astype(f32)
    flat = []
    for gW, gb in reversed(grads):
        flat += [gW.ravel(), gb]
    flat += [ins[-1] @ r + f32(l2) * v.astype(f32), np.array([r.sum()])]
    g32 = np.concatenate(flat)
    assert np.all(np.abs(g32 - g64) <= 1e-5 * gsc + 1e-12)
