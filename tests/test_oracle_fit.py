"""Pins for the oracle's occupancy fit (Sec. 3.1: BCE with gradient descent).

- the loss at w = 0, beta = 0 is log 2 whatever the labels;
- the analytic gradient against Richardson-extrapolated central differences;
- gradient descent and Adam reach the minimiser that Newton's method (IRLS, a
  different algorithm) finds on a small strictly convex problem;
- one Adam update equals torch.optim.Adam's in FP64;
- the logit backward equals the exact finite change of the (linear) logit in w.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O


def _problem(dim=2, M=9, n=150, seed=0, ell=0.8):
    rng = np.random.default_rng(seed)
    g = np.linspace(-1.5, 1.5, int(round(M ** (1 / dim))))
    h = np.stack(np.meshgrid(*([g] * dim), indexing="ij")).reshape(dim, -1)
    pts = rng.uniform(-2, 2, (dim, n))
    y = (np.sin(2 * pts[0]) + 0.5 * pts[1] + 0.3 * rng.normal(size=n) > 0).astype(np.uint8)
    return h, ell, pts, y


def test_loss_at_zero_is_log2():
    h, ell, pts, y = _problem()
    L, g, _ = O.fit_loss_grad(h, ell, np.zeros(h.shape[1] + 1), pts, y, 1e-3)
    assert L == pytest.approx(math.log(2), rel=1e-15)
    # at w = 0: r_i = 1/2 - y_i, so grad_beta = 1/2 - mean(y)
    assert g[-1] == pytest.approx(0.5 - y.mean(), rel=1e-13)


def test_bce_limits():
    s = np.array([0.0, 40.0, -40.0, 3.0])
    y = np.array([1, 1, 0, 0], np.uint8)
    L, g = O.bce_logits(s, y)
    ref = (math.log(2) + math.log1p(math.exp(-40)) + math.log1p(math.exp(-40)) +
           3.0 + math.log1p(math.exp(-3))) / 4
    assert L == pytest.approx(ref, rel=1e-14)
    assert g[0] == pytest.approx(-0.125, rel=1e-15)


def test_gradient_matches_finite_differences():
    h, ell, pts, y = _problem(dim=3, M=8, n=120, seed=1, ell=0.9)
    M = h.shape[1]
    rng = np.random.default_rng(2)
    wb = rng.normal(0, 1.0, M + 1)
    l2 = 0.05
    _, g, gsc = O.fit_loss_grad(h, ell, wb, pts, y, l2)
    fd = np.zeros(M + 1)
    for j in range(M + 1):
        def L(d):
            v = wb.copy()
            v[j] += d
            return O.fit_loss_grad(h, ell, v, pts, y, l2)[0]
        f1 = (L(2e-4) - L(-2e-4)) / 4e-4
        f2 = (L(1e-4) - L(-1e-4)) / 2e-4
        fd[j] = (4 * f2 - f1) / 3
    np.testing.assert_allclose(g, fd, atol=1e-9)
    assert np.all(np.abs(g) <= gsc * (1 + 1e-13))


def _newton_minimiser(h, ell, pts, y, l2):
    """Minimise the same loss by Newton's method (IRLS) on a feature matrix read
    off the oracle's own logit (Phi[:, j] = s with w = e_j, beta = 0)."""
    M = h.shape[1]
    n = pts.shape[1]
    Phi = np.zeros((n, M + 1))
    for j in range(M):
        e = np.zeros(M)
        e[j] = 1.0
        Phi[:, j] = O.occ_eval(O.Occupancy(h, e, 0.0, ell), pts)[0]
    Phi[:, M] = 1.0
    reg = np.full(M + 1, l2)
    reg[M] = 0.0
    wb = np.zeros(M + 1)
    for _ in range(100):
        p = 1 / (1 + np.exp(-Phi @ wb))
        grad = Phi.T @ (p - y) / n + reg * wb
        H = (Phi * (p * (1 - p))[:, None]).T @ Phi / n + np.diag(reg)
        step = np.linalg.solve(H, grad)
        wb -= step
        if np.abs(step).max() < 1e-15:
            break
    return wb


def test_gradient_descent_reaches_newton_minimiser():
    h, ell, pts, y = _problem(seed=3)
    l2 = 0.02
    ref = _newton_minimiser(h, ell, pts, y, l2)
    wb, _, _, loss = O.fit(h, ell, pts, y, 0, 6000, 1.0, l2, lr_bias=1.0)
    assert np.all(np.diff(loss) <= 1e-15)  # monotone at a stable step
    np.testing.assert_allclose(wb, ref, atol=1e-8)


def test_adam_reaches_newton_minimiser():
    h, ell, pts, y = _problem(seed=4)
    l2 = 0.02
    ref = _newton_minimiser(h, ell, pts, y, l2)
    wb, m, v, loss = O.fit(h, ell, pts, y, 1, 4000, 0.02, l2)
    wb, _, _, _ = O.fit(h, ell, pts, y, 1, 4000, 0.002, l2, wb0=wb, m=m, v=v, t0=4000)
    np.testing.assert_allclose(wb, ref, atol=1e-6)


def test_adam_step_matches_torch():
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=50)
    p = p0.copy()
    m, v = np.zeros(50), np.zeros(50)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 8):
        g = rng.normal(size=50)
        O.adam_step(p, g, m, v, t, 0.01, 0.9, 0.999, 1e-8)
        opt.zero_grad()
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_logit_backward_is_exact_change_of_logit():
    h, ell, pts, _ = _problem(dim=3, M=8, n=40, seed=6)
    M = h.shape[1]
    rng = np.random.default_rng(7)
    w = rng.normal(size=M)
    g = rng.normal(size=40)
    gw, gx = O.logit_bwd(h, w, ell, pts, g)
    # s is linear in (w, beta): d/dw_j sum_i g_i s_i = sum_i g_i phi_ij
    for j in range(M):
        e = np.zeros(M)
        e[j] = 1.0
        phi_j = O.occ_eval(O.Occupancy(h, e, 0.0, ell), pts)[0]
        assert gw[j] == pytest.approx(float(g @ phi_j), rel=1e-12, abs=1e-14)
    assert gw[M] == pytest.approx(g.sum(), rel=1e-13)
    _, _, gs, _ = O.occ_grad(O.Occupancy(h, w, 0.0, ell), pts)
    np.testing.assert_allclose(gx, g[None, :] * gs, rtol=1e-14, atol=1e-16)


def test_logit_backward_subset_equals_full_backward_bit_for_bit():
    """The subset form sums the same terms in the same order as the full weight
    backward (itself pinned above against the exact change of the logit), so every
    listed hinge's value is identical; the absolute form equals the full backward of
    |g|.  Repeated and unordered hinge indices included."""
    h, ell, pts, _ = _problem(dim=3, M=27, n=301, seed=8, ell=0.7)
    M = h.shape[1]
    rng = np.random.default_rng(9)
    g = rng.normal(size=pts.shape[1])
    js = np.r_[rng.permutation(M)[:11], 4, 4, 0, M - 1]
    out, ab = O.logit_bwd_w_subset(h, ell, pts, g, js)
    gw, _ = O.logit_bwd(h, np.zeros(M), ell, pts, g, want_x=False)
    gw_abs, _ = O.logit_bwd(h, np.zeros(M), ell, pts, np.abs(g), want_x=False)
    assert np.array_equal(out, gw[js])
    assert np.array_equal(ab, gw_abs[js])


def test_logit_backward_subset_closed_form():
    """One hinge at the origin and points on the axes at r = 0, l, 2l, 3l: the
    features are 1, e^-1/2, e^-2, e^-9/2, so the sums are written out by hand, with
    mixed-sign upstream gradients for the absolute form."""
    ell = 0.625
    h = np.zeros((2, 1))
    x = np.array([[0.0, ell, 0.0, -2 * ell, 0.0],
                  [0.0, 0.0, -ell, 0.0, 3 * ell]])
    g = np.array([0.5, -2.0, 3.0, 1.25, -0.75])
    phi = np.array([1.0, math.exp(-0.5), math.exp(-0.5), math.exp(-2.0), math.exp(-4.5)])
    out, ab = O.logit_bwd_w_subset(h, ell, x, g, [0])
    assert out[0] == pytest.approx(float(np.dot(g, phi)), rel=1e-15)
    assert ab[0] == pytest.approx(float(np.dot(np.abs(g), phi)), rel=1e-15)
    # a hinge far from every point: every feature underflows to zero
    out, ab = O.logit_bwd_w_subset(np.array([[1e3], [0.0]]), ell, x, g, [0])
    assert out[0] == 0.0 and ab[0] == 0.0
