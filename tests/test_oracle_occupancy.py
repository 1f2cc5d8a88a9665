"""Pins for the oracle's occupancy c = sigma(w^T phi(x) + beta) (Sec. 3.1).

Closed forms for one hinge, superposition over hinges, central finite differences
(h = 1e-3 and Richardson-extrapolated) for the gradient and Hessian, translation
invariance, and the error scales used by the parity metrics.
"""
import math

import numpy as np
import pytest

import oracle as O


def _occ(dim, M, seed=0, ell=0.5, scale=1.0, beta=-0.3):
    rng = np.random.default_rng(seed)
    h = rng.uniform(-2, 2, (dim, M))
    w = rng.normal(0, scale, M)
    return O.Occupancy(h, w, beta, ell)


def test_single_hinge_closed_forms():
    ell, w, beta = 0.7, 1.3, -0.4
    h = np.array([[0.25], [-1.5], [2.0]])
    occ = O.Occupancy(h, np.array([w]), beta, ell)
    u = np.array([0.6, 0.0, -0.8])  # unit vector
    # r = 0: phi = 1;  r = l: phi = e^{-1/2};  r = 2l: phi = e^{-2}
    for r, phi in ((0.0, 1.0), (ell, math.exp(-0.5)), (2 * ell, math.exp(-2.0))):
        x = h[:, 0] + r * u
        s, c, sabs = O.occ_eval(occ, x[:, None])
        assert s[0] == pytest.approx(w * phi + beta, rel=1e-14, abs=1e-15)
        assert c[0] == pytest.approx(1 / (1 + math.exp(-(w * phi + beta))), rel=1e-14)
        assert sabs[0] == pytest.approx(abs(w) * phi + abs(beta), rel=1e-14)
        cc, gc, gs, _ = O.occ_grad(occ, x[:, None])
        gs_ref = -w * phi * (r * u) / ell ** 2
        np.testing.assert_allclose(gs[:, 0], gs_ref, rtol=1e-13, atol=1e-15)
        sp = 1 / (1 + math.exp(-(w * phi + beta)))
        np.testing.assert_allclose(gc[:, 0], sp * (1 - sp) * gs_ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("beta", [36.0, -36.0, 45.0, -80.0])
def test_gradient_keeps_relative_accuracy_at_large_logits(beta):
    """Where sigma(s) rounds to within a few ulp of 1, sigma'(s) must still be
    e^{-|s|} / (1 + e^{-|s|})^2 to FP64 relative accuracy (c (1 - c) would be off by
    up to 50 % at s = 36): the closed form for one hinge."""
    ell, w = 0.5, 1.1
    occ = O.Occupancy(np.zeros((2, 1)), np.array([w]), beta, ell)
    x = np.array([[0.3], [-0.2]])
    phi = math.exp(-0.13 / (2 * ell ** 2))
    e = math.exp(-abs(w * phi + beta))
    sp = e / (1 + e) ** 2
    _, gc, gs, _ = O.occ_grad(occ, x)
    np.testing.assert_allclose(gs[:, 0], -w * phi * x[:, 0] / ell ** 2, rtol=1e-13)
    np.testing.assert_allclose(gc[:, 0], sp * gs[:, 0], rtol=1e-13)


def test_single_hinge_gradient_peaks_at_lengthscale():
    ell = 0.4
    occ = O.Occupancy(np.zeros((2, 1)), np.array([2.0]), 0.0, ell)
    r = np.linspace(0.05, 3 * ell, 2001)
    x = np.stack([r, np.zeros_like(r)])
    _, _, gs, _ = O.occ_grad(occ, x)
    k = int(np.argmax(np.abs(gs[0])))
    assert abs(r[k] - ell) <= (r[1] - r[0])


def test_superposition_over_hinges():
    occ = _occ(3, 17, seed=1)
    x = np.random.default_rng(2).uniform(-2, 2, (3, 50))
    s, _, _ = O.occ_eval(occ, x)
    _, _, gs, _ = O.occ_grad(occ, x)
    acc_s = np.full(50, occ.beta)
    acc_g = np.zeros((3, 50))
    for j in range(17):
        one = O.Occupancy(occ.hinges[:, j:j + 1], occ.weights[j:j + 1], 0.0, occ.lengthscale)
        sj, _, _ = O.occ_eval(one, x)
        _, _, gj, _ = O.occ_grad(one, x)
        acc_s += sj
        acc_g += gj
    np.testing.assert_allclose(s, acc_s, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(gs, acc_g, rtol=1e-12, atol=1e-13)


def _central(f, x, h):
    dim, n = x.shape
    out = np.zeros((dim,) + f(x).shape)
    for k in range(dim):
        e = np.zeros((dim, 1))
        e[k] = h
        out[k] = (f(x + e) - f(x - e)) / (2 * h)
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_matches_central_differences(dim):
    occ = _occ(dim, 40, seed=3, ell=0.5, scale=2.0)
    x = np.random.default_rng(4).uniform(-2, 2, (dim, 64))
    c_of = lambda y: O.occ_eval(occ, y)[1]
    s_of = lambda y: O.occ_eval(occ, y)[0]
    _, gc, gs, gabs = O.occ_grad(occ, x)
    # h = 1e-3, truncation error h^2 |f'''|/6 is about 1e-5 relative at l = 0.5
    fd = _central(c_of, x, 1e-3)
    scale = np.abs(gc).max()
    assert np.abs(fd - gc).max() <= 1e-4 * scale
    # Richardson extrapolation removes the h^2 term
    f1, f2 = _central(s_of, x, 2e-3), _central(s_of, x, 1e-3)
    rich = (4 * f2 - f1) / 3
    assert np.abs(rich - gs).max() <= 1e-8 * np.abs(gs).max()
    # G_abs bounds |grad c| (it is a sum of absolute values)
    assert np.all(np.sqrt((gc ** 2).sum(0)) <= gabs * (1 + 1e-12) + 1e-300)


@pytest.mark.parametrize("dim", [2, 3])
def test_hessian_matches_differences_of_gradient(dim):
    occ = _occ(dim, 25, seed=5, ell=0.6, scale=1.5)
    x = np.random.default_rng(6).uniform(-2, 2, (dim, 32))
    hc, hs = O.occ_hess(occ, x)
    g_of = lambda y: O.occ_grad(occ, y)[1]
    gs_of = lambda y: O.occ_grad(occ, y)[2]
    for fun, H in ((g_of, hc), (gs_of, hs)):
        f1, f2 = _central(fun, x, 2e-4), _central(fun, x, 1e-4)
        rich = (4 * f2 - f1) / 3  # rich[b, a, i] = d g_a / d x_b
        np.testing.assert_allclose(np.transpose(rich, (1, 0, 2)), H, atol=1e-7 * np.abs(H).max())
        np.testing.assert_allclose(H, np.transpose(H, (1, 0, 2)), atol=1e-12 * np.abs(H).max())


def test_translation_invariance():
    occ = _occ(2, 30, seed=7)
    x = np.random.default_rng(8).uniform(-2, 2, (2, 40))
    t = np.array([[3.25], [-1.75]])
    moved = O.Occupancy(occ.hinges + t, occ.weights, occ.beta, occ.lengthscale)
    s0, _, _ = O.occ_eval(occ, x)
    s1, _, _ = O.occ_eval(moved, x + t)
    np.testing.assert_allclose(s0, s1, rtol=0, atol=1e-12)


def test_logit_scale_bounds_logit():
    occ = _occ(3, 60, seed=9, scale=3.0)
    x = np.random.default_rng(10).uniform(-2, 2, (3, 100))
    s, c, sabs = O.occ_eval(occ, x)
    assert np.all(np.abs(s) <= sabs * (1 + 1e-14))
    np.testing.assert_allclose(c, 1 / (1 + np.exp(-s)), rtol=1e-15)
