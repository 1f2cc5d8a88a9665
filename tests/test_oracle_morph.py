"""Pins for the oracle's workspace morph (Sec. 3.2: Eq. 1 solved by Euler's method).

- identities: eta = 0, T = 0, w = 0;
- one hinge: the path stays on the ray from the hinge and follows the scalar
  radial recurrence;
- convergence to the integral curve of Eq. 1 computed by a library ODE solver,
  with first-order error in eta (explicit Euler);
- each Euler step is a diffeomorphism when eta * Lip(grad c) < 1 (Sec. 3.4 needs
  the map to be one): det(I - eta Hess c) > 0 along every path;
- samples are independent of each other and of the batch;
- the collision-free fraction rises after the morph (the trend of Table 1).
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle as O
from paper_2108_11775_amd import configs as K, inputs as I


def _scene(dim=2, M=36, seed=0, ell=0.6, scale=2.0):
    rng = np.random.default_rng(seed)
    h = rng.uniform(-3, 3, (dim, M))
    w = rng.normal(0, scale, M)
    return O.Occupancy(h, w, -0.5, ell)


def test_identities():
    occ = _scene()
    x = np.random.default_rng(1).uniform(-3, 3, (2, 64))
    assert np.array_equal(O.morph_ws(occ, x, 20, 0.0), x)
    assert np.array_equal(O.morph_ws(occ, x, 0, 0.1), x)
    flat = O.Occupancy(occ.hinges, np.zeros(occ.M), 1.7, occ.lengthscale)
    assert np.array_equal(O.morph_ws(flat, x, 20, 0.1), x)


def test_single_hinge_radial_recurrence():
    ell, w, beta, eta, T = 0.5, 3.0, -1.0, 0.05, 40
    hc = np.array([0.3, -0.2])
    occ = O.Occupancy(hc[:, None], np.array([w]), beta, ell)
    u = np.array([0.8, 0.6])
    r0 = np.array([0.1, 0.4, 0.5, 0.9, 1.6])
    x0 = hc[:, None] + u[:, None] * r0[None, :]
    xT = O.morph_ws(occ, x0, T, eta)
    # scalar recurrence r <- r (1 + eta sigma'(s) w e^{-r^2/2l^2} / l^2)
    r = r0.copy()
    for _ in range(T):
        phi = np.exp(-r ** 2 / (2 * ell ** 2))
        c = 1 / (1 + np.exp(-(w * phi + beta)))
        r = r * (1 + eta * c * (1 - c) * w * phi / ell ** 2)
    ref = hc[:, None] + u[:, None] * r[None, :]
    np.testing.assert_allclose(xT, ref, rtol=0, atol=1e-13)


def test_converges_to_integral_curve_first_order():
    occ = _scene(seed=2)
    x0 = np.array([[0.4], [-0.7]])
    t_end = 1.0

    def f(t, y):
        return -O.occ_grad(occ, y.reshape(2, 1))[1][:, 0]

    sol = solve_ivp(f, (0, t_end), x0[:, 0], method="DOP853", rtol=1e-12, atol=1e-12)
    exact = sol.y[:, -1]
    errs = []
    for T in (50, 100, 200, 400):
        xT = O.morph_ws(occ, x0, T, t_end / T)[:, 0]
        errs.append(np.linalg.norm(xT - exact))
    ratios = [errs[k + 1] / errs[k] for k in range(3)]
    assert errs[-1] < 1e-2 * max(1.0, np.linalg.norm(exact - x0[:, 0]))
    for q in ratios:
        assert 0.4 < q < 0.6  # global error O(eta)


def _lip_bound(occ):
    w = np.abs(occ.weights)
    ell = occ.lengthscale
    b1 = math.exp(-0.5) * w.sum() / ell
    b2 = w.sum() / ell ** 2
    return 0.25 * b2 + b1 ** 2 / (6 * math.sqrt(3))


@pytest.mark.parametrize("dim", [2, 3])
def test_each_step_is_a_diffeomorphism(dim):
    occ = _scene(dim=dim, M=20, seed=3, scale=1.0)
    L = _lip_bound(occ)
    eta = 0.9 / L
    x = np.random.default_rng(4).uniform(-3, 3, (dim, 200))
    _, amp, mdet, meh = O.morph_ws(occ, x, 30, eta, diag=True)
    assert np.all(meh <= eta * L + 1e-12)
    # eigenvalues of I - eta H lie in [1 - eta L, 1 + eta L]
    assert np.all(mdet >= (1 - eta * L) ** dim - 1e-12)
    assert np.all(mdet > 0)
    assert np.all(amp <= (1 + eta * L) ** 30 * (1 + 1e-12))


def test_batch_independence():
    occ = _scene(seed=5)
    x = np.random.default_rng(6).uniform(-3, 3, (2, 33))
    full = O.morph_ws(occ, x, 15, 0.05)
    for i in (0, 17, 32):
        one = O.morph_ws(occ, x[:, i:i + 1], 15, 0.05)
        assert np.array_equal(one[:, 0], full[:, i])


def test_translation_commutes_with_morph():
    occ = _scene(seed=7)
    t = np.array([[2.5], [-4.0]])
    moved = O.Occupancy(occ.hinges + t, occ.weights, occ.beta, occ.lengthscale)
    x = np.random.default_rng(8).uniform(-3, 3, (2, 40))
    a = O.morph_ws(occ, x, 25, 0.05)
    b = O.morph_ws(moved, x + t, 25, 0.05)
    np.testing.assert_allclose(a + t, b, rtol=0, atol=1e-10)


@pytest.mark.slow
def test_free_fraction_rises_on_config1():
    cfg = K.C1
    h = I.hinge_grid(2, cfg.grid, cfg.lo, cfg.hi)
    M = h.shape[1]
    pts = I.uniform_points(cfg.cfg_id, K.STREAM_FIT, 2, cfg.fit_points, cfg.lo, cfg.hi)
    dc, dr = I.discs(cfg.cfg_id, cfg.n_discs, cfg.lo, cfg.hi, cfg.r_min, cfg.r_max)
    y = O.label_discs(dc, dr, pts)
    wb, _, _, loss = O.fit(h, cfg.lengthscale, pts, y, 0, cfg.fit_steps, cfg.fit_lr, cfg.fit_l2,
                           lr_bias=cfg.fit_lr_bias)
    assert loss[-1] < 0.5 * loss[0]
    occ = O.Occupancy(h, wb[:M], wb[M], cfg.lengthscale)
    x0 = O.uniform_samples(I.philox_seed(cfg.cfg_id), 0, [cfg.lo] * 2, [cfg.hi] * 2, cfg.n_samples)
    x1 = O.morph_ws(occ, x0, cfg.T, cfg.eta)
    before = 1 - O.label_discs(dc, dr, x0).mean()
    after = 1 - O.label_discs(dc, dr, x1).mean()
    assert after > before + 0.03
