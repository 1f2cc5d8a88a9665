"""Pins of the oracle's inverse morph, log-determinant and epsilon mixture (Sec. 3.2:
the inverse of the flow and the density of the morphed distribution; Sec. 3.3: the
epsilon bias toward the prior) to finite differences, the change-of-variables
identity and the published Philox stream."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2108_11775_amd import configs as K, inputs as I

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _c1():
    cfg = K.C1
    h = I.hinge_grid(2, cfg.grid, cfg.lo, cfg.hi)
    wb = np.load(os.path.join(GOLDEN, "ws2d_4096.npy")).astype(np.float64)
    return cfg, O.Occupancy(h, wb[:-1], wb[-1], cfg.lengthscale)


def _small(seed=0):
    rng = np.random.default_rng(seed)
    ax = np.linspace(-1.2, 1.2, 3)
    j = np.arange(9)
    h = np.stack([ax[j % 3], ax[j // 3]])
    return O.Occupancy(h, rng.normal(0, 3.0, 9), -1.0, 0.6)


def test_logdet_matches_finite_difference_jacobian():
    cfg, occ = _c1()
    x = I.uniform_points(1, K.STREAM_EVAL, 2, 8, cfg.lo, cfg.hi).astype(np.float64)
    xT, ld, _ = O.morph_logdet(occ, x, cfg.T, cfg.eta)
    assert np.allclose(xT, O.morph_ws(occ, x, cfg.T, cfg.eta), rtol=0, atol=1e-13)
    hstep = 1e-6
    for i in range(x.shape[1]):
        J = np.zeros((2, 2))
        for k in range(2):
            xp, xm = x[:, i:i + 1].copy(), x[:, i:i + 1].copy()
            xp[k] += hstep
            xm[k] -= hstep
            J[:, k] = (O.morph_ws(occ, xp, cfg.T, cfg.eta) -
                       O.morph_ws(occ, xm, cfg.T, cfg.eta))[:, 0] / (2 * hstep)
        assert abs(np.log(abs(np.linalg.det(J))) - ld[i]) <= 1e-6 * (1 + abs(ld[i]))


def test_round_trip_and_consistent_logdet():
    cfg, occ = _c1()
    y = I.uniform_points(1, K.STREAM_EVAL, 2, 300, cfg.lo, cfg.hi)
    z, ld_f, _ = O.morph_logdet(occ, y, cfg.T, cfg.eta)
    y2, ld_i, _, resid = O.morph_inverse(occ, z, cfg.T, cfg.eta, 60)
    assert np.all(np.abs(y2 - y) <= 1e-10 * (1 + np.abs(y)))
    assert np.all(resid <= 1e-12)
    assert np.allclose(ld_i, ld_f, rtol=0, atol=1e-9)


def test_zero_step_is_the_identity():
    _, occ = _c1()
    z = np.random.default_rng(1).uniform(-10, 10, (2, 20))
    y, ld, _, r = O.morph_inverse(occ, z, 5, 0.0, 3)
    assert np.array_equal(y, z) and np.all(ld == 0) and np.all(r == 0)


def test_density_of_the_morphed_distribution_integrates_to_one():
    """p_z(z) = p_y(phi^-1(z)) exp(-logdet) with a Gaussian prior integrates to 1."""
    occ = _small()
    T, eta, sig = 10, 0.1, 0.35
    # the step is a contraction-backed diffeomorphism here: eta |Hc| < 1 on the path
    g = np.linspace(-3, 3, 241)
    X, Y = np.meshgrid(g, g)
    z = np.stack([X.ravel(), Y.ravel()])
    _, _, _, meh = O.morph_ws(occ, z, T, eta, diag=True)
    assert meh.max() < 0.5
    y, ld, _, resid = O.morph_inverse(occ, z, T, eta, 40)
    assert resid.max() < 1e-12
    py = np.exp(-(y ** 2).sum(axis=0) / (2 * sig ** 2)) / (2 * np.pi * sig ** 2)
    pz = py * np.exp(-ld)
    dA = (g[1] - g[0]) ** 2
    assert abs(pz.sum() * dA - 1.0) < 1e-4


def test_mixture_coins_follow_the_philox_stream():
    seed, sid = I.philox_seed(2), 5
    keep = O.mixture_coins(seed, sid, 100000, 0.1)
    assert abs(keep.mean() - 0.1) < 5 * np.sqrt(0.09 / 100000)
    assert not O.mixture_coins(seed, sid, 1000, 0.0).any()
    assert O.mixture_coins(seed, sid, 1000, 1.0).all()
    key = [seed & 0xffffffff, seed >> 32]
    for i in (0, 1, 77777):
        w = O.philox4x32_10([i & 0xffffffff, i >> 32, 0xffffffff, sid], key)[0]
        assert keep[i] == ((w >> 8) * 2.0 ** -24 < 0.1)


def test_logdet_3d_matches_finite_difference_jacobian():
    rng = np.random.default_rng(3)
    h = rng.uniform(-1, 1, (3, 12))
    occ = O.Occupancy(h, rng.normal(0, 2.0, 12), 0.3, 0.5)
    x = rng.uniform(-1, 1, (3, 5))
    T, eta = 6, 0.05
    _, ld, _ = O.morph_logdet(occ, x, T, eta)
    for i in range(5):
        J = np.zeros((3, 3))
        for k in range(3):
            xp, xm = x[:, i:i + 1].copy(), x[:, i:i + 1].copy()
            xp[k] += 1e-6
            xm[k] -= 1e-6
            J[:, k] = (O.morph_ws(occ, xp, T, eta) - O.morph_ws(occ, xm, T, eta))[:, 0] / 2e-6
        assert abs(np.log(abs(np.linalg.det(J))) - ld[i]) <= 1e-7 * (1 + abs(ld[i]))
    z = O.morph_ws(occ, x, T, eta)
    y, ld_i, _, r = O.morph_inverse(occ, z, T, eta, 50)
    assert np.allclose(y, x, rtol=0, atol=1e-11) and np.allclose(ld_i, ld, rtol=0, atol=1e-10)


def test_mixture_coins_strict_threshold_and_counter():
    seed, sid = I.philox_seed(3), 11
    key = [seed & 0xffffffff, seed >> 32]
    us = np.array([(O.philox4x32_10([i, 0, 0xffffffff, sid], key)[0] >> 8) * 2.0 ** -24
                   for i in range(300)])
    # the coin is u < eps, taken on the counter with third word 0xffffffff
    keep = O.mixture_coins(seed, sid, 300, 0.3)
    assert np.array_equal(keep, (us < 0.3).astype(np.uint8))
    j = int(np.argmax(us))
    at = O.mixture_coins(seed, sid, 300, float(us[j]))
    assert at[j] == 0 and at.sum() == int((us < us[j]).sum())
