"""GPU parity of the morph's log-determinant, its inverse by fixed point and the
epsilon mixture (Sec. 3.2, Sec. 3.3) against the FP64 oracle, through the C ABI
(grid path: both split schemes of the matrix-core contractions).

Tolerances (FP32 against FP64):
  x_T          as the plain morph: 1e-5 max(1, A) max(1, |x_T|_inf), A the oracle's
               product of |I - eta Hc|_2 along its path;
  logdet       1e-5 (L_abs + max(1, A) T), L_abs the oracle's sum over steps of the
               per-step scale eta |dHc| dim (1 + eta |Hc| dim)^(dim-1) / |det|, the
               second term for the evaluation points carrying the path's own error;
  inverse      y against the oracle's inverse of the same z: 1e-5 max(1, A) max(1, |y|);
               the fixed-point residual below 4 ulp of the coordinates;
  mixture      prior batch, coins and kept samples bit-exact; morphed samples equal to
               the plain morph of the same batch bit for bit.
"""
import os

import numpy as np
import pytest

import oracle as O
import paper_2108_11775_amd as P
from paper_2108_11775_amd import configs as K, inputs as I

from helpers import dev, gpu_occ, host, oracle_occ, require_gpu, ws_scene

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _scene(cfg, grid):
    sc = ws_scene(cfg)
    g = (cfg.grid, cfg.grid) if grid else None
    return sc, gpu_occ(sc["h"], sc["wb"], sc["ell"], grid=g), oracle_occ(sc["h"], sc["wb"], sc["ell"])


def _check_logdet(go, oo, x0, T, eta):
    out, ld = P.morph_logdet(go, dev(x0), T, eta)
    out, ld = host(out), host(ld)
    ref, ld_r, ldsc = O.morph_logdet(oo, x0, T, eta)
    _, amp, _, _ = O.morph_ws(oo, x0, T, eta, diag=True)
    A = np.maximum(1, amp)
    err = np.abs(out - ref).max(axis=0)
    assert np.all(err <= TOL * A * np.maximum(1, np.abs(ref).max(axis=0))), np.max(err)
    bound = TOL * (ldsc + A * T)
    e2 = np.abs(ld - ld_r)
    assert np.all(e2 <= bound), np.max(e2 / bound)
    # the plain morph kernel gives the same points up to rounding order
    return out, ld


@pytest.mark.parametrize("grid", [True, False], ids=["grid", "pairwise"])
def test_logdet_config1(grid):
    require_gpu()
    cfg = K.C1
    _, go, oo = _scene(cfg, grid)
    x0 = O.uniform_samples(I.philox_seed(cfg.cfg_id), 0, [cfg.lo] * 2, [cfg.hi] * 2, 3001)
    _check_logdet(go, oo, x0, cfg.T, cfg.eta)


def test_logdet_config2_grid_sampled():
    require_gpu()
    cfg = K.C2
    _, go, oo = _scene(cfg, True)
    x0 = O.uniform_samples(I.philox_seed(cfg.cfg_id), 0, [cfg.lo] * 2, [cfg.hi] * 2, 1 << 16)
    out, ld = P.morph_logdet(go, dev(x0), cfg.T, cfg.eta)
    idx = np.unique(np.r_[0, np.arange(1, 1 << 16, 331), (1 << 16) - 1])
    _check_logdet(go, oo, x0[:, idx], cfg.T, cfg.eta)
    # a sample's result does not depend on the batch
    o2, l2 = P.morph_logdet(go, dev(np.ascontiguousarray(x0[:, idx])), cfg.T, cfg.eta)
    assert np.array_equal(host(o2), host(out)[:, idx]) and np.array_equal(host(l2), host(ld)[idx])


@pytest.mark.parametrize("grid", [True, False], ids=["grid", "pairwise"])
def test_inverse_config1(grid):
    require_gpu()
    cfg = K.C1
    _, go, oo = _scene(cfg, grid)
    y0 = O.uniform_samples(I.philox_seed(cfg.cfg_id), 0, [cfg.lo] * 2, [cfg.hi] * 2, 2049)
    z = O.morph_ws(oo, y0, cfg.T, cfg.eta).astype(np.float32)
    y, ld, resid = P.morph_inverse(go, dev(z), cfg.T, cfg.eta, 30)
    y, ld, resid = host(y), host(ld), host(resid)
    y_r, ld_r, ldsc, r_r = O.morph_inverse(oo, z, cfg.T, cfg.eta, 30)
    _, amp, _, _ = O.morph_ws(oo, y_r, cfg.T, cfg.eta, diag=True)
    A = np.maximum(1, amp)
    err = np.abs(y - y_r).max(axis=0)
    assert np.all(err <= TOL * A * np.maximum(1, np.abs(y_r).max(axis=0))), np.max(err)
    assert np.all(np.abs(ld - ld_r) <= TOL * (ldsc + A * cfg.T))
    assert np.all(resid <= 4 * 2.0 ** -23 * np.maximum(1, np.abs(y).max(axis=0)))
    # round trip back to the prior samples (FP32 forward on the oracle's path)
    assert np.all(np.abs(y - y0).max(axis=0) <= 1e-4 * A * np.maximum(1, np.abs(y0).max(axis=0)))


def test_inverse_config2_grid_sampled():
    """The inverse at the benchmark's grid size (64 x 64: two row tiles, four k-steps
    of the split contraction) and iteration count, on a sampled subset of a batch."""
    require_gpu()
    cfg = K.C2
    _, go, oo = _scene(cfg, True)
    y0 = O.uniform_samples(I.philox_seed(cfg.cfg_id), 0, [cfg.lo] * 2, [cfg.hi] * 2, 1 << 14)
    idx = np.unique(np.r_[0, np.arange(1, 1 << 14, 211), (1 << 14) - 1])
    z_all = P.morph_samples(go, dev(y0), cfg.T, cfg.eta)
    y, ld, resid = P.morph_inverse(go, z_all, cfg.T, cfg.eta, 10)
    y, ld, resid = host(y)[:, idx], host(ld)[idx], host(resid)[idx]
    z = host(z_all)[:, idx]
    y_r, ld_r, ldsc, _ = O.morph_inverse(oo, z, cfg.T, cfg.eta, 10)
    _, amp, _, _ = O.morph_ws(oo, y_r, cfg.T, cfg.eta, diag=True)
    A = np.maximum(1, amp)
    err = np.abs(y - y_r).max(axis=0)
    assert np.all(err <= TOL * A * np.maximum(1, np.abs(y_r).max(axis=0))), np.max(err)
    assert np.all(np.abs(ld - ld_r) <= TOL * (ldsc + A * cfg.T))
    assert np.all(resid <= 4 * 2.0 ** -23 * np.maximum(1, np.abs(y).max(axis=0)))


@pytest.mark.parametrize("gapped", [False, True], ids=["fp16-edge", "bf16-gapped-axis"])
def test_logdet_inverse_split_schemes(gapped):
    """Both split schemes on the log-determinant and the inverse (a hinge x-axis with a
    10-lengthscale gap takes the bf16 splits), weights down to 2^-18.9 of the largest
    with random signs and points up to 8 lengthscales outside the grid, where the FP16
    scheme scales ex dx^2 by 2^(c-k).  One step per decade of the Hessian's size, eta
    max|Hc| = 0.1: the log-det of a single step is taken at the input on both sides, so
    its error is the Hessian's, held to the oracle's per-step scale; the inverse of the
    oracle's forward step (a tenth of that eta, where the fixed point contracts) against
    the oracle's inverse."""
    require_gpu()
    rng = np.random.default_rng(2211 + gapped)
    g0, g1, ell = 64, 48, 0.3
    ax = (np.r_[np.linspace(-3, -1.5, 32), np.linspace(1.5, 3, 32)] if gapped
          else np.linspace(-3, 3, g0)).astype(np.float32)
    ay = np.linspace(-2, 2, g1).astype(np.float32)
    j = np.arange(g0 * g1)
    h = np.stack([ax[j % g0], ay[j // g0]]).astype(np.float32)
    wb = (10.0 * 2.0 ** rng.uniform(-18.9, 0, g0 * g1 + 1)
          * rng.choice([-1.0, 1.0], g0 * g1 + 1)).astype(np.float32)
    wb[-1] = 0.0
    far = np.stack([rng.uniform(-3 - 8 * ell, 3 + 8 * ell, 400),
                    rng.uniform(-2 - 8 * ell, 2 + 8 * ell, 400)])
    x = np.concatenate([rng.uniform(-3, 3, (2, 400)), far], axis=1).astype(np.float32)
    go = P.Occupancy(dev(h), dev(wb), ell, grid=(g0, g1))
    oo = oracle_occ(h, wb, ell)
    hc, _ = O.occ_hess(oo, x)
    dec = np.floor(np.log10(np.abs(hc).max(axis=(0, 1)))).astype(int)
    for d in np.unique(dec):
        sel = np.flatnonzero(dec == d)
        eta = float(np.float32(0.1 * 10.0 ** (-d)))
        xs = np.ascontiguousarray(x[:, sel])
        _, ld = P.morph_logdet(go, dev(xs), 1, eta)
        _, ld_r, ldsc = O.morph_logdet(oo, xs, 1, eta)
        e = np.abs(host(ld) - ld_r)
        assert np.all(e <= TOL * ldsc), (d, float(np.max(e / ldsc)))
        # the inverse with a tenth of that step, where the fixed point contracts
        ei = float(np.float32(0.1 * eta))
        z = O.morph_ws(oo, xs, 1, ei).astype(np.float32)
        y, _, _ = P.morph_inverse(go, dev(z), 1, ei, 30)
        y_r, _, _, r_r = O.morph_inverse(oo, z, 1, ei, 30)
        assert np.all(r_r <= 1e-6 * np.maximum(1, np.abs(y_r).max(axis=0)))
        _, amp, _, _ = O.morph_ws(oo, y_r, 1, ei, diag=True)
        err = np.abs(host(y) - y_r).max(axis=0)
        assert np.all(err <= TOL * np.maximum(1, amp) * np.maximum(1, np.abs(y_r).max(axis=0)))


@pytest.mark.parametrize("n", [1, 255, 1000])
def test_pairwise_3d(n):
    require_gpu()
    rng = np.random.default_rng(n)
    h = rng.uniform(-1, 1, (3, 50)).astype(np.float32)
    wb = np.r_[rng.normal(0, 2.0, 50), -0.5].astype(np.float32)
    go, oo = gpu_occ(h, wb, 0.4), oracle_occ(h, wb, 0.4)
    x0 = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    _check_logdet(go, oo, x0, 8, 0.02)
    z = O.morph_ws(oo, x0, 8, 0.02).astype(np.float32)
    y, _, resid = P.morph_inverse(go, dev(z), 8, 0.02, 25)
    y_r, _, _, _ = O.morph_inverse(oo, z, 8, 0.02, 25)
    assert np.all(np.abs(host(y) - y_r) <= 1e-5 * np.maximum(1, np.abs(y_r)))


def test_identities():
    require_gpu()
    cfg = K.C1
    _, go, _ = _scene(cfg, True)
    x = dev(I.uniform_points(1, K.STREAM_EVAL, 2, 777, cfg.lo, cfg.hi))
    out, ld = P.morph_logdet(go, x, 0, cfg.eta)
    assert np.array_equal(host(out), host(x)) and np.all(host(ld) == 0)
    y, ld, r = P.morph_inverse(go, x, 4, 0.0, 3)
    assert np.array_equal(host(y), host(x)) and np.all(host(ld) == 0) and np.all(host(r) == 0)


@pytest.mark.parametrize("eps", [0.0, 0.1, 1.0])
def test_mixture(eps):
    require_gpu()
    cfg = K.C2
    _, go, _ = _scene(cfg, True)
    seed, sid, n = I.philox_seed(cfg.cfg_id), 3, 100003
    x0, out, keep = P.mixture_samples(go, seed, sid, [cfg.lo] * 2, [cfg.hi] * 2, n, eps, cfg.T,
                                      cfg.eta)
    ref_x0 = P.uniform_samples(seed, sid, [cfg.lo] * 2, [cfg.hi] * 2, n)
    assert np.array_equal(host(x0), host(ref_x0))
    coins = O.mixture_coins(seed, sid, n, float(np.float32(eps)))
    assert np.array_equal(host(keep), coins)
    plain = host(P.morph_samples(go, ref_x0, cfg.T, cfg.eta))
    o = host(out)
    k = coins.astype(bool)
    assert np.array_equal(o[:, k], host(x0)[:, k])
    assert np.array_equal(o[:, ~k], plain[:, ~k])
