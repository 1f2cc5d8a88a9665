"""GPU parity of the grid-factorised 2-D path (FP32-accurate split contractions on the
matrix cores) against the oracle's pairwise definition, with the same condition-aware
tolerances as the pairwise path."""
import numpy as np
import pytest

import oracle as O
import paper_2108_11775_amd as P
from paper_2108_11775_amd import configs as K, inputs as I

from helpers import dev, host, one_step_grad_check, oracle_occ, require_gpu, split_rule, ws_scene

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _grid_occ(h, wb, ell, g0, g1):
    return P.Occupancy(dev(h), dev(wb), ell, grid=(g0, g1))


@pytest.mark.parametrize("cfg", [K.C1, K.C2])
@pytest.mark.parametrize("n", [1, 3001])
def test_grid_eval_grad(cfg, n):
    require_gpu()
    sc = ws_scene(cfg)
    go = _grid_occ(sc["h"], sc["wb"], sc["ell"], cfg.grid, cfg.grid)
    x = I.uniform_points(cfg.cfg_id, K.STREAM_EVAL, 2, n, cfg.lo - 0.5, cfg.hi + 0.5)
    c, s = P.occupancy_eval(go, dev(x))
    _, g = P.occupancy_grad(go, dev(x))
    oo = oracle_occ(sc["h"], sc["wb"], sc["ell"])
    s_r, c_r, sabs = O.occ_eval(oo, x)
    _, g_r, _, gabs = O.occ_grad(oo, x)
    assert np.all(np.abs(host(s) - s_r) <= TOL * sabs)
    assert np.all(np.abs(host(c) - c_r) <= TOL * (c_r + c_r * (1 - c_r) * sabs))
    assert np.all(np.abs(host(g) - g_r).max(axis=0) <= TOL * gabs)


@pytest.mark.parametrize("g0,g1", [(17, 45), (64, 33), (2, 1), (63, 64)])
def test_grid_shapes(g0, g1):
    require_gpu()
    rng = np.random.default_rng(g0 * 100 + g1)
    ax = np.sort(rng.uniform(-3, 3, g0)).astype(np.float32)
    ay = np.sort(rng.uniform(-2, 2, g1)).astype(np.float32)
    j = np.arange(g0 * g1)
    h = np.stack([ax[j % g0], ay[j // g0]]).astype(np.float32)
    wb = rng.normal(0, 1.5, g0 * g1 + 1).astype(np.float32)
    x = rng.uniform(-3.5, 3.5, (2, 777)).astype(np.float32)
    go = _grid_occ(h, wb, 0.5, g0, g1)
    _, s = P.occupancy_eval(go, dev(x))
    oo = oracle_occ(h, wb, 0.5)
    s_r, _, sabs = O.occ_eval(oo, x)
    assert np.all(np.abs(host(s) - s_r) <= TOL * sabs)
    out = host(P.morph_samples(go, dev(x), 10, 0.02))
    ref, amp, _, _ = O.morph_ws(oo, x, 10, 0.02, diag=True)
    err = np.abs(out - ref).max(axis=0)
    assert np.all(err <= TOL * np.maximum(1, amp) * np.maximum(1, np.abs(ref).max(axis=0)))


def test_grid_morph_config2_full_size_sampled():
    require_gpu()
    cfg = K.C2
    sc = ws_scene(cfg)
    seed = I.philox_seed(cfg.cfg_id)
    x0_d = P.uniform_samples(seed, 0, [cfg.lo] * 2, [cfg.hi] * 2, cfg.n_samples)
    go = _grid_occ(sc["h"], sc["wb"], sc["ell"], cfg.grid, cfg.grid)
    out = host(P.morph_samples(go, x0_d, cfg.T, cfg.eta))
    x0 = O.uniform_samples(seed, 0, [cfg.lo] * 2, [cfg.hi] * 2, cfg.n_samples)
    n = cfg.n_samples
    idx = np.unique(np.r_[0, np.arange(1, n, n // 300), n - 1])
    ref, amp, _, _ = O.morph_ws(oracle_occ(sc["h"], sc["wb"], sc["ell"]), x0[:, idx], cfg.T, cfg.eta,
                                diag=True)
    err = np.abs(out[:, idx] - ref).max(axis=0)
    assert np.all(err <= TOL * np.maximum(1, amp) * np.maximum(1, np.abs(ref).max(axis=0)))
    # the same launch again gives the same bits, and a sample's result does not depend
    # on its place in the batch (the batch rolled by 12,345, same kernel)
    assert np.array_equal(host(P.morph_samples(go, x0_d, cfg.T, cfg.eta)), out)
    rolled = host(P.morph_samples(go, dev(np.ascontiguousarray(np.roll(x0, 12345, axis=1))),
                                  cfg.T, cfg.eta))
    assert np.array_equal(np.roll(rolled, -12345, axis=1), out)


def test_grid_morph_config1_full_and_deterministic():
    require_gpu()
    cfg = K.C1
    sc = ws_scene(cfg)
    x0 = O.uniform_samples(I.philox_seed(cfg.cfg_id), 0, [cfg.lo] * 2, [cfg.hi] * 2, cfg.n_samples)
    go = _grid_occ(sc["h"], sc["wb"], sc["ell"], cfg.grid, cfg.grid)
    a = host(P.morph_samples(go, dev(x0), cfg.T, cfg.eta))
    b = host(P.morph_samples(go, dev(x0), cfg.T, cfg.eta))
    assert np.array_equal(a, b)
    ref, amp, _, _ = O.morph_ws(oracle_occ(sc["h"], sc["wb"], sc["ell"]), x0, cfg.T, cfg.eta,
                                diag=True)
    err = np.abs(a - ref).max(axis=0)
    assert np.all(err <= TOL * np.maximum(1, amp) * np.maximum(1, np.abs(ref).max(axis=0)))


def test_grid_split_precision_wide_range():
    """Weights over six decades (wider than the FP16 scheme's 2^-19, so the three-way
    bf16 splits run) with random signs and samples up to 8 lengthscales outside the
    grid (every feature tiny but normal in FP32) still meet the FP32 tolerance of the
    absolute sums.
    Weights stay below 10 so that sigma' stays a normal FP32 number."""
    require_gpu()
    rng = np.random.default_rng(2108)
    g0, g1, ell = 64, 48, 0.3
    ax = np.linspace(-3, 3, g0).astype(np.float32)
    ay = np.linspace(-2, 2, g1).astype(np.float32)
    j = np.arange(g0 * g1)
    h = np.stack([ax[j % g0], ay[j // g0]]).astype(np.float32)
    mag = 10.0 ** rng.uniform(-5, 1, g0 * g1 + 1)
    wb = (mag * rng.choice([-1.0, 1.0], g0 * g1 + 1)).astype(np.float32)
    wb[-1] = 0.0  # no bias: the tolerance of far samples is then set by their tiny sums
    far = np.stack([rng.uniform(-3 - 8 * ell, 3 + 8 * ell, 500),
                    rng.uniform(-2 - 8 * ell, 2 + 8 * ell, 500)])
    x = np.concatenate([rng.uniform(-3.2, 3.2, (2, 500)), far], axis=1).astype(np.float32)
    go = _grid_occ(h, wb, ell, g0, g1)
    _, s = P.occupancy_eval(go, dev(x))
    _, g = P.occupancy_grad(go, dev(x))
    oo = oracle_occ(h, wb, ell)
    s_r, _, sabs = O.occ_eval(oo, x)
    _, g_r, _, gabs = O.occ_grad(oo, x)
    assert np.all(np.abs(host(s) - s_r) <= TOL * sabs)
    assert np.all(np.abs(host(g) - g_r).max(axis=0) <= TOL * gabs)
    one_step_grad_check(go, oo, x)


def _wide_case(rng, g0, g1, ell, ax, ay, log2_range):
    j = np.arange(g0 * g1)
    h = np.stack([ax[j % g0], ay[j // g0]]).astype(np.float32)
    mag = 10.0 * 2.0 ** rng.uniform(-log2_range, 0, g0 * g1 + 1)
    wb = (mag * rng.choice([-1.0, 1.0], g0 * g1 + 1)).astype(np.float32)
    # a tenth of the weights exactly +0 or -0: the range test skips zeros
    zero = rng.random(g0 * g1) < 0.1
    wb[:-1][zero] = np.where(rng.random(zero.sum()) < 0.5, 0.0, -0.0).astype(np.float32)
    wb[-1] = 0.0
    lo, hi = ax.min(), ax.max()
    far = np.stack([rng.uniform(lo - 8 * ell, hi + 8 * ell, 500),
                    rng.uniform(ay.min() - 8 * ell, ay.max() + 8 * ell, 500)])
    x = np.concatenate([rng.uniform(lo - 0.2, hi + 0.2, (2, 500)), far], axis=1).astype(np.float32)
    go = _grid_occ(h, wb, ell, g0, g1)
    oo = oracle_occ(h, wb, ell)
    # single evaluations keep the bf16 splits
    _, s = P.occupancy_eval(go, dev(x))
    _, g = P.occupancy_grad(go, dev(x))
    s_r, _, sabs = O.occ_eval(oo, x)
    _, g_r, _, gabs = O.occ_grad(oo, x)
    assert np.all(np.abs(host(s) - s_r) <= TOL * sabs)
    assert np.all(np.abs(host(g) - g_r).max(axis=0) <= TOL * gabs)
    # morphs take the block's scheme: one step per decade of G_abs checks the gradient
    # to the same tolerance, far points included
    one_step_grad_check(go, oo, x)
    # a 10-step morph of fewer than 2^17 samples runs the 16-sample waves, far points
    # included
    out = host(P.morph_samples(go, dev(x), 10, 0.002))
    ref, amp, _, _ = O.morph_ws(oo, x, 10, 0.002, diag=True)
    err = np.abs(out - ref).max(axis=0)
    assert np.all(err <= TOL * np.maximum(1, amp) * np.maximum(1, np.abs(ref).max(axis=0)))


def test_grid_fp16_scheme_range_edge():
    """The FP16 split scheme (morphs) at the edge of its range: nonzero weights down to
    2^-18.9 of the largest (the scheme takes 2^-19), random signs, a tenth of them +-0,
    samples up to 8 lengthscales outside the grid, where each sample's operand scale
    2^c carries the features that FP16 alone could not hold."""
    require_gpu()
    rng = np.random.default_rng(1619)
    g0, g1, ell = 64, 48, 0.3
    _wide_case(rng, g0, g1, ell, np.linspace(-3, 3, g0).astype(np.float32),
               np.linspace(-2, 2, g1).astype(np.float32), 18.9)


def test_grid_bf16_fallback_gapped_axis():
    """A hinge x-axis with a gap of 3 (10 lengthscales, above the FP16 scheme's 6 kappa
    units) takes the three-part bf16 splits; weights within the FP16 range."""
    require_gpu()
    rng = np.random.default_rng(1620)
    g0, g1, ell = 40, 30, 0.3
    ax = np.r_[np.linspace(-3, -1.5, 20), np.linspace(1.5, 3, 20)].astype(np.float32)
    _wide_case(rng, g0, g1, ell, ax, np.linspace(-2, 2, g1).astype(np.float32), 10.0)


@pytest.mark.parametrize("scheme", ["fp16", "bf16"])
def test_grid_large_batch_ragged_grid_sampled(scheme):
    """Morphs of 2^17 samples and more take the 32-sample waves (smaller morphs the
    16-sample waves, which the other morph cases here exercise): a ragged 45 x 37
    grid, 2^17 + 333 samples, outputs sampled every 293rd sample; on the FP16 splits,
    and on the bf16 splits with one weight at 2^-30 of the largest."""
    require_gpu()
    rng = np.random.default_rng(4537)
    g0, g1 = 45, 37
    ax = np.sort(rng.uniform(-3, 3, g0)).astype(np.float32)
    ay = np.sort(rng.uniform(-2, 2, g1)).astype(np.float32)
    j = np.arange(g0 * g1)
    h = np.stack([ax[j % g0], ay[j // g0]]).astype(np.float32)
    wb = rng.normal(0, 1.5, g0 * g1 + 1).astype(np.float32)
    if scheme == "bf16":
        wb[100] = np.float32(np.abs(wb[:-1]).max() * 2.0 ** -30)
    n = (1 << 17) + 333
    x = rng.uniform(-3.5, 3.5, (2, n)).astype(np.float32)
    go = _grid_occ(h, wb, 0.5, g0, g1)
    assert split_rule(ax, wb[:-1], 0.5)[0] == scheme == P.split_scheme(go)[0]
    _, s = P.occupancy_eval(go, dev(x))
    out = host(P.morph_samples(go, dev(x), 5, 0.02))
    idx = np.unique(np.r_[0, np.arange(1, n, 293), n - 1])
    oo = oracle_occ(h, wb, 0.5)
    s_r, _, sabs = O.occ_eval(oo, x[:, idx])
    assert np.all(np.abs(host(s)[idx] - s_r) <= TOL * sabs)
    ref, amp, _, _ = O.morph_ws(oo, x[:, idx], 5, 0.02, diag=True)
    err = np.abs(out[:, idx] - ref).max(axis=0)
    assert np.all(err <= TOL * np.maximum(1, amp) * np.maximum(1, np.abs(ref).max(axis=0)))
