"""GPU parity of the paper's tanh-network occupancy (Sec. 3.1) and of the morph on
it (Eq. 1) against the FP64 oracle, through the C ABI on identical inputs.

Tolerances (FP32 against FP64, 1e-5 relative to the scale the rounding acts on;
S_abs and G_abs are the oracle's error scales of s and grad s, which propagate
|W| |a| sums and the rounding of each tanh through the layers):
  logit     |s_gpu - s| <= 1e-5 S_abs
  occupancy |c_gpu - c| <= 1e-5 (c + sigma' S_abs)
  gradient  |g_gpu - g|_inf <= 1e-5 (sigma' G_abs + |sigma''| |grad s| S_abs)
  morph     |x_gpu - x|_inf <= 1e-5 max(1, A) max(1, |x_T|_inf) per sample, with A
            the product of |I - eta Hess c|_2 along the oracle's path.
"""
import os

import numpy as np
import pytest

import oracle as O
import paper_2108_11775_amd as P
from paper_2108_11775_amd import configs as K, inputs as I

from helpers import GOLDEN, dev, host, require_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _golden(cfg):
    name = {1: "tanh_c1.npy", 2: "tanh_c2.npy"}[cfg.cfg_id]
    return np.load(os.path.join(GOLDEN, name)).astype(np.float32)


def _pair(dim, H, L, params):
    params = np.asarray(params, np.float32)
    return P.TanhNet(dim, H, L, dev(params)), O.TanhNet(dim, H, L, params.astype(np.float64))


def _check_eval_grad(gnet, onet, x):
    c, s = P.tanh_occupancy_eval(gnet, dev(x))
    c2, g = P.tanh_occupancy_grad(gnet, dev(x))
    s_r, gs_r, gc_r, sabs, gabs = O.tanh_grad(onet, x)
    c_r = 1 / (1 + np.exp(-s_r))
    e = np.exp(-np.abs(s_r))
    sp = e / (1 + e) ** 2  # sigma'(s) without the cancellation of c (1 - c)
    assert np.all(np.abs(host(s) - s_r) <= TOL * sabs), np.max(np.abs(host(s) - s_r) / sabs)
    assert np.all(np.abs(host(c) - c_r) <= TOL * (c_r + sp * sabs))
    assert np.array_equal(host(c), host(c2))
    scale = sp * gabs + np.abs(sp * (1 - 2 * c_r)) * np.abs(gs_r).max(axis=0) * sabs
    err = np.abs(host(g) - gc_r).max(axis=0)
    assert np.all(err <= TOL * scale + 1e-30), np.max(err / scale)


@pytest.mark.parametrize("cfg", [K.C1, K.C2], ids=["config1", "config2"])
@pytest.mark.parametrize("n", [1, 17, 5001])
def test_eval_grad_fitted_networks(cfg, n):
    require_gpu()
    tc = K.TANH
    gnet, onet = _pair(2, tc.hidden, tc.layers, _golden(cfg))
    x = I.uniform_points(cfg.cfg_id, K.STREAM_EVAL, 2, n, cfg.lo, cfg.hi)
    _check_eval_grad(gnet, onet, x)


# every width class (1, 2 and 4 row tiles of 16, padded and full) and depth
@pytest.mark.parametrize("dim,H,L", [(2, 1, 1), (2, 7, 2), (3, 16, 3), (2, 17, 4), (3, 32, 1),
                                     (2, 33, 3), (3, 48, 2), (2, 64, 4), (3, 64, 3)])
def test_eval_grad_shapes(dim, H, L):
    require_gpu()
    rng = np.random.default_rng(100 * dim + 10 * L + H)
    n_p = O.tanh_nparams(dim, H, L)
    params = rng.normal(0, 1.0 / np.sqrt(max(H, dim)), n_p) * 1.5
    gnet, onet = _pair(dim, H, L, params)
    x = rng.uniform(-2, 2, (dim, 1237)).astype(np.float32)
    _check_eval_grad(gnet, onet, x)


def _tanh_rule(params, dim, H, L):
    """The documented rule for the forward hidden products' scheme, stated here
    independently of the library: FP16 parts (three products) when every hidden-to-
    hidden W_l and b_l is finite, every nonzero |w| of W_l is at least 2^-19 of its
    largest, and with m 2^e its largest (m in [0.5, 1)) the layer's scale exponent
    z = 29 - e lies in [0, 100] with 2^z max|b_l| <= 2^120; BF16 parts otherwise."""
    p = np.asarray(params, dtype=np.float32)
    ok = L > 1
    off = H * dim + H
    for _ in range(1, L):
        w = np.abs(p[off:off + H * H])
        b = np.abs(p[off + H * H:off + H * H + H])
        off += H * H + H
        if not (np.all(np.isfinite(w)) and np.all(np.isfinite(b))):
            ok = False
            continue
        e = 0
        if w.max() > 0:
            e = int(np.frexp(w.max())[1])
            ok &= float(w[w > 0].min()) >= float(w.max()) * 2.0 ** -19
        z = (15 - e if w.max() > 0 else 0) + 14
        ok &= 0 <= z <= 100 and float(b.max()) * 2.0 ** z <= 2.0 ** 120
    return ("fp16", 3) if ok else ("bf16", 6)


FWD_CASES = ["fp16-edge", "fp16-small-layer", "bf16-tiny-weight", "bf16-huge-weight",
             "bf16-tiny-layer", "bf16-large-layer", "bf16-large-bias"]


@pytest.mark.parametrize("case", FWD_CASES)
def test_eval_grad_forward_schemes(case):
    """The forward hidden products run on FP16 parts of 2^fsw W_l when every nonzero
    hidden weight is within 2^-19 of its layer's largest and the layer's scale keeps
    its bias finite, on BF16 parts otherwise (the backward always on BF16 parts).  Both
    schemes at their edges: weights spread over 2^-18.9 of the largest with random
    signs, or a whole layer scaled by 2^-60 (FP16); one weight at 2^-20 of the largest,
    one weight of 1e30 (the units it feeds saturate), a layer scaled by 2^-110 or 2^40,
    a bias of 1e30 (BF16): the library reports the scheme the rule gives and matches
    the oracle either way."""
    require_gpu()
    rng = np.random.default_rng(1 + FWD_CASES.index(case))
    dim, H, L = 2, 64, 3
    n_p = O.tanh_nparams(dim, H, L)
    params = rng.normal(0, 1.0 / np.sqrt(H), n_p) * 1.5
    w1 = H * dim + H  # W_1 starts after W_0, b_0
    blk = params[w1:w1 + H * H]
    if case == "fp16-edge":
        blk[:] = np.sign(blk) * 0.4 * 2.0 ** rng.uniform(-18.9, 0, H * H)
    elif case == "fp16-small-layer":
        blk *= 2.0 ** -60
    elif case == "bf16-tiny-weight":
        blk[17] = np.abs(blk).max() * 2.0 ** -20
    elif case == "bf16-huge-weight":
        blk[5] = 1e30
    elif case == "bf16-tiny-layer":
        blk *= 2.0 ** -110
    elif case == "bf16-large-layer":
        blk *= 2.0 ** 40
    else:
        params[w1 + H * H + 3] = 1e30
    params[w1:w1 + H * H] = blk
    gnet, onet = _pair(dim, H, L, params)
    want = {"fp16": ("fp16", 3), "bf16": ("bf16", 6)}[case[:4]]
    assert _tanh_rule(params, dim, H, L) == want == P.tanh_split_scheme(gnet)
    x = rng.uniform(-3, 3, (dim, 2049)).astype(np.float32)
    _check_eval_grad(gnet, onet, x)


def test_forward_scheme_of_the_trained_shapes():
    """The networks the morph tests and the bench fit (Xavier-style weights, small
    biases) take the FP16 forward products, one hidden layer none (no hidden-to-hidden
    product: reported as BF16)."""
    require_gpu()
    rng = np.random.default_rng(11)
    for dim, H, L in [(2, 64, 3), (3, 64, 2), (3, 32, 4), (2, 16, 1)]:
        params = rng.normal(0, 1.0 / np.sqrt(H), O.tanh_nparams(dim, H, L))
        gnet, _ = _pair(dim, H, L, params)
        assert P.tanh_split_scheme(gnet) == _tanh_rule(params, dim, H, L), (dim, H, L)
        assert P.tanh_split_scheme(gnet)[0] == ("fp16" if L > 1 else "bf16")


def _morph_check(onet, x0, T, eta, out, idx=None):
    if idx is not None:
        x0, out = x0[:, idx], out[:, idx]
    ref, amp = O.tanh_morph(onet, x0, T, eta, diag=True)
    err = np.abs(out - ref).max(axis=0)
    bound = TOL * np.maximum(1, amp) * np.maximum(1, np.abs(ref).max(axis=0))
    assert np.all(err <= bound), np.max(err / bound)


def test_morph_config1_full():
    require_gpu()
    cfg = K.C1
    tc = K.TANH
    gnet, onet = _pair(2, tc.hidden, tc.layers, _golden(cfg))
    x0 = O.uniform_samples(I.philox_seed(cfg.cfg_id), 0, [cfg.lo] * 2, [cfg.hi] * 2, cfg.n_samples)
    out = host(P.tanh_morph_samples(gnet, dev(x0), cfg.T, cfg.eta))
    _morph_check(onet, x0, cfg.T, cfg.eta, out)


def test_morph_config2_full_size_sampled():
    """The 2^20-sample, T = 50 morph in the launch configuration of the benchmark."""
    require_gpu()
    cfg = K.C2
    tc = K.TANH
    gnet, onet = _pair(2, tc.hidden, tc.layers, _golden(cfg))
    seed = I.philox_seed(cfg.cfg_id)
    x0_d = P.uniform_samples(seed, 0, [cfg.lo] * 2, [cfg.hi] * 2, cfg.n_samples)
    out = host(P.tanh_morph_samples(gnet, x0_d, cfg.T, cfg.eta))
    x0 = O.uniform_samples(seed, 0, [cfg.lo] * 2, [cfg.hi] * 2, cfg.n_samples)
    n = cfg.n_samples
    idx = np.unique(np.r_[0, np.arange(1, n, n // 400), n - 1])
    _morph_check(onet, x0, cfg.T, cfg.eta, out, idx)


@pytest.mark.parametrize("n", [1, 15, 16, 4097])
def test_morph_3d_ragged(n):
    require_gpu()
    rng = np.random.default_rng(n)
    params = rng.normal(0, 0.4, O.tanh_nparams(3, 24, 2))
    gnet, onet = _pair(3, 24, 2, params)
    x0 = rng.uniform(-2, 2, (3, n)).astype(np.float32)
    out = host(P.tanh_morph_samples(gnet, dev(x0), 12, 0.05))
    _morph_check(onet, x0, 12, 0.05, out)


def test_identities_in_place_and_determinism():
    require_gpu()
    cfg = K.C1
    tc = K.TANH
    gnet, _ = _pair(2, tc.hidden, tc.layers, _golden(cfg))
    x = dev(I.uniform_points(1, K.STREAM_EVAL, 2, 5000, cfg.lo, cfg.hi))
    assert np.array_equal(host(P.tanh_morph_samples(gnet, x, 0, 0.05)), host(x))
    assert np.array_equal(host(P.tanh_morph_samples(gnet, x, 7, 0.0)), host(x))
    a = host(P.tanh_morph_samples(gnet, x, cfg.T, cfg.eta))
    b = host(P.tanh_morph_samples(gnet, x, cfg.T, cfg.eta))
    assert np.array_equal(a, b)
    y = x.clone()
    P.tanh_morph_samples(gnet, y, cfg.T, cfg.eta, out=y)
    assert np.array_equal(host(y), a)
    # a constant network (all weights zero) leaves the points where they are
    z = np.zeros(O.tanh_nparams(2, tc.hidden, tc.layers), np.float32)
    z[-1] = 1.5
    znet, _ = _pair(2, tc.hidden, tc.layers, z)
    assert np.array_equal(host(P.tanh_morph_samples(znet, x, 10, 0.5)), host(x))
    c, s = P.tanh_occupancy_eval(znet, x)
    assert np.all(host(s) == np.float32(1.5))


def test_free_fraction_rises_after_gpu_morph():
    require_gpu()
    cfg = K.C2
    tc = K.TANH
    gnet, _ = _pair(2, tc.hidden, tc.layers, _golden(cfg))
    dc, dr = I.discs(cfg.cfg_id, cfg.n_discs, cfg.lo, cfg.hi, cfg.r_min, cfg.r_max)
    x0 = P.uniform_samples(I.philox_seed(cfg.cfg_id), 0, [cfg.lo] * 2, [cfg.hi] * 2, 1 << 18)
    x1 = P.tanh_morph_samples(gnet, x0, cfg.T, cfg.eta)
    _, h0 = P.label_points_discs(dev(dc), dev(dr), x0, count=True)
    _, h1 = P.label_points_discs(dev(dc), dev(dr), x1, count=True)
    before = 1 - int(host(h0)[0]) / x0.shape[1]
    after = 1 - int(host(h1)[0]) / x0.shape[1]
    assert after > before + 0.1, (before, after)


# ---------------------------------------------------------------- the fit ---

def _fit_data(cfg, n):
    dc, dr = I.discs(cfg.cfg_id, cfg.n_discs, cfg.lo, cfg.hi, cfg.r_min, cfg.r_max)
    pts = I.uniform_points(cfg.cfg_id, K.STREAM_FIT, 2, n, cfg.lo, cfg.hi)
    return pts, O.label_discs(dc, dr, pts)


def _check_loss_grad(gnet, onet, pts, y, l2):
    loss, g = P.tanh_loss_grad(gnet, dev(pts), dev(y), l2)
    L, g_r, gsc = O.tanh_loss_grad(onet, pts, y, l2, with_scale=True)
    assert abs(host(loss)[0] - L) <= 1e-6 * L
    err = np.abs(host(g) - g_r)
    assert np.all(err <= TOL * gsc + 1e-12), np.max(err / (gsc + 1e-30))


@pytest.mark.parametrize("n", [1, 63, 10000])
def test_loss_grad_fitted_network(n):
    require_gpu()
    tc = K.TANH
    gnet, onet = _pair(2, tc.hidden, tc.layers, _golden(K.C2))
    pts, y = _fit_data(K.C2, n)
    _check_loss_grad(gnet, onet, pts, y, tc.l2[1])


@pytest.mark.parametrize("dim,H,L", [(2, 5, 1), (3, 16, 2), (2, 40, 3), (3, 64, 4)])
def test_loss_grad_shapes(dim, H, L):
    require_gpu()
    rng = np.random.default_rng(7 * H + L)
    params = rng.normal(0, 1.0 / np.sqrt(max(H, dim)), O.tanh_nparams(dim, H, L))
    gnet, onet = _pair(dim, H, L, params)
    pts = rng.uniform(-2, 2, (dim, 3001)).astype(np.float32)
    y = (rng.uniform(size=3001) < 0.35).astype(np.uint8)
    _check_loss_grad(gnet, onet, pts, y, 1e-3)


def test_fit_adam_one_step_from_identical_state():
    require_gpu()
    tc = K.TANH
    params = _golden(K.C1)
    gnet, onet = _pair(2, tc.hidden, tc.layers, params)
    pts, y = _fit_data(K.C1, 4000)
    rng = np.random.default_rng(5)
    m0 = (rng.normal(size=params.size) * 1e-3).astype(np.float32)
    v0 = (rng.uniform(size=params.size) * 1e-5).astype(np.float32)
    m_d, v_d = dev(m0), dev(v0)
    lr, l2 = float(np.float32(tc.lr)), float(np.float32(tc.l2[0]))
    b1, b2, eps = (float(np.float32(v)) for v in (tc.beta1, tc.beta2, tc.eps))
    P.tanh_fit(gnet, dev(pts), dev(y), 1, lr, l2, b1, b2, eps, adam_m=m_d, adam_v=v_d, t0=3)
    _, g, gsc = O.tanh_loss_grad(onet, pts, y, l2, with_scale=True)
    p_r, m_r, v_r = params.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64)
    O.adam_step(p_r, g, m_r, v_r, 4, lr, b1, b2, eps)
    # the moments follow the gradient tightly; Adam's step direction m/sqrt(v) is
    # ill-conditioned where the gradient is near zero, so the step is compared to lr
    assert np.all(np.abs(host(m_d) - m_r) <= TOL * (0.1 * gsc + np.abs(m_r)) + 1e-12)
    assert np.abs(host(gnet.params) - p_r).max() <= 2e-3 * lr


def test_fit_reduces_the_loss_and_is_deterministic():
    require_gpu()
    tc = K.TANH
    cfg = K.C1
    pts, y = _fit_data(cfg, cfg.fit_points)
    init = I.tanh_init(cfg.cfg_id, 2, tc.hidden, tc.layers, cfg.hi)
    runs = []
    for _ in range(2):
        gnet = P.TanhNet(2, tc.hidden, tc.layers, dev(init.copy()))
        loss = P.tanh_fit(gnet, dev(pts), dev(y), 200, tc.lr, tc.l2[0])
        runs.append((host(loss), host(gnet.params)))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    loss = runs[0][0]
    assert loss[-1] < 0.5 * loss[0]
    # the loss the GPU reports for step 0 is the oracle's at the initial parameters
    L0, _ = O.tanh_loss_grad(O.TanhNet(2, tc.hidden, tc.layers, init.astype(np.float64)), pts, y,
                             tc.l2[0])
    assert abs(loss[0] - L0) <= 1e-6 * L0
