"""Pins for the oracle's residual MLP and amortised morph.

The forward is pinned by a hand-evaluated one-unit network and by torch's FP64
linear/SiLU layers; the MSE gradient by torch autograd in FP64 (a different
differentiation route); the amortised morph by its fallback rule: with a zero
network, flagged samples take exactly the plain morph and the rest stay put.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2108_11775_amd import configs as K, inputs as I


def test_one_unit_network_by_hand():
    widths = (1, 1, 1)
    P = O.mlp_pack([(np.array([[2.0]]), np.array([0.0])), (np.array([[3.0]]), np.array([0.5]))])
    out = O.mlp_forward(widths, P, np.array([[1.0]]))
    silu2 = 2.0 / (1.0 + math.exp(-2.0))
    assert out[0, 0] == pytest.approx(1.0 + 3.0 * silu2 + 0.5, rel=1e-15)


def _torch_mlp(layers, q):
    x = torch.tensor(q.T, dtype=torch.float64)
    h = x
    for li, (W, b) in enumerate(layers):
        h = torch.nn.functional.linear(h, W, b)
        if li < len(layers) - 1:
            h = torch.nn.functional.silu(h)
    return x + h


def test_forward_and_gradient_match_torch():
    widths = (7, 32, 32, 32, 7)
    layers = I.mlp_init(5, widths, zero_last=False)
    P = O.mlp_pack(layers)
    rng = np.random.default_rng(0)
    q = rng.uniform(-math.pi, math.pi, (7, 40))
    tgt = rng.normal(size=(7, 40))
    out = O.mlp_forward(widths, P, q)
    tl = [(torch.tensor(W, dtype=torch.float64, requires_grad=True),
           torch.tensor(b, dtype=torch.float64, requires_grad=True)) for W, b in layers]
    ref = _torch_mlp(tl, q)
    np.testing.assert_allclose(out, ref.detach().numpy().T, rtol=1e-13, atol=1e-14)
    L, g = O.mlp_loss_grad(widths, P, q, tgt)
    loss = ((ref - torch.tensor(tgt.T)) ** 2).mean()
    loss.backward()
    assert L == pytest.approx(loss.item(), rel=1e-13)
    gref = np.concatenate([np.concatenate([W.grad.numpy().reshape(-1), b.grad.numpy()])
                           for W, b in tl])
    np.testing.assert_allclose(g, gref, rtol=1e-11, atol=1e-15)


def test_zero_last_layer_is_identity():
    widths = K.C5.widths
    P = O.mlp_pack(I.mlp_init(5, widths))
    q = np.random.default_rng(1).uniform(-3, 3, (7, 10))
    assert np.array_equal(O.mlp_forward(widths, P, q), q)


def test_amortised_zero_network_falls_back_to_plain_morph():
    rng = np.random.default_rng(2)
    arm = O.Arm(rng.uniform(0.1, 0.4, 7), np.zeros(7), np.array(K.C3.alpha), np.zeros(7), 8)
    h = rng.uniform(-1.2, 1.2, (3, 48))
    occ = O.Occupancy(h, rng.normal(0, 3.0, 48), -0.5, 0.3)
    widths = (7, 16, 16, 7)
    P = O.mlp_pack(I.mlp_init(5, widths))
    q = rng.uniform(-math.pi, math.pi, (7, 24))
    out, flag, maxc = O.amortised_morph(widths, P, arm, occ, q, 5, 0.01, 0.5)
    plain = O.morph_arm(arm, occ, q, 5, 0.01)
    pts = O.fk_points(arm, q)
    for s in range(24):
        cmax = O.occ_eval(occ, pts[:, :, s])[1].max()
        assert maxc[s] == pytest.approx(cmax, rel=1e-14)
        assert flag[s] == (cmax > 0.5)
        if flag[s]:
            np.testing.assert_array_equal(out[:, s], plain[:, s])
        else:
            np.testing.assert_array_equal(out[:, s], q[:, s])
    assert 0 < flag.sum() < 24


def test_weighted_mse_is_the_mse_over_duplicated_samples():
    """A sample of integer weight u counts as u copies of itself: with the batch
    normalisation of each side, B L_w(batch) = B' L(batch with the hard samples
    repeated u times), B' the repeated batch's size, and likewise for the gradient.
    No weight (or no hard sample) is the plain MSE, bit for bit."""
    widths = (7, 24, 24, 7)
    layers = I.mlp_init(8, widths, zero_last=False)
    P = O.mlp_pack(layers)
    rng = np.random.default_rng(4)
    B, u = 30, 3
    q = rng.uniform(-math.pi, math.pi, (7, B))
    t = q + rng.normal(0, 0.2, (7, B))
    hard = (rng.uniform(size=B) < 0.4).astype(np.uint8)
    assert 0 < hard.sum() < B
    Lw, gw = O.mlp_loss_grad_weighted(widths, P, q, t, hard, float(u))
    rep = np.concatenate([np.arange(B)] + [np.flatnonzero(hard)] * (u - 1))
    Ld, gd = O.mlp_loss_grad(widths, P, q[:, rep], t[:, rep])
    assert B * Lw == pytest.approx(len(rep) * Ld, rel=1e-12)
    np.testing.assert_allclose(B * gw, len(rep) * gd, rtol=1e-10, atol=1e-14)
    L0, g0 = O.mlp_loss_grad(widths, P, q, t)
    L1, g1 = O.mlp_loss_grad_weighted(widths, P, q, t, np.zeros(B, np.uint8), 7.0)
    L2, g2 = O.mlp_loss_grad_weighted(widths, P, q, t, hard, 1.0)
    assert L1 == L0 and L2 == L0
    assert np.array_equal(g1, g0) and np.array_equal(g2, g0)


def test_refining_amortised_morph_pins():
    """The refining variant (flagged configurations take the plain steps from q_hat):
    with a zero network q_hat = q, so it is the plain-fallback amortised morph bit for
    bit; with no steps it returns q_hat everywhere; and each flagged configuration's
    result is the plain morph of its q_hat."""
    rng = np.random.default_rng(12)
    arm = O.Arm(rng.uniform(0.1, 0.4, 7), np.zeros(7), np.array(K.C3.alpha), np.zeros(7), 8)
    h = rng.uniform(-1.2, 1.2, (3, 48))
    occ = O.Occupancy(h, rng.normal(0, 3.0, 48), -0.5, 0.3)
    widths = (7, 16, 16, 7)
    q = rng.uniform(-math.pi, math.pi, (7, 24))
    P0 = O.mlp_pack(I.mlp_init(5, widths))
    a, fa, ma = O.amortised_morph(widths, P0, arm, occ, q, 5, 0.01, 0.5)
    r, fr, mr = O.amortised_morph(widths, P0, arm, occ, q, 5, 0.01, 0.5, refine=True)
    assert np.array_equal(a, r) and np.array_equal(fa, fr) and np.array_equal(ma, mr)
    layers = I.mlp_init(6, widths, zero_last=False)
    layers[-1] = (layers[-1][0] * 0.1, layers[-1][1] * 0.1)
    P1 = O.mlp_pack(layers)
    qh = O.mlp_forward(widths, P1, q)
    r0, f0, _ = O.amortised_morph(widths, P1, arm, occ, q, 0, 0.01, 0.5, refine=True)
    assert np.array_equal(r0, qh)
    r5, f5, _ = O.amortised_morph(widths, P1, arm, occ, q, 5, 0.01, 0.5, refine=True)
    assert np.array_equal(f5, f0) and 0 < f5.sum() < 24
    fb = f5 == 1
    np.testing.assert_array_equal(r5[:, ~fb], qh[:, ~fb])
    ref = O.morph_arm(arm, occ, np.ascontiguousarray(qh[:, fb]), 5, 0.01)
    np.testing.assert_allclose(r5[:, fb], ref, rtol=0, atol=1e-12)
