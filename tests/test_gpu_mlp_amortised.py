"""GPU parity: BF16-MFMA residual MLP (forward, MSE gradient), the body-point
occupancy check and the amortised morph with its plain-morph fallback.

BF16 bar (FP32 accumulate against the FP64 oracle on the same BF16-valued weights
and inputs): |f_gpu - f| <= 2e-2 * (|f| + F_abs), F_abs = sum_k |W_L| |h_{L-1}| + |b_L|;
per-layer weight gradients within 2e-2 relative (Frobenius).
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_2108_11775_amd as P
from paper_2108_11775_amd import configs as K, inputs as I

from helpers import arm_scene, dev, gpu_occ, host, oracle_occ, require_gpu

pytestmark = pytest.mark.gpu


def _bf16(a):
    """Round FP32 values to BF16 (nearest even) and return them as FP32."""
    a = np.ascontiguousarray(np.asarray(a, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def _net(widths, seed=5, zero_last=False):
    layers = I.mlp_init(seed, widths, zero_last=zero_last)
    if not zero_last:  # give the last layer a realistic, non-zero scale
        W, b = layers[-1]
        layers[-1] = (W * 0.5, b * 0.5)
    return layers


@pytest.mark.parametrize("widths,B", [((7, 256, 256, 256, 7), 1000), ((7, 64, 64, 7), 4099),
                                      ((3, 96, 96, 96, 3), 77)])
def test_forward_bf16(widths, B):
    require_gpu()
    layers = _net(widths)
    mlp = P.Mlp.from_layers(layers)
    q = I.uniform_points(5, K.STREAM_EVAL, widths[0], B, -math.pi, math.pi)
    got = host(mlp.forward(dev(q)))
    # oracle on the BF16-valued weights and inputs (exact upcast); biases stay FP32
    lb = [(_bf16(W), b) for W, b in layers]
    f, fs = O.mlp_forward(widths, O.mlp_pack(lb), _bf16(q), residual=False, with_scale=True)
    fg = got.astype(np.float64) - q.astype(np.float64)
    err = np.abs(fg - f)
    assert np.all(err <= 2e-2 * (np.abs(f) + fs)), np.max(err / (np.abs(f) + fs))


def test_zero_last_layer_is_exact_identity():
    require_gpu()
    mlp = P.Mlp.from_layers(I.mlp_init(5, K.C5.widths))
    q = dev(I.uniform_points(5, K.STREAM_EVAL, 7, 3000, -math.pi, math.pi))
    assert np.array_equal(host(mlp.forward(q)), host(q))


@pytest.mark.parametrize("widths,B", [((7, 256, 256, 256, 7), 2048), ((7, 64, 64, 7), 3001)])
def test_mse_gradient_per_layer(widths, B):
    require_gpu()
    layers = _net(widths, seed=6)
    mlp = P.Mlp.from_layers(layers)
    q = I.uniform_points(6, K.STREAM_EVAL, widths[0], B, -math.pi, math.pi)
    t = q + 0.3 * I.rng(6, 13).normal(size=q.shape).astype(np.float32)
    acts = mlp.acts_buffer(B)
    qh = mlp.forward(dev(q), acts=acts)
    loss, grad = mlp.backward(qh, dev(t), acts)
    grad = host(grad)
    lb = [(_bf16(W), b) for W, b in layers]
    Pb = O.mlp_pack(lb)
    L, gref = O.mlp_loss_grad(widths, Pb, q, t)
    assert abs(host(loss)[0] - L) <= 2e-2 * L
    off = 0
    for li in range(len(widths) - 1):
        fi, fo = widths[li], widths[li + 1]
        for n_el in (fi * fo, fo):  # W then b
            a, b = grad[off:off + n_el], gref[off:off + n_el]
            assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b) + 1e-12, (li, n_el)
            off += n_el


def test_weighted_mse_gradient_matches_oracle():
    """The sample-weighted MSE (hard samples weigh 4) against the oracle's, at the BF16
    bar; no hard sample, or weight 1, gives the plain backward's bits."""
    require_gpu()
    widths, B = (7, 256, 256, 256, 7), 3000
    layers = _net(widths, seed=7)
    mlp = P.Mlp.from_layers(layers)
    q = I.uniform_points(7, K.STREAM_EVAL, 7, B, -math.pi, math.pi)
    t = q + 0.3 * I.rng(7, 13).normal(size=q.shape).astype(np.float32)
    hard = (I.rng(7, 14).uniform(size=B) < 0.3).astype(np.uint8)
    acts = mlp.acts_buffer(B)
    qh = mlp.forward(dev(q), acts=acts)
    loss, grad = mlp.backward(qh, dev(t), acts, hard=dev(hard), hard_weight=4.0)
    grad = host(grad)
    Pb = O.mlp_pack([(_bf16(W), b) for W, b in layers])
    L, gref = O.mlp_loss_grad_weighted(widths, Pb, q, t, hard, 4.0)
    assert abs(host(loss)[0] - L) <= 2e-2 * L
    off = 0
    for li in range(len(widths) - 1):
        fi, fo = widths[li], widths[li + 1]
        for n_el in (fi * fo, fo):
            a, b = grad[off:off + n_el], gref[off:off + n_el]
            assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b) + 1e-12, (li, n_el)
            off += n_el
    l0, g0 = mlp.backward(qh, dev(t), acts)
    l1, g1 = mlp.backward(qh, dev(t), acts, hard=dev(np.zeros(B, np.uint8)), hard_weight=4.0)
    l2, g2 = mlp.backward(qh, dev(t), acts, hard=dev(hard), hard_weight=1.0)
    g0, g1, g2 = host(g0), host(g1), host(g2)
    assert np.array_equal(g0, g1) and np.array_equal(g0, g2)
    assert host(l0)[0] == host(l1)[0] == host(l2)[0]


def test_arm_max_occupancy_matches_oracle():
    require_gpu()
    sc = arm_scene()
    a, d, al, th = sc["dh"]
    arm_o, arm_g = O.Arm(a, d, al, th, 8), P.Arm(a, d, al, th, 8)
    q = I.uniform_points(3, K.STREAM_EVAL, 7, 3000, -math.pi, math.pi)
    maxc, flag = P.arm_max_occupancy(gpu_occ(sc["h"], sc["wb"], sc["ell"]), arm_g, dev(q), 0.5)
    maxc, flag = host(maxc), host(flag)
    oo = oracle_occ(sc["h"], sc["wb"], sc["ell"])
    pts = O.fk_points(arm_o, q)
    ref = np.array([O.occ_eval(oo, pts[:, :, s])[1].max() for s in range(q.shape[1])])
    assert np.abs(maxc - ref).max() <= 1e-4
    sure = np.abs(ref - 0.5) > 1e-4
    assert np.array_equal(flag[sure], (ref[sure] > 0.5).astype(np.uint8))


def test_amortised_zero_network_is_plain_morph_on_flagged():
    require_gpu()
    sc = arm_scene()
    a, d, al, th = sc["dh"]
    arm_g = P.Arm(a, d, al, th, 8)
    occ = gpu_occ(sc["h"], sc["wb"], sc["ell"])
    mlp = P.Mlp.from_layers(I.mlp_init(5, K.C5.widths))
    q = dev(I.uniform_points(3, K.STREAM_EVAL, 7, 5000, -math.pi, math.pi))
    out, flag, nf = P.amortised_morph(mlp, occ, arm_g, q, K.C3.T, K.C3.eta)
    _, flag_ref = P.arm_max_occupancy(occ, arm_g, q, 0.5)
    plain = host(P.morph_samples(occ, q, K.C3.T, K.C3.eta, arm=arm_g))
    out, flag, qh = host(out), host(flag), host(q)
    assert np.array_equal(flag, host(flag_ref))
    assert int(host(nf)[0]) == int(flag.sum()) and 0 < flag.sum() < 5000
    f = flag.astype(bool)
    assert np.array_equal(out[:, f], plain[:, f])       # same kernel, same per-config arithmetic
    assert np.array_equal(out[:, ~f], qh[:, ~f])        # q_hat = q exactly


def test_amortised_matches_oracle():
    require_gpu()
    sc = arm_scene()
    a, d, al, th = sc["dh"]
    arm_o, arm_g = O.Arm(a, d, al, th, 8), P.Arm(a, d, al, th, 8)
    widths = (7, 64, 64, 7)
    layers = _net(widths, seed=8)
    layers[-1] = (layers[-1][0] * 0.05, layers[-1][1] * 0.05)
    mlp = P.Mlp.from_layers(layers)
    n = 48
    q = I.uniform_points(3, K.STREAM_EVAL, 7, n, -math.pi, math.pi)
    out, flag, _ = P.amortised_morph(mlp, gpu_occ(sc["h"], sc["wb"], sc["ell"]), arm_g, dev(q),
                                     K.C3.T, K.C3.eta)
    out, flag = host(out), host(flag)
    lb = [(_bf16(W), b) for W, b in layers]
    ref, fref, maxc = O.amortised_morph(widths, O.mlp_pack(lb), arm_o,
                                        oracle_occ(sc["h"], sc["wb"], sc["ell"]), q, K.C3.T,
                                        K.C3.eta)
    # the flag is decided in FP32 from a BF16 network: compare where the oracle's
    # max occupancy is clear of the threshold
    sure = np.abs(maxc - 0.5) > 2e-2
    assert np.array_equal(flag[sure], fref[sure])
    both = sure & (flag == 1)
    if both.any():
        _, amp, _ = O.morph_arm(arm_o, oracle_occ(sc["h"], sc["wb"], sc["ell"]), q[:, both],
                                K.C3.T, K.C3.eta, diag=True)
        err = np.abs(out[:, both] - ref[:, both]).max(axis=0)
        assert np.all(err <= 1e-5 * np.maximum(1, amp) * np.maximum(1, np.abs(ref[:, both]).max(axis=0)))
    keep = sure & (flag == 0)
    assert np.all(np.abs(out[:, keep] - ref[:, keep]) <= 2e-2 * (np.abs(ref[:, keep] - q[:, keep]) + 0.05))


def test_amortised_config5_full_batch_sampled():
    """The amortised morph at the workload's size and network: 7-256-256-256-7 (random
    initialisation, last layer scaled down) on 65,536 configurations in one call, its
    outputs sampled every 1,600th against the oracle's amortised morph of those
    configurations (a configuration's result does not depend on the rest of the
    batch)."""
    require_gpu()
    sc = arm_scene()
    a, d, al, th = sc["dh"]
    arm_o, arm_g = O.Arm(a, d, al, th, 8), P.Arm(a, d, al, th, 8)
    widths = (7, 256, 256, 256, 7)
    layers = _net(widths, seed=9)
    layers[-1] = (layers[-1][0] * 0.05, layers[-1][1] * 0.05)
    mlp = P.Mlp.from_layers(layers)
    c3 = K.C3
    n = c3.n_samples
    q = O.uniform_samples(I.philox_seed(c3.cfg_id), 11, [c3.q_lo] * 7, [c3.q_hi] * 7, n)
    out, flag, _ = P.amortised_morph(mlp, gpu_occ(sc["h"], sc["wb"], sc["ell"]), arm_g,
                                     dev(q), c3.T, c3.eta)
    idx = np.unique(np.r_[0, np.arange(1, n, 1600), n - 1])
    out, flag, qs = host(out)[:, idx], host(flag)[idx], np.ascontiguousarray(q[:, idx])
    oo = oracle_occ(sc["h"], sc["wb"], sc["ell"])
    lb = [(_bf16(W), b) for W, b in layers]
    ref, fref, maxc = O.amortised_morph(widths, O.mlp_pack(lb), arm_o, oo, qs, c3.T, c3.eta)
    sure = np.abs(maxc - 0.5) > 2e-2
    assert sure.sum() >= 0.8 * idx.size
    assert np.array_equal(flag[sure], fref[sure])
    both = sure & (flag == 1)
    assert both.any() and (sure & (flag == 0)).any()
    _, amp, _ = O.morph_arm(arm_o, oo, qs[:, both], c3.T, c3.eta, diag=True)
    err = np.abs(out[:, both] - ref[:, both]).max(axis=0)
    assert np.all(err <= 1e-5 * np.maximum(1, amp) * np.maximum(1, np.abs(ref[:, both]).max(axis=0)))
    keep = sure & (flag == 0)
    assert np.all(np.abs(out[:, keep] - ref[:, keep]) <= 2e-2 * (np.abs(ref[:, keep] - qs[:, keep]) + 0.05))


def test_training_reduces_loss_and_fallbacks():
    """The trained network beats the method without it: fewer fallbacks than the
    zero network (q_hat = q) on held-out configurations."""
    require_gpu()
    from paper_2108_11775_amd import amortise
    sc = arm_scene()
    a, d, al, th = sc["dh"]
    arm_g = P.Arm(a, d, al, th, 8)
    occ = gpu_occ(sc["h"], sc["wb"], sc["ell"])
    c3 = K.C3
    pairs = amortise.make_pairs(occ, arm_g, 8, 8192, c3.T, c3.eta, I.philox_seed(5), c3.q_lo, c3.q_hi)
    mlp = P.Mlp.from_layers(I.mlp_init(5, (7, 128, 128, 128, 7)))
    losses = host(amortise.train(mlp, pairs, 40, 2e-3))
    assert losses[-8:].mean() < 0.8 * losses[:8].mean()
    q = P.uniform_samples(I.philox_seed(5), 999, [c3.q_lo] * 7, [c3.q_hi] * 7, 8192)
    zero = P.Mlp.from_layers(I.mlp_init(5, (7, 128, 128, 128, 7)))
    _, f_zero, _ = P.amortised_morph(zero, occ, arm_g, q, c3.T, c3.eta)
    _, f_net, _ = P.amortised_morph(mlp, occ, arm_g, q, c3.T, c3.eta)
    assert host(f_net).mean() < host(f_zero).mean()


def test_amortised_config5_grid_path_sampled():
    """The amortised morph on the bench's own path: the 16^3 hinge grid (the check of
    q_hat on the grid arm kernel, the fallback morph on the grid arm kernel with the
    FP16 split scheme this world's weights take) and a non-zero 7-256-256-256-7
    network, 65,536 configurations in one call, every 1,600th compared with the
    oracle's amortised morph; the fallbacks are also the plain grid morph's bits."""
    require_gpu()
    sc = arm_scene()
    a, d, al, th = sc["dh"]
    arm_o, arm_g = O.Arm(a, d, al, th, 8), P.Arm(a, d, al, th, 8)
    widths = (7, 256, 256, 256, 7)
    layers = _net(widths, seed=9)
    layers[-1] = (layers[-1][0] * 0.05, layers[-1][1] * 0.05)
    mlp = P.Mlp.from_layers(layers)
    c3 = K.C3
    n = c3.n_samples
    q = O.uniform_samples(I.philox_seed(c3.cfg_id), 11, [c3.q_lo] * 7, [c3.q_hi] * 7, n)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"], (16, 16, 16))
    assert P.split_scheme(go) == ("fp16", 3)
    q_d = dev(q)
    out, flag, nf = P.amortised_morph(mlp, go, arm_g, q_d, c3.T, c3.eta)
    plain = host(P.morph_samples(go, q_d, c3.T, c3.eta, arm=arm_g))
    out, flag = host(out), host(flag)
    P.sync()
    assert int(host(nf)[0]) == int(flag.sum()) and 0 < flag.sum() < n
    fb = flag.astype(bool)
    assert np.array_equal(out[:, fb], plain[:, fb])
    idx = np.unique(np.r_[0, np.arange(1, n, 1600), n - 1])
    out, flag, qs = out[:, idx], flag[idx], np.ascontiguousarray(q[:, idx])
    oo = oracle_occ(sc["h"], sc["wb"], sc["ell"])
    lb = [(_bf16(W), b) for W, b in layers]
    ref, fref, maxc = O.amortised_morph(widths, O.mlp_pack(lb), arm_o, oo, qs, c3.T, c3.eta)
    sure = np.abs(maxc - 0.5) > 2e-2
    assert sure.sum() >= 0.8 * idx.size
    assert np.array_equal(flag[sure], fref[sure])
    both = sure & (flag == 1)
    assert both.any() and (sure & (flag == 0)).any()
    _, amp, _ = O.morph_arm(arm_o, oo, qs[:, both], c3.T, c3.eta, diag=True)
    err = np.abs(out[:, both] - ref[:, both]).max(axis=0)
    assert np.all(err <= 1e-5 * np.maximum(1, amp) * np.maximum(1, np.abs(ref[:, both]).max(axis=0)))
    keep = sure & (flag == 0)
    assert np.all(np.abs(out[:, keep] - ref[:, keep]) <= 2e-2 * (np.abs(ref[:, keep] - qs[:, keep]) + 0.05))


def test_refining_variant_on_the_grid_path():
    """The refining amortised morph (flagged configurations take T_refine plain steps
    from q_hat) on the bench's path: 16^3 grid, 7-256-256-256-7 network, 65,536
    configurations.  Unflagged outputs are q_hat's bits; flagged ones are the plain
    grid morph of q_hat (same bits) and, sampled, the oracle's morph of the GPU's q_hat
    within the arm tolerance; the flags agree with the oracle's occupancy at the GPU's
    q_hat away from the threshold.  A zero network gives the plain-fallback amortised
    morph's bits."""
    require_gpu()
    sc = arm_scene()
    a, d, al, th = sc["dh"]
    arm_o, arm_g = O.Arm(a, d, al, th, 8), P.Arm(a, d, al, th, 8)
    widths = (7, 256, 256, 256, 7)
    layers = _net(widths, seed=10)
    layers[-1] = (layers[-1][0] * 0.05, layers[-1][1] * 0.05)
    mlp = P.Mlp.from_layers(layers)
    c3 = K.C3
    n, Tr, thr = c3.n_samples, 8, 0.3
    q = O.uniform_samples(I.philox_seed(c3.cfg_id), 12, [c3.q_lo] * 7, [c3.q_hi] * 7, n)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"], (16, 16, 16))
    q_d = dev(q)
    out, flag, nf = P.amortised_morph(mlp, go, arm_g, q_d, Tr, c3.eta, thr, refine=True)
    qh = mlp.forward(q_d)
    polished = host(P.morph_samples(go, qh, Tr, c3.eta, arm=arm_g))
    out, flag, qh = host(out), host(flag), host(qh)
    P.sync()
    fb = flag.astype(bool)
    assert int(host(nf)[0]) == int(fb.sum()) and 0 < fb.sum() < n
    assert np.array_equal(out[:, ~fb], qh[:, ~fb])
    assert np.array_equal(out[:, fb], polished[:, fb])
    idx = np.unique(np.r_[0, np.arange(1, n, 1600), n - 1])
    oo = oracle_occ(sc["h"], sc["wb"], sc["ell"])
    qhs = np.ascontiguousarray(qh[:, idx]).astype(np.float64)
    pts = O.fk_points(arm_o, qhs)
    maxc = np.array([O.occ_eval(oo, pts[:, :, s])[1].max() for s in range(idx.size)])
    sure = np.abs(maxc - thr) > 1e-4
    assert np.array_equal(flag[idx][sure], (maxc[sure] > thr).astype(np.uint8))
    sel = idx[fb[idx]]
    assert sel.size > 0
    ref, amp, _ = O.morph_arm(arm_o, oo, np.ascontiguousarray(qh[:, sel]).astype(np.float64), Tr,
                              c3.eta, diag=True)
    err = np.abs(out[:, sel] - ref).max(axis=0)
    assert np.all(err <= 1e-5 * np.maximum(1, amp) * np.maximum(1, np.abs(ref).max(axis=0)))
    # a zero network: q_hat = q, so the refining variant is the plain-fallback one
    zero = P.Mlp.from_layers(I.mlp_init(5, widths))
    z1, f1, _ = P.amortised_morph(zero, go, arm_g, q_d, c3.T, c3.eta, 0.5)
    z2, f2, _ = P.amortised_morph(zero, go, arm_g, q_d, c3.T, c3.eta, 0.5, refine=True)
    assert np.array_equal(host(f1), host(f2)) and np.array_equal(host(z1), host(z2))


def test_amortised_trained_network_grid_path_sampled():
    """A network trained by the library itself (plain-morph pairs on the 16^3 grid path,
    Adam through the BF16 forward/backward kernels) in the amortised morph on the grid
    path, 65,536 configurations, every 1,600th against the oracle's amortised morph
    with the same (BF16-rounded) weights: the trained f(q) is far from zero, so the
    BF16 bar on the network's output and the flags are tested where they matter."""
    from paper_2108_11775_amd import amortise
    require_gpu()
    sc = arm_scene()
    a, d, al, th = sc["dh"]
    arm_o, arm_g = O.Arm(a, d, al, th, 8), P.Arm(a, d, al, th, 8)
    c3, c5 = K.C3, K.C5
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"], (16, 16, 16))
    pairs = amortise.make_pairs(go, arm_g, 4, 8192, c3.T, c3.eta, I.philox_seed(c5.cfg_id, 77),
                                c3.q_lo, c3.q_hi)
    mlp = P.Mlp.from_layers(I.mlp_init(c5.cfg_id, c5.widths))
    losses = host(amortise.train(mlp, pairs, 40, 3e-3, schedule="cosine"))
    assert losses[-1] < 0.9 * losses[0]  # from f = 0 (MSE 0.06) towards the targets
    n = c3.n_samples
    q = O.uniform_samples(I.philox_seed(c3.cfg_id), 13, [c3.q_lo] * 7, [c3.q_hi] * 7, n)
    out, flag, nf = P.amortised_morph(mlp, go, arm_g, dev(q), c3.T, c3.eta)
    out, flag = host(out), host(flag)
    idx = np.unique(np.r_[0, np.arange(1, n, 1600), n - 1])
    out, flag, qs = out[:, idx], flag[idx], np.ascontiguousarray(q[:, idx])
    layers = O.mlp_unpack(host(mlp.params).astype(np.float64), c5.widths)
    Pb = O.mlp_pack([(_bf16(W), b) for W, b in layers])
    oo = oracle_occ(sc["h"], sc["wb"], sc["ell"])
    ref, fref, maxc = O.amortised_morph(c5.widths, Pb, arm_o, oo, qs, c3.T, c3.eta)
    fq, fs = O.mlp_forward(c5.widths, Pb, qs, residual=False, with_scale=True)
    assert np.abs(fq).max() > 0.1  # a trained, non-trivial correction
    sure = np.abs(maxc - 0.5) > 2e-2
    assert sure.sum() >= 0.8 * idx.size
    assert np.array_equal(flag[sure], fref[sure])
    both = sure & (flag == 1)
    assert both.any() and (sure & (flag == 0)).any()
    _, amp, _ = O.morph_arm(arm_o, oo, qs[:, both], c3.T, c3.eta, diag=True)
    err = np.abs(out[:, both] - ref[:, both]).max(axis=0)
    assert np.all(err <= 1e-5 * np.maximum(1, amp) * np.maximum(1, np.abs(ref[:, both]).max(axis=0)))
    # kept configurations: q + f(q), f at the BF16 bar of the forward tests (relative to
    # |f| + F_abs, F_abs = sum |W_L| |h| + |b_L|), plus the rounding of q + f in FP32
    keep = sure & (flag == 0)
    bound = 2e-2 * (np.abs(fq[:, keep]) + fs[:, keep]) + 2.0 ** -22 * np.abs(qs[:, keep])
    assert np.all(np.abs(out[:, keep] - ref[:, keep]) <= bound)
