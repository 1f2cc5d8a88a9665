"""GPU parity: prior samples and collision labels, bit-exact against the oracle."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import paper_2108_11775_amd as P
from paper_2108_11775_amd import configs as K, inputs as I

from helpers import GOLDEN, arm_scene, dev, host, require_gpu, ws_scene

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,n,lo,hi", [
    (2, 10007, [-10.0, -10.0], [10.0, 10.0]),
    (7, 4099, [-math.pi] * 7, [math.pi] * 7),
    (3, 1, [-1.0, -0.5, 0.0], [1.0, 0.5, 3.0]),
])
def test_uniform_samples_bit_exact(dim, n, lo, hi):
    require_gpu()
    seed = I.philox_seed(2)
    got = host(P.uniform_samples(seed, 5, lo, hi, n))
    ref = O.uniform_samples(seed, 5, lo, hi, n)
    assert got.dtype == np.float32 and np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_uniform_samples_full_size_sampled():
    require_gpu()
    cfg = K.C2
    seed = I.philox_seed(cfg.cfg_id)
    got = host(P.uniform_samples(seed, 0, [cfg.lo] * 2, [cfg.hi] * 2, cfg.n_samples))
    ref = O.uniform_samples(seed, 0, [cfg.lo] * 2, [cfg.hi] * 2, cfg.n_samples)
    assert np.array_equal(got, ref)


def test_label_discs_bit_exact_and_count():
    require_gpu()
    cfg = K.C2
    sc = ws_scene(cfg)
    dc, dr = sc["discs"]
    x = O.uniform_samples(I.philox_seed(cfg.cfg_id), 1, [cfg.lo] * 2, [cfg.hi] * 2, 70001)
    lab, hit = P.label_points_discs(dev(dc), dev(dr), dev(x), count=True)
    ref = O.label_discs(dc, dr, x)
    assert np.array_equal(host(lab), ref)
    assert int(host(hit)[0]) == int(ref.sum())


def test_label_tiny_scenes_bit_exact():
    require_gpu()
    d = json.load(open(os.path.join(GOLDEN, "labels_tiny.json")))
    ds, bs = d["discs"], d["boxes"]
    lab = P.label_points_discs(dev(np.asarray(ds["centres"], np.float32)),
                               dev(np.asarray(ds["radii"], np.float32)),
                               dev(np.asarray(ds["points"], np.float32).T.copy()))
    assert host(lab).tolist() == ds["expected"]
    lab = P.label_points_boxes(dev(np.asarray(bs["centres"], np.float32)),
                               dev(np.asarray(bs["half"], np.float32)),
                               dev(np.asarray(bs["points"], np.float32).T.copy()))
    assert host(lab).tolist() == bs["expected"]


def test_label_boxes_bit_exact():
    require_gpu()
    sc = arm_scene()
    bc, be = sc["boxes"]
    x = I.uniform_points(K.C4.cfg_id, K.STREAM_FIT, 3, 100003, -1.0, 1.0)
    lab, hit = P.label_points_boxes(dev(bc), dev(be), dev(x), count=True)
    ref = O.label_boxes(bc, be, x)
    assert np.array_equal(host(lab), ref)
    assert int(host(hit)[0]) == int(ref.sum())


def test_label_configs_match_outside_rounding_band():
    require_gpu()
    sc = arm_scene()
    a, d, al, th = sc["dh"]
    bc, be = sc["boxes"]
    arm_o = O.Arm(a, d, al, th, 8)
    arm_g = P.Arm(a, d, al, th, 8)
    q = O.uniform_samples(I.philox_seed(3), 0, [K.C3.q_lo] * 7, [K.C3.q_hi] * 7, 20011)
    lab, hit = P.label_configs(arm_g, dev(bc), dev(be), dev(q), count=True)
    ref = O.label_configs(arm_o, bc, be, q)
    margin = O.config_label_margin(arm_o, bc, be, q)
    # Both sides decide in FP64; only the sine/cosine libraries differ (about 1 ulp),
    # so labels may differ only for body points within ~1e-12 of a box face.
    sure = margin > 1e-12
    got = host(lab)
    assert np.array_equal(got[sure], ref[sure])
    assert (~sure).sum() <= 2
    assert int(host(hit)[0]) == int(got.sum())


def test_empty_label_batch_counts_zero():
    require_gpu()
    import torch
    sc = ws_scene(K.C1)
    dc, dr = sc["discs"]
    lab, hit = P.label_points_discs(dev(dc), dev(dr), torch.empty((2, 0), device="cuda"), count=True)
    assert lab.numel() == 0 and int(host(hit)[0]) == 0
