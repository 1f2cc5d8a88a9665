"""The tensor-grid statement of an occupancy is checked on the device: hinges that are
not the grid the `grid` field states are reported by the next pdmp_sync as
PDMP_EINVAL (the launch itself runs to completion; its results are undefined), for
every entry point that may take the grid factorisation.  A valid grid raises nothing,
and the report is cleared once taken."""
import math

import numpy as np
import pytest

import paper_2108_11775_amd as P
from paper_2108_11775_amd import _lib, configs as K, inputs as I

from helpers import arm_scene, dev, gpu_occ, host, require_gpu, ws_scene

pytestmark = pytest.mark.gpu


def _expect_einval():
    with pytest.raises(P.PdmpError) as e:
        P.sync()
    assert e.value.status == _lib.PDMP_EINVAL
    assert "tensor grid" in str(e.value)
    P.sync()  # taken: the next sync reports nothing


def _bad(h, j, k):
    h = h.copy()
    h[k, j] = np.nextafter(h[k, j], np.float32(np.inf), dtype=np.float32)
    return h


@pytest.mark.parametrize("j,k", [(0, 0), (777, 1), (4095, 0), (130, 1)])
def test_2d_non_grid_hinges_reported(j, k):
    require_gpu()
    cfg = K.C2
    sc = ws_scene(cfg)
    x = dev(I.uniform_points(cfg.cfg_id, K.STREAM_EVAL, 2, 5000, cfg.lo, cfg.hi))
    good = gpu_occ(sc["h"], sc["wb"], sc["ell"], (cfg.grid, cfg.grid))
    ref = host(P.morph_samples(good, x, 5, cfg.eta))
    P.sync()
    bad = gpu_occ(_bad(sc["h"], j, k), sc["wb"], sc["ell"], (cfg.grid, cfg.grid))
    P.morph_samples(bad, x, 5, cfg.eta)
    _expect_einval()
    P.occupancy_eval(bad, x)
    _expect_einval()
    P.occupancy_grad(bad, x)
    _expect_einval()
    P.morph_logdet(bad, x, 3, cfg.eta)
    _expect_einval()
    # the device is fine afterwards: a valid call gives the same bits as before
    assert np.array_equal(host(P.morph_samples(good, x, 5, cfg.eta)), ref)
    P.sync()


def test_3d_and_arm_non_grid_hinges_reported():
    require_gpu()
    sc = arm_scene()
    a, d, al, th = sc["dh"]
    arm = P.Arm(a, d, al, th, 8)
    q = dev(I.uniform_points(3, K.STREAM_EVAL, 7, 300, -math.pi, math.pi))
    x = dev(I.uniform_points(3, K.STREAM_EVAL, 3, 300, -1.0, 1.0))
    good = gpu_occ(sc["h"], sc["wb"], sc["ell"], (16, 16, 16))
    P.morph_samples(good, q, 2, 0.01, arm=arm)
    P.occupancy_bwd(good, x, dev(np.ones(300, np.float32)), want_x=False)
    P.sync()
    bad = gpu_occ(_bad(sc["h"], 16 * 16 * 9 + 3, 2), sc["wb"], sc["ell"], (16, 16, 16))
    P.morph_samples(bad, q, 2, 0.01, arm=arm)
    _expect_einval()
    P.arm_max_occupancy(bad, arm, q, 0.5)
    _expect_einval()
    P.occupancy_bwd(bad, x, dev(np.ones(300, np.float32)), want_x=False)
    _expect_einval()
    P.morph_samples(bad, x, 2, 0.002)
    _expect_einval()


def test_nan_hinge_reported_and_no_grid_not_checked():
    require_gpu()
    cfg = K.C1
    sc = ws_scene(cfg)
    h = sc["h"].copy()
    h[1, 40] = np.nan
    x = dev(I.uniform_points(cfg.cfg_id, K.STREAM_EVAL, 2, 100, cfg.lo, cfg.hi))
    P.morph_samples(gpu_occ(h, sc["wb"], sc["ell"], (cfg.grid, cfg.grid)), x, 2, cfg.eta)
    _expect_einval()
    # without the grid statement the pairwise kernel reads every hinge: nothing to check
    P.morph_samples(gpu_occ(_bad(sc["h"], 3, 0), sc["wb"], sc["ell"]), x, 2, cfg.eta)
    P.sync()
