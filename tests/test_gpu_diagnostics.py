"""The library's own reports about how it ran: the split scheme the grid morph kernels
take (held to the documented rule, stated independently in the tests' helpers) and
the measured issue costs the benchmark states its ceilings with."""
import math

import numpy as np
import pytest

import paper_2108_11775_amd as P
from paper_2108_11775_amd import configs as K

from helpers import arm_scene, gpu_occ, require_gpu, split_rule, ws_scene

pytestmark = pytest.mark.gpu


def _grid2(ax, ay):
    j = np.arange(ax.size * ay.size)
    return np.stack([ax[j % ax.size], ay[j // ax.size]]).astype(np.float32)


def test_split_scheme_reported_by_the_library():
    require_gpu()
    for cfg in (K.C1, K.C2):
        sc = ws_scene(cfg)
        go = gpu_occ(sc["h"], sc["wb"], sc["ell"], (cfg.grid, cfg.grid))
        assert P.split_scheme(go) == ("fp16", 3) == split_rule(sc["h"][0, :cfg.grid],
                                                                sc["wb"][:-1], sc["ell"])
        assert P.split_scheme(gpu_occ(sc["h"], sc["wb"], sc["ell"])) == ("pairwise", None)
    a = arm_scene()
    assert P.split_scheme(gpu_occ(a["h"], a["wb"], a["ell"], (16, 16, 16))) == ("fp16", 3)
    rng = np.random.default_rng(77)
    ell = 0.5
    kappa = math.sqrt(math.log2(math.e) / 2.0) / ell
    for case in range(12):
        g0, g1 = int(rng.integers(1, 65)), int(rng.integers(1, 65))
        ax = np.sort(rng.uniform(-3, 3, g0)).astype(np.float32)
        if case % 3 == 1 and g0 > 1:  # a gap just above or below the limit
            ax[g0 // 2:] += np.float32((6.0 + rng.choice([-0.05, 0.05])) / kappa)
        ay = np.sort(rng.uniform(-2, 2, g1)).astype(np.float32)
        wb = rng.normal(0, 1, g0 * g1 + 1).astype(np.float32)
        if case % 3 == 2:  # one weight just inside or outside the 2^-19 range
            wb[0] = np.float32(np.abs(wb[:-1]).max() * 2.0 ** (-19 + rng.choice([-0.01, 0.01])))
        go = gpu_occ(_grid2(ax, ay), wb, ell, (g0, g1))
        assert P.split_scheme(go) == split_rule(ax, wb[:-1], ell), (case, g0, g1)


def test_issue_rates_measured():
    """Plausible figures: each class costs at least a full-rate wave64 instruction's
    2 cycles on a 32-lane SIMD issue (the FP32 vector peak counts 64 flops per SIMD per
    cycle) and the transcendental no less than the FMA; the clock lies in the part's
    range."""
    require_gpu()
    r = P.issue_rates()
    assert all(np.isfinite(v) and v > 0 for v in r.values()), r
    assert 0.5 <= r["clock_ghz"] <= 2.6
    assert r["v_exp_f32"] >= r["v_fma_f32"] >= 1.5
    assert r["v_mfma_f32_32x32x16_f16"] >= 16
    print(f"\n[issue rates] {r}", flush=True)
