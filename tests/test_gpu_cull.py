"""GPU parity of the culled morph (compact-support hinge culling, a variant beyond the
paper) against the oracle's culled morph on the same cell grid (FP32 tolerance as
the plain morph), plus the grid definition, determinism and batch independence."""
import math

import numpy as np
import pytest

import oracle as O
import paper_2108_11775_amd as P
from paper_2108_11775_amd import configs as K, inputs as I

from helpers import dev, gpu_occ, host, oracle_occ, require_gpu, ws_scene

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _grids(dim, lo, hi, rc):
    g = P.cull_grid(dim, lo, hi, rc)
    og = O.CullGrid.make(lo, hi, rc)
    assert g.inv_cell == np.float32(og.inv_cell)
    assert [g.nc[k] for k in range(dim)] == list(og.nc)
    return g, og


def _check(go, oo, g, og, x0, T, eta):
    out = host(P.morph_culled(go, g, dev(x0), T, eta))
    ref = O.morph_culled(oo, og, x0, T, eta)
    _, amp, _, _ = O.morph_ws(oo, x0, T, eta, diag=True)
    err = np.abs(out - ref).max(axis=0)
    bound = TOL * np.maximum(1, amp) * np.maximum(1, np.abs(ref).max(axis=0))
    assert np.all(err <= bound), np.max(err / bound)
    return out


@pytest.mark.parametrize("n", [1, 63, 5001])
def test_culled_morph_config2_scene(n):
    require_gpu()
    cfg = K.C2
    sc = ws_scene(cfg)
    go, oo = gpu_occ(sc["h"], sc["wb"], sc["ell"]), oracle_occ(sc["h"], sc["wb"], sc["ell"])
    g, og = _grids(2, [cfg.lo] * 2, [cfg.hi] * 2, 5.5 * cfg.lengthscale)
    x0 = I.uniform_points(cfg.cfg_id, K.STREAM_EVAL, 2, n, cfg.lo, cfg.hi)
    _check(go, oo, g, og, x0, cfg.T, cfg.eta)


def test_culled_morph_full_size_sampled_and_deterministic():
    require_gpu()
    cfg = K.C2
    sc = ws_scene(cfg)
    go, oo = gpu_occ(sc["h"], sc["wb"], sc["ell"]), oracle_occ(sc["h"], sc["wb"], sc["ell"])
    g, og = _grids(2, [cfg.lo] * 2, [cfg.hi] * 2, 5.5 * cfg.lengthscale)
    x0 = P.uniform_samples(I.philox_seed(cfg.cfg_id), 0, [cfg.lo] * 2, [cfg.hi] * 2, cfg.n_samples)
    a = host(P.morph_culled(go, g, x0, cfg.T, cfg.eta))
    b = host(P.morph_culled(go, g, x0, cfg.T, cfg.eta))
    assert np.array_equal(a, b)
    n = cfg.n_samples
    idx = np.unique(np.r_[0, np.arange(1, n, n // 300), n - 1])
    x0h = host(x0)[:, idx]
    ref = O.morph_culled(oo, og, x0h, cfg.T, cfg.eta)
    _, amp, _, _ = O.morph_ws(oo, x0h, cfg.T, cfg.eta, diag=True)
    err = np.abs(a[:, idx] - ref).max(axis=0)
    assert np.all(err <= TOL * np.maximum(1, amp) * np.maximum(1, np.abs(ref).max(axis=0)))
    # a point's result does not depend on the rest of the batch
    c = host(P.morph_culled(go, g, dev(np.ascontiguousarray(x0h)), cfg.T, cfg.eta))
    assert np.array_equal(c, a[:, idx])
    # and the culled morph stays close to the dense one (within the tail bound's effect)
    dense = host(P.morph_samples(go, x0, cfg.T, cfg.eta))
    assert np.median(np.abs(dense - a).max(axis=0)) < 1e-3


@pytest.mark.parametrize("n", [17, 3000])
def test_culled_morph_3d(n):
    require_gpu()
    rng = np.random.default_rng(n)
    h = rng.uniform(-1, 1, (3, 600)).astype(np.float32)
    wb = np.r_[rng.normal(0, 1.5, 600), -0.4].astype(np.float32)
    go, oo = gpu_occ(h, wb, 0.15), oracle_occ(h, wb, 0.15)
    g, og = _grids(3, [-1] * 3, [1] * 3, 4.0 * 0.15)
    x0 = rng.uniform(-1.1, 1.1, (3, n)).astype(np.float32)
    _check(go, oo, g, og, x0, 10, 0.005)


def test_culled_morph_many_cells():
    """More than 8192 cells (100 x 100 of side >= 0.2 on the config-2 box): the samples'
    counting sort takes its global-atomic path instead of the per-block LDS
    histograms; the result is the oracle's culled morph on the same cells.  A cutoff
    of half a lengthscale makes the culled field jump at cell faces, so one step
    (both sides choose cells from the same input) keeps the comparison free of a
    rounding-decided cell change."""
    require_gpu()
    cfg = K.C2
    sc = ws_scene(cfg)
    go, oo = gpu_occ(sc["h"], sc["wb"], sc["ell"]), oracle_occ(sc["h"], sc["wb"], sc["ell"])
    g, og = _grids(2, [cfg.lo] * 2, [cfg.hi] * 2, 0.2)
    assert g.nc[0] * g.nc[1] > 8192
    x0 = I.uniform_points(cfg.cfg_id, K.STREAM_EVAL, 2, 3000, cfg.lo, cfg.hi)
    _check(go, oo, g, og, x0, 1, cfg.eta)
