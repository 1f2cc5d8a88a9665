"""The largest batches.  A prior batch of 2^31 + 2^20 + 3 samples, so that sample
indices and label offsets use the top bit of 32 with a ragged tail: its samples
against the oracle's indexed form at sampled indices (the two ends, both sides of
2^31, random ones), its labels likewise and their count against their sum.  A morph of
that batch exceeds one kernel dispatch (2^32 - 1 work-items at two threads per point)
and must fail with PDMP_EINVAL, not run a truncated grid.  At the largest batch the
grid paths take, 2^31 - 1029 samples (ragged for the 8 parts and the 128-sample
blocks), the ordered morph and log-determinant must give the unordered kernels' bits
over the whole batch, and the morph the oracle's parity at the sampled points.  About
80 GB of device memory (skipped where less is free)."""
import numpy as np
import pytest

import oracle as O
import paper_2108_11775_amd as P
from paper_2108_11775_amd import _lib, configs as K, inputs as I

from helpers import dev, gpu_occ, host, oracle_occ, require_gpu, ws_scene

pytestmark = pytest.mark.gpu

N_BIG = (1 << 31) + (1 << 20) + 3
N_MAX = (1 << 31) - 1029


def _indices(rng, n, extra):
    return np.unique(np.r_[0, 1, 2, n - 3, n - 2, n - 1, extra,
                           rng.integers(0, n, 3000)]).astype(np.int64)


def test_batch_past_2_31_samples():
    require_gpu()
    import torch
    free, _ = torch.cuda.mem_get_info()
    if free < 90e9:
        pytest.skip(f"needs about 90 GB of free device memory ({free / 1e9:.0f} GB free)")
    cfg = K.C2
    sc = ws_scene(cfg)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"], (cfg.grid, cfg.grid))
    oo = oracle_occ(sc["h"], sc["wb"], sc["ell"])
    dc, dr = sc["discs"]
    seed, lo, hi = I.philox_seed(cfg.cfg_id), [cfg.lo] * 2, [cfg.hi] * 2
    rng = np.random.default_rng(231)

    # the prior batch and its labels past 2^31 samples
    idx = _indices(rng, N_BIG, [(1 << 31) - 1, 1 << 31, (1 << 31) + 1, (1 << 32) - 1 - (1 << 31)])
    idx_d = dev(idx)
    x = P.uniform_samples(seed, 9, lo, hi, N_BIG)
    xs = host(x[:, idx_d])
    assert np.array_equal(xs, O.uniform_at(seed, 9, lo, hi, idx))
    lab, hit = P.label_points_discs(dev(dc), dev(dr), x, count=True)
    assert np.array_equal(host(lab[idx_d]), O.label_discs(dc, dr, xs))
    assert int(host(hit)[0]) == int(lab.sum(dtype=torch.int64).item())
    del lab
    # a morph of it would need more than one dispatch: a clean error, whichever path
    for call in (lambda: P.morph_samples(go, x, 2, cfg.eta),
                 lambda: P.morph_samples_ws(go, x, 2, cfg.eta),
                 lambda: P.morph_logdet(go, x, 1, cfg.eta, ordered=True)):
        with pytest.raises(P.PdmpError) as e:
            call()
        assert e.value.status == _lib.PDMP_EINVAL
        assert "dispatch" in str(e.value)
    del x
    torch.cuda.empty_cache()

    # the largest batch the grid paths take
    idx = _indices(rng, N_MAX, [(1 << 30), (1 << 31) - 1030])
    idx_d = dev(idx)
    x = P.uniform_samples(seed, 9, lo, hi, N_MAX)
    xs = host(x[:, idx_d])
    T = 2
    ws = P.morph_workspace(go, N_MAX, T)
    assert ws is not None
    a = P.morph_samples_ws(go, x, T, cfg.eta, ws=ws)
    b = P.morph_samples(go, x, T, cfg.eta)
    assert torch.equal(a, b)
    got = host(a[:, idx_d])
    del a, b
    ref, amp, _, _ = O.morph_ws(oo, xs, T, cfg.eta, diag=True)
    err = np.abs(got - ref).max(axis=0)
    tol = 1e-5 * np.maximum(1, amp) * np.maximum(1, np.abs(ref).max(axis=0))
    assert np.all(err <= tol), float(np.max(err / tol))
    # the ordered log-determinant over one step, against the unordered kernel's bits
    o1, l1 = P.morph_logdet(go, x, 1, cfg.eta, ordered=True, ws=ws)
    o2, l2 = P.morph_logdet(go, x, 1, cfg.eta)
    assert torch.equal(o1, o2) and torch.equal(l1, l2)
    del o1, o2, l1, l2, x, ws
    torch.cuda.empty_cache()
    P.sync()
