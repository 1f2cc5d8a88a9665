"""GPU side of the producer/consumer (Sec. 3.3): the background sampler's bucket holds
exactly the morph of its Philox prior batches, a stalled producer leaves the consumer
on the prior without waiting, and the RRT consumer matches the oracle's replay."""
import time

import numpy as np
import pytest

import oracle as O
from oracle import rrt as R
import paper_2108_11775_amd as P
from paper_2108_11775_amd import configs as K, inputs as I

from helpers import dev, gpu_occ, host, require_gpu, ws_scene

pytestmark = pytest.mark.gpu


def _sampler(batch=4096, capacity=1 << 14, paused=False):
    cfg = K.C2
    sc = ws_scene(cfg)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"], grid=(cfg.grid, cfg.grid))
    s = P.Sampler(go, 2, [cfg.lo] * 2, [cfg.hi] * 2, cfg.T, cfg.eta, batch, capacity,
                  seed=I.philox_seed(2), stream_id=100, prior_stream_id=7)
    if paused:
        s.pause(True)
    s.start()
    return cfg, sc, go, s


def _wait(s, produced, timeout=20.0):
    t0 = time.time()
    while s.stats()["produced"] < produced:
        assert time.time() - t0 < timeout, s.stats()
        time.sleep(0.005)


def test_bucket_holds_the_morph_of_the_prior_batches():
    require_gpu()
    cfg, sc, go, s = _sampler()
    _wait(s, 3 * 4096)
    x, idx, fb = s.pop(3 * 4096)
    assert fb.all() and np.array_equal(idx, np.arange(3 * 4096))
    for b in range(3):
        x0 = P.uniform_samples(I.philox_seed(2), 100 + b, [cfg.lo] * 2, [cfg.hi] * 2, 4096)
        ref = host(P.morph_samples(go, x0, cfg.T, cfg.eta))
        assert np.array_equal(x[b * 4096:(b + 1) * 4096].T, ref)
    st = s.stats()
    assert st["status"] == 0 and st["popped_bucket"] == 3 * 4096
    assert s.close() == 0


def test_stalled_producer_never_blocks_the_consumer():
    require_gpu()
    cfg, sc, go, s = _sampler(paused=True)
    t0 = time.perf_counter()
    x, idx, fb = s.pop(200000)
    dt = time.perf_counter() - t0
    assert not fb.any() and dt < 2.0
    ref = O.uniform_samples(I.philox_seed(2), 7, [cfg.lo] * 2, [cfg.hi] * 2, 200000)
    assert np.array_equal(x.T, ref)
    assert s.stats()["produced"] == 0
    s.pause(False)
    _wait(s, 4096)
    _, _, fb2 = s.pop(100)
    assert fb2.all()
    assert s.close() == 0


def test_rrt_on_the_sampler_matches_the_oracle_replay():
    require_gpu()
    cfg, sc, go, s = _sampler(batch=16384, capacity=1 << 16)
    _wait(s, 16384)
    dc, dr = sc["discs"]
    start, goal = K.RRT_START_GOAL[2]
    res = P.rrt_run(s, start, goal, 0.5, -1.0, (dc, dr), 6000)
    cen = np.asarray(dc, np.float64)
    nodes, parents, solved, it = R.rrt_replay(res["samples"], start, goal, 0.5, -1.0,
                                              (cen[0], cen[1], np.asarray(dr, np.float64)))
    assert it == res["iters"] and bool(solved) == bool(res["solved"])
    assert np.array_equal(nodes, res["nodes"]) and np.array_equal(parents, res["parent"])
    assert res["from_bucket"] > 0
    assert s.close() == 0


def test_producer_failure_reaches_the_consumer():
    """A producer whose device allocation fails (a batch far beyond device memory:
    hipMalloc returns an error, nothing is launched) stops with PDMP_EDEVICE; the
    consumer sees the status and the producer's message, and keeps drawing from
    the prior without waiting."""
    require_gpu()
    cfg = K.C2
    sc = ws_scene(cfg)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"], grid=(cfg.grid, cfg.grid))
    s = P.Sampler(go, 2, [cfg.lo] * 2, [cfg.hi] * 2, cfg.T, cfg.eta, 1 << 42, 1 << 10,
                  seed=I.philox_seed(2), stream_id=100, prior_stream_id=7)
    s.start()
    t0 = time.time()
    while s.stats()["running"]:
        assert time.time() - t0 < 20.0
        time.sleep(0.005)
    st = s.stats()
    assert st["status"] == 3 and st["produced"] == 0
    assert st["error"].startswith("sampler producer: hipMalloc"), st["error"]
    x, idx, fb = s.pop(5)
    assert not fb.any() and list(idx) == [-1, -2, -3, -4, -5]
    ref = O.uniform_samples(I.philox_seed(2), 7, [cfg.lo] * 2, [cfg.hi] * 2, 5)
    assert np.array_equal(x, ref.T)
    # a second start after the failure is refused with the failure's message (the
    # stopped producer thread is joined, not replaced)
    with pytest.raises(P.PdmpError) as e:
        s.start()
    assert e.value.status == 1 and "hipMalloc" in str(e.value)
    assert s.stats()["status"] == 3
    assert s.close() == 3
