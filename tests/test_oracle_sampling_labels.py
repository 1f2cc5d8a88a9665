"""Pins for the oracle's prior sampler (Sec. 3.3) and collision labels (Table 1).

Philox4x32-10 is pinned to the published known-answer vectors; the labels to a
hand-built scene whose answers follow from exact arithmetic.
"""
import json
import os

import numpy as np
import pytest

import oracle as O


def _kat(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(golden_dir):
    rows = _kat(golden_dir)
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(O.philox4x32_10(ctr, key)) == out


def test_uniform_samples_grid_and_range():
    lo, hi = [-10.0, -np.pi], [10.0, np.pi]
    x = O.uniform_samples(12345, 0, lo, hi, 4096)
    assert x.dtype == np.float32 and x.shape == (2, 4096)
    lo32, hi32 = np.float32(lo), np.float32(hi)
    assert np.all(x[0] >= lo32[0]) and np.all(x[0] < hi32[0])
    assert np.all(x[1] >= lo32[1]) and np.all(x[1] <= hi32[1])
    # Coordinate 0 of sample i is lo + span*u with u = (word0 >> 8) 2^-24 of
    # Philox({i, 0, 0, stream}, key); check a few samples against the raw block.
    seed = 12345
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in (0, 1, 777, 4095):
        r = O.philox4x32_10([i, 0, 0, 0], key)
        for k in range(2):
            u = (int(r[k]) >> 8) / 2.0 ** 24
            ref = np.float32(float(lo32[k]) + (float(hi32[k]) - float(lo32[k])) * u)
            assert x[k, i] == ref


def test_uniform_samples_independent_of_batch_and_stream():
    a = O.uniform_samples(7, 3, [0, 0, 0, 0, 0, 0, 0], [1] * 7, 100)
    b = O.uniform_samples(7, 3, [0] * 7, [1] * 7, 37)
    assert np.array_equal(a[:, :37], b)
    c = O.uniform_samples(7, 4, [0] * 7, [1] * 7, 37)
    assert not np.array_equal(b, c)
    # dims 4..6 come from the second Philox block of each sample
    r = O.philox4x32_10([5, 0, 1, 3], [7, 0])
    assert a[4, 5] == np.float32((int(r[0]) >> 8) / 2.0 ** 24)


def test_uniform_at_matches_the_batch_and_the_high_counter_word():
    """The indexed form gives the batch's samples at any index, the counter's high word
    included (indices at and past 2^32 from the raw Philox block)."""
    lo, hi = [-10.0, -3.0, 0.5, 2.0, -1.0], [10.0, 3.0, 1.5, 9.0, 1.0]
    a = O.uniform_samples(4242, 6, lo, hi, 3001)
    idx = np.array([0, 1, 17, 1023, 3000, 2999, 5])
    assert np.array_equal(O.uniform_at(4242, 6, lo, hi, idx), a[:, idx])
    lo32, hi32 = np.float32(lo), np.float32(hi)
    for i in ((1 << 31) + 7, (1 << 32) - 1, 1 << 32, (1 << 33) + 12345):
        got = O.uniform_at(4242, 6, lo, hi, [i])[:, 0]
        for k in range(5):
            r = O.philox4x32_10([i & 0xFFFFFFFF, i >> 32, k // 4, 6], [4242, 0])
            u = (int(r[k % 4]) >> 8) / 2.0 ** 24
            assert got[k] == np.float32(float(lo32[k]) + (float(hi32[k]) - float(lo32[k])) * u)


def test_uniform_samples_moments():
    x = O.uniform_samples(99, 0, [0.0], [1.0], 1 << 18)[0].astype(np.float64)
    n = x.size
    # mean 1/2, variance 1/12; 6-sigma bands
    assert abs(x.mean() - 0.5) < 6 * np.sqrt(1 / 12 / n)
    assert abs(x.var() - 1 / 12) < 6 * np.sqrt(1 / 180 / n)
    hist = np.histogram(x, bins=16, range=(0, 1))[0]
    e = n / 16
    assert ((hist - e) ** 2 / e).sum() < 60  # chi^2, 15 dof


def test_label_discs_tiny_scene(golden_dir):
    d = json.load(open(os.path.join(golden_dir, "labels_tiny.json")))["discs"]
    pts = np.asarray(d["points"], np.float32).T
    got = O.label_discs(np.asarray(d["centres"], np.float32), np.asarray(d["radii"], np.float32), pts)
    assert got.tolist() == d["expected"]


def test_label_boxes_tiny_scene(golden_dir):
    d = json.load(open(os.path.join(golden_dir, "labels_tiny.json")))["boxes"]
    pts = np.asarray(d["points"], np.float32).T
    got = O.label_boxes(np.asarray(d["centres"], np.float32), np.asarray(d["half"], np.float32), pts)
    assert got.tolist() == d["expected"]


def test_label_discs_union_of_single_discs():
    rng = np.random.default_rng(0)
    c = rng.uniform(-5, 5, (2, 6)).astype(np.float32)
    r = rng.uniform(0.5, 2, 6).astype(np.float32)
    x = rng.uniform(-6, 6, (2, 2000)).astype(np.float32)
    each = np.stack([O.label_discs(c[:, k:k + 1], r[k:k + 1], x) for k in range(6)])
    assert np.array_equal(O.label_discs(c, r, x), each.max(axis=0))
    # a single disc: inside iff distance <= r, checked on points well away from the rim
    dist = np.hypot(x[0].astype(np.float64) - c[0, 0], x[1].astype(np.float64) - c[1, 0])
    far = np.abs(dist - r[0]) > 1e-6
    assert np.array_equal(each[0][far], (dist <= r[0])[far].astype(np.uint8))
