"""Pins of the oracle's compact-support culling (a variant beyond the paper): with one
cell per axis it is the dense sum; otherwise it stays within the tail bound
sum_j |w_j| exp(-r_c^2 / (2 l^2)) of the dense logit (and the matching gradient bound)."""
import math

import numpy as np
import pytest

import oracle as O


def _occ(dim, M, seed, ell=0.4):
    rng = np.random.default_rng(seed)
    h = rng.uniform(-3, 3, (dim, M))
    w = rng.normal(0, 1.0, M)
    return O.Occupancy(h, w, -0.3, ell), rng


@pytest.mark.parametrize("dim", [2, 3])
def test_one_cell_is_the_dense_sum(dim):
    occ, rng = _occ(dim, 300, dim)
    g = O.CullGrid.make([-3.5] * dim, [3.5] * dim, 20.0)
    assert list(g.nc) == [1] * dim
    x = rng.uniform(-3, 3, (dim, 200))
    s, gc = O.cull_eval(occ, g, x)
    s_d, _, _ = O.occ_eval(occ, x)
    _, gc_d, _, _ = O.occ_grad(occ, x)
    assert np.array_equal(s, s_d) and np.array_equal(gc, gc_d)
    assert np.array_equal(O.morph_culled(occ, g, x, 5, 0.05), O.morph_ws(occ, x, 5, 0.05))


@pytest.mark.parametrize("dim,rc_l", [(2, 3.0), (2, 5.5), (3, 4.0)])
def test_within_the_tail_bound(dim, rc_l):
    ell = 0.4
    occ, rng = _occ(dim, 2000, 10 + dim, ell)
    rc = rc_l * ell
    g = O.CullGrid.make([-3.0] * dim, [3.0] * dim, rc)
    assert 1.0 / g.inv_cell >= rc
    x = rng.uniform(-3.5, 3.5, (dim, 500))  # also points outside the box
    s, gc = O.cull_eval(occ, g, x)
    s_d, _, _ = O.occ_eval(occ, x)
    _, gc_d, gs_d, _ = O.occ_grad(occ, x)
    W = np.abs(occ.weights).sum()
    tail_s = W * math.exp(-rc * rc / (2 * ell * ell))
    # per dropped hinge |grad phi| = r/l^2 phi, and r e^{-r^2/2l^2} falls for r > l
    tail_g = W * (rc / ell ** 2) * math.exp(-rc * rc / (2 * ell * ell))
    assert np.all(np.abs(s - s_d) <= tail_s * (1 + 1e-9))
    # grad c = sigma'(s) grad s with sigma' <= 1/4 and |sigma''| <= 1/(6 sqrt 3):
    # |d grad c| <= tail_g / 4 + tail_s |grad s| / (6 sqrt 3)
    bound = 0.25 * tail_g + tail_s * np.abs(gs_d).max(axis=0) / (6 * math.sqrt(3))
    assert np.all(np.abs(gc - gc_d).max(axis=0) <= bound * (1 + 1e-9) + 1e-15)
    # and the culling really drops hinges: the sums differ somewhere
    assert np.any(s != s_d)


def test_points_beyond_the_box_take_the_last_cell():
    # box [0, 10] with unit cells: 11 cells, the last one [10, 11).  A point at
    # x = 11.5 belongs to the clamped cell 10, so it takes the hinges of cells 9 and 10
    # only: the hinge at 9.5 (distance 2) is kept, the one at 8.5 (cell 8) is not.
    h = np.array([[8.5, 9.5, 1.5, 2.5], [0.5, 0.5, 0.5, 0.5]])
    w = np.array([1.0, 2.0, 3.0, 4.0])
    occ = O.Occupancy(h, w, 0.25, 5.0)
    g = O.CullGrid.make([0.0, 0.0], [10.0, 10.0], 1.0)
    assert list(g.nc) == [11, 11]
    s, _ = O.cull_eval(occ, g, np.array([[11.5], [0.5]]))
    assert abs(s[0] - (0.25 + 2.0 * math.exp(-4.0 / 50.0))) <= 1e-15
    # x = -1.5 is clamped to cell 0: cells 0 and 1 only, so the hinge at 1.5 is kept
    # and the one at 2.5 (cell 2) is not
    s2, _ = O.cull_eval(occ, g, np.array([[-1.5], [0.5]]))
    assert abs(s2[0] - (0.25 + 3.0 * math.exp(-9.0 / 50.0))) <= 1e-15
