"""Pins for the oracle's arm path (Sec. 3.2: body points, FK Jacobians, Eq. 3).

- q = 0 with d = 0 puts every joint origin on the base x axis (closed form);
- alpha = 0, d = 0 reduces standard DH to the textbook planar arm;
- the positional Jacobian against central differences of the body points;
- the suffix-sum pull-back against the column-by-column sum of J^T grad c;
- the joint gradient against finite differences of the summed occupancy;
- the joint-space morph: identities and positive step determinants for small eta;
- configuration labels against point labels of the oracle's own body points.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2108_11775_amd import configs as K, inputs as I


def _arm(seed=0, ndof=7, ppl=8, planar=False):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.1, 0.4, ndof)
    alpha = np.zeros(ndof) if planar else np.array(K.C3.alpha[:ndof])
    return O.Arm(a, np.zeros(ndof), alpha, np.zeros(ndof), ppl)


def _occ3(seed=1, M=64, ell=0.3, scale=2.0):
    rng = np.random.default_rng(seed)
    h = rng.uniform(-1.2, 1.2, (3, M))
    return O.Occupancy(h, rng.normal(0, scale, M), -0.5, ell)


def test_zero_configuration_closed_form():
    arm = _arm()
    pts = O.fk_points(arm, np.zeros((7, 1)))[:, :, 0]
    ends = np.concatenate([[0.0], np.cumsum(arm.a)])
    for i in range(7):
        for k in range(8):
            x = ends[i] + (k + 1) / 8 * (ends[i + 1] - ends[i])
            np.testing.assert_allclose(pts[:, i * 8 + k], [x, 0, 0], atol=1e-15)


def test_planar_reduction():
    arm = _arm(seed=2, planar=True)
    q = np.random.default_rng(3).uniform(-math.pi, math.pi, (7, 20))
    pts = O.fk_points(arm, q)
    for s in range(20):
        ang = np.cumsum(q[:, s])
        ox = np.concatenate([[0.0], np.cumsum(arm.a * np.cos(ang))])
        oy = np.concatenate([[0.0], np.cumsum(arm.a * np.sin(ang))])
        for i in range(7):
            f = (np.arange(8) + 1) / 8
            np.testing.assert_allclose(pts[0, i * 8:(i + 1) * 8, s], ox[i] + f * (ox[i + 1] - ox[i]),
                                       atol=1e-14)
            np.testing.assert_allclose(pts[1, i * 8:(i + 1) * 8, s], oy[i] + f * (oy[i + 1] - oy[i]),
                                       atol=1e-14)
            np.testing.assert_allclose(pts[2, i * 8:(i + 1) * 8, s], 0.0, atol=1e-15)


def test_jacobian_matches_central_differences():
    arm = _arm(seed=4)
    q = np.random.default_rng(5).uniform(-math.pi, math.pi, 7)
    for body in (0, 9, 27, 55):
        J = O.fk_jacobian(arm, q, body)
        fd = np.zeros((3, 7))
        for j in range(7):
            def P(d):
                qq = q.copy()
                qq[j] += d
                return O.fk_points(arm, qq[:, None])[:, body, 0]
            f1 = (P(2e-4) - P(-2e-4)) / 4e-4
            f2 = (P(1e-4) - P(-1e-4)) / 2e-4
            fd[:, j] = (4 * f2 - f1) / 3
        np.testing.assert_allclose(J, fd, atol=1e-10)
        # joints beyond the point's link do not move it
        assert np.all(J[:, body // 8 + 1:] == 0)


def test_pullback_forms_agree_and_match_explicit_sum():
    arm = _arm(seed=6)
    occ = _occ3()
    q = np.random.default_rng(7).uniform(-math.pi, math.pi, (7, 16))
    c0, g0 = O.arm_cost_grad(arm, occ, q, form=0)
    c1, g1 = O.arm_cost_grad(arm, occ, q, form=1)
    np.testing.assert_allclose(g1, g0, rtol=0, atol=1e-12 * max(1.0, np.abs(g0).max()))
    assert np.array_equal(c0, c1)
    # explicit sum_p J_p^T grad c(p) with the Jacobian routine
    pts = O.fk_points(arm, q)
    for s in (0, 5, 15):
        _, gc, _, _ = O.occ_grad(occ, pts[:, :, s])
        ref = np.zeros(7)
        for p in range(56):
            ref += O.fk_jacobian(arm, q[:, s], p).T @ gc[:, p]
        np.testing.assert_allclose(g0[:, s], ref, atol=1e-12 * max(1.0, np.abs(ref).max()))
        cc = O.occ_eval(occ, pts[:, :, s])[1]
        assert c0[s] == pytest.approx(cc.sum(), rel=1e-14)


def test_joint_gradient_matches_finite_differences():
    arm = _arm(seed=8)
    occ = _occ3(seed=9)
    q = np.random.default_rng(10).uniform(-math.pi, math.pi, (7, 6))
    _, g = O.arm_cost_grad(arm, occ, q)
    for j in range(7):
        def C(d):
            qq = q.copy()
            qq[j] += d
            return O.arm_cost_grad(arm, occ, qq)[0]
        f1 = (C(2e-4) - C(-2e-4)) / 4e-4
        f2 = (C(1e-4) - C(-1e-4)) / 2e-4
        np.testing.assert_allclose(g[j], (4 * f2 - f1) / 3, atol=1e-8 * max(1, np.abs(g).max()))


def test_arm_morph_identities_and_steps():
    arm = _arm(seed=11)
    occ = _occ3(seed=12)
    q = np.random.default_rng(13).uniform(-math.pi, math.pi, (7, 8))
    assert np.array_equal(O.morph_arm(arm, occ, q, 10, 0.0), q)
    assert np.array_equal(O.morph_arm(arm, occ, q, 0, 0.01), q)
    # T steps = T single steps
    a = O.morph_arm(arm, occ, q, 3, 0.01)
    b = q
    for _ in range(3):
        b = b - 0.01 * O.arm_cost_grad(arm, occ, b)[1]
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)
    _, amp, mdet = O.morph_arm(arm, occ, q, 5, 1e-3, diag=True)
    assert np.all(mdet > 0) and np.all(np.isfinite(amp))


def test_config_labels_match_point_labels_of_body_points():
    c3 = K.C3
    a, d, al, th = I.dh_params(c3.cfg_id, c3.n_dof, c3.link_min, c3.link_max, c3.alpha)
    arm = O.Arm(a, d, al, th, c3.pts_per_link)
    bc, be = I.boxes(c3.cfg_id, c3.n_boxes, c3.box_lo, c3.box_hi, c3.half_min, c3.half_max)
    q = I.uniform_points(c3.cfg_id, K.STREAM_EVAL, 7, 2000, c3.q_lo, c3.q_hi)
    lab = O.label_configs(arm, bc, be, q)
    pts = O.fk_points(arm, q)
    per_pt = np.stack([O.label_boxes(bc, be, pts[:, p, :]) for p in range(56)])
    assert np.array_equal(lab, per_pt.max(axis=0))
    free = 1 - lab.mean()
    assert 0.10 <= free <= 0.60  # within the span of Table 1's prior feasibility
    margin = O.config_label_margin(arm, bc, be, q)
    assert np.all(margin >= 0)


def _line_arm():
    """Two links of length 1 along the base x axis at q = 0 (alpha = d = theta0 = 0),
    four body points per link: the points are (k/4, 0, 0), k = 1..8, all exact."""
    return O.Arm(np.array([1.0, 1.0]), np.zeros(2), np.zeros(2), np.zeros(2), 4)


@pytest.mark.parametrize("centre,half,margin,label", [
    # box beyond the arm tip: nearest point (2,0,0), 3 - 2 - 0.5 = 0.5 outside
    ((3.0, 0.0, 0.0), (0.5, 0.5, 0.5), 0.5, 0),
    # the tip lies exactly on the box's face x = 2: inside (closed), margin 0
    ((2.5, 0.0, 0.0), (0.5, 1.0, 1.0), 0.0, 1),
    # points 0.75, 1, 1.25 inside a box of half-width 0.125 around x = 1: the deepest
    # point (1,0,0) is 0.125 from the x faces; 0.75 and 1.25 lie on them -> 0
    ((1.0, 0.25, 0.0), (0.25, 0.5, 0.5), 0.0, 1),
    ((1.0, 0.25, 0.0), (0.125, 0.5, 0.5), 0.125, 1),
    # a slab above the arm: every point is 2 - 1.5 = 0.5 below its y face
    ((1.0, 2.0, 0.0), (5.0, 1.5, 5.0), 0.5, 0),
    # a box below in z, corner side: max over axes of |p_a - c_a| - e_a is 0.25 (z)
    ((1.0, 0.0, -0.75), (4.0, 4.0, 0.5), 0.25, 0),
])
def test_config_label_margin_hand_built_scene(centre, half, margin, label):
    arm = _line_arm()
    c = np.array(centre, np.float64).reshape(3, 1)
    e = np.array(half, np.float64).reshape(3, 1)
    q = np.zeros((2, 1))
    assert O.config_label_margin(arm, c, e, q)[0] == margin
    assert O.label_configs(arm, c, e, q)[0] == label


def test_config_label_margin_is_the_flip_distance():
    """Moving the box toward the arm by just over the margin flips an outside label;
    by just under it does not (the margin is a distance, taken over all boxes)."""
    arm = _line_arm()
    q = np.zeros((2, 1))
    e = np.array([[0.5], [0.5], [0.5]])
    far = np.array([[3.0, 0.0], [0.0, 5.0], [0.0, 0.0]])   # two boxes: x at 0.5, y far
    ef = np.array([[0.5, 0.5], [0.5, 0.5], [0.5, 0.5]])
    mg = O.config_label_margin(arm, far, ef, q)[0]
    assert mg == 0.5
    for shift, lab in [(mg - 1e-9, 0), (mg + 1e-9, 1)]:
        c = far.copy()
        c[0, 0] -= shift
        assert O.label_configs(arm, c, ef, q)[0] == lab
    # one box only, moved along y onto the arm by the same rule
    c = np.array([[1.0], [0.75], [0.0]])
    mg = O.config_label_margin(arm, c, e, q)[0]
    assert mg == 0.25
    assert O.label_configs(arm, c - [[0], [mg - 1e-9], [0]], e, q)[0] == 0
    assert O.label_configs(arm, c - [[0], [mg + 1e-9], [0]], e, q)[0] == 1


def test_arm_step_scale_against_jacobian_columns():
    """The per-configuration gradient scale written out from the positional
    Jacobians (themselves pinned against central differences) and the workspace
    gradient scale of each body point."""
    arm = _arm(seed=5)
    occ = _occ3(seed=6)
    q = np.random.default_rng(7).uniform(-math.pi, math.pi, (7, 5))
    got = O.arm_step_scale(arm, occ, q)
    pts = O.fk_points(arm, q)
    for s in range(q.shape[1]):
        _, _, _, gabs = O.occ_grad(occ, pts[:, :, s])
        lever = np.array([np.abs(O.fk_jacobian(arm, q[:, s], p)).sum(axis=0).max()
                          for p in range(56)])
        assert got[s] == pytest.approx(float((lever * gabs).sum()), rel=1e-12)


def test_arm_step_hessian_norm_bounds_the_step_jacobian():
    """For one step, |I - eta H|_2 <= 1 + eta |H|_2 and det(I - eta H) >= (1 - eta |H|_2)^7
    when eta |H|_2 < 1 (eigenvalues of the symmetrised step Jacobian)."""
    arm = _arm(seed=8)
    occ = _occ3(seed=9)
    q = np.random.default_rng(10).uniform(-math.pi, math.pi, (7, 6))
    for eta in (1e-3, 2e-2):
        _, amp, mdet, meh = O.morph_arm(arm, occ, q, 1, eta, diag=True, with_eh=True)
        assert np.all(meh > 0)
        assert np.all(amp <= 1 + meh + 1e-12)
        small = meh < 1
        assert np.all(mdet[small] >= (1 - meh[small]) ** 7 - 1e-12)
