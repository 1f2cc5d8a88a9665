"""GPU parity along the GPU's own explicit-Euler paths (Sec. 3.2, Eq. 1; Eq. 3 for the arm).

A T-step comparison against the oracle's own path has to allow for the map's
amplification of rounding differences (the product A of |I - eta Hc| along the path,
in the thousands on the arm).  Here the recording morph writes every state of a
strided subset of samples from the very kernels and launch of the plain morph (its
output is checked to be the same bits), and the oracle takes one step from each
recorded GPU state: that step must land on the GPU's next state within the one-step
tolerance 1e-5 (|x'| + eta G_abs(x)) per coordinate (the arm: eta times the
body-point scale sum_p max_j |J_p[:, j]|_1 G_abs(p)), with no amplification in the
bound.  Beside that the tests report, from the oracle at the visited states: the share
of samples whose final state is within the unscaled 1e-5 of the oracle's own T-step
path, the largest eta |Hc|_2, and the number of steps with det(I - eta Hc) <= 0 (where
the discrete map folds, so it is not a diffeomorphism there).  With PDMP_REPORT set to
a directory the figures are also written there as JSON.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import paper_2108_11775_amd as P
from paper_2108_11775_amd import configs as K, inputs as I

from helpers import arm_scene, dev, gpu_occ, host, oracle_occ, require_gpu, ws_scene

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _report(name, rec):
    print(f"\n[trajectory] {name}: {json.dumps(rec)}", flush=True)
    d = os.environ.get("PDMP_REPORT")
    if d:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, f"trajectory_{name}.json"), "w") as f:
            json.dump(rec, f, indent=1)


def _check_recording(out, traj, x0, stride):
    """traj's first state is the input and its last the output, bit for bit."""
    assert np.array_equal(traj[0], x0[:, ::stride])
    assert np.array_equal(traj[-1], out[:, ::stride])


def _ws_along_path(oo, traj, eta):
    """One oracle step from every recorded state but the last, against the next state."""
    T1, dim, nt = traj.shape
    X = np.ascontiguousarray(traj[:-1].transpose(1, 0, 2).reshape(dim, -1)).astype(np.float64)
    Y = traj[1:].transpose(1, 0, 2).reshape(dim, -1)
    ref = O.morph_ws(oo, X, 1, eta)
    _, _, _, gabs = O.occ_grad(oo, X)
    err = np.abs(Y - ref)
    tol = TOL * (np.abs(ref) + eta * gabs[None, :])
    return X, err, tol


def _ws_stats(oo, X, traj, eta, T):
    """Figures of the visited states and of the final states against the oracle's own
    T-step paths from the same inputs."""
    _, _, mdet, meh = O.morph_ws(oo, X, 1, eta, diag=True)
    ref_T = O.morph_ws(oo, traj[0].astype(np.float64), T, eta)
    errT = np.abs(traj[-1] - ref_T).max(axis=0)
    within = errT <= TOL * np.maximum(1.0, np.abs(ref_T).max(axis=0))
    return {"samples": int(traj.shape[2]), "steps": int(T), "states": int(X.shape[1]),
            "max_eta_hess": float(meh.max()), "steps_det_nonpositive": int((mdet <= 0).sum()),
            "min_step_det": float(mdet.min()),
            "share_final_within_unscaled_1e-5": float(within.mean()),
            "final_err_max": float(errT.max()), "final_err_median": float(np.median(errT))}


@pytest.mark.parametrize("cfg", [K.C1, K.C2])
def test_ws2d_one_step_along_gpu_path(cfg):
    """Config 1 (small-batch 16-sample waves) in full; config 2 at its full batch of
    2^20 (the headline launch) with every 256th sample recorded."""
    require_gpu()
    sc = ws_scene(cfg)
    seed = I.philox_seed(cfg.cfg_id)
    n = cfg.n_samples
    stride = 1 if n <= 4096 else 256
    x0_d = P.uniform_samples(seed, 0, [cfg.lo] * 2, [cfg.hi] * 2, n)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"], (cfg.grid, cfg.grid))
    out_d, traj_d = P.morph_trajectory(go, x0_d, cfg.T, cfg.eta, stride=stride)
    out, traj, x0 = host(out_d), host(traj_d), host(x0_d)
    assert np.array_equal(out, host(P.morph_samples(go, x0_d, cfg.T, cfg.eta)))
    _check_recording(out, traj, x0, stride)
    oo = oracle_occ(sc["h"], sc["wb"], sc["ell"])
    X, err, tol = _ws_along_path(oo, traj, cfg.eta)
    rec = _ws_stats(oo, X, traj, cfg.eta, cfg.T)
    rec["one_step_max_err_over_tol"] = float((err / tol).max())
    rec["one_step_share_within_unscaled_1e-5"] = float(
        (err <= TOL * np.maximum(1.0, np.abs(X))).all(axis=0).mean())
    _report(f"ws2d_config{cfg.cfg_id}", rec)
    assert np.all(err <= tol), float((err / tol).max())


def test_ws3d_one_step_along_gpu_path():
    """The 3-D workspace morph on the box world's 16^3 grid."""
    require_gpu()
    sc = arm_scene()
    n, T, eta, stride = 20001, 12, 0.002, 8
    x0 = I.uniform_points(3, K.STREAM_EVAL, 3, n, -1.2, 1.2)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"], (16, 16, 16))
    out_d, traj_d = P.morph_trajectory(go, dev(x0), T, eta, stride=stride)
    out, traj = host(out_d), host(traj_d)
    assert np.array_equal(out, host(P.morph_samples(go, dev(x0), T, eta)))
    _check_recording(out, traj, x0, stride)
    _, err, tol = _ws_along_path(oracle_occ(sc["h"], sc["wb"], sc["ell"]), traj, eta)
    assert np.all(err <= tol), float((err / tol).max())


@pytest.mark.parametrize("n,stride", [(3001, 3), (9000, 7)])
def test_pairwise_ws_one_step_along_gpu_path(n, stride):
    """Hinges given without a grid take the pairwise kernel (both of its launch shapes)."""
    require_gpu()
    cfg = K.C2
    sc = ws_scene(cfg)
    x0 = I.uniform_points(cfg.cfg_id, K.STREAM_EVAL, 2, n, cfg.lo, cfg.hi)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"])
    out_d, traj_d = P.morph_trajectory(go, dev(x0), 8, cfg.eta, stride=stride)
    out, traj = host(out_d), host(traj_d)
    assert np.array_equal(out, host(P.morph_samples(go, dev(x0), 8, cfg.eta)))
    _check_recording(out, traj, x0, stride)
    _, err, tol = _ws_along_path(oracle_occ(sc["h"], sc["wb"], sc["ell"]), traj, cfg.eta)
    assert np.all(err <= tol), float((err / tol).max())


def _arms(sc):
    a, d, al, th = sc["dh"]
    return O.Arm(a, d, al, th, 8), P.Arm(a, d, al, th, 8)


def _arm_along_path(ao, oo, traj, eta):
    T1, nd, nt = traj.shape
    Q = np.ascontiguousarray(traj[:-1].transpose(1, 0, 2).reshape(nd, -1)).astype(np.float64)
    Y = traj[1:].transpose(1, 0, 2).reshape(nd, -1)
    ref = O.morph_arm(ao, oo, Q, 1, eta)
    scale = O.arm_step_scale(ao, oo, Q)
    err = np.abs(Y - ref)
    tol = TOL * (np.abs(ref) + eta * scale[None, :])
    return Q, err, tol


def test_arm_one_step_along_gpu_path_config3():
    """Config 3 at its full batch (65,536 configurations, the grid arm kernel on the
    FP16 split scheme), every 256th configuration recorded over its 30 steps."""
    require_gpu()
    sc = arm_scene()
    ao, ag = _arms(sc)
    c3 = K.C3
    seed = I.philox_seed(c3.cfg_id)
    stride = 256
    q0_d = P.uniform_samples(seed, 0, [c3.q_lo] * 7, [c3.q_hi] * 7, c3.n_samples)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"], (16, 16, 16))
    out_d, traj_d = P.morph_trajectory(go, q0_d, c3.T, c3.eta, stride=stride, arm=ag)
    out, traj, q0 = host(out_d), host(traj_d), host(q0_d)
    assert np.array_equal(out, host(P.morph_samples(go, q0_d, c3.T, c3.eta, arm=ag)))
    _check_recording(out, traj, q0, stride)
    oo = oracle_occ(sc["h"], sc["wb"], sc["ell"])
    Q, err, tol = _arm_along_path(ao, oo, traj, c3.eta)
    # figures of the visited states (step Jacobians by central differences) on every
    # fourth recorded configuration, and of the final states against the oracle's paths
    sub = traj[:, :, ::4]
    Qs = np.ascontiguousarray(sub[:-1].transpose(1, 0, 2).reshape(7, -1)).astype(np.float64)
    _, amp1, mdet, meh = O.morph_arm(ao, oo, Qs, 1, c3.eta, diag=True, with_eh=True)
    ref_T = O.morph_arm(ao, oo, traj[0].astype(np.float64), c3.T, c3.eta)
    errT = np.abs(traj[-1] - ref_T).max(axis=0)
    within = errT <= TOL * np.maximum(1.0, np.abs(ref_T).max(axis=0))
    folded = (mdet.reshape(c3.T, -1) <= 0).any(axis=0)
    rec = {"configs": int(traj.shape[2]), "steps": int(c3.T), "states": int(Q.shape[1]),
           "one_step_max_err_over_tol": float((err / tol).max()),
           "one_step_share_within_unscaled_1e-5": float(
               (err <= TOL * np.maximum(1.0, np.abs(Q))).all(axis=0).mean()),
           "share_final_within_unscaled_1e-5": float(within.mean()),
           "final_err_max": float(errT.max()), "final_err_median": float(np.median(errT)),
           "diag_configs": int(sub.shape[2]), "diag_states": int(Qs.shape[1]),
           "max_eta_hess": float(meh.max()), "max_step_norm": float(amp1.max()),
           "steps_det_nonpositive": int((mdet <= 0).sum()),
           "paths_with_a_folding_step": int(folded.sum()), "min_step_det": float(mdet.min())}
    _report("arm_config3", rec)
    assert np.all(err <= tol), float((err / tol).max())


def test_pairwise_arm_one_step_along_gpu_path():
    """The same arm with hinges given without a grid: the pairwise arm kernel."""
    require_gpu()
    sc = arm_scene()
    ao, ag = _arms(sc)
    c3 = K.C3
    q0 = O.uniform_samples(I.philox_seed(c3.cfg_id), 9, [c3.q_lo] * 7, [c3.q_hi] * 7, 301)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"])
    out_d, traj_d = P.morph_trajectory(go, dev(q0), 6, c3.eta, stride=10, arm=ag)
    out, traj = host(out_d), host(traj_d)
    assert np.array_equal(out, host(P.morph_samples(go, dev(q0), 6, c3.eta, arm=ag)))
    _check_recording(out, traj, q0, 10)
    _, err, tol = _arm_along_path(ao, oracle_occ(sc["h"], sc["wb"], sc["ell"]), traj, c3.eta)
    assert np.all(err <= tol), float((err / tol).max())


def test_recording_edge_cases():
    """T = 0 records the input only; a stride beyond n records sample 0 alone; a batch
    that is not a multiple of the stride records its ragged tail's first sample."""
    require_gpu()
    cfg = K.C2
    sc = ws_scene(cfg)
    go = gpu_occ(sc["h"], sc["wb"], sc["ell"], (cfg.grid, cfg.grid))
    x0 = I.uniform_points(cfg.cfg_id, K.STREAM_EVAL, 2, 1000, cfg.lo, cfg.hi)
    out, traj = P.morph_trajectory(go, dev(x0), 0, cfg.eta, stride=3)
    assert np.array_equal(host(out), x0) and host(traj).shape == (1, 2, 334)
    assert np.array_equal(host(traj)[0], x0[:, ::3])
    out, traj = P.morph_trajectory(go, dev(x0), 4, cfg.eta, stride=5000)
    assert host(traj).shape == (5, 2, 1)
    assert np.array_equal(host(traj)[-1, :, 0], host(out)[:, 0])
    out, traj = P.morph_trajectory(go, dev(x0), 4, cfg.eta, stride=999)
    assert host(traj).shape == (5, 2, 2)
    assert np.array_equal(host(traj)[-1], host(out)[:, [0, 999]])
