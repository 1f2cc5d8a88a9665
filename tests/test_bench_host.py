"""Host-side checks (CPU): the documented split-scheme rule of the grid kernels (the
rule each kernel block applies to the same weights and hinges, stated in the tests'
helpers; the GPU tests hold the library's own report to it) and bench.py's command
line refusals."""
import math
import os
import subprocess
import sys

import numpy as np

from paper_2108_11775_amd import configs as K

from helpers import arm_scene, split_rule, ws_scene

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _axis(n, lo=-3.0, hi=3.0):
    return np.linspace(lo, hi, n).astype(np.float32)


def test_split_scheme_on_the_workloads():
    # the fitted weights of the 2-D configs and the arm world span about 2^-11 of
    # their largest magnitude, on regular grids: the FP16 scheme
    for cfg in (K.C1, K.C2):
        sc = ws_scene(cfg)
        assert split_rule(sc["h"][0, :cfg.grid], sc["wb"][:-1], sc["ell"]) == ("fp16", 3)
    a = arm_scene()
    assert split_rule(a["h"][0, :16], a["wb"][:-1], a["ell"]) == ("fp16", 3)


def test_split_scheme_weight_range_threshold():
    w = np.ones(64, dtype=np.float32)
    w[5] = np.float32(2.0 ** -19)            # exactly the limit: still FP16
    assert split_rule(_axis(8), w, 0.5)[0] == "fp16"
    w[5] = np.float32(2.0 ** -19) * np.float32(0.999)
    assert split_rule(_axis(8), w, 0.5)[0] == "bf16"
    w[5] = 0.0                                # zeros are exact in any format
    assert split_rule(_axis(8), w, 0.5)[0] == "fp16"
    assert split_rule(_axis(8), np.zeros(64, np.float32), 0.5)[0] == "fp16"
    for bad in (np.nan, np.inf):
        w[5] = bad
        assert split_rule(_axis(8), w, 0.5) == ("bf16", 6)


def test_split_scheme_axis_gap():
    ell = 0.5
    kappa = math.sqrt(math.log2(math.e) / 2.0) / ell
    w = np.ones(64, dtype=np.float32)
    gap = 6.0 / kappa                          # the largest gap allowed, in x units
    ok = np.array([0.0, 0.98 * gap, 1.96 * gap], dtype=np.float32)
    assert split_rule(ok, w, ell)[0] == "fp16"
    wide = np.array([0.0, 1.05 * gap], dtype=np.float32)
    assert split_rule(wide, w, ell)[0] == "bf16"
    # order and repeats do not matter: the gap is between consecutive distinct values
    assert split_rule(ok[::-1].copy(), w, ell)[0] == "fp16"
    assert split_rule(np.r_[ok, ok].astype(np.float32), w, ell)[0] == "fp16"
    # a single coordinate has no gap
    assert split_rule(np.array([1.0], np.float32), w, ell)[0] == "fp16"


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_cli_refusals():
    r = _run("--gpus", "2")
    assert r.returncode == 2 and '"n_gpus": 2' in r.stdout
    r = _run("--workloads", "arm,nonsense")
    assert r.returncode != 0 and "nonsense" in r.stderr

