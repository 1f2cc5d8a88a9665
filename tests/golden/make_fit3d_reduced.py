"""Write the oracle's reference trajectory of the reduced 3-D occupancy fit.

Calls only the FP64 oracle (oracle/) on seeded synthetic inputs: the box world of the
7-DOF arm, 16^3 hinges, l = 0.15, BCE + (l2/2)|w|^2 with l2 = 1e-4, 500 full-batch
Adam steps (lr 1e-2, betas 0.9 / 0.999, eps 1e-8; every hyperparameter rounded to
FP32 first, the values the library's fit receives) from w = 0 on 65,536 uniform
labelled points -- the 2^20-point fit at a size the oracle finishes in minutes.
fit3d_65536.npz holds the loss before each step [500] and the final weights [M+1]
(bias last), both FP64.

    python tests/golden/make_fit3d_reduced.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2108_11775_amd import configs as K, inputs as I  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))
N_POINTS = 65536


def problem():
    """Hinges, lengthscale, points and labels of the reduced fit (shared with its test)."""
    c3, c4 = K.C3, K.C4
    h = I.hinge_grid(3, c3.grid, c3.box_lo, c3.box_hi)
    bc, be = I.boxes(c3.cfg_id, c3.n_boxes, c3.box_lo, c3.box_hi, c3.half_min, c3.half_max)
    pts = I.uniform_points(c4.cfg_id, K.STREAM_FIT, 3, N_POINTS, c3.box_lo, c3.box_hi)
    y = O.label_boxes(bc, be, pts)
    return h, c3.lengthscale, pts, y


def hyper():
    c4 = K.C4
    return {k: float(np.float32(v)) for k, v in
            dict(lr=c4.lr, l2=c4.l2, b1=c4.beta1, b2=c4.beta2, eps=c4.eps).items()}


if __name__ == "__main__":
    t = time.time()
    h, ell, pts, y = problem()
    hp = hyper()
    wb, _, _, loss = O.fit(h, ell, pts, y, 1, K.C4.steps, hp["lr"], hp["l2"], b1=hp["b1"],
                           b2=hp["b2"], eps=hp["eps"])
    np.savez(os.path.join(OUT, "fit3d_65536.npz"), loss=loss, wb=wb)
    print(f"loss {loss[0]:.6f} -> {loss[-1]:.6f}, max|w| {np.abs(wb).max():.4f}, "
          f"{time.time() - t:.0f} s")
