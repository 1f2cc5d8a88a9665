"""Write the occupancy weights the parity tests use as fixed inputs.

Calls only the FP64 oracle (oracle/) on the seeded synthetic scenes:
  ws2d_4096.npy  -- 2-D disc world, 30x30 hinges, l=0.7: 200 GD steps (lr_w 64,
                    lr_beta 2, l2 1e-3) on 10^4 labelled points;
  ws2d_1M.npy    -- 2-D disc world, 64x64 hinges, l=0.4: the same protocol
                    (lr_w 128);
  arm7_box.npy   -- 3-D box world of the 7-DOF arm, 16^3 hinges, l=0.15: 60 Adam
                    steps (lr 1e-2, l2 1e-4) on 2^15 labelled points, a reduced
                    version of the 2^20-point, 500-step fit.
Each file holds [M+1] float32 weights with the bias last.

    python tests/golden/make_fits.py
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


def fit_ws(cfg):
    h = I.hinge_grid(2, cfg.grid, cfg.lo, cfg.hi)
    pts = I.uniform_points(cfg.cfg_id, K.STREAM_FIT, 2, cfg.fit_points, cfg.lo, cfg.hi)
    dc, dr = I.discs(cfg.cfg_id, cfg.n_discs, cfg.lo, cfg.hi, cfg.r_min, cfg.r_max)
    y = O.label_discs(dc, dr, pts)
    wb, _, _, loss = O.fit(h, cfg.lengthscale, pts, y, 0, cfg.fit_steps, cfg.fit_lr, cfg.fit_l2,
                           lr_bias=cfg.fit_lr_bias)
    print(f"{cfg.name}: loss {loss[0]:.4f} -> {loss[-1]:.4f}")
    return wb.astype(np.float32)


def fit_arm(n_pts=1 << 15, steps=60):
    c3, c4 = K.C3, K.C4
    h = I.hinge_grid(3, c3.grid, c3.box_lo, c3.box_hi)
    bc, be = I.boxes(c3.cfg_id, c3.n_boxes, c3.box_lo, c3.box_hi, c3.half_min, c3.half_max)
    pts = I.uniform_points(c4.cfg_id, K.STREAM_FIT, 3, n_pts, c3.box_lo, c3.box_hi)
    y = O.label_boxes(bc, be, pts)
    wb, _, _, loss = O.fit(h, c3.lengthscale, pts, y, 1, steps, c4.lr, c4.l2, b1=c4.beta1,
                           b2=c4.beta2, eps=c4.eps)
    print(f"arm7 box world: loss {loss[0]:.4f} -> {loss[-1]:.4f}")
    return wb.astype(np.float32)


if __name__ == "__main__":
    t = time.time()
    np.save(os.path.join(OUT, "ws2d_4096.npy"), fit_ws(K.C1))
    np.save(os.path.join(OUT, "ws2d_1M.npy"), fit_ws(K.C2))
    np.save(os.path.join(OUT, "arm7_box.npy"), fit_arm())
    print(f"done in {time.time() - t:.1f} s")
