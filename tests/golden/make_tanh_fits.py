"""Write the tanh-network occupancy weights (Sec. 3.1) the parity tests and the
benchmark use as fixed inputs.

Calls only the FP64 oracle (oracle/) on the seeded synthetic disc worlds of
configs 1 and 2: full-batch Adam (lr 1e-2) on mean BCE + (l2/2)|weights|^2 over the
10^4 labelled fit points, from the seeded initialisation of inputs.tanh_init:
  tanh_c1.npy -- 3 hidden tanh layers of 64, 1000 steps, l2 1e-5;
  tanh_c2.npy -- the same network, 1500 steps, l2 1e-6.
Each file holds the flat float32 parameters (W_l, b_l per layer, then v, b_o).

    python tests/golden/make_tanh_fits.py
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


def fit_tanh(cfg, steps, l2):
    tc = K.TANH
    pts = I.uniform_points(cfg.cfg_id, K.STREAM_FIT, 2, cfg.fit_points, cfg.lo, cfg.hi)
    dc, dr = I.discs(cfg.cfg_id, cfg.n_discs, cfg.lo, cfg.hi, cfg.r_min, cfg.r_max)
    y = O.label_discs(dc, dr, pts)
    P0 = I.tanh_init(cfg.cfg_id, 2, tc.hidden, tc.layers, cfg.hi)
    P, loss = O.tanh_fit(O.TanhNet(2, tc.hidden, tc.layers, P0), pts, y, steps, tc.lr, l2,
                         tc.beta1, tc.beta2, tc.eps)
    print(f"{cfg.name} tanh: loss {loss[0]:.4f} -> {loss[-1]:.4f}")
    return P.astype(np.float32)


if __name__ == "__main__":
    t = time.time()
    np.save(os.path.join(OUT, "tanh_c1.npy"), fit_tanh(K.C1, K.TANH.steps[0], K.TANH.l2[0]))
    np.save(os.path.join(OUT, "tanh_c2.npy"), fit_tanh(K.C2, K.TANH.steps[1], K.TANH.l2[1]))
    print(f"done in {time.time() - t:.1f} s")
