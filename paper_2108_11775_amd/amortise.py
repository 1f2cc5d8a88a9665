"""Learned amortised morph: training data from the plain morph and the MLP training
loop.  Every arithmetic step runs in libpdmp's kernels (Philox prior batches, the
joint-space morph, BF16-MFMA forward/backward, Adam, BF16 repacking); this module
only sequences the calls.

Training pairs are (q, morph_T(q)) for prior batches q ~ U[q_lo, q_hi)^n_dof drawn
with Philox streams 0, 1, 2, ...; each batch is its own contiguous [n_dof][B]
tensor, so epochs iterate over the batches without any gather or shuffle copy
(the batches are independent uniform draws).
"""
from __future__ import annotations

import time

import torch

from . import Arm, Mlp, Occupancy, adam_step, arm_max_occupancy, morph_samples, uniform_samples


def make_pairs(occ: Occupancy, arm: Arm, n_batches: int, batch: int, T: int, eta: float,
               seed: int, q_lo: float, q_hi: float, first_stream: int = 0, device="cuda"):
    pairs = []
    lo, hi = [q_lo] * arm.n_dof, [q_hi] * arm.n_dof
    for b in range(n_batches):
        q = uniform_samples(seed, first_stream + b, lo, hi, batch, device=device)
        t = morph_samples(occ, q, T, eta, arm=arm)
        pairs.append((q, t))
    return pairs


def train(mlp: Mlp, pairs, epochs: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
          log=None, schedule: str = "constant", hard_weight=None, occ: Occupancy = None,
          arm: Arm = None, hard_thresh: float = 0.5, restarts: int = 4):
    """Adam on the MSE between q + f(q) and the plain-morph target.

    schedule "cosine" anneals the step as lr * (1 + cos(pi t / steps)) / 2;
    "cosine_restarts" does so over each of `restarts` equal periods.  With hard_weight,
    every step first checks the network's own outputs (pdmp_arm_max_occupancy on occ,
    arm) and weighs the samples whose q + f(q) lands above hard_thresh by hard_weight.
    Returns the per-step loss as a device tensor [epochs * len(pairs)].
    """
    import math
    if schedule not in ("constant", "cosine", "cosine_restarts"):
        raise ValueError(f"unknown schedule {schedule!r}")
    if hard_weight is not None and (occ is None or arm is None):
        raise ValueError("hard_weight needs the occupancy and the arm")
    dev = mlp.params.device
    B = int(pairs[0][0].shape[1])
    steps = epochs * len(pairs)
    period = max(1, steps // max(1, restarts))
    losses = torch.empty(steps, dtype=torch.float32, device=dev)
    m = torch.zeros_like(mlp.params)
    v = torch.zeros_like(mlp.params)
    grad = torch.empty_like(mlp.params)
    acts = mlp.acts_buffer(B, dev)
    qhat = torch.empty_like(pairs[0][0])
    t = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        for q, tgt in pairs:
            mlp.forward(q, acts=acts, out=qhat)
            hard = None
            if hard_weight is not None:
                _, hard = arm_max_occupancy(occ, arm, qhat, hard_thresh)
            mlp.backward(qhat, tgt, acts, grad=grad, loss=losses[t:t + 1], hard=hard,
                         hard_weight=1.0 if hard_weight is None else hard_weight)
            t += 1
            if schedule == "constant":
                lr_t = lr
            elif schedule == "cosine":
                lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * (t - 1) / steps))
            else:
                lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * ((t - 1) % period) / period))
            adam_step(mlp.params, grad, m, v, t, lr_t, beta1, beta2, eps)
            mlp.pack()
        if log is not None:
            log(f"epoch {ep + 1}/{epochs}: loss {losses[t - 1].item():.5f} "
                f"({time.perf_counter() - t0:.1f} s)")
    return losses
