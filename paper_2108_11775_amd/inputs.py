"""Seeded synthetic inputs shared by the HIP path, the oracle tests and the bench.

This module draws scenes, hinge grids, arm parameters, fit points and network
initialisations from numpy generators keyed by (config, stream).  It holds none of
the method's arithmetic: no features, costs, gradients, labels, kinematics or
updates.  Base samples that the method itself draws on the GPU (Sec. 3.3 samples
the prior in batches on the device) are not produced here; both sides derive them
from the same Philox4x32-10 counter scheme, and this module only supplies the seed.

The paper's environments (Divider, Cupboard, Lab-setup and the Jaco arm) are not
available, so every workload is synthetic, with obstacle densities chosen so that
the fraction of collision-free prior samples falls inside the span the paper
reports for its own scenes (Table 1, 12.8 % to 52.2 %).
"""
from __future__ import annotations

import numpy as np

from .configs import (ENTROPY, STREAM_SCENE, STREAM_FIT, STREAM_BASE, STREAM_DH,
                      STREAM_MLP, STREAM_SHUFFLE, STREAM_EVAL, STREAM_TANH)

__all__ = ["rng", "philox_seed", "discs", "boxes", "hinge_grid", "dh_params",
           "uniform_points", "mlp_init", "STREAM_SCENE", "STREAM_FIT", "STREAM_BASE",
           "STREAM_DH", "STREAM_MLP", "STREAM_SHUFFLE", "STREAM_EVAL", "STREAM_TANH",
           "tanh_init"]


def rng(cfg_id: int, stream: int) -> np.random.Generator:
    """Independent generator for (config, stream)."""
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence(entropy=ENTROPY, spawn_key=(cfg_id, stream))))


def philox_seed(cfg_id: int, stream: int = STREAM_BASE) -> int:
    """64-bit Philox key for the on-device base-sample generator."""
    return int(rng(cfg_id, stream).integers(0, 2**63 - 1, dtype=np.int64))


def discs(cfg_id: int, k: int, lo: float, hi: float, r_min: float, r_max: float):
    """k discs with centres U[lo,hi]^2 and radii U(r_min, r_max).

    Returns (centres [2][k], radii [k]) as float32.
    """
    g = rng(cfg_id, STREAM_SCENE)
    c = g.uniform(lo, hi, size=(2, k)).astype(np.float32)
    r = g.uniform(r_min, r_max, size=k).astype(np.float32)
    return np.ascontiguousarray(c), r


def boxes(cfg_id: int, k: int, lo: float, hi: float, e_min: float, e_max: float):
    """k axis-aligned boxes: centres U[lo,hi]^3, half-extents U(e_min, e_max) per axis.

    A box that contains the origin (the arm's base) is redrawn.  Returns
    (centres [3][k], half-extents [3][k]) as float32.
    """
    g = rng(cfg_id, STREAM_SCENE)
    cs, es = [], []
    while len(cs) < k:
        c = g.uniform(lo, hi, size=3).astype(np.float32)
        e = g.uniform(e_min, e_max, size=3).astype(np.float32)
        if np.all(np.abs(c.astype(np.float64)) <= e.astype(np.float64)):
            continue
        cs.append(c)
        es.append(e)
    return (np.ascontiguousarray(np.stack(cs, axis=1)),
            np.ascontiguousarray(np.stack(es, axis=1)))


def hinge_grid(dim: int, g: int, lo: float, hi: float) -> np.ndarray:
    """Regular hinge grid, g points per axis including both ends, x fastest.

    Returns [dim][g**dim] float32; hinge j = ix + g*iy (+ g*g*iz).
    """
    axis = np.linspace(lo, hi, g).astype(np.float32)
    j = np.arange(g ** dim)
    out = np.empty((dim, g ** dim), dtype=np.float32)
    for k in range(dim):
        out[k] = axis[(j // g ** k) % g]
    return np.ascontiguousarray(out)


def dh_params(cfg_id: int, n_dof: int, l_min: float, l_max: float, alpha):
    """Standard DH parameters: a_i ~ U(l_min, l_max), d_i = 0, alpha fixed, theta0 = 0.

    Returns float32 arrays (a, d, alpha, theta0), each [n_dof].
    """
    g = rng(cfg_id, STREAM_DH)
    a = g.uniform(l_min, l_max, size=n_dof).astype(np.float32)
    d = np.zeros(n_dof, np.float32)
    al = np.asarray(alpha, dtype=np.float32)
    th = np.zeros(n_dof, np.float32)
    return a, d, al, th


def uniform_points(cfg_id: int, stream: int, dim: int, n: int, lo, hi) -> np.ndarray:
    """n points U[lo,hi]^dim as [dim][n] float32 (fit data, evaluation sets)."""
    g = rng(cfg_id, stream)
    lo = np.broadcast_to(np.asarray(lo, np.float64), (dim,))
    hi = np.broadcast_to(np.asarray(hi, np.float64), (dim,))
    x = g.uniform(size=(dim, n))
    x = lo[:, None] + (hi - lo)[:, None] * x
    return np.ascontiguousarray(x.astype(np.float32))


def mlp_init(cfg_id: int, widths, zero_last: bool = True):
    """Weights W_l [out][in] ~ U(+-1/sqrt(in)), biases likewise; last layer zero.

    Returns a list of (W, b) float32 pairs.
    """
    g = rng(cfg_id, STREAM_MLP)
    layers = []
    for li in range(len(widths) - 1):
        fin, fout = widths[li], widths[li + 1]
        bound = 1.0 / np.sqrt(fin)
        w = g.uniform(-bound, bound, size=(fout, fin)).astype(np.float32)
        b = g.uniform(-bound, bound, size=fout).astype(np.float32)
        if zero_last and li == len(widths) - 2:
            w[:] = 0
            b[:] = 0
        layers.append((np.ascontiguousarray(w), b))
    return layers


def tanh_init(cfg_id: int, dim: int, H: int, L: int, in_scale: float) -> np.ndarray:
    """Flat float32 parameters of a tanh occupancy network (L hidden layers of width H).

    Layout: W_l [H][n_l], b_l [H] per hidden layer (n_0 = dim), then v [H], b_o.
    Weights ~ U(+-sqrt(6 / (fan_in + fan_out))) (Glorot), the first layer's divided
    by in_scale (the half-width of the domain, so W_0 x is O(1)); first-layer
    biases ~ U(-1, 1), the others zero.
    """
    g = rng(cfg_id, STREAM_TANH)
    parts = []
    nin = dim
    for li in range(L):
        bound = np.sqrt(6.0 / (nin + H))
        w = g.uniform(-bound, bound, size=(H, nin))
        if li == 0:
            w /= in_scale
        b = g.uniform(-1.0, 1.0, size=H) if li == 0 else np.zeros(H)
        parts += [w.ravel(), b]
        nin = H
    bound = np.sqrt(6.0 / (H + 1))
    parts += [g.uniform(-bound, bound, size=H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)
