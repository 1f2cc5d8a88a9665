"""Frozen workload configurations and the readings taken where the paper is silent.

The method (Lai, Zhi, Hermans, Ramos: Parallelised Diffeomorphic Sampling-based
Motion Planning) morphs base samples by explicit-Euler integration of the negative
gradient of a learned occupancy cost (Sec. 3.2, Eq. 1 and the Euler remark after
Eq. 2), pulled back into joint space through forward-kinematics Jacobians for an arm
(Sec. 3.2, Eq. 3).  The occupancy is a logistic classifier trained with binary
cross-entropy (Sec. 3.1); here it is the Hilbert-map form sigma(w^T phi(x) + beta)
over Gaussian RBF features on a hinge grid.

Every constant below is a workload parameter, not a result.  Nothing here computes
any part of the method.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

# Seed entropy shared by every generator (the arXiv number of the paper).
ENTROPY = 2108_11775

# Generator streams (spawn keys), one per kind of input.
STREAM_SCENE = 0
STREAM_FIT = 1
STREAM_BASE = 2
STREAM_DH = 3
STREAM_MLP = 4
STREAM_SHUFFLE = 5
STREAM_EVAL = 6
STREAM_TANH = 7


@dataclass(frozen=True)
class Workspace2D:
    """2-D disc world: plain morph of workspace points (configs 1 and 2)."""
    cfg_id: int
    name: str
    lo: float = -10.0
    hi: float = 10.0
    n_discs: int = 20
    r_min: float = 0.5
    r_max: float = 1.5
    grid: int = 30               # hinges per axis; M = grid**2
    lengthscale: float = 0.7
    fit_points: int = 10_000
    fit_steps: int = 200
    fit_l2: float = 1e-3
    fit_lr: float = 64.0         # GD step on w, see the `gd_learning_rate` reading
    fit_lr_bias: float = 2.0     # GD step on beta
    n_samples: int = 4096
    T: int = 20
    eta: float = 0.05

    @property
    def n_hinges(self) -> int:
        return self.grid ** 2


@dataclass(frozen=True)
class Arm7:
    """7-DOF arm in a 3-D box world (config 3) and its occupancy fit (config 4)."""
    cfg_id: int = 3
    name: str = "arm7-65536"
    n_dof: int = 7
    pts_per_link: int = 8
    link_min: float = 0.1
    link_max: float = 0.4
    # Standard DH twist pattern, base at the origin, all offsets d = 0.
    alpha: tuple = (math.pi / 2, -math.pi / 2, math.pi / 2, -math.pi / 2,
                    math.pi / 2, -math.pi / 2, 0.0)
    q_lo: float = -math.pi
    q_hi: float = math.pi
    box_lo: float = -1.0
    box_hi: float = 1.0
    n_boxes: int = 40
    half_min: float = 0.05
    half_max: float = 0.35      # raised once from 0.15 (prior free 86 % -> 45 %)
    grid: int = 16               # 16^3 = 4096 hinges
    lengthscale: float = 0.15
    n_samples: int = 65_536
    T: int = 30
    eta: float = 0.01

    @property
    def n_hinges(self) -> int:
        return self.grid ** 3

    @property
    def n_body(self) -> int:
        return self.n_dof * self.pts_per_link


@dataclass(frozen=True)
class Fit3D:
    """Config 4: occupancy fit of the arm's box world on labelled 3-D points."""
    cfg_id: int = 4
    name: str = "fit3d-1M"
    n_points: int = 1 << 20
    steps: int = 500
    l2: float = 1e-4
    lr: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


@dataclass(frozen=True)
class Amortised:
    """Config 5: residual MLP q_hat = q + f(q), f = 7-256-256-256-7 SiLU."""
    cfg_id: int = 5
    name: str = "amortised-arm7"
    widths: tuple = (7, 256, 256, 256, 7)
    train_pairs: int = 1 << 22
    batch: int = 65_536
    epochs: int = 50
    lr: float = 3e-3
    schedule: str = "cosine"  # lr (1 + cos(pi t / steps)) / 2 over the 3,200 Adam steps
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    threshold: float = 0.5
    eval_samples: int = 65_536


@dataclass(frozen=True)
class TanhOcc:
    """The paper's own occupancy (Sec. 3.1): a fully connected network with tanh
    between hidden layers and a sigmoid output, on the 2-D disc worlds of configs 1
    and 2 (same scenes, fit points, samples, T and eta as the RBF occupancy)."""
    name: str = "tanh-occ"
    hidden: int = 64
    layers: int = 3
    lr: float = 1e-2        # full-batch Adam on mean BCE + (l2/2)|weights|^2
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    steps: tuple = (1000, 1500)   # configs 1, 2
    l2: tuple = (1e-5, 1e-6)


C1 = Workspace2D(cfg_id=1, name="ws2d-4096")
C2 = Workspace2D(cfg_id=2, name="ws2d-1M", n_discs=100, grid=64, lengthscale=0.4,
                 fit_lr=128.0, n_samples=1 << 20, T=50, eta=0.02)
C3 = Arm7()
C4 = Fit3D()
C5 = Amortised()
TANH = TanhOcc()

CONFIGS = {1: C1, 2: C2, 3: C3, 4: C4, 5: C5}

# RRT consumer of the producer/consumer workload: start and goal in the disc worlds,
# points of largest clearance on a 0.5 lattice near opposite corners.
RRT_START_GOAL = {1: ((-10.0, -10.0), (8.0, 10.0)), 2: ((-10.0, -8.0), (10.0, 10.0))}

# Readings of points the paper leaves open (each is listed with its reason in the
# design notes).  They are frozen here so that every side uses the same ones.
READINGS = {
    "tanh_network": "3 hidden tanh layers of 64 on raw coordinates (the paper gives no "
                    "widths); Glorot init with the first layer divided by the domain "
                    "half-width; Adam lr 1e-2 on all parameters, L2 on weights only",
    "rbf": "phi_j(x) = exp(-|x-h_j|^2 / (2 l^2))",
    "bias": "scalar beta, unregularised, stored as weights[M]",
    "grid": "linspace(lo, hi, g) per axis, both ends included, x fastest",
    "euler": "explicit forward Euler, gradient at the current state, fixed eta, "
             "T steps, no clipping, joints not wrapped",
    "eq3": "grad_q c = sum_p J_p(q)^T grad_x c(psi_p(q)); cost = sum of body-point "
           "occupancies",
    "body_points": "8 per link at k/8, k=1..8, along o_{i-1} -> o_i",
    "labels": "closed obstacles, decided in FP64; a configuration collides iff any "
              "body point lies in any box",
    "gd_learning_rate": "gradient descent with one step for w and one for beta: "
                        "lr_w = 1/(0.25*lambda_max(Phi^T Phi/n) + l2) rounded down to a "
                        "power of two (50 power iterations on the config's own fit "
                        "data: 64 for config 1, 128 for config 2); lr_beta = 2, half of "
                        "1/(0.25*1) for the constant feature, so the preconditioned "
                        "step stays below 2/L",
    "adam": "Kingma & Ba Algorithm 1 with bias correction, eps added to sqrt(v_hat)",
    "fallback": "max over body points of c(psi_p(q_hat)) > 0.5 re-runs the plain morph "
                "from the base q",
}
