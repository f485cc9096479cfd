"""Seeded synthetic inputs shared by the HIP path and the FP64 oracle.

This module holds data only: the robot description, the sphere model, the
scene and start/goal generators and the per-workload parameters.  It holds none
of the method's arithmetic (no integrator, kinematics, cost or update), so that
the two implementations it feeds stay independent.  Everything is drawn from
``numpy.random.default_rng(seed)`` on the host.

The paper (STORM, arXiv 2104.13542) controls a 7-joint Franka Panda; it does not
print the arm's kinematic constants, so the published Franka modified (Craig)
Denavit-Hartenberg table and joint limits are used.  Its learned self-collision
and scene-collision networks are not available, so a synthetic 52-sphere body
model and random sphere/cuboid scenes stand in for them (Sec. 3.2, Eq. 13-14).

Goal poses are given as joint configurations ``q_goal``: the caller turns them
into a pose with whichever forward kinematics it owns, so that goals are
reachable by construction without this module computing kinematics.
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

DOF = 7

# Franka Panda, modified DH: one row per frame k = 1..8 holding
# (a_{k-1} [m], d_k [m], alpha_{k-1} [rad]).  Frame 8 is the flange (theta = 0).
PANDA_DH = np.array(
    [
        [0.0, 0.333, 0.0],
        [0.0, 0.0, -math.pi / 2],
        [0.0, 0.316, math.pi / 2],
        [0.0825, 0.0, math.pi / 2],
        [-0.0825, 0.384, -math.pi / 2],
        [0.0, 0.0, math.pi / 2],
        [0.088, 0.0, math.pi / 2],
        [0.0, 0.107, 0.0],
    ],
    dtype=np.float64,
)

PANDA_Q_MIN = np.array([-2.8973, -1.7628, -2.8973, -3.0718, -2.8973, -0.0175, -2.8973])
PANDA_Q_MAX = np.array([2.8973, 1.7628, 2.8973, -0.0698, 2.8973, 3.7525, 2.8973])
PANDA_QD_MAX = np.array([2.1750, 2.1750, 2.1750, 2.1750, 2.6100, 2.6100, 2.6100])

# A collision-free reference configuration used by examples and the closed loop.
PANDA_READY = np.array([0.0, -0.785, 0.0, -2.356, 0.0, 1.571, 0.785])


def _segment(body, p0, p1, n, r0, r1):
    rows = []
    for i in range(n):
        t = i / (n - 1) if n > 1 else 0.0
        p = [p0[c] * (1.0 - t) + p1[c] * t for c in range(3)]
        rows.append([float(body), p[0], p[1], p[2], r0 * (1.0 - t) + r1 * t])
    return rows


def panda_spheres() -> np.ndarray:
    """Synthetic 52-sphere body model, rows (body, x, y, z, r) in the body frame.

    Bodies 1..7 are the links (attached to DH frame k), body 8 the hand on the
    flange frame.  Sphere counts per body are 6, 6, 6, 8, 10, 6, 4, 6 and radii
    lie in [0.04, 0.08] m.  Spheres sit along each link's segment, pulled back
    from the joints so that the ready configuration is free of self-contact.
    Rows are sorted by body.
    """
    s = []
    s += _segment(1, (0, 0, -0.30), (0, 0, -0.12), 6, 0.08, 0.06)
    s += _segment(2, (0, -0.02, 0), (0, -0.17, 0), 6, 0.07, 0.06)
    s += _segment(3, (0, 0, -0.22), (0.03, 0, -0.10), 6, 0.06, 0.05)
    s += _segment(4, (-0.02, 0.06, 0), (-0.08, 0.22, 0), 8, 0.06, 0.05)
    s += _segment(5, (0, 0.05, -0.30), (0, 0.0, -0.14), 10, 0.06, 0.045)
    s += _segment(6, (0.0, 0, -0.03), (0.07, 0, 0.0), 6, 0.05, 0.045)
    s += _segment(7, (0, 0, 0.01), (0, 0, 0.07), 4, 0.045, 0.04)
    s += _segment(8, (0, -0.05, 0.09), (0, 0.05, 0.09), 3, 0.04, 0.04)
    s += _segment(8, (0, 0, 0.05), (0, 0, 0.14), 3, 0.04, 0.04)
    return np.array(s, dtype=np.float64)


# Obstacle record: 16 values [kind, cx, cy, cz, e0, e1, e2, R00..R22].
# kind 0 = sphere (e0 = radius), kind 1 = cuboid (e = half extents,
# R = rotation of the box frame into the world frame, row-major).
OBSTACLE_STRIDE = 16
OBS_SPHERE = 0
OBS_CUBOID = 1

# Cost-term switches (bit mask) for Sec. 3.2, Eq. 15.
COST_POSE = 1 << 0
COST_JOINT = 1 << 1
COST_VEL = 1 << 2
COST_STOP = 1 << 3
COST_MANIP = 1 << 4
COST_SELF = 1 << 5
COST_ENV = 1 << 6
COST_ALL = 0x7F  # the reaching task's terms (the ball term is separate)
COST_BALL = 1 << 7


@dataclasses.dataclass
class Params:
    """Parameters of one MPC problem (all SI units)."""

    n_particles: int
    horizon: int
    dt: np.ndarray  # [H] step lengths
    n_halton: int = 0  # particles [0, n_halton) use Halton + B-spline noise
    n_null: int = 0  # particles [N - n_null, N) are zero-acceleration
    n_knots: int = 8  # B-spline control points
    seed: int = 0
    beta: float = 0.1
    gamma: float = 1.0
    alpha_mu: float = 1.0
    alpha_sigma: float = 0.1
    w_term: float = 1.0
    sigma2_min: float = 0.0
    sigma_init: np.ndarray = dataclasses.field(default_factory=lambda: np.full(DOF, 0.1))
    acc_stop: float = 2.0
    k_jl: float = 0.1
    k_vl: float = 0.1
    k_m: float = 0.05
    w_pos: float = 150.0
    w_rot: float = 20.0
    alpha_pos: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(3))
    alpha_rot: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(3))
    a_stop: float = 10.0
    a_joint: float = 100.0
    a_vel: float = 10.0
    a_manip: float = 30.0
    a_coll: float = 1000.0
    cost_mask: int = COST_POSE | COST_JOINT
    grad_mask: int = 0  # terms of the differentiable form; 0 = cost_mask
    comb_filter: int = 0  # 1: comb-filter the Gaussian particles' noise along the horizon (Sec. 3.3)
    comb: tuple = (1.0, 0.0, 0.0)  # (c1, c2, c3): e'_h = c1 e_h + c2 e'_{h-1} + c3 e'_{h-2}
    cov_per_step: int = 0  # 1: one diagonal covariance per (step, joint), each updated by Eq. 5
    # ball on the tray (dynamic object balancing): the ball term (COST_BALL) is
    # w_ball times the ball's distance from the tray centre in the tray plane
    w_ball: float = 0.0
    ball_gravity: tuple = (0.0, 0.0, -9.81)  # world frame, m/s^2
    ball_center: tuple = (0.0, 0.0)  # tray centre in the flange frame (x, y), m
    self_model: int = 0  # self-collision term: 0 sphere pairs, 1 the learned network (Problem.self_mlp)


@dataclasses.dataclass
class Problem:
    params: Params
    q0: np.ndarray  # [7]
    v0: np.ndarray  # [7]
    a0: np.ndarray  # [7]
    q_goal: np.ndarray  # [7] joint configuration whose flange pose is the goal
    obstacles: np.ndarray  # [O, 16]
    spheres: np.ndarray  # [S, 5]
    # ball state in the flange frame of q0: position (x, y, z) and velocity;
    # the caller moves it to the world frame with its own forward kinematics
    ball_tray: np.ndarray = None
    # parameters of the learned self-collision network (self_model = 1), the
    # layout of SELF_MLP_LAYOUT
    self_mlp: np.ndarray = None


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation (normalised Gaussian quaternion)."""
    w, x, y, z = rng.standard_normal(4)
    n = math.sqrt(w * w + x * x + y * y + z * z)
    w, x, y, z = w / n, x / n, y / n, z / n
    return np.array(
        [
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ]
    )


def random_scene(rng: np.random.Generator, n_spheres: int, n_cuboids: int) -> np.ndarray:
    """Spheres r ~ U(0.03, 0.15) m and cuboids with half extents ~ U(0.03, 0.15) m,
    random orientation, centres ~ U([0,1] x [-0.5,0.5] x [0,1]) m."""
    rows = []
    lo = np.array([0.0, -0.5, 0.0])
    hi = np.array([1.0, 0.5, 1.0])
    for _ in range(n_spheres):
        c = rng.uniform(lo, hi)
        r = rng.uniform(0.03, 0.15)
        row = np.zeros(OBSTACLE_STRIDE)
        row[0] = OBS_SPHERE
        row[1:4] = c
        row[4] = r
        row[7:16] = np.eye(3).reshape(-1)
        rows.append(row)
    for _ in range(n_cuboids):
        c = rng.uniform(lo, hi)
        e = rng.uniform(0.03, 0.15, size=3)
        row = np.zeros(OBSTACLE_STRIDE)
        row[0] = OBS_CUBOID
        row[1:4] = c
        row[4:7] = e
        row[7:16] = random_rotation(rng).reshape(-1)
        rows.append(row)
    if not rows:
        return np.zeros((0, OBSTACLE_STRIDE))
    return np.array(rows)


def random_q(rng: np.random.Generator) -> np.ndarray:
    return rng.uniform(PANDA_Q_MIN, PANDA_Q_MAX)


def config1(seed: int = 0, v0_random: bool = False) -> Problem:
    """Plain single step: N=64, H=16, dt=0.02, Gaussian noise sigma=0.1,
    pose + joint-limit costs, beta=0.1."""
    rng = np.random.default_rng(seed)
    q0 = random_q(rng)
    q_goal = random_q(rng)
    v0 = rng.uniform(-0.5, 0.5, DOF) if v0_random else np.zeros(DOF)
    p = Params(n_particles=64, horizon=16, dt=np.full(16, 0.02), seed=seed,
               cost_mask=COST_POSE | COST_JOINT)
    return Problem(p, q0, v0, np.zeros(DOF), q_goal, np.zeros((0, OBSTACLE_STRIDE)), panda_spheres())


def config2(seed: int = 0, n_particles: int = 500, horizon: int = 30,
            n_obs_spheres: int = 30, n_obs_cuboids: int = 20) -> Problem:
    """STORM-shaped step: N=500 (half Halton + cubic B-spline with 8 control
    points, half Gaussian), H=30, dt = linspace(0.01, 0.1, 30), every cost term,
    52 body spheres, 30 sphere + 20 cuboid obstacles."""
    rng = np.random.default_rng(seed)
    q0 = random_q(rng)
    q_goal = random_q(rng)
    obstacles = random_scene(rng, n_obs_spheres, n_obs_cuboids)
    p = Params(n_particles=n_particles, horizon=horizon,
               dt=np.linspace(0.01, 0.1, horizon), n_halton=n_particles // 2,
               n_knots=8, seed=seed, sigma_init=np.full(DOF, 0.3), cost_mask=COST_ALL)
    return Problem(p, q0, np.zeros(DOF), np.zeros(DOF), q_goal, obstacles, panda_spheres())


def config3_problem(p_index: int) -> Problem:
    """One problem of the batched workload: problem p uses seed 1000 + p,
    N ~ U{128..1024}, H ~ U{20..40}, O ~ U{10..50} obstacles (half spheres)."""
    rng = np.random.default_rng(1000 + p_index)
    n = int(rng.integers(128, 1025))
    h = int(rng.integers(20, 41))
    o = int(rng.integers(10, 51))
    q0 = random_q(rng)
    q_goal = random_q(rng)
    obstacles = random_scene(rng, o // 2, o - o // 2)
    p = Params(n_particles=n, horizon=h, dt=np.linspace(0.01, 0.1, h), n_halton=n // 2,
               n_knots=8, seed=1000 + p_index, sigma_init=np.full(DOF, 0.3), cost_mask=COST_ALL)
    return Problem(p, q0, np.zeros(DOF), np.zeros(DOF), q_goal, obstacles, panda_spheres())


def config4(seed: int = 0) -> Problem:
    """Differentiable workload: N=1024, H=30, the costs and dt of the plain step."""
    rng = np.random.default_rng(seed)
    q0 = random_q(rng)
    q_goal = random_q(rng)
    p = Params(n_particles=1024, horizon=30, dt=np.full(30, 0.02), seed=seed,
               cost_mask=COST_POSE | COST_JOINT)
    return Problem(p, q0, np.zeros(DOF), np.zeros(DOF), q_goal, np.zeros((0, OBSTACLE_STRIDE)),
                   panda_spheres())


def config5_problem(p_index: int) -> Problem:
    """One problem of the large workload: N=4096, H=64, 100 obstacles (50/50)."""
    rng = np.random.default_rng(5000 + p_index)
    q0 = random_q(rng)
    q_goal = random_q(rng)
    obstacles = random_scene(rng, 50, 50)
    p = Params(n_particles=4096, horizon=64, dt=np.linspace(0.01, 0.1, 64), n_halton=2048,
               n_knots=8, seed=5000 + p_index, sigma_init=np.full(DOF, 0.3),
               cost_mask=COST_ALL)
    return Problem(p, q0, np.zeros(DOF), np.zeros(DOF), q_goal, obstacles, panda_spheres())


def config_ball(seed: int = 0, n_particles: int = 500, horizon: int = 30) -> Problem:
    """Ball-on-tray workload: the arm near its ready configuration holds the
    tray level; a ball at a random place on the tray with a small random
    velocity.  N=500 (half Halton + B-spline), H=30, dt = linspace(0.01, 0.1),
    ball + joint + velocity + stop + manipulability + self-collision terms."""
    rng = np.random.default_rng(7000 + seed)
    q0 = PANDA_READY + rng.uniform(-0.1, 0.1, DOF)
    ball = np.concatenate([rng.uniform(-0.08, 0.08, 2), [0.02], rng.uniform(-0.05, 0.05, 2), [0.0]])
    p = Params(n_particles=n_particles, horizon=horizon, dt=np.linspace(0.01, 0.1, horizon),
               n_halton=n_particles // 2, n_knots=8, seed=7000 + seed, sigma_init=np.full(DOF, 0.3),
               cost_mask=COST_BALL | COST_JOINT | COST_VEL | COST_STOP | COST_MANIP | COST_SELF, w_ball=100.0)
    return Problem(p, q0, np.zeros(DOF), np.zeros(DOF), PANDA_READY.copy(), np.zeros((0, OBSTACLE_STRIDE)),
                   panda_spheres(), ball)


# The learned self-collision network (Eq. 13, jointNERF form): input
# [sin q, cos q], hidden layers of 256, 128 and 64 units (ReLU), one output.
# Parameters in one flat array, in this order (weights [out][in]).
SELF_MLP_LAYOUT = (("W1", (256, 14)), ("b1", (256,)), ("W2", (128, 256)), ("b2", (128,)),
                   ("W3", (64, 128)), ("b3", (64,)), ("w4", (64,)), ("b4", (1,)))
SELF_MLP_SIZE = sum(int(np.prod(s)) for _, s in SELF_MLP_LAYOUT)


def random_self_mlp(seed: int = 0) -> np.ndarray:
    """Seeded network parameters with He-scaled weights, every value exactly
    representable in FP16 (so a half-precision evaluation starts from the
    same weights)."""
    rng = np.random.default_rng(9000 + seed)
    out = []
    for name, shape in SELF_MLP_LAYOUT:
        if name.startswith("W") or name == "w4":
            fan_in = shape[-1]
            v = rng.normal(scale=math.sqrt(2.0 / fan_in), size=shape)
        else:
            v = rng.uniform(-0.1, 0.1, size=shape)
        out.append(v.reshape(-1))
    return np.concatenate(out).astype(np.float16).astype(np.float64)


# Parameters of the network fitted to the Panda sphere model's signed link
# distance (written by oracle/train_self_mlp.py; FP16-exact values).
PANDA_SELF_MLP = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "self_mlp_panda.npy")


def panda_self_mlp() -> np.ndarray:
    return np.load(PANDA_SELF_MLP).astype(np.float64)


def config_self_mlp(seed: int = 0, n_particles: int = 500, horizon: int = 30, trained: bool = True) -> Problem:
    """The STORM-shaped step with the learned self-collision network in place
    of the sphere pairs: the network fitted to the sphere model (trained), or
    seeded random parameters of the same shape."""
    prob = config2(seed, n_particles=n_particles, horizon=horizon)
    prob.params.self_model = 1
    prob.self_mlp = panda_self_mlp() if trained else random_self_mlp(seed)
    return prob


def standard_normal(seed: int, shape) -> np.ndarray:
    """Seeded standard-normal array, used as an explicit noise input."""
    return np.random.default_rng(seed).standard_normal(shape)
