"""Seeded synthetic workloads for the trajectory optimizer.

This module only draws inputs: a serial arm with collision spheres, cuboid
worlds, start configurations, goal poses and initial seed trajectories.  It
holds none of the optimizer's arithmetic (no kinematics, no distances, no
costs), so the HIP path and the FP64 reference can both consume its output
without sharing any computation.

The shapes follow the paper's setting where it gives them (7-DOF arm, T=32
waypoints, 4 line-search magnitudes, history 4, 100 iterations; the
'Line Search' and L-BFGS history ablations and appendix 'cuRobo Parameters').  The paper's datasets (MotionBenchMaker, MpiNets)
and its Franka sphere model are not available, so these draws stand in for
them; every recipe is fixed by a numpy PCG64 seed and a fixed draw order.

Conventions:
  * a pose is 7 floats: x, y, z, qw, qx, qy, qz (unit quaternion, sign free);
  * a fixed transform is a row-major 3x4 matrix [R | p] (12 floats);
  * link l is actuated by joint ``joint[l]`` rotating about the local z axis
    after its fixed transform (joint frame = parent frame * fixed_tf[l]).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# Line-search magnitudes of the paper (its 'Line Search' ablation) and the
# eight-value set used for the larger candidate sweep.
ALPHA_4 = (0.01, 0.3, 0.7, 1.0)
ALPHA_8 = (0.01, 0.1, 0.2, 0.3, 0.5, 0.7, 0.9, 1.0)


@dataclass
class Robot:
    parent: np.ndarray       # [L] int32, -1 = base
    joint: np.ndarray        # [L] int32, -1 = fixed link
    fixed_tf: np.ndarray     # [L,12] float64
    sphere_link: np.ndarray  # [M] int32
    sphere: np.ndarray       # [M,4] float64 local xyz + radius
    ee_link: np.ndarray      # [n_ee] int32
    ee_tf: np.ndarray        # [n_ee,12] float64
    q_lo: np.ndarray         # [D]
    q_hi: np.ndarray         # [D]

    @property
    def dof(self) -> int:
        return int(self.q_lo.shape[0])

    @property
    def n_links(self) -> int:
        return int(self.parent.shape[0])

    @property
    def n_spheres(self) -> int:
        return int(self.sphere.shape[0])

    @property
    def n_ee(self) -> int:
        return int(self.ee_link.shape[0])


@dataclass
class Worlds:
    offsets: np.ndarray      # [W+1] int32 prefix sums of cuboid counts
    pose: np.ndarray         # [n,7] float64 box->world, xyz + wxyz
    dims: np.ndarray         # [n,3] float64 full side lengths

    @property
    def n_worlds(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def world(self, w: int):
        a, b = int(self.offsets[w]), int(self.offsets[w + 1])
        return self.pose[a:b], self.dims[a:b]


@dataclass
class Batch:
    seeds: np.ndarray        # [P] int32 seeds per problem
    horizon: np.ndarray      # [P] int32 waypoints T per problem
    world: np.ndarray        # [P] int32 world index per problem
    q_start: np.ndarray      # [P,D] float64
    goal: np.ndarray         # [P,n_ee,7] float64
    x0: np.ndarray           # [sum_p S_p*T_p*D] float64, seed-major rows
    meta: dict = field(default_factory=dict)

    @property
    def n_problems(self) -> int:
        return int(self.seeds.shape[0])

    def row_offsets(self, dof: int) -> np.ndarray:
        """Float offset of each seed's [T,D] block in ``x0`` ([sum S+1])."""
        offs = [0]
        for s, t in zip(self.seeds, self.horizon):
            for _ in range(int(s)):
                offs.append(offs[-1] + int(t) * dof)
        return np.asarray(offs, dtype=np.int64)

    def seed_slices(self, dof: int):
        offs = self.row_offsets(dof)
        out, k = [], 0
        for p, (s, t) in enumerate(zip(self.seeds, self.horizon)):
            for i in range(int(s)):
                out.append((p, i, int(t), int(offs[k]), int(offs[k + 1])))
                k += 1
        return out


def _trans_rotx(z: float, angle: float) -> np.ndarray:
    """Fixed transform Trans(0,0,z) * RotX(angle) as a 3x4 row-major array."""
    c, s = math.cos(angle), math.sin(angle)
    return np.array([1, 0, 0, 0,
                     0, c, -s, 0,
                     0, s, c, z], dtype=np.float64)


def _random_quaternion(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random unit quaternions (Shoemake, Graphics Gems III), wxyz."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    qx = a * np.sin(2 * math.pi * u2)
    qy = a * np.cos(2 * math.pi * u2)
    qz = b * np.sin(2 * math.pi * u3)
    qw = b * np.cos(2 * math.pi * u3)
    return np.stack([qw, qx, qy, qz], axis=1)


def asymmetric_limits(seed: int, dof: int):
    """Per-joint limits that differ from joint to joint and are not
    symmetric about 0: q_lo ~ U(-2.9, -0.6), q_hi ~ U(0.6, 2.9) rad."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-2.9, -0.6, size=dof), rng.uniform(0.6, 2.9, size=dof)


def make_arm(seed: int = 0, dof: int = 7, n_spheres: int = 52,
             limit: float = 2.8, limits=None) -> Robot:
    """Synthetic serial arm with revolute z joints.

    Link l (0-based) carries joint l.  Link 0 sits on the base z axis at
    height l_0; links 1.. add Trans(0,0,l_i)*RotX(+-pi/2) with alternating
    sign so that consecutive axes are orthogonal (an arm with only parallel
    axes could not reach random orientations).  Offsets l ~ U(0.05, 0.35) m,
    tool = Trans(0,0,0.10).  Sphere m hangs on link (m mod D) at a fraction
    U(0.1, 0.9) of the segment to the next joint, with N(0, 0.02^2) lateral
    scatter and radius U(0.03, 0.08) m.  Limits are +-limit on every joint,
    or the per-joint arrays ``limits = (q_lo, q_hi)``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lengths = rng.uniform(0.05, 0.35, size=dof)
    fixed = np.zeros((dof, 12))
    for i in range(dof):
        twist = 0.0 if i == 0 else (math.pi / 2 if i % 2 == 1 else -math.pi / 2)
        fixed[i] = _trans_rotx(lengths[i], twist)
    tool_len = 0.10
    seg = np.append(lengths[1:], tool_len)  # segment of link i reaches joint i+1
    link = np.arange(n_spheres) % dof
    frac = rng.uniform(0.1, 0.9, size=n_spheres)
    lateral = rng.normal(0.0, 0.02, size=(n_spheres, 2))
    radius = rng.uniform(0.03, 0.08, size=n_spheres)
    sph = np.zeros((n_spheres, 4))
    sph[:, 0] = lateral[:, 0]
    sph[:, 1] = lateral[:, 1]
    sph[:, 2] = frac * seg[link]
    sph[:, 3] = radius
    ee_tf = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, tool_len]], dtype=np.float64)
    return Robot(parent=np.arange(-1, dof - 1, dtype=np.int32),
                 joint=np.arange(dof, dtype=np.int32),
                 fixed_tf=fixed,
                 sphere_link=link.astype(np.int32),
                 sphere=sph,
                 ee_link=np.array([dof - 1], dtype=np.int32),
                 ee_tf=ee_tf,
                 q_lo=np.full(dof, -limit) if limits is None else np.asarray(limits[0], dtype=np.float64).copy(),
                 q_hi=np.full(dof, limit) if limits is None else np.asarray(limits[1], dtype=np.float64).copy())


def make_two_arm(seed: int = 0, dof_per_arm: int = 7, n_spheres: int = 120,
                 limit: float = 2.8) -> Robot:
    """Two 7-joint arms on a shared base (a kinematic tree, 14 DOF).

    Each branch is built like :func:`make_arm`; the second branch's root is
    offset 0.5 m along base y.  Spheres alternate between the two branches.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    d2 = 2 * dof_per_arm
    fixed = np.zeros((d2, 12))
    parent = np.zeros(d2, dtype=np.int32)
    seglen = np.zeros(d2)
    tool_len = 0.10
    for arm in range(2):
        lengths = rng.uniform(0.05, 0.35, size=dof_per_arm)
        for i in range(dof_per_arm):
            l = arm * dof_per_arm + i
            twist = 0.0 if i == 0 else (math.pi / 2 if i % 2 == 1 else -math.pi / 2)
            fixed[l] = _trans_rotx(lengths[i], twist)
            parent[l] = -1 if i == 0 else l - 1
            seglen[l] = lengths[i + 1] if i + 1 < dof_per_arm else tool_len
        fixed[arm * dof_per_arm, 7] = -0.25 if arm == 0 else 0.25
    link = np.array([(m % 2) * dof_per_arm + (m // 2) % dof_per_arm
                     for m in range(n_spheres)], dtype=np.int32)
    frac = rng.uniform(0.1, 0.9, size=n_spheres)
    lateral = rng.normal(0.0, 0.02, size=(n_spheres, 2))
    radius = rng.uniform(0.03, 0.08, size=n_spheres)
    sph = np.zeros((n_spheres, 4))
    sph[:, 0] = lateral[:, 0]
    sph[:, 1] = lateral[:, 1]
    sph[:, 2] = frac * seglen[link]
    sph[:, 3] = radius
    tool = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, tool_len], dtype=np.float64)
    return Robot(parent=parent,
                 joint=np.arange(d2, dtype=np.int32),
                 fixed_tf=fixed,
                 sphere_link=link,
                 sphere=sph,
                 ee_link=np.array([dof_per_arm - 1, d2 - 1], dtype=np.int32),
                 ee_tf=np.stack([tool, tool]),
                 q_lo=np.full(d2, -limit),
                 q_hi=np.full(d2, limit))


def make_worlds(seed: int, counts, oriented: bool = True, base_clear: float = 0.12) -> Worlds:
    """Cuboid worlds: sides U(0.05,0.4) m, centers U([-.5,.5]^2 x [0,1]) m.

    ``oriented`` draws a uniform random orientation per cuboid (Shoemake),
    otherwise boxes are axis aligned.  Cuboids whose centre lies below 0.6 m
    and whose enclosing ball comes within ``base_clear`` of the vertical axis
    through the robot base are redrawn, so the base column is free.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = [int(c) for c in counts]
    n = sum(counts)
    dims = rng.uniform(0.05, 0.4, size=(n, 3))
    centers = np.empty((n, 3))
    centers[:, 0:2] = rng.uniform(-0.5, 0.5, size=(n, 2))
    centers[:, 2] = rng.uniform(0.0, 1.0, size=n)
    if base_clear > 0:
        half_diag = 0.5 * np.linalg.norm(dims, axis=1)
        for i in range(n):
            while centers[i, 2] < 0.6 and np.hypot(centers[i, 0], centers[i, 1]) < base_clear + half_diag[i]:
                centers[i, 0:2] = rng.uniform(-0.5, 0.5, size=2)
                centers[i, 2] = rng.uniform(0.0, 1.0)
    if oriented:
        quat = _random_quaternion(rng, n)
    else:
        quat = np.tile(np.array([1.0, 0.0, 0.0, 0.0]), (n, 1))
    offsets = np.zeros(len(counts) + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(counts)
    return Worlds(offsets=offsets, pose=np.concatenate([centers, quat], axis=1), dims=dims)


def _goal_poses(rng: np.random.Generator, n: int, r_lo=0.3, r_hi=0.8) -> np.ndarray:
    """Positions uniform in the spherical shell r_lo..r_hi, random orientation."""
    r = np.cbrt(rng.uniform(r_lo ** 3, r_hi ** 3, size=n))
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return np.concatenate([v * r[:, None], _random_quaternion(rng, n)], axis=1)


def make_batch(robot: Robot, seed: int, seeds, horizon, world,
               start_range: float = 1.0, noise: float = 0.05) -> Batch:
    """Problems with a random start, a random goal pose per end effector and
    seeds that interpolate linearly from the start to a random endpoint
    U(-2.5,2.5)^D plus N(0, noise^2) per waypoint, clipped to the limits.
    For a horizon of 1 (inverse kinematics) a seed is a single random
    configuration U(0.9*limits)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    seeds = np.asarray(seeds, dtype=np.int32)
    horizon = np.asarray(horizon, dtype=np.int32)
    world = np.asarray(world, dtype=np.int32)
    P, D = seeds.shape[0], robot.dof
    q_start = rng.uniform(-start_range, start_range, size=(P, D))
    goal = _goal_poses(rng, P * robot.n_ee).reshape(P, robot.n_ee, 7)
    rows = []
    for p in range(P):
        T = int(horizon[p])
        for _ in range(int(seeds[p])):
            if T == 1:
                rows.append(rng.uniform(0.9 * robot.q_lo, 0.9 * robot.q_hi).reshape(1, D))
                continue
            end = rng.uniform(-2.5, 2.5, size=D)
            frac = (np.arange(1, T + 1) / T)[:, None]
            traj = q_start[p][None, :] * (1 - frac) + end[None, :] * frac
            traj += rng.normal(0.0, noise, size=(T, D))
            rows.append(np.clip(traj, robot.q_lo, robot.q_hi))
    x0 = np.concatenate([r.reshape(-1) for r in rows]) if rows else np.zeros(0)
    return Batch(seeds=seeds, horizon=horizon, world=world, q_start=q_start,
                 goal=goal, x0=x0)


# ---------------------------------------------------------------------------
# Named workloads.  Each returns (robot, worlds, batch, settings).

def cfg_plain(seed: int = 1):
    """One problem: 7-DOF arm with 20 spheres, 10 axis-aligned cuboids,
    T=32, 4 seeds, 100 iterations, 4 line-search magnitudes."""
    robot = make_arm(seed=0, n_spheres=20)
    worlds = make_worlds(seed, [10], oriented=False)
    batch = make_batch(robot, seed + 100, [4], [32], [0])
    return robot, worlds, batch, dict(name="plain-1x4x32", alpha=ALPHA_4, iters=100)


def cfg_cost_adjoint(seed: int = 2):
    """Cost+adjoint throughput: 52 spheres, 40 oriented cuboids,
    32 seeds x T=32 x 8 line-search candidates."""
    robot = make_arm(seed=0, n_spheres=52)
    worlds = make_worlds(seed, [40], oriented=True)
    batch = make_batch(robot, seed + 100, [32], [32], [0])
    return robot, worlds, batch, dict(name="cost-adjoint-32x32x8", alpha=ALPHA_8, iters=100)


def cfg_ik(seed: int = 3, n_goals: int = 4096, n_seeds: int = 32):
    """Collision-free IK batch: T=1, n_goals goal poses x n_seeds seeds, one
    shared world of 40 oriented cuboids, 52 spheres."""
    robot = make_arm(seed=0, n_spheres=52)
    worlds = make_worlds(seed, [40], oriented=True)
    batch = make_batch(robot, seed + 100, [n_seeds] * n_goals, [1] * n_goals, [0] * n_goals)
    return robot, worlds, batch, dict(name=f"ik-{n_goals}x{n_seeds}", alpha=ALPHA_4, iters=100)


def goal_configs(robot: Robot, seed: int, n: int, spread: float = 2.5) -> np.ndarray:
    """n joint configurations U(-spread, spread)^D (clipped to the limits);
    their end-effector poses are goals reachable by construction."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = rng.uniform(-spread, spread, size=(n, robot.dof))
    return np.clip(q, robot.q_lo, robot.q_hi)


def self_pairs(robot: Robot, min_gap: int = 2) -> np.ndarray:
    """Sphere pairs checked for self-collision: spheres on links at least
    `min_gap` apart along the kinematic tree (adjacent links may touch).
    Returns [n, 2] int32, i < j."""
    L = robot.n_links
    depth = np.zeros(L, dtype=np.int64)
    for l in range(L):
        depth[l] = 0 if robot.parent[l] < 0 else depth[robot.parent[l]] + 1

    def gap(a, b):
        # tree distance between links a and b
        n = 0
        while a != b:
            if depth[a] >= depth[b]:
                a = robot.parent[a]
            else:
                b = robot.parent[b]
            n += 1
            if a < 0 or b < 0:
                return 1 << 20     # different roots
        return n
    lk = robot.sphere_link
    out = [(i, j) for i in range(robot.n_spheres) for j in range(i + 1, robot.n_spheres)
           if gap(int(lk[i]), int(lk[j])) >= min_gap]
    return np.asarray(out, dtype=np.int32).reshape(-1, 2)


def normal_draws(seed: int, shape) -> np.ndarray:
    """Standard normal draws (float32) for the particle stage."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size=shape, dtype=np.float32)


def cfg_uneven(seed: int = 4, n_problems: int = 64):
    """Uneven batch: per problem seeds U{4..64}, T in {24,32,48}, its own
    world of U{5..200} oriented cuboids."""
    rng = np.random.Generator(np.random.PCG64(seed))
    robot = make_arm(seed=0, n_spheres=52)
    seeds = rng.integers(4, 65, size=n_problems)
    horizon = rng.choice(np.array([24, 32, 48]), size=n_problems)
    counts = rng.integers(5, 201, size=n_problems)
    worlds = make_worlds(seed + 1, counts, oriented=True)
    batch = make_batch(robot, seed + 100, seeds, horizon, np.arange(n_problems))
    return robot, worlds, batch, dict(name=f"uneven-{n_problems}", alpha=ALPHA_4, iters=100)


def cfg_large(seed: int = 5):
    """Large: 14-DOF two-arm tree, 120 spheres, 500 oriented cuboids,
    128 seeds x T=48."""
    robot = make_two_arm(seed=0, n_spheres=120)
    worlds = make_worlds(seed, [500], oriented=True)
    batch = make_batch(robot, seed + 100, [128], [48], [0])
    return robot, worlds, batch, dict(name="large-128x48-tree", alpha=ALPHA_4, iters=100)


def to_f32(batch: Batch) -> Batch:
    """Round every floating input of a batch to float32 (and back to float64
    storage), so that the FP32 device path and the FP64 reference see
    identical values."""
    return Batch(seeds=batch.seeds, horizon=batch.horizon, world=batch.world,
                 q_start=batch.q_start.astype(np.float32).astype(np.float64),
                 goal=batch.goal.astype(np.float32).astype(np.float64),
                 x0=batch.x0.astype(np.float32).astype(np.float64), meta=batch.meta)


def robot_f32(robot: Robot) -> Robot:
    f = lambda a: a.astype(np.float32).astype(np.float64)
    return Robot(parent=robot.parent, joint=robot.joint, fixed_tf=f(robot.fixed_tf),
                 sphere_link=robot.sphere_link, sphere=f(robot.sphere),
                 ee_link=robot.ee_link, ee_tf=f(robot.ee_tf), q_lo=f(robot.q_lo),
                 q_hi=f(robot.q_hi))


def worlds_f32(w: Worlds) -> Worlds:
    f = lambda a: a.astype(np.float32).astype(np.float64)
    return Worlds(offsets=w.offsets, pose=f(w.pose), dims=f(w.dims))
