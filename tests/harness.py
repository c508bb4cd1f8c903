"""Shared helpers of the parity tests: build identical fp32 inputs for the HIP
path and the FP64 reference, and compare their outputs.

Tolerances (written here once, used by every parity test):
  cost      |c - c_ref| <= 1e-4 |c_ref| + 1e-6               (per seed)
  gradient  |g - g_ref|_2 <= 1e-3 |g_ref|_2 + 1e-6           (per seed block)
  verdict   (min_clear >= 0) equal unless |min_clear_ref| <= 1e-5 m
"""
from __future__ import annotations

import numpy as np

from paper_2310_17274_amd import workloads as wl

COST_RTOL = 1e-4
GRAD_RTOL = 1e-3
ABS_TOL = 1e-6
CONTACT_TOL = 1e-5


def f32_inputs(robot, worlds, batch):
    return wl.robot_f32(robot), wl.worlds_f32(worlds), wl.to_f32(batch)


def rows_of(batch, dof):
    return batch.x0.reshape(-1, dof)


def problem_rows(batch):
    """(p, first row, S, T) per problem."""
    out, r = [], 0
    for p, (s, t) in enumerate(zip(batch.seeds, batch.horizon)):
        out.append((p, r, int(s), int(t)))
        r += int(s) * int(t)
    return out


def oracle_cost_grad(ref, worlds, batch, q_rows, nthreads=8, grad=True):
    """Reference cost [seeds], grad [rows, D], min clearance [seeds]."""
    D = ref.robot.dof
    costs, grads, mcs = [], [], []
    for p, r0, S, T in problem_rows(batch):
        w = int(batch.world[p])
        q = q_rows[r0:r0 + S * T].reshape(-1)
        c, g, mc = ref.cost_grad_batch(worlds.world(w), batch.q_start[p], batch.goal[p], T, q,
                                       nthreads=nthreads, grad=grad)
        costs.append(c)
        mcs.append(mc)
        if grad:
            grads.append(g.reshape(-1, D))
    return (np.concatenate(costs), np.concatenate(grads) if grad else None, np.concatenate(mcs))


def seed_blocks(batch):
    out, r = [], 0
    for s, t in zip(batch.seeds, batch.horizon):
        for _ in range(int(s)):
            out.append((r, r + int(t)))
            r += int(t)
    return out


def assert_cost_close(c, c_ref, what="cost"):
    c, c_ref = np.asarray(c, np.float64), np.asarray(c_ref, np.float64)
    err = np.abs(c - c_ref)
    tol = COST_RTOL * np.abs(c_ref) + ABS_TOL
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, f"{what}: {bad.size} seeds off, worst rel {np.max(err / (np.abs(c_ref) + 1e-30)):.3e} at {bad[:5]}"


def block_index(blocks):
    """Row indices of the listed (first, end) blocks, concatenated, and each
    block's start in that list (for np.add.reduceat; blocks are non-empty)."""
    lens = np.array([b - a for a, b in blocks], dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    firsts = np.array([a for a, _ in blocks], dtype=np.int64)
    rows = np.repeat(firsts - starts, lens) + np.arange(int(lens.sum()))
    return rows, starts


def block_sums(v, starts):
    """Per-block sums of the per-row values v."""
    return np.add.reduceat(v, starts)


def assert_grad_close(g, g_ref, batch, what="grad"):
    g, g_ref = np.asarray(g, np.float64), np.asarray(g_ref, np.float64)
    _, starts = block_index(seed_blocks(batch))
    e = np.sqrt(block_sums(((g - g_ref) ** 2).sum(1), starts))
    n = np.sqrt(block_sums((g_ref ** 2).sum(1), starts))
    bad = np.nonzero(e > GRAD_RTOL * n + ABS_TOL)[0]
    worst = float(np.max(e / (n + 1e-30))) if e.size else 0.0
    assert bad.size == 0, f"{what}: {bad.size} seed blocks off, worst rel {worst:.3e} at {bad[:5]}"


def assert_verdicts(mc, mc_ref):
    mc, mc_ref = np.asarray(mc, np.float64), np.asarray(mc_ref, np.float64)
    differ = (mc >= 0) != (mc_ref >= 0)
    near = np.abs(mc_ref) <= CONTACT_TOL
    assert not np.any(differ & ~near), f"collision verdicts differ at {np.nonzero(differ & ~near)[0][:5]}"
