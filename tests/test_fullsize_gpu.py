"""Element-wise parity at the full sizes of the workloads, through the
launches the solver makes: every candidate of every seed of one line-search
evaluation (cost, directional derivative, gradient block, collision
verdict) against the FP64 reference, and the line-search choice against the
reference's rule fed the reference's candidate values.

  cost+adjoint  32 seeds x 32 waypoints x 8 candidates, every layout and the
                autotuned one (the launch the benchmark times)
  IK            4096 goals x 32 seeds, T = 1, 4 candidates (and the choice)
  uneven        all 64 problems (seeds 4..64, T in {24,32,48}, 5..200 cuboids)
  large         two-arm tree, 500 cuboids, swept: 16 of the 128 seeds, all
                4 candidates
"""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_2310_17274_amd import workloads as wl
from tests import harness as H
from tests.test_parity_gpu import LAYOUTS, SWEPT, Case, _dev

pytestmark = pytest.mark.gpu


def _direction(case, scale, seed):
    rng = np.random.default_rng(seed)
    d = rng.normal(0, scale, case.batch.x0.shape).astype(np.float32).astype(np.float64)
    return d.reshape(-1, case.robot.dof)


def _oracle_candidates(case, x_rows, d_rows, alpha, seeds=None):
    """Reference cost, <g, d>, gradient rows and clearance of every
    candidate clip(x + alpha_k d): lists over k of [seeds] / [rows, D]
    (seeds: restrict to these seed indices of a one-problem batch)."""
    lo, hi = case.robot.q_lo, case.robot.q_hi
    out = []
    for a in alpha:
        xk = np.clip(x_rows + a * d_rows, lo, hi)
        if seeds is None:
            c, g, mc = H.oracle_cost_grad(case.ref, case.worlds, case.batch, xk)
        else:
            T = int(case.batch.horizon[0])
            q = np.concatenate([xk[s * T:(s + 1) * T] for s in seeds]).reshape(-1)
            c, g, mc = case.ref.cost_grad_batch(case.worlds.world(0), case.batch.q_start[0], case.batch.goal[0],
                                                T, q, nthreads=8)
            g = g.reshape(-1, case.robot.dof)
        out.append((c, g, mc))
    return out


def _seed_rows(batch):
    return H.seed_blocks(batch)


def _check_candidates(case, cost, gd, grad, mc, ref_k, d_rows, seeds=None):
    """Per seed block (vectorised over blocks): cost, verdict, gradient and
    <g, d> of every candidate against the reference's."""
    blocks = _seed_rows(case.batch)
    if seeds is not None:
        blocks = [blocks[s] for s in seeds]
    rows, starts = H.block_index(blocks)
    dsel = d_rows[rows]
    nd = np.sqrt(H.block_sums((dsel ** 2).sum(1), starts))
    sel = slice(None) if seeds is None else list(seeds)
    for k, (cr, gr, mcr) in enumerate(ref_k):
        H.assert_cost_close(cost[k][sel], cr, f"candidate {k} cost")
        H.assert_verdicts(mc[k][sel], mcr)
        gk = grad[k][rows].astype(np.float64)
        e = np.sqrt(H.block_sums(((gk - gr) ** 2).sum(1), starts))
        n = np.sqrt(H.block_sums((gr ** 2).sum(1), starts))
        bad = np.nonzero(e > H.GRAD_RTOL * n + H.ABS_TOL)[0]
        assert bad.size == 0, f"candidate {k}: gradient blocks {bad[:5]} off"
        gd_ref = H.block_sums((gr * dsel).sum(1), starts)
        bad = np.nonzero(np.abs(gd[k][sel] - gd_ref) > H.GRAD_RTOL * n * nd + H.ABS_TOL)[0]
        assert bad.size == 0, f"candidate {k}: <g,d> of seeds {bad[:5]} off"


def _gpu_candidates(case, dd, alpha):
    cost, gd, g, mc = case.ctx.mg_linesearch_eval(case.b, case.q_start, case.goal, case.x, dd, alpha)
    torch.cuda.synchronize()
    return cost.cpu().numpy(), gd.cpu().numpy(), g.cpu().numpy(), mc.cpu().numpy()


def _check_choice(case, alpha, mode, dd, d_rows, ref_k, seeds):
    """mg_linesearch's index against the reference rule on the reference's
    candidate values; a different index is accepted only when the deciding
    candidate's condition is met within rounding (cost margin 1e-4 |c0|,
    derivative margin 1e-3 |g||d|)."""
    c0, g0, _ = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x)
    xo, co, go, ch, mco = case.ctx.mg_linesearch(case.b, case.q_start, case.goal, case.x, c0, g0, dd, alpha, mode)
    torch.cuda.synchronize()
    ch = ch.cpu().numpy()
    blocks = _seed_rows(case.batch)
    x_rows = case.batch.x0.reshape(-1, case.robot.dof)
    if case.batch.n_problems == 1:
        # the listed seeds only (one problem: seed s owns rows s T .. s T + T - 1)
        T = int(case.batch.horizon[0])
        q = np.concatenate([x_rows[s * T:(s + 1) * T] for s in seeds]).reshape(-1)
        c_sub, g_sub, _ = case.ref.cost_grad_batch(case.worlds.world(0), case.batch.q_start[0],
                                                   case.batch.goal[0], T, q, nthreads=8)
        c0r = np.zeros(len(blocks))
        g0r = np.zeros_like(x_rows)
        for i, s in enumerate(seeds):
            c0r[s] = c_sub[i]
            g0r[s * T:(s + 1) * T] = g_sub.reshape(-1, case.robot.dof)[i * T:(i + 1) * T]
    else:
        c0r, g0r, _ = H.oracle_cost_grad(case.ref, case.worlds, case.batch, x_rows)
    rows, starts = H.block_index([blocks[s] for s in seeds])
    ds = d_rows[rows]
    dn = np.sqrt(H.block_sums((ds ** 2).sum(1), starts))
    g0d = H.block_sums((g0r[rows] * ds).sum(1), starts)
    K = len(alpha)
    ck = np.stack([np.asarray(ref_k[k][0], np.float64) for k in range(K)], 1)
    gdk = np.stack([H.block_sums((ref_k[k][1] * ds).sum(1), starts) for k in range(K)], 1)
    gn = np.stack([np.sqrt(H.block_sums((ref_k[k][1] ** 2).sum(1), starts)) for k in range(K)], 1)
    n_diff = 0
    for i, s in enumerate(seeds):
        want = ref.ls_select(alpha, float(c0r[s]), float(g0d[i]), ck[i], gdk[i], mode)
        got = int(ch[s])
        if got == want:
            continue
        n_diff += 1
        k = max(got, want)
        arm = abs(ck[i, k] - (c0r[s] + ref.ETA1 * alpha[k] * g0d[i])) <= 1e-4 * abs(c0r[s]) + 1e-6
        wolfe = abs(gdk[i, k] - ref.ETA_W * g0d[i]) <= 1e-3 * gn[i, k] * dn[i] + 1e-6
        assert arm or (mode > 0 and wolfe), f"seed {s}: gpu chose {got}, reference {want}"
    assert n_diff <= max(1, len(seeds) // 16)


def _adjoint_case(layout):
    robot, worlds, batch, meta = wl.cfg_cost_adjoint()
    return Case(robot, worlds, batch, layout=layout), meta["alpha"]


@pytest.mark.parametrize("layout", LAYOUTS + [pytest.param("auto", id="autotuned")])
def test_cost_adjoint_every_candidate(layout):
    """32 seeds x 32 waypoints x 8 candidates, one launch: all 256
    (seed, candidate) costs, gradient blocks, <g, d> and verdicts."""
    case, alpha = _adjoint_case(None if layout == "auto" else layout)
    d = _direction(case, 0.05, 0)
    dd = _dev(d)
    if layout == "auto":
        case.ctx.mg_autotune(case.b, case.q_start, case.goal, case.x, dd, alpha, launches=3)
    cost, gd, g, mc = _gpu_candidates(case, dd, alpha)
    x = case.batch.x0.reshape(-1, 7)
    ref_k = _oracle_candidates(case, x, d, alpha)
    _check_candidates(case, cost, gd, g, mc, ref_k, d)
    _check_choice(case, alpha, 1, dd, d, ref_k, list(range(32)))


def test_ik_every_seed_and_candidate():
    """4096 goals x 32 seeds at T = 1 (131,072 rows), 4 candidates, and
    the line-search choice of every seed."""
    robot, worlds, batch, meta = wl.cfg_ik()
    case = Case(robot, worlds, batch)
    c, g, mc = (t.cpu().numpy() for t in case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x))
    x = case.batch.x0.reshape(-1, 7)
    cr, gr, mcr = H.oracle_cost_grad(case.ref, case.worlds, case.batch, x)
    H.assert_cost_close(c, cr)
    H.assert_grad_close(g, gr, case.batch)
    H.assert_verdicts(mc, mcr)
    d = _direction(case, 0.1, 1)
    dd = _dev(d)
    cost, gd, gk, mck = _gpu_candidates(case, dd, meta["alpha"])
    ref_k = _oracle_candidates(case, x, d, meta["alpha"])
    _check_candidates(case, cost, gd, gk, mck, ref_k, d)
    _check_choice(case, meta["alpha"], 1, dd, d, ref_k, list(range(case.batch.x0.size // 7)))


def test_uneven_all_problems():
    """All 64 problems of the uneven batch in one evaluation, then every
    candidate of one line-search launch."""
    robot, worlds, batch, meta = wl.cfg_uneven()
    case = Case(robot, worlds, batch)
    c, g, mc = (t.cpu().numpy() for t in case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x))
    x = case.batch.x0.reshape(-1, 7)
    cr, gr, mcr = H.oracle_cost_grad(case.ref, case.worlds, case.batch, x, nthreads=16)
    H.assert_cost_close(c, cr)
    H.assert_grad_close(g, gr, case.batch)
    H.assert_verdicts(mc, mcr)
    d = _direction(case, 0.05, 2)
    cost, gd, gk, mck = _gpu_candidates(case, _dev(d), meta["alpha"])
    _check_candidates(case, cost, gd, gk, mck, _oracle_candidates(case, x, d, meta["alpha"]), d)


@pytest.mark.parametrize("layout", [pytest.param((0, 0), id="lane"), pytest.param((3, 0), id="groups2"), pytest.param((4, 0), id="groups4")])
def test_large_tree_swept_sixteen_seeds_every_candidate(layout):
    """Two-arm tree, 120 spheres, 500 cuboids, swept collision, 128 seeds x
    48 waypoints x 4 candidates in one launch: 16 seeds, every candidate,
    and the line-search choice of those seeds."""
    robot, worlds, batch, meta = wl.cfg_large()
    case = Case(robot, worlds, batch, params=SWEPT, layout=layout)
    alpha = meta["alpha"]
    d = _direction(case, 0.03, 3)
    dd = _dev(d)
    cost, gd, gk, mck = _gpu_candidates(case, dd, alpha)
    seeds = [int(s) for s in np.random.default_rng(4).choice(128, 16, replace=False)]
    x = case.batch.x0.reshape(-1, robot.dof)
    ref_k = _oracle_candidates(case, x, d, alpha, seeds=seeds)
    _check_candidates(case, cost, gd, gk, mck, ref_k, d, seeds=seeds)
    _check_choice(case, alpha, 0, dd, d, ref_k, seeds)


@pytest.mark.parametrize("params", [pytest.param(None, id="plain"), pytest.param(SWEPT, id="swept"),
                                    pytest.param(dict(speed=1), id="speed")])
@pytest.mark.parametrize("kind", ["adjoint_small", "tree"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_directional_derivative_is_gradient_dot_direction(layout, kind, params):
    """The line-search launch forms <g_k, d> by its own route (link
    velocities under d against the link wrenches); it must equal the inner
    product of the same launch's gradient with d, to fp32 rounding of the
    terms (relative to sum |g_i d_i|)."""
    from tests.test_parity_gpu import make_case
    case = make_case(kind, layout=layout, params=params)
    d = _direction(case, 0.05, 5)
    alpha = wl.ALPHA_4
    cost, gd, g, mc = _gpu_candidates(case, _dev(d), alpha)
    for k in range(len(alpha)):
        for i, (a, b) in enumerate(H.seed_blocks(case.batch)):
            prod = g[k][a:b].astype(np.float64) * d[a:b]
            assert abs(gd[k][i] - prod.sum()) <= 2e-5 * np.abs(prod).sum() + 1e-3, (k, i, gd[k][i], prod.sum())
