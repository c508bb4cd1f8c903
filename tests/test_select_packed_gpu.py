"""Line-search choice (Alg.1) and the fused L-BFGS step (Alg.6) with several
seeds per wavefront: row blocks of at most 32 floats (inverse kinematics at
T = 1, short horizons) take 8, 16 or 32 lanes per seed.

  ik     5 goals x 9 seeds at T = 1 (45 seeds: eight per wavefront, the
         last wavefront ragged), one world of 40 oriented cuboids
  short  horizons 1..4 (blocks of 7..28 floats, per-seed table), odd seed
         counts, two worlds
"""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_2310_17274_amd import workloads as wl
from tests import harness as H
from tests.test_fullsize_gpu import _direction, _oracle_candidates
from tests.test_parity_gpu import Case, _dev

pytestmark = pytest.mark.gpu


def _short_case(kind):
    robot = wl.make_arm(seed=0, n_spheres=52)
    if kind == "ik":
        worlds = wl.make_worlds(3, [40], oriented=True)
        batch = wl.make_batch(robot, 103, [9] * 5, [1] * 5, [0] * 5)
    else:
        worlds = wl.make_worlds(5, [12, 30])
        batch = wl.make_batch(robot, 41, [3, 5, 1, 7], [1, 2, 3, 4], [0, 1, 1, 0])
    return Case(robot, worlds, batch)


def _alpha(K):
    return list(wl.ALPHA_4) if K == 4 else [float(a) for a in np.linspace(0.01, 1.0, K)]


@pytest.mark.parametrize("K,mode", [(4, 0), (4, 1), (8, 2), (16, 1)])
@pytest.mark.parametrize("kind", ["ik", "short"])
def test_packed_linesearch_parity(kind, K, mode):
    """Every seed's choice against the reference rule fed the reference's
    candidate values (a different index only where the deciding condition
    holds within rounding), and the chosen iterate, cost, gradient and
    clearance."""
    case = _short_case(kind)
    alpha = _alpha(K)
    D = case.robot.dof
    x_rows = case.batch.x0.reshape(-1, D)
    d = _direction(case, 0.1, 11)
    dd = _dev(d)
    c0, g0, _ = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x)
    xo, co, go, ch, mco = case.ctx.mg_linesearch(case.b, case.q_start, case.goal, case.x, c0, g0, dd, alpha, mode)
    torch.cuda.synchronize()
    xo, co, go, ch, mco = (t.cpu().numpy() for t in (xo, co, go, ch, mco))
    c0r, g0r, _ = H.oracle_cost_grad(case.ref, case.worlds, case.batch, x_rows)
    ref_k = _oracle_candidates(case, x_rows, d, alpha)
    blocks = H.seed_blocks(case.batch)
    n_diff = 0
    for s, (a, b) in enumerate(blocks):
        g0d = float(np.sum(g0r[a:b] * d[a:b]))
        ck = [float(ref_k[k][0][s]) for k in range(K)]
        gk = [ref_k[k][1][a:b] for k in range(K)]
        gdk = [float(np.sum(g * d[a:b])) for g in gk]
        want = ref.ls_select(alpha, float(c0r[s]), g0d, ck, gdk, mode)
        got = int(ch[s])
        if got != want:
            n_diff += 1
            k = max(got, want)
            arm = abs(ck[k] - (c0r[s] + ref.ETA1 * alpha[k] * g0d)) <= 1e-4 * abs(c0r[s]) + 1e-6
            wolfe = abs(gdk[k] - ref.ETA_W * g0d) <= 1e-3 * np.linalg.norm(gk[k]) * np.linalg.norm(d[a:b]) + 1e-6
            assert arm or (mode > 0 and wolfe), f"seed {s}: gpu chose {got}, reference {want}"
            continue
        xk = np.clip(x_rows[a:b] + alpha[got] * d[a:b], case.robot.q_lo, case.robot.q_hi)
        np.testing.assert_allclose(xo[a:b], xk, atol=2e-6, err_msg=f"seed {s}")
        H.assert_cost_close([co[s]], [ck[got]], f"seed {s} cost")
        assert np.linalg.norm(go[a:b] - gk[got]) <= H.GRAD_RTOL * np.linalg.norm(gk[got]) + H.ABS_TOL, s
        H.assert_verdicts([mco[s]], [ref_k[got][2][s]])
    assert n_diff <= max(1, len(blocks) // 16)


@pytest.mark.parametrize("m", [4, 8])
@pytest.mark.parametrize("kind", ["ik", "short"])
def test_packed_fused_step_equals_separate_launches(kind, m):
    """The solver's iteration (choice and the next L-BFGS direction in one
    launch, several seeds per wavefront) against the same iterations as
    separate line-search and L-BFGS launches (one wavefront per seed for the
    direction): identical bits for the best cost and trajectory of every
    seed (the group sums add the same partial sums; the lanes beyond a
    block add zeros)."""
    case = _short_case(kind)
    alpha, iters = list(wl.ALPHA_4), 12
    x0 = case.x.clone()
    xs, bc, _, _ = case.ctx.mg_solve(case.b, case.q_start, case.goal, x0.clone(), iters, m, alpha, mode=1,
                                     use_graph=False)
    torch.cuda.synchronize()
    xs, bc = xs.cpu().numpy(), bc.cpu().numpy()

    x = x0.clone()
    c, g, _ = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, x)
    d = case.ctx.mg_lbfgs_step(case.b, m, True, x, g)
    best_c, best_x = c.cpu().numpy().copy(), x.cpu().numpy().copy()
    blocks = H.seed_blocks(case.batch)
    for _ in range(iters):
        x, c, g, _, _ = case.ctx.mg_linesearch(case.b, case.q_start, case.goal, x, c, g, d, alpha, 1)
        d = case.ctx.mg_lbfgs_step(case.b, m, False, x, g)
        torch.cuda.synchronize()
        cn, xn = c.cpu().numpy(), x.cpu().numpy()
        for s, (a, b) in enumerate(blocks):
            if cn[s] < best_c[s]:
                best_c[s] = cn[s]
                best_x[a:b] = xn[a:b]
    assert np.array_equal(bc, best_c)
    assert np.array_equal(xs, best_x)
