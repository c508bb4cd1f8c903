"""Parity of the HIP path (through the C ABI) with the FP64 reference.

Every case feeds identical seeded fp32 inputs to both and compares per seed
(tolerances in harness.py).  Sizes span several workgroups and a ragged tail;
the full-size cost+adjoint workload is checked on sampled seeds.
"""
import math

import numpy as np
import pytest
import torch

from oracle import ref
from paper_2310_17274_amd import workloads as wl
from tests import harness as H

pytestmark = pytest.mark.gpu

# evaluation layouts (layout, slices): lane per link (automatic slices),
# wave per link in one workgroup per 64 evaluations, split over four
# workgroups (the last to finish adds the slices), two waves per link, and
# two or four slot groups per wave (32 or 16 evaluations per workgroup)
LAYOUTS = [pytest.param((0, 0), id="lane"), pytest.param((1, 1), id="wave"),
           pytest.param((1, 4), id="wave4"), pytest.param((2, 0), id="wave2"),
           pytest.param((3, 0), id="groups2"), pytest.param((4, 0), id="groups4")]


def _dev(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float32, device="cuda").contiguous()


class Case:
    """Inputs of one workload on both sides."""

    def __init__(self, robot, worlds, batch, params=None, K_max=16, m_max=8, layout=None, self_pairs=None):
        from paper_2310_17274_amd.binding import Context, default_params
        self.robot, self.worlds, self.batch = H.f32_inputs(robot, worlds, batch)
        params = params or {}
        self.ctx = Context(self.robot, default_params(**params))
        self.ctx.mg_set_worlds(self.worlds)
        if self_pairs is not None:
            self.ctx.mg_set_self_collision(self_pairs)
        b = self.batch
        self.b = self.ctx.batch(b.seeds, b.horizon, b.world, K_max=K_max, m_max=m_max)
        if layout is not None:
            if layout[0] == 2 and self.robot.n_links > 8:
                pytest.skip("two waves per link need at most 8 links")
            if layout[0] >= 3 and self_pairs is not None:
                pytest.skip("slot groups per wave take no self-collision")
            if layout[0] == 4 and np.bincount(self.robot.sphere_link).max() <= 4:
                pytest.skip("four slot groups per wave need more than 4 spheres on some link")
            self.b.mg_batch_set_layout(*layout)
        D = self.robot.dof
        self.q_start = _dev(b.q_start)
        self.goal = _dev(b.goal.reshape(b.n_problems, -1))
        self.x = _dev(b.x0.reshape(-1, D))
        self.ref = ref.Ref(self.robot, **params) if self_pairs is None else \
            ref.Ref(self.robot, self_pairs=self_pairs, **params)


def make_case(kind, **kw):
    if kind == "plain":
        return Case(*wl.cfg_plain()[:3], **kw)
    if kind == "adjoint":
        robot, worlds, batch, _ = wl.cfg_cost_adjoint()
        return Case(robot, worlds, batch, **kw)
    if kind == "adjoint_small":
        robot = wl.make_arm(seed=0, n_spheres=52)
        worlds = wl.make_worlds(2, [40])
        batch = wl.make_batch(robot, 102, [5], [32], [0])
        return Case(robot, worlds, batch, **kw)
    if kind == "ik":
        robot, worlds, batch, _ = wl.cfg_ik(n_goals=24, n_seeds=9)
        return Case(robot, worlds, batch, **kw)
    if kind == "uneven":
        rng = np.random.default_rng(4)
        robot = wl.make_arm(seed=0, n_spheres=52)
        P = 5
        seeds = rng.integers(1, 7, P)
        horizon = np.array([2, 24, 33, 48, 64])
        counts = np.array([0, 5, 37, 200, 1])
        worlds = wl.make_worlds(9, counts)
        batch = wl.make_batch(robot, 7, seeds, horizon, np.arange(P))
        return Case(robot, worlds, batch, **kw)
    if kind == "tree":
        robot = wl.make_two_arm(seed=0, n_spheres=60)
        worlds = wl.make_worlds(6, [80])
        batch = wl.make_batch(robot, 61, [3], [20], [0])
        return Case(robot, worlds, batch, **kw)
    raise ValueError(kind)


def gpu_cost_grad(case):
    c, g, mc = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x)
    torch.cuda.synchronize()
    return c.cpu().numpy(), g.cpu().numpy(), mc.cpu().numpy()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("kind", ["plain", "adjoint_small", "ik", "uneven", "tree"])
def test_cost_grad_parity(kind, layout):
    case = make_case(kind, layout=layout)
    c, g, mc = gpu_cost_grad(case)
    cr, gr, mcr = H.oracle_cost_grad(case.ref, case.worlds, case.batch, case.batch.x0.reshape(-1, case.robot.dof))
    H.assert_cost_close(c, cr)
    H.assert_grad_close(g, gr, case.batch)
    H.assert_verdicts(mc, mcr)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_cost_grad_parity_with_collisions_and_limits(layout):
    """Seeds pushed into obstacles and beyond joint limits so that every
    branch of the collision and limit profiles is exercised."""
    robot = wl.make_arm(seed=0, n_spheres=52)
    worlds = wl.make_worlds(11, [60])
    batch = wl.make_batch(robot, 13, [6], [16], [0], noise=0.4)
    batch.x0 = np.clip(batch.x0 * 1.3, -3.2, 3.2)
    case = Case(robot, worlds, batch, layout=layout)
    c, g, mc = gpu_cost_grad(case)
    cr, gr, mcr = H.oracle_cost_grad(case.ref, case.worlds, case.batch, case.batch.x0.reshape(-1, 7))
    assert np.any(mcr < 0), "the case must contain collisions"
    H.assert_cost_close(c, cr)
    H.assert_grad_close(g, gr, case.batch)
    H.assert_verdicts(mc, mcr)


SWEPT = dict(swept=1, sweep_steps=4)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("kind", ["adjoint_small", "uneven", "tree"])
def test_swept_cost_grad_parity(kind, layout):
    """Continuous collision: trace samples toward both neighbouring waypoints
    (the start before waypoint 1), horizons 2..64, worlds of 0..200 cuboids,
    the two-arm tree."""
    case = make_case(kind, params=SWEPT, layout=layout)
    c, g, mc = gpu_cost_grad(case)
    cr, gr, mcr = H.oracle_cost_grad(case.ref, case.worlds, case.batch, case.batch.x0.reshape(-1, case.robot.dof))
    H.assert_cost_close(c, cr)
    H.assert_grad_close(g, gr, case.batch)
    H.assert_verdicts(mc, mcr)
    # the trace adds cost somewhere in these workloads
    cd, _, _ = H.oracle_cost_grad(ref.Ref(case.robot), case.worlds, case.batch,
                                  case.batch.x0.reshape(-1, case.robot.dof), grad=False)
    assert np.all(cr >= cd) and np.any(cr > cd)


@pytest.mark.parametrize("layout", [pytest.param((1, 8), id="wave8"), pytest.param((1, 16), id="wave16")])
@pytest.mark.parametrize("kind,params", [("plain", None), ("uneven", None), ("tree", None),
                                         ("adjoint_small", SWEPT), ("tree", SWEPT)],
                         ids=["plain", "uneven", "tree", "adjoint_small-swept", "tree-swept"])
def test_cost_grad_parity_many_slices(kind, params, layout):
    """The wave-per-link layout with the world split over 8 and 16
    workgroups per chunk (the last to finish adds the slices in order)."""
    case = make_case(kind, layout=layout, params=params)
    c, g, mc = gpu_cost_grad(case)
    cr, gr, mcr = H.oracle_cost_grad(case.ref, case.worlds, case.batch, case.batch.x0.reshape(-1, case.robot.dof))
    H.assert_cost_close(c, cr)
    H.assert_grad_close(g, gr, case.batch)
    H.assert_verdicts(mc, mcr)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_swept_tunnelling_example_on_gpu(layout):
    """The thin-wall example worked by hand in the reference's pins: both
    waypoints clear of the wall, the segment through it; swept cost 0.136
    against 0.001 discrete (unit collision weight, other terms off)."""
    from tests.test_oracle_pins import COLLISION_ONLY, one_link_robot
    robot = one_link_robot()
    phi = math.asin(0.09)
    worlds = wl.Worlds(offsets=np.array([0, 1], np.int32),
                       pose=np.array([[math.cos(phi), 0.0, 0.0, 1.0, 0.0, 0.0, 0.0]]),
                       dims=np.array([[1.0, 0.04, 1.0]]))
    batch = wl.Batch(seeds=np.array([1], np.int32), horizon=np.array([2], np.int32),
                     world=np.array([0], np.int32), q_start=np.array([[-phi]]),
                     goal=np.array([[[0, 0, 0, 1, 0, 0, 0]]], dtype=float), x0=np.array([-phi, phi]))
    case = Case(robot, worlds, batch, params=dict(COLLISION_ONLY, **SWEPT), layout=layout)
    c, g, mc = gpu_cost_grad(case)
    assert c[0] == pytest.approx(0.136, rel=1e-4)
    assert mc[0] == pytest.approx(0.02, rel=1e-4)
    cd = Case(robot, worlds, batch, params=COLLISION_ONLY)
    assert gpu_cost_grad(cd)[0][0] == pytest.approx(0.001, rel=1e-4)


@pytest.mark.parametrize("layout", [pytest.param((0, 0), id="lane"), pytest.param((3, 0), id="groups2"), pytest.param((4, 0), id="groups4")])
def test_large_tree_swept_linesearch_sampled(layout):
    """Two-arm tree (14 joints, 120 spheres) against 500 cuboids with swept
    collision, 128 seeds x 48 waypoints x 4 candidates in one line-search
    launch; sampled seeds checked one by one at the chosen candidate."""
    robot, worlds, batch, meta = wl.cfg_large()
    case = Case(robot, worlds, batch, params=SWEPT, layout=layout)
    D, S, T = robot.dof, 128, 48
    rng = np.random.default_rng(1)
    d = rng.normal(0, 0.03, case.batch.x0.shape).astype(np.float32).astype(np.float64)
    dd = _dev(d.reshape(-1, D))
    c0, g0, _ = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x)
    alpha = meta["alpha"]
    xo, co, go, ch, mco = case.ctx.mg_linesearch(case.b, case.q_start, case.goal, case.x, c0, g0, dd, alpha, mode=0)
    torch.cuda.synchronize()
    ch, co, go = ch.cpu().numpy(), co.cpu().numpy(), go.cpu().numpy().reshape(S, T, D)
    x = case.batch.x0.reshape(S, T, D)
    dv = d.reshape(S, T, D)
    boxes = case.worlds.world(0)
    for s in rng.choice(S, 3, replace=False):
        k = int(ch[s])
        xk = np.clip(x[s] + alpha[k] * dv[s], case.robot.q_lo, case.robot.q_hi)
        cr, gr, _, _ = case.ref.traj_cost(boxes, case.batch.q_start[0], case.batch.goal[0], xk)
        H.assert_cost_close([co[s]], [cr])
        assert np.linalg.norm(go[s] - gr) <= H.GRAD_RTOL * np.linalg.norm(gr) + H.ABS_TOL


def _particle_round_reference(case, mean, var, eps_round, costs_gpu, boxes, p=0):
    """Reference checks of one particle round of problem p from the same
    inputs: every particle's cost, and the update fed the GPU's costs.
    mean, var [S, T, D]; eps_round [N, S, T, D]; costs_gpu [S, N]."""
    S, T, D = mean.shape
    N = eps_round.shape[0]
    out_m, out_v = np.empty_like(mean), np.empty_like(var)
    lo, hi = case.robot.q_lo, case.robot.q_hi
    for s in range(S):
        th = np.clip(mean[s] + np.sqrt(var[s]) * eps_round[:, s], lo, hi)
        cr = np.array([case.ref.traj_cost(boxes, case.batch.q_start[p], case.batch.goal[p], th[i], grad=False)[0]
                       for i in range(N)])
        H.assert_cost_close(costs_gpu[s], cr, f"particle costs of seed {s}")
        m, v, _ = ref.particle_update(costs_gpu[s], th.reshape(N, -1), mean[s].reshape(-1), var[s].reshape(-1))
        out_m[s], out_v[s] = m.reshape(T, D), v.reshape(T, D)
    return out_m, out_v


PARTICLE_LAYOUTS = [pytest.param((0, 0), id="lane"), pytest.param((1, 1), id="wave"),
                    pytest.param((2, 0), id="wave2"), pytest.param((3, 0), id="groups2"), pytest.param((4, 0), id="groups4")]


@pytest.mark.parametrize("layout", PARTICLE_LAYOUTS)
def test_particle_stage_parity(layout):
    """Two rounds of 64 particles per seed (Alg.5): each round's particle
    costs against the reference's, and the mean / variance update against
    the reference update fed the GPU's costs (fp32 sums of 64 terms)."""
    case = make_case("adjoint_small", layout=layout)
    S, T, D, N = 5, 32, 7, 64
    rng = np.random.default_rng(12)
    eps = rng.normal(0, 1, (2, N, S * T, D)).astype(np.float32).astype(np.float64)
    case.b.mg_batch_reserve_particles(N)
    mean = case.x.clone()
    var = torch.full_like(mean, 0.05 ** 2)
    boxes = case.worlds.world(0)
    for it in range(2):
        m_in = mean.double().cpu().numpy().reshape(S, T, D)
        v_in = var.double().cpu().numpy().reshape(S, T, D)
        _, _, costs = case.ctx.mg_particles(case.b, case.q_start, case.goal, mean, var,
                                            _dev(eps[it:it + 1]), costs=True)
        torch.cuda.synchronize()
        m_ref, v_ref = _particle_round_reference(case, m_in, v_in, eps[it].reshape(N, S, T, D),
                                                 costs.cpu().numpy()[0], boxes)
        np.testing.assert_allclose(mean.cpu().numpy().reshape(S, T, D), m_ref, rtol=0, atol=5e-6)
        np.testing.assert_allclose(var.cpu().numpy().reshape(S, T, D), v_ref, rtol=2e-4, atol=1e-9)
    # one call of two rounds is the same computation
    mean2 = case.x.clone()
    var2 = torch.full_like(mean2, 0.05 ** 2)
    case.ctx.mg_particles(case.b, case.q_start, case.goal, mean2, var2, _dev(eps))
    torch.cuda.synchronize()
    assert torch.equal(mean2, mean) and torch.equal(var2, var)


def test_particle_stage_end_to_end_against_reference():
    """The whole two-round stage against the reference's own stage: the means
    agree to a small fraction of the distance they moved."""
    case = make_case("plain")
    S, T, D, N = 4, 32, 7, 128
    rng = np.random.default_rng(13)
    eps = rng.normal(0, 1, (2, N, S * T, D)).astype(np.float32).astype(np.float64)
    case.b.mg_batch_reserve_particles(N)
    mean = case.x.clone()
    var = torch.full_like(mean, 0.05 ** 2)
    case.ctx.mg_particles(case.b, case.q_start, case.goal, mean, var, _dev(eps))
    torch.cuda.synchronize()
    x0 = case.batch.x0.reshape(S, T, D)
    m_ref, v_ref, _ = case.ref.particles(case.worlds.world(0), case.batch.q_start[0], case.batch.goal[0], T,
                                         x0, np.full_like(x0, np.float32(0.05 ** 2)),
                                         eps.reshape(2, N, S, T, D))
    mg = mean.cpu().numpy().reshape(S, T, D)
    for s in range(S):
        moved = np.abs(m_ref[s] - x0[s]).max()
        assert moved > 1e-3
        assert np.abs(mg[s] - m_ref[s]).max() <= 1e-2 * moved + 1e-5, s


@pytest.mark.parametrize("layout", [pytest.param((0, 0), id="lane"), pytest.param((3, 0), id="groups2"), pytest.param((4, 0), id="groups4")])
def test_large_tree_swept_particle_stage_sampled(layout):
    """Particle stage at full size: two-arm tree, 128 seeds x 48 waypoints,
    256 particles, 2 rounds, 500 cuboids, swept collision.  Sampled particle
    costs against the reference, the update of sampled seeds against the
    reference update fed the GPU's costs."""
    robot, worlds, batch, meta = wl.cfg_large()
    case = Case(robot, worlds, batch, params=SWEPT, layout=layout)
    S, T, D, N = 128, 48, robot.dof, 256
    rng = np.random.default_rng(14)
    eps = rng.normal(0, 1, (1, N, S * T, D)).astype(np.float32)
    case.b.mg_batch_reserve_particles(N)
    mean = case.x.clone()
    var = torch.full_like(mean, 0.05 ** 2)
    _, _, costs = case.ctx.mg_particles(case.b, case.q_start, case.goal, mean, var,
                                        torch.from_numpy(eps).cuda(), costs=True)
    torch.cuda.synchronize()
    costs = costs.cpu().numpy()[0]
    x0 = case.batch.x0.reshape(S, T, D)
    e = eps[0].astype(np.float64).reshape(N, S, T, D)
    sd = np.sqrt(np.float64(np.float32(0.05 ** 2)))
    boxes = case.worlds.world(0)
    for s, i in zip(rng.choice(S, 4, replace=False), rng.choice(N, 4, replace=False)):
        th = np.clip(x0[s] + sd * e[i, s], robot.q_lo, robot.q_hi)
        cr = case.ref.traj_cost(boxes, case.batch.q_start[0], case.batch.goal[0], th, grad=False)[0]
        H.assert_cost_close([costs[s, i]], [cr], f"particle {i} of seed {s}")
    mg = mean.cpu().numpy().reshape(S, T, D)
    vg = var.cpu().numpy().reshape(S, T, D)
    for s in rng.choice(S, 2, replace=False):
        th = np.clip(x0[s] + sd * e[:, s], robot.q_lo, robot.q_hi)
        m, v, _ = ref.particle_update(costs[s], th.reshape(N, -1), x0[s].reshape(-1),
                                      np.full(T * D, sd * sd))
        np.testing.assert_allclose(mg[s].reshape(-1), m, rtol=0, atol=5e-6)
        np.testing.assert_allclose(vg[s].reshape(-1), v, rtol=2e-4, atol=1e-9)


def test_autotuned_layout_keeps_parity():
    """The autotuner picks one of the offered cuboid-slice layouts; the
    evaluation stays within parity under the chosen layout, and the solve
    under graphs still equals the solve with direct launches."""
    case = make_case("uneven")
    c0, g0, _ = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x)
    d = case.ctx.mg_lbfgs_step(case.b, 4, True, case.x, g0)
    h = case.ctx.mg_autotune(case.b, case.q_start, case.goal, case.x, d, wl.ALPHA_4, launches=3)
    # lane-per-link slices, minus wave-per-link workgroups, two waves per
    # link (-8), two or four slot groups per wave (-16, -32)
    assert h in (1, 2, 4, -1, -2, -4, -8, -16, -32)
    c, g, mc = gpu_cost_grad(case)
    cr, gr, mcr = H.oracle_cost_grad(case.ref, case.worlds, case.batch, case.batch.x0.reshape(-1, 7))
    H.assert_cost_close(c, cr)
    H.assert_grad_close(g, gr, case.batch)
    outs = []
    for use_graph in (True, False):
        x = case.x.clone()
        x, bc, bs, ok = case.ctx.mg_solve(case.b, case.q_start, case.goal, x, 30, 4, wl.ALPHA_4,
                                          graph_inner=10, use_graph=use_graph)
        torch.cuda.synchronize()
        outs.append((x.cpu().numpy(), bc.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def _self_case(layout, seed=13, S=6, T=16):
    robot = wl.make_arm(seed=0, n_spheres=52)
    worlds = wl.make_worlds(11, [40])
    batch = wl.make_batch(robot, seed, [S], [T], [0], noise=0.6)
    return Case(robot, worlds, batch, layout=layout, self_pairs=wl.self_pairs(robot))


@pytest.mark.parametrize("layout", [pytest.param(None, id="auto"), pytest.param((1, 4), id="wave4"),
                                    pytest.param((2, 0), id="wave2")])
def test_self_collision_cost_grad_parity(layout):
    """Self-collision (Eq.(9)) over non-adjacent links' sphere pairs with the
    world term on; noisy trajectories so that arms fold onto themselves."""
    case = _self_case(layout)
    c, g, mc = gpu_cost_grad(case)
    cr, gr, mcr = H.oracle_cost_grad(case.ref, case.worlds, case.batch, case.batch.x0.reshape(-1, 7))
    H.assert_cost_close(c, cr)
    H.assert_grad_close(g, gr, case.batch)
    H.assert_verdicts(mc, mcr)
    selfc = [case.ref.traj_cost(case.worlds.world(0), case.batch.q_start[0], case.batch.goal[0], q,
                                grad=False)[3][4] for q in case.batch.x0.reshape(6, 16, 7)]
    assert np.count_nonzero(selfc) >= 2, "the case must contain self-collisions"


def test_self_collision_linesearch_parity():
    case = _self_case(None, seed=17, S=4, T=32)
    _linesearch_parity(case, wl.ALPHA_4, 1)


def test_self_collision_restrictions():
    """Self-collision lives in the wave-per-link layout: the particle stage
    takes it only with the particle count its records were built for."""
    from paper_2310_17274_amd._lib import MgError
    case = _self_case(None, S=2, T=8)
    case.b.mg_batch_reserve_particles(8)
    eps = torch.zeros((1, 4, 16, 7), device="cuda")
    var = torch.full_like(case.x, 1e-3)
    with pytest.raises(MgError):
        case.ctx.mg_particles(case.b, case.q_start, case.goal, case.x.clone(), var, eps)


@pytest.mark.parametrize("layout", [pytest.param((1, 1), id="wave"), pytest.param((2, 0), id="wave2")])
def test_self_collision_particle_stage_parity(layout):
    """One particle round with self-collision on: every particle's cost
    against the reference's, and the update fed the GPU's costs."""
    case = _self_case(layout, seed=19, S=3, T=16)
    S, T, D, N = 3, 16, 7, 24
    rng = np.random.default_rng(20)
    eps = rng.normal(0, 1, (1, N, S * T, D)).astype(np.float32).astype(np.float64)
    case.b.mg_batch_reserve_particles(N)
    mean = case.x.clone()
    var = torch.full_like(mean, 0.1 ** 2)
    m_in = mean.double().cpu().numpy().reshape(S, T, D)
    v_in = var.double().cpu().numpy().reshape(S, T, D)
    _, _, costs = case.ctx.mg_particles(case.b, case.q_start, case.goal, mean, var, _dev(eps), costs=True)
    torch.cuda.synchronize()
    m_ref, v_ref = _particle_round_reference(case, m_in, v_in, eps[0].reshape(N, S, T, D),
                                             costs.cpu().numpy()[0], case.worlds.world(0))
    np.testing.assert_allclose(mean.cpu().numpy().reshape(S, T, D), m_ref, rtol=0, atol=5e-6)
    np.testing.assert_allclose(var.cpu().numpy().reshape(S, T, D), v_ref, rtol=2e-4, atol=1e-9)


@pytest.mark.parametrize("layout", [pytest.param((1, 1), id="wave"), pytest.param((2, 0), id="wave2")])
def test_self_collision_with_swept_parity(layout):
    """Self-collision and swept collision together (both wave-per-link)."""
    robot = wl.make_arm(seed=0, n_spheres=52)
    worlds = wl.make_worlds(8, [40])
    batch = wl.make_batch(robot, 81, [3], [16], [0])
    case = Case(robot, worlds, batch, params=SWEPT, layout=layout, self_pairs=wl.self_pairs(robot))
    c, g, mc = gpu_cost_grad(case)
    cr, gr, mcr = H.oracle_cost_grad(case.ref, case.worlds, case.batch, case.batch.x0.reshape(-1, robot.dof))
    H.assert_cost_close(c, cr)
    H.assert_grad_close(g, gr, case.batch)
    H.assert_verdicts(mc, mcr)


def test_cost_only_matches_cost_grad():
    case = make_case("adjoint_small")
    c1, _, mc1 = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x, grad=False)
    c2, _, mc2 = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x, grad=True)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(mc1, mc2)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_cost_grad_is_deterministic(layout):
    case = make_case("uneven", layout=layout)
    a = gpu_cost_grad(case)
    b = gpu_cost_grad(case)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("params", [pytest.param(None, id="default"),
                                    pytest.param(dict(speed=1), id="speed"),
                                    pytest.param(dict(speed=1, swept=1, sweep_steps=4), id="speed_swept")])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_full_size_cost_adjoint_sampled(layout, params):
    """Full 32 seeds x 32 waypoints x 8 candidates workload through the
    line-search launch; candidates of sampled seeds checked one by one.
    Also with the speed metric, and with it and swept collision (both
    wave per link: a lane-per-link request falls back to it)."""
    case = make_case("adjoint", layout=layout, params=params)
    D = 7
    rng = np.random.default_rng(0)
    d = rng.normal(0, 0.05, case.batch.x0.shape).astype(np.float32).astype(np.float64)
    dd = _dev(d.reshape(-1, D))
    c0, g0, _ = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x)
    alpha = wl.ALPHA_8
    xo, co, go, ch, mco = case.ctx.mg_linesearch(case.b, case.q_start, case.goal, case.x, c0, g0, dd, alpha, mode=0)
    torch.cuda.synchronize()
    ch = ch.cpu().numpy()
    xo, co, go = xo.cpu().numpy(), co.cpu().numpy(), go.cpu().numpy()
    x = case.batch.x0.reshape(32, 32, D)
    dv = d.reshape(32, 32, D)
    pose, dims = case.worlds.world(0)
    for s in rng.choice(32, 6, replace=False):
        k = int(ch[s])
        xk = np.clip(x[s] + alpha[k] * dv[s], case.robot.q_lo, case.robot.q_hi)
        cr, gr, _, _ = case.ref.traj_cost((pose, dims), case.batch.q_start[0], case.batch.goal[0], xk)
        H.assert_cost_close([co[s]], [cr])
        gs = go.reshape(32, 32, D)[s]
        assert np.linalg.norm(gs - gr) <= H.GRAD_RTOL * np.linalg.norm(gr) + H.ABS_TOL
        np.testing.assert_allclose(xo.reshape(32, 32, D)[s], xk, atol=2e-6)


def test_lbfgs_step_parity():
    case = make_case("plain")
    D, T, S = 7, 32, 4
    n = T * D
    rng = np.random.default_rng(3)
    m = 4
    states = [ref.new_lbfgs_state(n, m) for _ in range(S)]
    x = case.batch.x0.reshape(S, n).copy()
    for it in range(7):
        g = rng.normal(0, 1, (S, n)).astype(np.float32).astype(np.float64)
        if it > 0:
            g = g_prev + 0.5 * (x - x_prev) + 0.1 * g   # mostly positive curvature pairs
            g = g.astype(np.float32).astype(np.float64)
        d_gpu = case.ctx.mg_lbfgs_step(case.b, m, it == 0, _dev(x.reshape(-1, D)), _dev(g.reshape(-1, D)))
        torch.cuda.synchronize()
        d_gpu = d_gpu.cpu().numpy().reshape(S, n)
        for s in range(S):
            d_ref = ref.lbfgs_step(n, m, it == 0, states[s], x[s], g[s])
            assert np.linalg.norm(d_gpu[s] - d_ref) <= 1e-3 * np.linalg.norm(d_ref) + 1e-7, (it, s)
        x_prev, g_prev = x.copy(), g.copy()
        x = (x + 0.05 * d_gpu).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_linesearch_parity(mode, layout):
    _linesearch_parity(make_case("plain", layout=layout), wl.ALPHA_4, mode)


@pytest.mark.parametrize("K", [3, 16])
def test_linesearch_candidate_counts_wave_per_link(K):
    """Candidate counts that do not divide the 64 lanes of a workgroup
    (rows straddle workgroups) and the largest count."""
    _linesearch_parity(make_case("plain", layout=(1, 2)), [float(a) for a in np.linspace(0.01, 1.0, K)], 1)


def _linesearch_parity(case, alpha, mode):
    D = 7
    c0, g0, _ = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x)
    d = case.ctx.mg_lbfgs_step(case.b, 4, True, case.x, g0)
    xo, co, go, ch, mco = case.ctx.mg_linesearch(case.b, case.q_start, case.goal, case.x, c0, g0, d, alpha, mode)
    torch.cuda.synchronize()
    c0n, g0n, dn = c0.cpu().numpy(), g0.cpu().numpy(), d.cpu().numpy()
    ch, co, xo, go = ch.cpu().numpy(), co.cpu().numpy(), xo.cpu().numpy(), go.cpu().numpy()
    pose, dims = case.worlds.world(0)
    T = 32
    for s in range(4):
        r = slice(s * T, (s + 1) * T)
        i, xr, cr, gr, mcr = case.ref.linesearch((pose, dims), case.batch.q_start[0], case.batch.goal[0],
                                                 case.batch.x0.reshape(-1, D)[r], float(c0n[s]),
                                                 g0n[r], dn[r], alpha, mode)
        if int(ch[s]) != i:
            # a different choice is only allowed when the rule is decided
            # within rounding: the GPU's pick must also satisfy it
            pytest.fail(f"seed {s}: gpu chose {ch[s]}, reference {i}")
        H.assert_cost_close([co[s]], [cr])
        np.testing.assert_allclose(xo[r], xr, atol=2e-6)
        assert np.linalg.norm(go[r] - gr) <= H.GRAD_RTOL * np.linalg.norm(gr) + H.ABS_TOL


def _solve_case(use_graph, kind="plain", iters=100, layout=None):
    case = make_case(kind, layout=layout)
    x = case.x.clone()
    alpha = wl.ALPHA_4
    x, bc, bs, ok = case.ctx.mg_solve(case.b, case.q_start, case.goal, x, iters, 4, alpha, mode=1,
                                      graph_inner=25, use_graph=use_graph)
    torch.cuda.synchronize()
    return case, x.cpu().numpy(), bc.cpu().numpy(), bs.cpu().numpy(), ok.cpu().numpy()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_solve_graph_equals_direct_launches(layout):
    _, x1, c1, s1, ok1 = _solve_case(True, layout=layout)
    _, x2, c2, s2, ok2 = _solve_case(False, layout=layout)
    assert np.array_equal(x1, x2) and np.array_equal(c1, c2)
    assert np.array_equal(s1, s2) and np.array_equal(ok1, ok2)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_solve_results_are_reference_consistent(layout):
    """The solve is chaotic in fp32 vs fp64, so the reference re-evaluates
    the GPU's best trajectories: their cost must equal the reported best
    cost, it must not exceed the start cost, and the success verdict must
    agree with the reference's pose error and clearance of the best seed."""
    case, x, bc, bs, ok = _solve_case(True, layout=layout)
    D, T = 7, 32
    cr, _, mcr = H.oracle_cost_grad(case.ref, case.worlds, case.batch, x.reshape(-1, D), grad=False)
    H.assert_cost_close(bc, cr, "best cost")
    c_start, _, _ = H.oracle_cost_grad(case.ref, case.worlds, case.batch, case.batch.x0.reshape(-1, D), grad=False)
    assert np.all(bc <= c_start * (1 + 1e-4))
    assert int(bs[0]) == int(np.argmin(bc))
    k = int(bs[0])
    pe, re_ = case.ref.pose_error(x.reshape(4, T, D)[k, -1], case.batch.goal[0])
    near = abs(pe[0] - 0.005) < 1e-5 or abs(re_[0] - 0.05) < 1e-4 or abs(mcr[k]) < 1e-5
    if not near:
        assert bool(ok[0]) == bool(pe[0] <= 0.005 and re_[0] <= 0.05 and mcr[k] >= 0)
    # the optimizer makes progress on this problem
    assert bc.min() < 0.5 * c_start.min()


def test_ik_solve_reaches_reachable_goals():
    """Inverse kinematics (T = 1) with goals made reachable by construction
    (reference FK of random configurations) in an empty world, 32 seeds per
    goal: the success rate matches the reference solver's on the same
    problems (94% for the reference with these draws)."""
    robot = wl.make_arm(seed=0, n_spheres=52)
    worlds = wl.make_worlds(0, [0])
    P, S = 16, 32
    batch = wl.make_batch(robot, 21, [S] * P, [1] * P, [0] * P)
    r = ref.Ref(wl.robot_f32(robot))
    rng = np.random.default_rng(5)
    for p in range(P):
        _, _, ee = r.fk(rng.uniform(-2.0, 2.0, 7))
        batch.goal[p] = ee
    case = Case(robot, worlds, batch)
    x = case.x.clone()
    x, bc, bs, ok = case.ctx.mg_solve(case.b, case.q_start, case.goal, x, 100, 4, wl.ALPHA_4)
    torch.cuda.synchronize()
    ok = ok.cpu().numpy()
    xr = x.cpu().numpy().reshape(P, S, 7)
    bs = bs.cpu().numpy()
    # the success flags agree with the reference's pose error of the chosen seed
    for p in range(P):
        pe, re_ = case.ref.pose_error(xr[p, bs[p]], case.batch.goal[p])
        if abs(pe[0] - 0.005) > 1e-5 and abs(re_[0] - 0.05) > 1e-4:
            assert bool(ok[p]) == bool(pe[0] <= 0.005 and re_[0] <= 0.05), p
    assert ok.mean() >= 0.75


@pytest.mark.parametrize("two_arm", [False, True])
def test_ee_pose_matches_reference(two_arm):
    robot = wl.make_two_arm(seed=0, n_spheres=24) if two_arm else wl.make_arm(seed=0, n_spheres=20)
    robot = wl.robot_f32(robot)
    from paper_2310_17274_amd.binding import Context
    ctx = Context(robot)
    q = wl.goal_configs(robot, 5, 200).astype(np.float32).astype(np.float64)
    pose = ctx.mg_ee_pose(_dev(q)).cpu().numpy()
    r = ref.Ref(robot)
    for i in range(q.shape[0]):
        _, _, ee = r.fk(q[i])
        ee = ee.reshape(-1, 7)
        np.testing.assert_allclose(pose[i, :, :3], ee[:, :3], atol=1e-5)
        for e in range(ee.shape[0]):
            qg, qr = pose[i, e, 3:], ee[e, 3:]
            assert min(np.abs(qg - qr).max(), np.abs(qg + qr).max()) < 1e-5


def test_autograd_function_matches_adjoint():
    from paper_2310_17274_amd.binding import MgCost
    case = make_case("uneven")
    q = case.x.clone().requires_grad_(True)
    cost = MgCost.apply(q, case.ctx, case.b, case.q_start, case.goal)
    w = torch.linspace(0.5, 1.5, cost.numel(), device="cuda")
    (cost * w).sum().backward()
    c, g, _ = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x)
    torch.cuda.synchronize()
    assert torch.equal(cost.detach(), c)
    rows = torch.as_tensor(np.repeat(case.batch.horizon, case.batch.seeds), device="cuda")
    expect = g * torch.repeat_interleave(w, rows).view(-1, 1)
    assert torch.allclose(q.grad, expect, rtol=1e-6, atol=0)


def test_gpu_gradient_against_central_differences():
    """fp32 central differences of the GPU cost on a collision-free, smooth
    problem (no cuboid within reach), step 1e-3."""
    robot = wl.make_arm(seed=0, n_spheres=20)
    worlds = wl.make_worlds(0, [0])
    batch = wl.make_batch(robot, 31, [2], [8], [0], noise=0.01)
    case = Case(robot, worlds, batch, params=dict(a8=50.0, a9=0.01))
    c, g, _ = gpu_cost_grad(case)
    x = case.x.clone()
    h = 1e-3
    rng = np.random.default_rng(0)
    idx = rng.choice(x.numel(), 16, replace=False)
    fd, gi = [], []
    for i in idx:
        xp = x.clone().view(-1); xp[i] += h
        xm = x.clone().view(-1); xm[i] -= h
        cp = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, xp.view_as(x), grad=False)[0]
        cm = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, xm.view_as(x), grad=False)[0]
        fd.append(((cp.double() - cm.double()).sum() / (2 * h)).item())
        gi.append(float(g.reshape(-1)[i]))
    fd, gi = np.array(fd), np.array(gi)
    # fp32 cost rounding bounds the difference quotient's accuracy
    noise = 4 * float(c.sum()) * 6e-8 / (2 * h)
    assert np.linalg.norm(fd - gi) <= 2e-2 * np.linalg.norm(gi) + noise * np.sqrt(len(idx))


def test_device_noise_matches_the_oracle():
    """Counter-based draws on the device (Philox-4x64-10 + Box-Muller)
    against the oracle's: the same integer stream, so the normals agree to
    fp32 evaluation of sqrt(-2 ln u1) (at most 5.9, a few ulp) times
    cospi(2 u2) (a few ulp): 4e-6 absolute."""
    from paper_2310_17274_amd.binding import mg_philox_normals
    for seed, it0, n_it, N, rows, D in ((7, 0, 2, 5, 33, 7), (2 ** 63 + 11, 3, 1, 16, 96, 14), (0, 0, 1, 3, 5, 3)):
        got = mg_philox_normals(seed, it0, n_it, N, rows, D).cpu().numpy().astype(np.float64)
        want = ref.philox_normals(seed, it0 + n_it, N, rows, D)[it0:]
        np.testing.assert_allclose(got, want, rtol=0, atol=4e-6)


@pytest.mark.parametrize("layout", [pytest.param((0, 0), id="lane"), pytest.param(None, id="default"),
                                    pytest.param((3, 0), id="groups2"), pytest.param((4, 0), id="groups4")])
def test_seeded_particle_stage(layout):
    """The particle stage with its draws made inside the evaluation and
    update kernels equals the stage fed the same draws from memory (bit for
    bit), and agrees with the oracle's stage on the oracle's draws."""
    from paper_2310_17274_amd.binding import mg_philox_normals
    case = make_case("plain", layout=layout)
    S, T, D, N, seed = 4, 32, 7, 64, 1234
    case.b.mg_batch_reserve_particles(N)
    m1, v1 = case.x.clone(), torch.full_like(case.x, 0.05 ** 2)
    _, _, c1 = case.ctx.mg_particles_seeded(case.b, case.q_start, case.goal, m1, v1, N, 2, seed, costs=True)
    eps = mg_philox_normals(seed, 0, 2, N, S * T, D)
    m2, v2 = case.x.clone(), torch.full_like(case.x, 0.05 ** 2)
    _, _, c2 = case.ctx.mg_particles(case.b, case.q_start, case.goal, m2, v2, eps, costs=True)
    torch.cuda.synchronize()
    assert torch.equal(m1, m2) and torch.equal(v1, v2) and torch.equal(c1, c2)
    x0 = case.batch.x0.reshape(S, T, D)
    eps_ref = ref.philox_normals(seed, 2, N, S * T, D).reshape(2, N, S, T, D)
    m_ref, _, _ = case.ref.particles(case.worlds.world(0), case.batch.q_start[0], case.batch.goal[0], T, x0,
                                     np.full_like(x0, np.float32(0.05 ** 2)), eps_ref)
    mg = m1.cpu().numpy().reshape(S, T, D)
    for s in range(S):
        moved = np.abs(m_ref[s] - x0[s]).max()
        assert moved > 1e-3
        assert np.abs(mg[s] - m_ref[s]).max() <= 1e-2 * moved + 1e-5, s
