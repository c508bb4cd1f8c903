"""Speed metric (Eq.(11)) on the GPU through the C ABI against the FP64
reference: each sphere's world collision cost times its central-difference
speed, with the exact gradient (the speed's own gradient acts on the
neighbouring waypoints; the reference's is pinned by finite differences).
The term lives in the wave-per-link layout; a lane-per-link request falls
back to it, and the cuboid split over workgroups is not used with it."""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_2310_17274_amd import workloads as wl
from tests import harness as H
from tests.test_parity_gpu import (Case, _dev, _linesearch_parity, _particle_round_reference, gpu_cost_grad,
                                   make_case)

pytestmark = pytest.mark.gpu

SPEED = dict(speed=1)
LAYOUTS = [pytest.param((0, 0), id="lane_request"), pytest.param((1, 1), id="wave"),
           pytest.param((1, 4), id="wave4"), pytest.param((2, 0), id="wave2"),
           pytest.param((3, 0), id="groups2"), pytest.param((4, 0), id="groups4")]


def _collision_case(params, layout, seed=13):
    """Seeds pushed into obstacles (noisy, scaled) so that the collision
    term, and with it the speed factor, is active."""
    robot = wl.make_arm(seed=0, n_spheres=52)
    worlds = wl.make_worlds(11, [60])
    batch = wl.make_batch(robot, seed, [6], [16], [0], noise=0.4)
    batch.x0 = np.clip(batch.x0 * 1.3, -3.2, 3.2)
    return Case(robot, worlds, batch, params=params, layout=layout)


def _check(case):
    c, g, mc = gpu_cost_grad(case)
    cr, gr, mcr = H.oracle_cost_grad(case.ref, case.worlds, case.batch, case.batch.x0.reshape(-1, case.robot.dof))
    H.assert_cost_close(c, cr)
    H.assert_grad_close(g, gr, case.batch)
    H.assert_verdicts(mc, mcr)
    return cr


@pytest.mark.parametrize("layout", LAYOUTS)
def test_speed_cost_grad_parity(layout):
    case = _collision_case(SPEED, layout)
    _check(case)
    # the factor changes the collision term of this case
    T, b = 16, case.batch
    args = (case.worlds.world(0), b.q_start[0], b.goal[0], b.x0.reshape(-1, 7)[:T])
    fast = case.ref.traj_cost(*args, grad=False)[3][2]
    plain = ref.Ref(case.robot).traj_cost(*args, grad=False)[3][2]
    assert plain > 0 and abs(fast - plain) > 1e-2 * plain


@pytest.mark.parametrize("layout", [pytest.param((1, 1), id="wave"), pytest.param((3, 0), id="groups2"), pytest.param((4, 0), id="groups4")])
@pytest.mark.parametrize("kind", ["uneven", "tree"])
def test_speed_cost_grad_parity_uneven_and_tree(kind, layout):
    """Horizons 2..64 (a one-waypoint speed uses the start and itself) and
    the two-arm tree."""
    _check(make_case(kind, params=SPEED, layout=layout))


@pytest.mark.parametrize("layout", [pytest.param((1, 1), id="wave"), pytest.param((2, 0), id="wave2"),
                                    pytest.param((3, 0), id="groups2"), pytest.param((4, 0), id="groups4")])
def test_speed_with_swept_parity(layout):
    _check(_collision_case(dict(speed=1, swept=1, sweep_steps=4), layout, seed=21))


def test_speed_with_self_collision_parity():
    robot = wl.make_arm(seed=0, n_spheres=52)
    worlds = wl.make_worlds(11, [40])
    batch = wl.make_batch(robot, 13, [6], [16], [0], noise=0.6)
    case = Case(robot, worlds, batch, params=SPEED, self_pairs=wl.self_pairs(robot))
    _check(case)


@pytest.mark.parametrize("layout", [pytest.param((1, 1), id="wave"), pytest.param((3, 0), id="groups2"), pytest.param((4, 0), id="groups4")])
def test_speed_linesearch_parity(layout):
    case = make_case("plain", params=SPEED, layout=layout)
    _linesearch_parity(case, wl.ALPHA_4, 1)


def test_speed_particle_round_parity():
    """One particle round with the speed metric: particle costs against the
    reference's and the update fed the GPU's costs."""
    case = make_case("adjoint_small", params=SPEED)
    S, T, D, N = 5, 32, 7, 32
    rng = np.random.default_rng(22)
    eps = rng.normal(0, 1, (1, N, S * T, D)).astype(np.float32).astype(np.float64)
    case.b.mg_batch_reserve_particles(N)
    mean = case.x.clone()
    var = torch.full_like(mean, 0.05 ** 2)
    m_in = mean.double().cpu().numpy().reshape(S, T, D)
    v_in = var.double().cpu().numpy().reshape(S, T, D)
    _, _, costs = case.ctx.mg_particles(case.b, case.q_start, case.goal, mean, var, _dev(eps), costs=True)
    torch.cuda.synchronize()
    m_ref, v_ref = _particle_round_reference(case, m_in, v_in, eps[0].reshape(N, S, T, D),
                                             costs.cpu().numpy()[0], case.worlds.world(0))
    np.testing.assert_allclose(mean.cpu().numpy().reshape(S, T, D), m_ref, rtol=0, atol=5e-6)
    np.testing.assert_allclose(var.cpu().numpy().reshape(S, T, D), v_ref, rtol=2e-4, atol=1e-9)
