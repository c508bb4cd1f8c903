"""The solve with each line-search choice (Alg.1) and L-BFGS direction
(Alg.6) folded into the next evaluation launch against the same solve with
separate launches: identical bits for the returned trajectories, best costs,
best seeds and success flags (the fused launch runs the same arithmetic).

  adjoint  32 seeds x 32 waypoints x 8 candidates (the benchmark's solve),
           wave per link with one slice, four slices, two and four slot groups
  plain    4 seeds x 32 waypoints x 4 candidates
"""
import numpy as np
import pytest
import torch

from paper_2310_17274_amd import workloads as wl
from tests.test_parity_gpu import make_case

pytestmark = pytest.mark.gpu


def _solve(case, fused, use_graph, iters, alpha, m=4, mode=1, graph_inner=25):
    case.b.mg_batch_set_fusion(fused)
    x = case.x.clone()
    x, bc, bs, ok = case.ctx.mg_solve(case.b, case.q_start, case.goal, x, iters, m, alpha, mode=mode,
                                      graph_inner=graph_inner, use_graph=use_graph)
    torch.cuda.synchronize()
    return x.cpu().numpy(), bc.cpu().numpy(), bs.cpu().numpy(), ok.cpu().numpy()


def _same(r1, r2):
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("layout", [pytest.param((1, 1), id="wave"), pytest.param((1, 4), id="wave4"),
                                    pytest.param((3, 0), id="groups2"), pytest.param((4, 0), id="groups4")])
@pytest.mark.parametrize("use_graph", [True, False], ids=["graph", "direct"])
def test_fused_solve_equals_separate_launches_adjoint(layout, use_graph):
    case = make_case("adjoint", layout=layout)
    alpha = list(wl.cfg_cost_adjoint()[3]["alpha"])
    _same(_solve(case, True, use_graph, 100, alpha), _solve(case, False, use_graph, 100, alpha))


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("iters", [1, 2, 27, 60])
def test_fused_solve_equals_separate_launches_plain(iters, mode):
    """Iteration counts around the graph length (26 fused iterations per
    replay), the smallest, and the other line-search rules."""
    case = make_case("plain", layout=(3, 0))
    alpha = list(wl.ALPHA_4)
    _same(_solve(case, True, True, iters, alpha, mode=mode), _solve(case, False, True, iters, alpha, mode=mode))


@pytest.mark.parametrize("K", [1, 2, 8])
def test_fused_solve_candidate_counts(K):
    """One, two and eight candidates (padded to 4 or 8 in the choice; with
    32 evaluations per workgroup a chunk holds 32 / K rows of one seed)."""
    case = make_case("adjoint", layout=(3, 0))
    alpha = [float(a) for a in np.linspace(0.05, 1.0, K)]
    assert case.ctx.mg_solve_fuses(case.b, K, 4, case.x)
    _same(_solve(case, True, True, 40, alpha), _solve(case, False, True, 40, alpha))


@pytest.mark.parametrize("m", [1, 2, 3])
def test_fused_solve_shorter_histories(m):
    """History lengths below the kernel's four register slots (the ring
    wraps sooner)."""
    case = make_case("plain", layout=(1, 1))
    alpha = list(wl.ALPHA_4)
    _same(_solve(case, True, True, 60, alpha, m=m), _solve(case, False, True, 60, alpha, m=m))


@pytest.mark.parametrize("layout", [pytest.param((1, 1), id="wave"), pytest.param((3, 0), id="groups2")])
def test_fused_solve_several_problems(layout):
    """Three problems of one horizon with different seed counts and worlds
    (workgroup chunks from the record table, seeds after the first
    problem's rows)."""
    from tests.test_parity_gpu import Case
    robot = wl.make_arm(seed=0, n_spheres=52)
    worlds = wl.make_worlds(8, [40, 12, 25])
    batch = wl.make_batch(robot, 77, [3, 5, 2], [32, 32, 32], [0, 1, 2])
    case = Case(robot, worlds, batch, layout=layout)
    alpha = list(wl.cfg_cost_adjoint()[3]["alpha"])
    assert case.ctx.mg_solve_fuses(case.b, len(alpha), 4, case.x)
    _same(_solve(case, True, True, 60, alpha), _solve(case, False, True, 60, alpha))


@pytest.mark.parametrize("layout", [pytest.param((1, 1), id="wave"), pytest.param((1, 4), id="wave4")])
def test_fused_solve_self_collision(layout):
    """Self-collision on (its phase runs after the folded choice, between
    the staging and the world tiles), horizon 32."""
    from tests.test_parity_gpu import _self_case
    case = _self_case(layout, T=32)
    alpha = list(wl.cfg_cost_adjoint()[3]["alpha"])
    assert case.ctx.mg_solve_fuses(case.b, len(alpha), 4, case.x)
    _same(_solve(case, True, True, 40, alpha), _solve(case, False, True, 40, alpha))


def test_fusion_applies_where_the_batch_qualifies():
    """The benchmark's batch in the two-slot-group layout folds the choice
    in; more than 4 history pairs, fusion switched off, an IK batch (7
    floats per seed) and the lane-per-link layout do not."""
    case = make_case("adjoint", layout=(3, 0))
    assert case.ctx.mg_solve_fuses(case.b, 8, 4, case.x)
    assert not case.ctx.mg_solve_fuses(case.b, 8, 5, case.x)      # more than 4 history pairs
    case.b.mg_batch_set_fusion(False)
    assert not case.ctx.mg_solve_fuses(case.b, 8, 4, case.x)
    ik = make_case("ik", layout=(1, 1))
    assert not ik.ctx.mg_solve_fuses(ik.b, 4, 4, ik.x)
    lane = make_case("adjoint", layout=(0, 0))
    assert not lane.ctx.mg_solve_fuses(lane.b, 8, 4, lane.x)
    from tests.test_parity_gpu import _self_case
    short = _self_case((1, 1), T=16)                              # 112 floats per seed: 2 per lane apart
    assert not short.ctx.mg_solve_fuses(short.b, 8, 4, short.x)
    halves = make_case("adjoint", layout=(2, 0))                  # two waves per link: no joint wave
    assert not halves.ctx.mg_solve_fuses(halves.b, 8, 4, halves.x)
    g4 = make_case("adjoint", layout=(4, 0))
    assert g4.ctx.mg_solve_fuses(g4.b, 8, 4, g4.x)


def test_fused_solve_repeated_calls():
    """Two solves in a row on one batch (the graph is replayed, and the
    second starts from the first's state sets) equal the separate path."""
    case = make_case("adjoint", layout=(3, 0))
    alpha = list(wl.cfg_cost_adjoint()[3]["alpha"])
    a1 = _solve(case, True, True, 60, alpha)
    a2 = _solve(case, True, True, 60, alpha)
    b1 = _solve(case, False, True, 60, alpha)
    _same(a1, b1)
    _same(a2, b1)
