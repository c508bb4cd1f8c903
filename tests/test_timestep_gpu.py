"""Time-step optimization (Alg.4) on the GPU through the C ABI: the
retiming kernel against the FP64 reference's retime, and the two-pass
driver against the same steps issued one by one."""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_2310_17274_amd import workloads as wl
from paper_2310_17274_amd.binding import default_params
from tests.test_parity_gpu import make_case

pytestmark = pytest.mark.gpu

# per-joint limits of a 7-joint arm (rad/s, rad/s^2, rad/s^3)
VMAX = np.array([2.175, 2.175, 2.175, 2.175, 2.61, 2.61, 2.61])
AMAX = np.array([15.0, 7.5, 10.0, 12.5, 15.0, 20.0, 20.0])
JMAX = np.array([7500.0, 3750.0, 5000.0, 6250.0, 7500.0, 10000.0, 10000.0])


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _retime_ref(case, x, dt, limits):
    """Per-seed reference retime of x [rows, D] (fp64 on the fp32 inputs)."""
    b, D = case.batch, case.robot.dof
    out, r0 = [], 0
    for p in range(b.n_problems):
        for _ in range(int(b.seeds[p])):
            T = int(b.horizon[p])
            out.append(ref.retime(_f32(b.q_start[p]), x[r0:r0 + T], dt, *limits))
            r0 += T
    return np.array(out)


@pytest.mark.parametrize("limits", [pytest.param((VMAX, AMAX, JMAX), id="all"),
                                    pytest.param((VMAX, 0 * AMAX, 0 * JMAX), id="velocity"),
                                    pytest.param((0 * VMAX, AMAX, 0 * JMAX), id="acceleration"),
                                    pytest.param((0 * VMAX, 0 * AMAX, JMAX), id="jerk")])
@pytest.mark.parametrize("kind", ["uneven", "adjoint"])
def test_retime_parity(kind, limits):
    """Every seed of an uneven batch (horizons 2..64, one problem of one
    seed) and of the full 32 x 32 cost+adjoint batch; each kind of limit
    alone and all three."""
    case = make_case(kind)
    x = case.x.clone()
    dt = float(np.float32(case.ctx.params.dt))
    got = case.ctx.mg_retime(case.b, case.q_start, x, *limits).cpu().numpy().astype(np.float64)
    want = _retime_ref(case, x.cpu().numpy().astype(np.float64), dt, limits)
    assert got.shape == want.shape and np.all(want > 0)
    np.testing.assert_allclose(got, want, rtol=1e-4, atol=0)


def test_retime_rest_and_scaling():
    """A seed that never leaves its start retimes to 0; the retimed spacing
    does not depend on the spacing the trajectory is read at."""
    case = make_case("adjoint_small")
    x = case.x.clone()
    T, D = 32, 7
    x[:T] = case.q_start[0]
    lim = (VMAX, AMAX, JMAX)
    a = case.ctx.mg_retime(case.b, case.q_start, x, *lim).cpu().numpy()
    assert a[0] == 0.0 and np.all(a[1:] > 0)
    case.ctx.mg_set_params(default_params(dt=0.05))
    b = case.ctx.mg_retime(case.b, case.q_start, x, *lim).cpu().numpy()
    np.testing.assert_allclose(b, a, rtol=1e-5, atol=0)


def test_retime_rejects_nan_limit():
    from paper_2310_17274_amd._lib import MgError
    case = make_case("adjoint_small")
    with pytest.raises(MgError):
        case.ctx.mg_retime(case.b, case.q_start, case.x, VMAX, np.full(7, np.nan), JMAX)


@pytest.mark.parametrize("use_graph", [True, False])
def test_solve_timestep_equals_its_steps(use_graph):
    """The driver against its steps issued one by one: a first solve
    without the jerk term, the retimed spacing of the problems' best seeds
    (also against the FP64 retime), the derivative weights rescaled to it,
    a second solve from the first one's best iterates, and the final
    retime.  Same kernels, so bit-identical; parameters restored after."""
    alpha = wl.ALPHA_4
    it1, it2, lim = 20, 15, (VMAX, AMAX, JMAX)
    drv = make_case("uneven")
    x = drv.x.clone()
    x, bc, bs, ok, (dt_opt, dt_f) = drv.ctx.mg_solve_timestep(drv.b, drv.q_start, drv.goal, x, it1, it2, 4, alpha,
                                                              *lim, use_graph=use_graph)
    torch.cuda.synchronize()
    p0 = default_params()
    # the parameters are back to what they were
    c0 = drv.ctx.mg_cost_grad(drv.b, drv.q_start, drv.goal, drv.x)[0]
    ref_case = make_case("uneven")
    assert torch.equal(c0, ref_case.ctx.mg_cost_grad(ref_case.b, ref_case.q_start, ref_case.goal, ref_case.x)[0])

    st = ref_case
    xs = st.x.clone()
    st.ctx.mg_set_params(default_params(a9=0.0))
    xs, bc1, bs1, _ = st.ctx.mg_solve(st.b, st.q_start, st.goal, xs, it1, 4, alpha, mode=1, graph_inner=25,
                                      use_graph=use_graph)
    dts = st.ctx.mg_retime(st.b, st.q_start, xs, *lim).cpu().numpy()
    seed0 = np.concatenate([[0], np.cumsum(st.batch.seeds)[:-1]])
    best = seed0 + bs1.cpu().numpy()
    want_opt = max(float(dts[best].max()), 1e-3)
    assert dt_opt == np.float32(want_opt)
    # FP64 retime of the first pass's best seeds
    dref = _retime_ref(st, xs.cpu().numpy().astype(np.float64), float(np.float32(p0.dt)), lim)
    np.testing.assert_allclose(dts, dref, rtol=1e-4, atol=0)
    f = np.float32
    rho = f(dt_opt) / f(p0.dt)
    rho2, rho3 = rho * rho, rho * rho * rho
    st.ctx.mg_set_params(default_params(dt=float(f(dt_opt)), a7=float(f(p0.a7) * rho),
                                        a8=float(f(p0.a8) * (rho2 * rho2)), a9=float(f(p0.a9) * (rho3 * rho3))))
    xs, bc2, bs2, ok2 = st.ctx.mg_solve(st.b, st.q_start, st.goal, xs, it2, 4, alpha, mode=1, graph_inner=25,
                                        use_graph=use_graph)
    dts2 = st.ctx.mg_retime(st.b, st.q_start, xs, *lim).cpu().numpy()
    torch.cuda.synchronize()
    assert torch.equal(xs, x) and torch.equal(bc2, bc) and torch.equal(bs2, bs) and torch.equal(ok2, ok)
    assert dt_f == np.float32(max(float(dts2[seed0 + bs2.cpu().numpy()].max()), 1e-3))
    # the retimed second pass sits on its limits: at dt_f no best seed exceeds them
    assert 0 < dt_f and dt_opt < 0.25


def test_retime_jerk_parity():
    """The largest |jerk| read at each seed's retimed spacing against the
    reference's (uneven batch: horizons 2..64)."""
    case = make_case("uneven")
    x = case.x.clone()
    lim = (VMAX, AMAX, JMAX)
    dt, jk = case.ctx.mg_retime(case.b, case.q_start, x, *lim, jerk=True)
    dt, jk = dt.cpu().numpy().astype(np.float64), jk.cpu().numpy().astype(np.float64)
    b, D = case.batch, 7
    xs = x.cpu().numpy().astype(np.float64)
    seed, r0 = 0, 0
    for p in range(b.n_problems):
        for _ in range(int(b.seeds[p])):
            T = int(b.horizon[p])
            q0 = _f32(b.q_start[p])
            dref = ref.retime(q0, xs[r0:r0 + T], 0.25, *lim)
            want = ref.max_jerk(q0, xs[r0:r0 + T], dref)
            assert abs(jk[seed] - want) <= 1e-3 * want + 1e-6, (p, seed, jk[seed], want)
            seed += 1
            r0 += T


def test_solve_timestep_against_the_oracle_driver():
    """mg_solve_timestep against the FP64 oracle's Alg.4 driver on the same
    inputs, with few iterations so that the fp32 and fp64 iterates stay
    close: dt_opt, dt_f and the best costs to 1e-3.  Independently of the
    iterates, the GPU's best costs must be the oracle's cost of the GPU's
    final trajectories at its dt_opt with the rescaled weights (a7 rho,
    a8 rho^4, a9 rho^6, jerk on): the exponents and the pass order."""
    from tests import harness as H
    case = make_case("plain")
    it1, it2, lim = 4, 3, (VMAX, AMAX, JMAX)
    x = case.x.clone()
    x, bc, bs, ok, (dt_opt, dt_f) = case.ctx.mg_solve_timestep(case.b, case.q_start, case.goal, x, it1, it2, 4,
                                                               wl.ALPHA_4, *lim, use_graph=False)
    torch.cuda.synchronize()
    bc = bc.cpu().numpy().astype(np.float64)
    xg = x.cpu().numpy().astype(np.float64).reshape(-1)
    b = case.batch
    boxes = case.worlds.world(0)
    xs_r, bc_r, (o_opt, o_f) = ref.solve_timestep(case.robot, [(boxes, b.q_start[0], b.goal[0], 32, b.x0)], it1,
                                                  it2, 4, wl.ALPHA_4, *lim, 1e-3, nthreads=4)
    assert abs(dt_opt - o_opt) <= 1e-3 * o_opt and abs(dt_f - o_f) <= 1e-3 * o_f, (dt_opt, o_opt, dt_f, o_f)
    np.testing.assert_allclose(bc, bc_r[0], rtol=1e-3)
    r2 = ref.Ref(case.robot, **ref.timestep_params({}, float(dt_opt)))
    c_re = r2.cost_grad_batch(boxes, b.q_start[0], b.goal[0], 32, xg, grad=False)[0]
    H.assert_cost_close(bc, c_re, "best cost at the rescaled weights")
    # the jerk weight matters here: without it the same trajectories cost less
    r_nj = ref.Ref(case.robot, **ref.timestep_params(dict(a9=0.0), float(dt_opt)))
    assert np.all(r_nj.cost_grad_batch(boxes, b.q_start[0], b.goal[0], 32, xg, grad=False)[0] < c_re)
