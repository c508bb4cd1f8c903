"""The allocation-free line search (mg_linesearch_noalloc) against
mg_linesearch through the C ABI: two calls in a row on one GPU, the second
with a smaller batch, in several evaluation layouts.  Where both calls run
the same kernels the results are bit-identical; the wave-per-link layout
split over workgroups (which the allocation-free call does not split) is
held to the parity tolerances.  Sizes beyond the static scratch are refused
on the host."""
import numpy as np
import pytest
import torch

from paper_2310_17274_amd import workloads as wl
from paper_2310_17274_amd._lib import MgError
from tests import harness as H
from tests.test_parity_gpu import Case, _dev

pytestmark = pytest.mark.gpu


def _case(S, T, layout, seed):
    robot = wl.make_arm(seed=0, n_spheres=52)
    worlds = wl.make_worlds(2, [40])
    batch = wl.make_batch(robot, seed, [S], [T], [0])
    return Case(robot, worlds, batch, layout=layout)


def _both(case, alpha, mode):
    c0, g0, _ = case.ctx.mg_cost_grad(case.b, case.q_start, case.goal, case.x)
    d = case.ctx.mg_lbfgs_step(case.b, 4, True, case.x, g0)
    ref_out = case.ctx.mg_linesearch(case.b, case.q_start, case.goal, case.x, c0, g0, d, alpha, mode)
    # poison the outputs so that a call that wrote nothing cannot pass
    out = tuple(torch.full_like(t, -7) for t in ref_out)
    na_out = case.ctx.mg_linesearch_noalloc(case.b, case.q_start, case.goal, case.x, c0, g0, d, alpha, mode,
                                            out=out)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ref_out], [t.cpu().numpy() for t in na_out]


@pytest.mark.parametrize("layout,exact", [((0, 0), True), ((1, 1), True), ((3, 0), True), ((4, 0), True),
                                          ((1, 4), False)],
                         ids=["lane", "wave", "groups2", "groups4", "wave4"])
def test_noalloc_linesearch_matches_linesearch(layout, exact):
    for S, T, K, seed in ((32, 32, 8, 11), (3, 12, 4, 12)):   # the second call is smaller
        case = _case(S, T, layout, seed)
        alpha = wl.ALPHA_8 if K == 8 else wl.ALPHA_4
        (xr, cr, gr, chr_, mcr), (xn, cn, gn, chn, mcn) = _both(case, alpha, 1)
        if exact:
            for a, b in ((xr, xn), (cr, cn), (gr, gn), (chr_, chn), (mcr, mcn)):
                assert np.array_equal(a, b)
            continue
        # other cuboid split: the same choice unless its margin is rounding
        same = chr_ == chn
        assert np.mean(same) >= 0.9
        H.assert_cost_close(cn[same], cr[same])
        blocks = [(s * T, (s + 1) * T) for s in range(S) if same[s]]
        for a, b in blocks:
            assert np.linalg.norm(gn[a:b] - gr[a:b]) <= H.GRAD_RTOL * np.linalg.norm(gr[a:b]) + H.ABS_TOL
            assert np.array_equal(xn[a:b], xr[a:b])
        H.assert_verdicts(mcn, mcr)


def test_noalloc_linesearch_refuses_sizes_beyond_the_scratch():
    """16 candidates x 32768 rows x (3 + 7) floats exceed the 4 Mi-float
    scratch: refused on the host before any launch."""
    case = _case(1024, 32, None, 13)
    c0 = torch.zeros(case.b.n_seeds, device="cuda")
    g0 = torch.zeros_like(case.x)
    alpha = [float(a) for a in np.linspace(0.01, 1.0, 16)]
    with pytest.raises(MgError) as e:
        case.ctx.mg_linesearch_noalloc(case.b, case.q_start, case.goal, case.x, c0, g0, g0, alpha, 1)
    assert e.value.status == -2 and "scratch" in str(e.value)
    # eight candidates fit
    (xr, cr, _, chr_, _), (xn, cn, _, chn, _) = _both(case, wl.ALPHA_8, 1)
    assert np.array_equal(xr, xn) and np.array_equal(cr, cn) and np.array_equal(chr_, chn)
