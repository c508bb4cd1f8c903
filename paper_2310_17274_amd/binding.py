"""Python binding of libmg with the C ABI's names (include/mg.h).

Argument marshalling only: torch provides device memory and the current
stream; every step of the method runs in the HIP kernels of libmg.so.

    ctx = Context(robot)                    # mg_create
    ctx.mg_set_worlds(worlds)               # mg_set_worlds
    b = ctx.batch(seeds, horizon, world)    # mg_batch_create
    cost, grad, mc = ctx.mg_cost_grad(b, q_start, goal, q)
    d = ctx.mg_lbfgs_step(b, m, reset, x, g)
    out = ctx.mg_linesearch(b, q_start, goal, x, c0, g0, d, alpha, mode)
    res = ctx.mg_solve(b, q_start, goal, x, iters, m, alpha, ...)
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check

_fp = C.POINTER(C.c_float)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return C.c_void_p(t.data_ptr())


def _f32(t, device):
    return torch.as_tensor(np.asarray(t), dtype=torch.float32, device=device).contiguous()


def default_params(**over) -> _lib.Params:
    p = _lib.Params()
    _lib.lib().mg_default_params(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


class Batch:
    """A batch of problems (mg_batch): seeds, horizon and world per problem."""

    def __init__(self, ctx: "Context", seeds, horizon, world, K_max=16, m_max=8):
        self.ctx = ctx
        self.seeds = np.ascontiguousarray(seeds, dtype=np.int32)
        self.horizon = np.ascontiguousarray(horizon, dtype=np.int32)
        self.world = np.ascontiguousarray(world, dtype=np.int32)
        self.P = int(self.seeds.shape[0])
        self.K_max, self.m_max = K_max, m_max
        h = C.c_void_p()
        ip = C.POINTER(C.c_int)
        check(_lib.lib().mg_batch_create(ctx.handle, self.P, self.seeds.ctypes.data_as(ip),
                                         self.horizon.ctypes.data_as(ip),
                                         self.world.ctypes.data_as(ip), K_max, m_max, C.byref(h)))
        self.handle = h
        self.n_seeds = int(self.seeds.sum())
        self.rows = int((self.seeds * self.horizon).sum())
        assert self.n_seeds == _lib.lib().mg_batch_seeds(h)
        assert self.rows == _lib.lib().mg_batch_rows(h)

    def mg_batch_set_layout(self, layout: int, slices: int = 0):
        """Fix the evaluation layout (-1 default, 0 lane per link, 1 wave per
        link, 2 two waves per link, 3 two slot groups per wave, 4 four slot
        groups per wave) and the cuboid slices (0 automatic, 1, 2, 4, and
        for layout 1 also 8 or 16; layouts 2, 3 and 4: 0 or 1)."""
        _lib.check(_lib.lib().mg_batch_set_layout(self.handle, int(layout), int(slices)))

    def mg_batch_set_fusion(self, enable: bool):
        """Fold each line-search choice of mg_solve into the next evaluation
        launch where the batch qualifies (default on)."""
        _lib.check(_lib.lib().mg_batch_set_fusion(self.handle, int(bool(enable))))

    def mg_batch_reserve_particles(self, n_particles: int):
        _lib.check(_lib.lib().mg_batch_reserve_particles(self.handle, int(n_particles)))

    def mg_set_timing(self, enable: bool):
        check(_lib.lib().mg_set_timing(self.handle, int(bool(enable))))

    def mg_eval_time(self):
        """(mean microseconds, count) of the recorded evaluation launches."""
        us, n = C.c_float(0.0), C.c_int(0)
        check(_lib.lib().mg_eval_time(self.handle, C.byref(us), C.byref(n)))
        return us.value, n.value

    def close(self):
        if self.handle:
            _lib.lib().mg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """Robot + parameters + worlds on the current device (mg_ctx)."""

    def __init__(self, robot, params: _lib.Params | None = None, device="cuda"):
        L = _lib.lib()
        self.device = torch.device(device)
        self.robot = robot
        self.dof = robot.dof
        self._keep = []

        def fa(a):
            a = np.ascontiguousarray(a, dtype=np.float32)
            self._keep.append(a)
            return a.ctypes.data_as(_fp)

        def ia(a):
            a = np.ascontiguousarray(a, dtype=np.int32)
            self._keep.append(a)
            return a.ctypes.data_as(C.POINTER(C.c_int))

        desc = _lib.RobotDesc(n_links=robot.n_links, dof=robot.dof, n_spheres=robot.n_spheres,
                              n_ee=robot.n_ee, parent=ia(robot.parent), joint=ia(robot.joint),
                              fixed_tf=fa(robot.fixed_tf), sphere_link=ia(robot.sphere_link),
                              sphere=fa(robot.sphere), ee_link=ia(robot.ee_link), ee_tf=fa(robot.ee_tf),
                              q_lo=fa(robot.q_lo), q_hi=fa(robot.q_hi))
        self.params = params if params is not None else default_params()
        h = C.c_void_p()
        check(L.mg_create(C.byref(desc), C.byref(self.params), C.byref(h)))
        self.handle = h
        self._keep = []
        self._worlds = None

    def close(self):
        if getattr(self, "handle", None):
            _lib.lib().mg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mg_set_params(self, params: _lib.Params):
        check(_lib.lib().mg_set_params(self.handle, C.byref(params)))
        self.params = params

    def mg_set_worlds(self, worlds):
        off = np.ascontiguousarray(worlds.offsets, dtype=np.int32)
        pose = _f32(worlds.pose, self.device).reshape(-1)
        dims = _f32(worlds.dims, self.device).reshape(-1)
        check(_lib.lib().mg_set_worlds(self.handle, int(off.shape[0] - 1),
                                       off.ctypes.data_as(C.POINTER(C.c_int)),
                                       _ptr(pose), _ptr(dims), _stream()))
        self._worlds = (pose, dims)   # kept until the stream has used them

    def batch(self, seeds, horizon, world, K_max=16, m_max=8) -> Batch:
        return Batch(self, seeds, horizon, world, K_max, m_max)

    # -- hot path ------------------------------------------------------------
    def mg_cost_grad(self, b: Batch, q_start, goal, q, grad=True, min_clear=True):
        dev = self.device
        cost = torch.empty(b.n_seeds, dtype=torch.float32, device=dev)
        g = torch.empty_like(q) if grad else None
        mc = torch.empty(b.n_seeds, dtype=torch.float32, device=dev) if min_clear else None
        check(_lib.lib().mg_cost_grad(self.handle, b.handle, _ptr(q_start), _ptr(goal), _ptr(q),
                                      _ptr(cost), _ptr(g), _ptr(mc), _stream()))
        return cost, g, mc

    def mg_lbfgs_step(self, b: Batch, m, reset, x, g, out=None):
        d = torch.empty_like(x) if out is None else out
        check(_lib.lib().mg_lbfgs_step(self.handle, b.handle, int(m), int(reset), _ptr(x), _ptr(g),
                                       _ptr(d), _stream()))
        return d

    def mg_linesearch(self, b: Batch, q_start, goal, x, c0, g0, d, alpha, mode=1, out=None):
        al = (C.c_float * len(alpha))(*alpha)
        if out is None:
            out = (torch.empty_like(x), torch.empty_like(c0), torch.empty_like(g0),
                   torch.empty(b.n_seeds, dtype=torch.int32, device=self.device),
                   torch.empty(b.n_seeds, dtype=torch.float32, device=self.device))
        xo, co, go, ch, mc = out
        check(_lib.lib().mg_linesearch(self.handle, b.handle, _ptr(q_start), _ptr(goal), _ptr(x),
                                       _ptr(c0), _ptr(g0), _ptr(d), len(alpha), al, int(mode),
                                       _ptr(xo), _ptr(co), _ptr(go), _ptr(ch), _ptr(mc), _stream()))
        return xo, co, go, ch, mc

    def mg_linesearch_eval(self, b: Batch, q_start, goal, x, d, alpha, grad=True, min_clear=True):
        """Every line-search candidate costed (no choice): cost, <g_k, d>,
        min clearance [K, seeds] and gradient [K, rows, D] (or None)."""
        K = len(alpha)
        al = (C.c_float * K)(*alpha)
        cost = torch.empty((K, b.n_seeds), dtype=torch.float32, device=self.device)
        gd = torch.empty_like(cost)
        mc = torch.empty_like(cost) if min_clear else None
        g = torch.empty((K, b.rows, self.dof), dtype=torch.float32, device=self.device) if grad else None
        check(_lib.lib().mg_linesearch_eval(self.handle, b.handle, _ptr(q_start), _ptr(goal), _ptr(x), _ptr(d),
                                            K, al, _ptr(cost), _ptr(gd), _ptr(g), _ptr(mc), _stream()))
        return cost, gd, g, mc

    def mg_linesearch_noalloc(self, b: Batch, q_start, goal, x, c0, g0, d, alpha, mode=1, out=None):
        """mg_linesearch with its per-candidate results in the library's static
        scratch (no device allocation in the call); out as mg_linesearch's."""
        al = (C.c_float * len(alpha))(*alpha)
        if out is None:
            out = (torch.empty_like(x), torch.empty_like(c0), torch.empty_like(g0),
                   torch.empty(b.n_seeds, dtype=torch.int32, device=self.device),
                   torch.empty(b.n_seeds, dtype=torch.float32, device=self.device))
        xo, co, go, ch, mc = out
        check(_lib.lib().mg_linesearch_noalloc(self.handle, b.handle, _ptr(q_start), _ptr(goal), _ptr(x),
                                               _ptr(c0), _ptr(g0), _ptr(d), len(alpha), al, int(mode),
                                               _ptr(xo), _ptr(co), _ptr(go), _ptr(ch), _ptr(mc), _stream()))
        return xo, co, go, ch, mc

    def mg_solve_fuses(self, b: Batch, K, m, x) -> bool:
        """Whether mg_solve folds each choice into the next evaluation launch."""
        return bool(_lib.lib().mg_solve_fuses(self.handle, b.handle, int(K), int(m), _ptr(x)))

    def mg_solve(self, b: Batch, q_start, goal, x, iters, m, alpha, mode=1, graph_inner=25,
                 use_graph=True, outputs=None):
        """Solve in place on x; returns (x, best_cost, best_seed, success)."""
        al = (C.c_float * len(alpha))(*alpha)
        if outputs is None:
            outputs = (torch.empty(b.n_seeds, dtype=torch.float32, device=self.device),
                       torch.empty(b.P, dtype=torch.int32, device=self.device),
                       torch.empty(b.P, dtype=torch.int32, device=self.device))
        bc, bs, ok = outputs
        check(_lib.lib().mg_solve(self.handle, b.handle, _ptr(q_start), _ptr(goal), _ptr(x), int(iters),
                                  int(m), len(alpha), al, int(mode), int(graph_inner),
                                  int(bool(use_graph)), _ptr(bc), _ptr(bs), _ptr(ok), _stream()))
        return x, bc, bs, ok

    def _limits(self, vmax, amax, jmax):
        D = self.robot.dof
        return tuple((C.c_float * D)(*np.broadcast_to(np.asarray(z, dtype=np.float32), (D,)).tolist())
                     for z in (vmax, amax, jmax))

    def mg_retime(self, b: Batch, q_start, x, vmax, amax, jmax, out=None, jerk=False):
        """Per-seed spacing [seeds] at which x's largest velocity,
        acceleration or jerk meets its limit (Alg.4 retime); with jerk=True
        also the largest |jerk| [seeds] read at that spacing."""
        lim = self._limits(vmax, amax, jmax)
        out = torch.empty(b.n_seeds, dtype=torch.float32, device=self.device) if out is None else out
        jk = torch.empty(b.n_seeds, dtype=torch.float32, device=self.device) if jerk else None
        check(_lib.lib().mg_retime(self.handle, b.handle, _ptr(q_start), _ptr(x), *lim, _ptr(out),
                                   _ptr(jk) if jerk else None, _stream()))
        return (out, jk) if jerk else out

    def mg_steer(self, b: Batch, q_from, q_to, res, n_max):
        """Parallel steering (Alg.3) of edges q_from -> q_to [n, D]; b holds
        one problem of horizon 1 with n (n_max + 1) seeds.  Returns
        (reach [n, D], last [n], dist [n])."""
        n = int(q_from.shape[0])
        reach = torch.empty_like(q_from)
        last = torch.empty(n, dtype=torch.int32, device=self.device)
        dist = torch.empty(n, dtype=torch.float32, device=self.device)
        check(_lib.lib().mg_steer(self.handle, b.handle, n, _ptr(q_from), _ptr(q_to), float(res), int(n_max),
                                  _ptr(reach), _ptr(last), _ptr(dist), _stream()))
        return reach, last, dist

    def mg_plan(self, b: Batch, start, goal, res, n_max, retract=None, n_samples=64, k_near=4, max_rounds=20,
                seed=0, max_waypoints=256):
        """Geometric plan (Alg.2) from start to goal (host [D]); b holds one
        problem of horizon 1 with a multiple of n_max + 1 seeds.  Returns the
        waypoints [n, D] (n = 0: none found)."""
        D = self.robot.dof
        f = lambda a: (C.c_float * D)(*np.asarray(a, dtype=np.float32).tolist())
        path = (C.c_float * (max_waypoints * D))()
        n = C.c_int(0)
        check(_lib.lib().mg_plan(self.handle, b.handle, f(start), f(goal), f(retract) if retract is not None else None,
                                 float(res), int(n_max), int(n_samples), int(k_near), int(max_rounds), int(seed),
                                 int(max_waypoints), path, C.byref(n), _stream()))
        return np.frombuffer(path, dtype=np.float32, count=n.value * D).reshape(n.value, D).copy()

    def mg_plan_batch(self, b: Batch, starts, goals, res, n_max, retract=None, n_samples=64, k_near=4,
                      max_rounds=40, refine_rounds=0, seed=0, max_waypoints=256):
        """Geometric plans (Alg.2) of several queries (host [n, D] starts and
        goals) on one shared roadmap.  Returns a list of waypoint arrays
        [n_i, D] (n_i = 0: none found)."""
        D = self.robot.dof
        st = np.ascontiguousarray(starts, dtype=np.float32).reshape(-1, D)
        gl = np.ascontiguousarray(goals, dtype=np.float32).reshape(-1, D)
        nq = st.shape[0]
        assert gl.shape[0] == nq
        fp = lambda a: a.ctypes.data_as(_lib._fp)
        paths = np.zeros((nq, max_waypoints, D), dtype=np.float32)
        nw = np.zeros(nq, dtype=np.int32)
        ret = np.ascontiguousarray(retract, dtype=np.float32) if retract is not None else None
        check(_lib.lib().mg_plan_batch(self.handle, b.handle, nq, fp(st), fp(gl),
                                       fp(ret) if ret is not None else None, float(res), int(n_max),
                                       int(n_samples), int(k_near), int(max_rounds), int(refine_rounds), int(seed),
                                       int(max_waypoints), fp(paths), nw.ctypes.data_as(_lib._ip), _stream()))
        return [paths[i, :nw[i]].copy() for i in range(nq)]

    def mg_ik_seeds(self, ik: Batch, to: Batch, q_start, goal, x_ik, w_dist=0.1):
        """Trajectory seeds [to rows, D] on the lines to the ranked IK
        solutions, and ik_ok [P]."""
        x_to = torch.empty((to.rows, self.robot.dof), dtype=torch.float32, device=self.device)
        ok = torch.empty(ik.P, dtype=torch.int32, device=self.device)
        check(_lib.lib().mg_ik_seeds(self.handle, ik.handle, to.handle, _ptr(q_start), _ptr(goal), _ptr(x_ik),
                                     float(w_dist), _ptr(x_to), _ptr(ok), _stream()))
        return x_to, ok

    def mg_traj_select(self, b: Batch, q_start, goal, x, vmax, amax, jmax, w_jerk=1e-3, w_time=1.0):
        """(best_seed [P], success [P], motion_time [P]) among x's seeds."""
        lim = self._limits(vmax, amax, jmax)
        bs = torch.empty(b.P, dtype=torch.int32, device=self.device)
        ok = torch.empty(b.P, dtype=torch.int32, device=self.device)
        mt = torch.empty(b.P, dtype=torch.float32, device=self.device)
        check(_lib.lib().mg_traj_select(self.handle, b.handle, _ptr(q_start), _ptr(goal), _ptr(x), *lim,
                                        float(w_jerk), float(w_time), _ptr(bs), _ptr(ok), _ptr(mt), _stream()))
        return bs, ok, mt

    def mg_motion_gen(self, ik: Batch, to: Batch, q_start, goal, x_ik, iters_ik, iters1, iters2, m, alpha,
                      vmax, amax, jmax, dt_min=1e-3, w_dist=0.1, w_jerk=1e-3, w_time=1.0, mode=1, x_to=None):
        """IK, seeds, time-step optimization, selection.  x_ik is updated in
        place; returns (x_to, ik_ok, best_seed, success, motion_time,
        (dt_opt, dt_f))."""
        al = (C.c_float * len(alpha))(*alpha)
        lim = self._limits(vmax, amax, jmax)
        if x_to is None:
            x_to = torch.empty((to.rows, self.robot.dof), dtype=torch.float32, device=self.device)
        ik_ok, bs, ok = (torch.empty(ik.P, dtype=torch.int32, device=self.device) for _ in range(3))
        mt = torch.empty(ik.P, dtype=torch.float32, device=self.device)
        dt = (C.c_float * 2)()
        check(_lib.lib().mg_motion_gen(self.handle, ik.handle, to.handle, _ptr(q_start), _ptr(goal), _ptr(x_ik),
                                       _ptr(x_to), int(iters_ik), int(iters1), int(iters2), int(m), len(alpha), al,
                                       int(mode), *lim, float(dt_min), float(w_dist), float(w_jerk),
                                       float(w_time), _ptr(ik_ok), _ptr(bs), _ptr(ok), _ptr(mt), dt, _stream()))
        return x_to, ik_ok, bs, ok, mt, (dt[0], dt[1])

    def mg_solve_timestep(self, b: Batch, q_start, goal, x, iters1, iters2, m, alpha, vmax, amax, jmax,
                          dt_min=1e-3, mode=1, graph_inner=25, use_graph=True):
        """Two-pass time-step optimization (Alg.4) in place on x; returns
        (x, best_cost, best_seed, success, (dt_opt, dt_f))."""
        al = (C.c_float * len(alpha))(*alpha)
        lim = self._limits(vmax, amax, jmax)
        bc = torch.empty(b.n_seeds, dtype=torch.float32, device=self.device)
        bs = torch.empty(b.P, dtype=torch.int32, device=self.device)
        ok = torch.empty(b.P, dtype=torch.int32, device=self.device)
        dt = (C.c_float * 2)()
        check(_lib.lib().mg_solve_timestep(self.handle, b.handle, _ptr(q_start), _ptr(goal), _ptr(x),
                                           int(iters1), int(iters2), int(m), len(alpha), al, int(mode),
                                           int(graph_inner), int(bool(use_graph)), *lim, float(dt_min),
                                           _ptr(bc), _ptr(bs), _ptr(ok), dt, _stream()))
        return x, bc, bs, ok, (dt[0], dt[1])

    def mg_set_self_collision(self, pairs):
        """Sphere pairs [n, 2] checked for self-collision (Eq.(9)); empty turns it off."""
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        check(_lib.lib().mg_set_self_collision(self.handle, pr.shape[0],
                                               pr.ctypes.data_as(C.POINTER(C.c_int))))

    def mg_ee_pose(self, q):
        """End-effector poses [rows, n_ee, 7] (xyz + wxyz) of configurations q [rows, D]."""
        rows = int(q.shape[0])
        out = torch.empty((rows, self.robot.n_ee, 7), dtype=torch.float32, device=self.device)
        check(_lib.lib().mg_ee_pose(self.handle, rows, _ptr(q), _ptr(out), _stream()))
        return out

    def mg_time_eval(self, b: Batch, q_start, goal, x, d, alpha, launches=30):
        """Mean microseconds per line-search evaluation launch, timed with
        HIP events around `launches` back-to-back launches."""
        al = (C.c_float * len(alpha))(*alpha)
        us = C.c_float(0.0)
        check(_lib.lib().mg_time_eval(self.handle, b.handle, _ptr(q_start), _ptr(goal), _ptr(x), _ptr(d),
                                      len(alpha), al, int(launches), C.byref(us), _stream()))
        return us.value

    def mg_autotune(self, b: Batch, q_start, goal, x, d, alpha, launches=10):
        """Fix the fastest cuboid-slice layout for this batch; returns it."""
        al = (C.c_float * len(alpha))(*alpha)
        h = C.c_int(0)
        check(_lib.lib().mg_autotune(self.handle, b.handle, _ptr(q_start), _ptr(goal), _ptr(x), _ptr(d),
                                     len(alpha), al, int(launches), C.byref(h), _stream()))
        return h.value

    def mg_particles_seeded(self, b: Batch, q_start, goal, mean, var, n_particles, n_iters, seed, beta=0.0,
                            k_mu=0.9, k_sigma=0.5, costs=False):
        """Particle stage with device-drawn noise (mg_philox_normals); in
        place on mean and var.  Returns (mean, var, costs or None)."""
        out = torch.empty((n_iters, b.n_seeds, n_particles), dtype=torch.float32, device=self.device) \
            if costs else None
        check(_lib.lib().mg_particles_seeded(self.handle, b.handle, _ptr(q_start), _ptr(goal), _ptr(mean),
                                             _ptr(var), int(n_particles), int(n_iters), C.c_ulonglong(seed),
                                             float(beta), float(k_mu), float(k_sigma),
                                             _ptr(out) if costs else None, _stream()))
        return mean, var, out

    def mg_particles(self, b: Batch, q_start, goal, mean, var, eps, beta=0.0, k_mu=0.9,
                     k_sigma=0.5, costs=False):
        """Particle stage in place on mean and var ([rows, D]); eps is
        [n_iters, N, rows, D].  Returns (mean, var, costs [n_iters, seeds, N]
        or None)."""
        n_iters, N = int(eps.shape[0]), int(eps.shape[1])
        out = torch.empty((n_iters, b.n_seeds, N), dtype=torch.float32, device=self.device) if costs else None
        check(_lib.lib().mg_particles(self.handle, b.handle, _ptr(q_start), _ptr(goal), _ptr(mean),
                                      _ptr(var), N, n_iters, _ptr(eps), float(beta), float(k_mu),
                                      float(k_sigma), _ptr(out) if costs else None, _stream()))
        return mean, var, out


def mg_philox_normals(seed, it0, n_iters, n_particles, rows, dof, device="cuda"):
    """Counter-based standard normal draws [n_iters, n_particles, rows, dof]
    of rounds it0.. (the particle stage's device noise)."""
    out = torch.empty((n_iters, n_particles, rows, dof), dtype=torch.float32, device=device)
    check(_lib.lib().mg_philox_normals(C.c_ulonglong(seed), int(it0), int(n_iters), int(n_particles), int(rows),
                                       int(dof), _ptr(out), _stream()))
    return out


def mg_knn(nodes, queries, k):
    """k nearest nodes [m, k] (int32, nearest first, -1 past the node count)
    and their squared distances [m, k] of each query, on the device."""
    n, D = int(nodes.shape[0]), int(nodes.shape[1])
    m = int(queries.shape[0])
    idx = torch.empty((m, k), dtype=torch.int32, device=queries.device)
    d2 = torch.empty((m, k), dtype=torch.float32, device=queries.device)
    check(_lib.lib().mg_knn(D, n, _ptr(nodes) if n else None, m, _ptr(queries), int(k), _ptr(idx), _ptr(d2),
                            _stream()))
    return idx, d2


class MgCost(torch.autograd.Function):
    """Total cost per seed as a differentiable function of the trajectories.

    forward runs the cost-only evaluation; backward runs the hand-written
    adjoint, which recomputes kinematics instead of saving link transforms,
    and scales each seed's rows by the incoming gradient of its cost.
    """

    @staticmethod
    def forward(fctx, q, ctx: Context, b: Batch, q_start, goal):
        cost, _, _ = ctx.mg_cost_grad(b, q_start, goal, q.detach().contiguous(), grad=False,
                                      min_clear=False)
        fctx.mg = (ctx, b, q_start, goal)
        fctx.save_for_backward(q)
        return cost

    @staticmethod
    def backward(fctx, grad_out):
        (q,) = fctx.saved_tensors
        ctx, b, q_start, goal = fctx.mg
        _, g, _ = ctx.mg_cost_grad(b, q_start, goal, q.detach().contiguous(), grad=True,
                                   min_clear=False)
        rows_per_seed = torch.as_tensor(np.repeat(b.horizon, b.seeds), device=q.device)
        scale = torch.repeat_interleave(grad_out, rows_per_seed)
        return g * scale.view(-1, 1).to(g.dtype), None, None, None, None
