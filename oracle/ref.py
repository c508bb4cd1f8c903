"""ctypes wrapper of the FP64 CPU reference (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It converts the seeded workload description into the
reference's plain double arrays and calls ``libmgref.so``.  The plain
definitions at the end (seed ranking, linear seeds, trajectory choice,
steering) are pinned by worked tables; the blend weights of the choice have
no paper values (parity unpinned beyond those tables).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import build as _build

_LIB = None

DEFAULTS = dict(
    # Eq.(14) pose weights (appendix 'Pose Reaching Cost')
    a0=2000.0, a1=350.0, a2=100.0, a3=100.0,
    # Eq.(16) smoothness weights (appendix 'Path-Length Minimization & Smoothness Costs')
    a6=5000.0, a7=50.0, a8=5000.0, a9=1.0,
    # Eq.(17): weight 5000 for every soft constraint (appendix 'cuRobo Parameters'), band 0.1
    w_bound=5000.0, eta2=0.1,
    # Eq.(10)/(11): activation distance 2.5 cm, weight 5000 (appendix 'cuRobo Parameters')
    w_coll=5000.0, eta=0.025,
    # first-pass time step of the dt re-optimisation (appendix 'Time-step Descretization and Temporal Weight Scaling')
    dt=0.25,
    vel_all=0, swept=0, sweep_steps=4,
    # Eq.(9) self-collision: weight 5000 like every soft constraint; the
    # checked sphere pairs are a robot property (none by default)
    w_self=5000.0, n_self=0,
    # Eq.(11) speed metric, off unless asked for
    speed=0,
)
# Line search constants (Reading: the Nocedal & Wright defaults).
ETA1 = 1e-4
ETA_W = 0.9

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Robot(C.Structure):
    _fields_ = [("n_links", C.c_int), ("dof", C.c_int), ("parent", _ip), ("joint", _ip),
                ("fixed_tf", _dp), ("n_spheres", C.c_int), ("sphere_link", _ip),
                ("sphere", _dp), ("n_ee", C.c_int), ("ee_link", _ip), ("ee_tf", _dp),
                ("q_lo", _dp), ("q_hi", _dp)]


class _Params(C.Structure):
    _fields_ = [("a0", C.c_double), ("a1", C.c_double), ("a2", C.c_double), ("a3", C.c_double),
                ("a6", C.c_double), ("a7", C.c_double), ("a8", C.c_double), ("a9", C.c_double),
                ("w_bound", C.c_double), ("eta2", C.c_double), ("w_coll", C.c_double),
                ("eta", C.c_double), ("dt", C.c_double), ("vel_all", C.c_int),
                ("swept", C.c_int), ("sweep_steps", C.c_int), ("w_self", C.c_double),
                ("n_self", C.c_int), ("self_pairs", _ip), ("speed", C.c_int)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.environ.get("MGREF_LIB") or _build.ensure()
        L = C.CDLL(path)
        L.mgref_traj_cost.restype = C.c_double
        L.mgref_box_sdf.restype = C.c_double
        L.mgref_dc.restype = C.c_double
        L.mgref_bound.restype = C.c_double
        L.mgref_ls_select.restype = C.c_int
        L.mgref_linesearch.restype = C.c_int
        L.mgref_retime.restype = C.c_double
        L.mgref_philox_normal.restype = C.c_double
        L.mgref_philox_normal.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_int64]
        _LIB = L
    return _LIB


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


class Ref:
    """Reference evaluator bound to one robot and one parameter set."""

    def __init__(self, robot, **params):
        p = dict(DEFAULTS)
        p.update(params)
        self.params = p
        self._keep = []
        def keep(x):
            self._keep.append(x[0])
            return x[1]
        self.robot = robot
        self._rb = _Robot(n_links=robot.n_links, dof=robot.dof,
                          parent=keep(_i(robot.parent)), joint=keep(_i(robot.joint)),
                          fixed_tf=keep(_d(robot.fixed_tf)), n_spheres=robot.n_spheres,
                          sphere_link=keep(_i(robot.sphere_link)), sphere=keep(_d(robot.sphere)),
                          n_ee=robot.n_ee, ee_link=keep(_i(robot.ee_link)),
                          ee_tf=keep(_d(robot.ee_tf)), q_lo=keep(_d(robot.q_lo)),
                          q_hi=keep(_d(robot.q_hi)))
        pairs = p.pop("self_pairs", None)
        self.params = dict(p, self_pairs=pairs)
        if pairs is not None and len(pairs):
            pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
            p["n_self"] = pairs.shape[0]
            p["self_pairs"] = keep(_i(pairs))
        self._pr = _Params(**p)

    # -- kinematics and geometry ---------------------------------------
    def fk(self, q):
        rb = self.robot
        q, qp = _d(q)
        tf = np.zeros((rb.n_links, 12)); sp = np.zeros((rb.n_spheres, 3)); ee = np.zeros((rb.n_ee, 7))
        lib().mgref_fk(C.byref(self._rb), qp, _d(tf)[1], _d(sp)[1], _d(ee)[1])
        return tf, sp, ee

    def pose_error(self, qT, goal):
        pe = np.zeros(self.robot.n_ee); re = np.zeros(self.robot.n_ee)
        g, gp = _d(goal)
        q, qp = _d(qT)
        lib().mgref_pose_error(C.byref(self._rb), qp, gp, _d(pe)[1], _d(re)[1])
        return pe, re

    # -- costs -----------------------------------------------------------
    def traj_cost(self, boxes, q0, goal, q, grad=True):
        """Cost, gradient [T,D] (or None), min clearance, terms[5]
        (smoothness, joint limits, world collision, pose, self-collision)."""
        pose, dims = boxes
        pose, pp = _d(np.asarray(pose).reshape(-1, 7)); dims, dp = _d(np.asarray(dims).reshape(-1, 3))
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, self.robot.dof)
        T = q.shape[0]
        g = np.zeros_like(q) if grad else None
        mc = C.c_double(0.0)
        terms = np.zeros(5)
        q0a, q0p = _d(q0)
        ga, gp_ = _d(goal)
        c = lib().mgref_traj_cost(C.byref(self._rb), C.byref(self._pr), pose.shape[0], pp, dp,
                                  q0p, gp_, T, _d(q)[1], _d(g)[1] if grad else None,
                                  C.byref(mc), _d(terms)[1])
        return c, g, mc.value, terms

    def cost_grad_batch(self, boxes, q0, goal, T, q, nthreads=1, grad=True):
        pose, dims = boxes
        pose, pp = _d(np.asarray(pose).reshape(-1, 7)); dims, dp = _d(np.asarray(dims).reshape(-1, 3))
        q = np.ascontiguousarray(q, dtype=np.float64)
        S = q.size // (T * self.robot.dof)
        cost = np.zeros(S); mc = np.zeros(S)
        g = np.zeros_like(q) if grad else None
        lib().mgref_cost_grad_batch(C.byref(self._rb), C.byref(self._pr), pose.shape[0], pp, dp,
                                    _d(q0)[1], _d(goal)[1], T, S, _d(q)[1], _d(cost)[1],
                                    _d(g)[1] if grad else None, _d(mc)[1], int(nthreads))
        return cost, g, mc

    # -- solver pieces -----------------------------------------------------
    def linesearch(self, boxes, q0, goal, x, c0, g0, d, alpha, mode=1, eta1=ETA1, eta_w=ETA_W):
        pose, dims = boxes
        pose, pp = _d(np.asarray(pose).reshape(-1, 7)); dims, dp = _d(np.asarray(dims).reshape(-1, 3))
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, self.robot.dof)
        T = x.shape[0]
        xo = np.zeros_like(x); go = np.zeros_like(x)
        co = C.c_double(0.0); mco = C.c_double(0.0)
        al = np.asarray(alpha, dtype=np.float64)
        i = lib().mgref_linesearch(C.byref(self._rb), C.byref(self._pr), pose.shape[0], pp, dp,
                                   _d(q0)[1], _d(goal)[1], T, _d(x)[1], C.c_double(c0),
                                   _d(g0)[1], _d(d)[1], len(al), _d(al)[1], int(mode),
                                   C.c_double(eta1), C.c_double(eta_w), _d(xo)[1],
                                   C.byref(co), _d(go)[1], C.byref(mco))
        return i, xo, co.value, go, mco.value

    def solve(self, boxes, q0, goal, T, x, iters, m, alpha, mode=1, eta1=ETA1, eta_w=ETA_W,
              nthreads=1, trace=False):
        pose, dims = boxes
        pose, pp = _d(np.asarray(pose).reshape(-1, 7)); dims, dp = _d(np.asarray(dims).reshape(-1, 3))
        x = np.array(x, dtype=np.float64, copy=True)
        S = x.size // (T * self.robot.dof)
        best = np.zeros(S)
        tr = np.zeros((iters, S)) if trace else None
        al = np.asarray(alpha, dtype=np.float64)
        lib().mgref_solve(C.byref(self._rb), C.byref(self._pr), pose.shape[0], pp, dp,
                          _d(q0)[1], _d(goal)[1], T, S, x.ctypes.data_as(_dp), iters, m, len(al),
                          _d(al)[1], int(mode), C.c_double(eta1), C.c_double(eta_w),
                          _d(best)[1], _d(tr)[1] if trace else None, int(nthreads))
        return x, best, tr

    def particles(self, boxes, q0, goal, T, mu, var, eps, beta=None, k_mu=None, k_sigma=None,
                  nthreads=1):
        """Particle stage of one problem: mu, var [S,T,D] in; eps
        [n_iters, N, S, T, D].  Returns (mu', var', costs [n_iters, S, N])."""
        pd = dict(PARTICLE_DEFAULTS)
        pd.update({k: v for k, v in dict(beta=beta, k_mu=k_mu, k_sigma=k_sigma).items() if v is not None})
        pose, dims = boxes
        pose, pp = _d(np.asarray(pose).reshape(-1, 7)); dims, dp = _d(np.asarray(dims).reshape(-1, 3))
        mu = np.array(mu, dtype=np.float64, copy=True)
        var = np.array(var, dtype=np.float64, copy=True)
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        n_iters, N = eps.shape[0], eps.shape[1]
        S = mu.size // (T * self.robot.dof)
        assert eps.size == n_iters * N * S * T * self.robot.dof
        costs = np.zeros((n_iters, S, N))
        lib().mgref_particles(C.byref(self._rb), C.byref(self._pr), pose.shape[0], pp, dp,
                              _d(q0)[1], _d(goal)[1], T, S, mu.ctypes.data_as(_dp),
                              var.ctypes.data_as(_dp), N, n_iters, eps.ctypes.data_as(_dp),
                              C.c_double(pd["beta"]), C.c_double(pd["k_mu"]),
                              C.c_double(pd["k_sigma"]), costs.ctypes.data_as(_dp), int(nthreads))
        return mu, var, costs


def timestep_params(params, dt_opt):
    """Second-pass parameters of Alg.4 (App. 'Time-step Descretization and
    Temporal Weight Scaling'): spacing dt_opt and, with rho = dt_opt / dt,
    the derivative weights a7 rho, a8 rho^4, a9 rho^6.  Reading: 'scale the
    weights by the new dt' keeps the cost of the same waypoints unchanged,
    since velocity, acceleration and jerk scale as rho^-1, rho^-2, rho^-3."""
    p = dict(DEFAULTS)
    p.update(params)
    rho = dt_opt / p["dt"]
    out = dict(params)
    out.update(dt=dt_opt, a7=p["a7"] * rho, a8=p["a8"] * rho ** 4, a9=p["a9"] * rho ** 6)
    return out


def solve_timestep(robot, problems, iters1, iters2, m, alpha, vmax, amax, jmax, dt_min, mode=1,
                   nthreads=1, **params):
    """Time-step optimization (Alg.4) of a batch of problems sharing one
    spacing, in the paper's order: (1) a solve at the first spacing dt with
    the jerk term off (a9 = 0); (2) dt_opt = the largest retime of the
    problems' best seeds (lowest index on ties), at least dt_min; (3) the
    derivative weights rescaled to dt_opt (timestep_params), jerk on; (4) a
    solve from the first pass's best iterates; (5) dt_f = the largest
    retime of the new best seeds.
    problems: list of (boxes, q0, goal, T, x [S*T*D]).  Returns (x per
    problem, best costs per problem, (dt_opt, dt_f))."""
    D = robot.dof
    p = dict(DEFAULTS)
    p.update(params)
    r1 = Ref(robot, **dict(params, a9=0.0))
    first = [r1.solve(b, q0, g, T, x, iters1, m, alpha, mode=mode, nthreads=nthreads)[:2]
             for b, q0, g, T, x in problems]

    def largest_retime(results, dt):
        out = 0.0
        for (b, q0, g, T, _), (x, best) in zip(problems, results):
            s = int(np.argmin(best))
            out = max(out, retime(q0, x.reshape(-1, T, D)[s], dt, vmax, amax, jmax))
        return max(out, dt_min)

    dt_opt = largest_retime(first, p["dt"])
    r2 = Ref(robot, **timestep_params(params, dt_opt))
    second = [r2.solve(b, q0, g, T, x1, iters2, m, alpha, mode=mode, nthreads=nthreads)[:2]
              for (b, q0, g, T, _), (x1, _) in zip(problems, first)]
    dt_f = largest_retime(second, dt_opt)
    return [x for x, _ in second], [c for _, c in second], (dt_opt, dt_f)


def knn(nodes, queries, k):
    """Brute-force k nearest nodes of each query (the planner's neighbour
    search, Alg.2): squared distances summed joint by joint in fp32 with every
    product and sum rounded, order by (distance, node index).  Returns
    (idx [m, k], d2 [m, k]), -1 / inf past the node count."""
    nodes = np.asarray(nodes, dtype=np.float32)
    queries = np.asarray(queries, dtype=np.float32)
    n, D = nodes.shape if nodes.size else (0, queries.shape[1])
    m = queries.shape[0]
    idx = np.full((m, k), -1, dtype=np.int64)
    d2o = np.full((m, k), np.inf, dtype=np.float32)
    for qi in range(m):
        d2 = np.zeros(n, dtype=np.float32)
        for j in range(D):
            u = (nodes[:, j] - queries[qi, j]).astype(np.float32)
            d2 = (d2 + (u * u).astype(np.float32)).astype(np.float32)
        order = np.lexsort((np.arange(n), d2))[:k]
        idx[qi, :order.size] = order
        d2o[qi, :order.size] = d2[order]
    return idx, d2o


def philox4x64(ctr, key):
    """Philox-4x64-10 of one counter block: four 64-bit words."""
    c = (C.c_uint64 * 4)(*[int(v) & ((1 << 64) - 1) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) & ((1 << 64) - 1) for v in key])
    o = (C.c_uint64 * 4)()
    lib().mgref_philox4x64(c, k, o)
    return [int(v) for v in o]


def philox_normals(seed, n_iters, N, rows, D):
    """Counter-based standard normal draws [n_iters, N, rows, D] of the
    particle stage (Philox-4x64-10 + Box-Muller, mgref.h)."""
    out = np.zeros((n_iters, N, rows, D))
    lib().mgref_philox_normals(C.c_uint64(seed), int(n_iters), int(N), int(rows), int(D),
                               out.ctypes.data_as(_dp))
    return out


# Particle stage constants.  The paper gives none of them (Alg.5 takes sigma0
# as an input); these are the documented builder choices: initial per-element
# variance 0.05^2 rad^2, adaptive temperature (beta <= 0: 0.1 x cost range),
# mean and variance step sizes 0.9 and 0.5.
PARTICLE_DEFAULTS = dict(sigma0=0.05 ** 2, beta=0.0, k_mu=0.9, k_sigma=0.5)


# -- standalone helpers (no robot needed) -----------------------------------

def particle_update(cost, theta, mu, var, beta=0.0, k_mu=0.9, k_sigma=0.5):
    """One Eq.(12)-(13) update: cost [N], theta [N, n], mu, var [n].
    Returns (mu', var', w)."""
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    N, n = theta.shape
    mu = np.array(mu, dtype=np.float64, copy=True).reshape(n)
    var = np.array(var, dtype=np.float64, copy=True).reshape(n)
    w = np.zeros(N)
    lib().mgref_particle_update(n, N, _d(cost)[1], _d(theta)[1], mu.ctypes.data_as(_dp),
                                var.ctypes.data_as(_dp), C.c_double(beta), C.c_double(k_mu),
                                C.c_double(k_sigma), w.ctypes.data_as(_dp))
    return mu, var, w


def box_sdf(pose, dims, c):
    g = np.zeros(3)
    v = lib().mgref_box_sdf(_d(pose)[1], _d(dims)[1], _d(c)[1], _d(g)[1])
    return v, g


def dc(d, eta):
    s = C.c_double(0.0)
    return lib().mgref_dc(C.c_double(d), C.c_double(eta), C.byref(s)), s.value


def bound(x, lo, hi, eta2):
    s = C.c_double(0.0)
    return lib().mgref_bound(C.c_double(x), C.c_double(lo), C.c_double(hi), C.c_double(eta2),
                             C.byref(s)), s.value


def mat_to_quat(R):
    q = np.zeros(4)
    lib().mgref_mat_to_quat(_d(np.asarray(R, dtype=np.float64).reshape(9))[1], _d(q)[1])
    return q


def derivatives(q0, q, dt):
    q = np.ascontiguousarray(q, dtype=np.float64)
    T, D = q.shape
    v = np.zeros((T + 1, D)); a = np.zeros((T + 1, D)); j = np.zeros((T + 1, D))
    lib().mgref_derivatives(T, D, _d(q0)[1], _d(q)[1], C.c_double(dt), _d(v)[1], _d(a)[1], _d(j)[1])
    return v, a, j


def retime(q0, q, dt, vmax, amax, jmax):
    """Alg.4 retime of one trajectory q [T, D] with start q0 at spacing dt."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    T, D = q.shape
    q0, vmax, amax, jmax = (_d(np.broadcast_to(np.asarray(z, dtype=np.float64), (D,)).copy())
                            for z in (q0, vmax, amax, jmax))
    return lib().mgref_retime(T, D, q0[1], _d(q)[1], C.c_double(dt), vmax[1], amax[1], jmax[1])


def lbfgs_step(n, m, reset, state, x, g):
    """state: dict with count, head, S, Y, rho, x_prev, g_prev (mutated)."""
    cnt = C.c_int(state["count"]); hd = C.c_int(state["head"])
    d = np.zeros(n)
    lib().mgref_lbfgs_step(n, m, int(reset), C.byref(cnt), C.byref(hd),
                           state["S"].ctypes.data_as(_dp), state["Y"].ctypes.data_as(_dp),
                           state["rho"].ctypes.data_as(_dp), state["x_prev"].ctypes.data_as(_dp),
                           state["g_prev"].ctypes.data_as(_dp), _d(x)[1], _d(g)[1], _d(d)[1])
    state["count"], state["head"] = cnt.value, hd.value
    return d


def new_lbfgs_state(n, m):
    mm = max(m, 1)
    return dict(count=0, head=0, S=np.zeros((mm, n)), Y=np.zeros((mm, n)), rho=np.zeros(mm),
                x_prev=np.zeros(n), g_prev=np.zeros(n))


def ls_select(alpha, c0, g0d, c, gd, mode, eta1=ETA1, eta_w=ETA_W):
    al = np.asarray(alpha, dtype=np.float64)
    return lib().mgref_ls_select(len(al), _d(al)[1], C.c_double(c0), C.c_double(g0d),
                                 _d(c)[1], _d(gd)[1], int(mode), C.c_double(eta1),
                                 C.c_double(eta_w))


# ---------------------------------------------------------------------------
# Motion generation around the solver (Sec. 'Global Motion Generation'
# overview, App. 'Evaluating Optimized Trajectories').  Plain definitions.

def max_jerk(q0, q, dt):
    """Largest |jerk| over t = 0..T and the joints at spacing dt."""
    return float(np.abs(derivatives(q0, q, dt)[2]).max())


def ik_rank(q, q0, pos_err, rot_err, clear, cost, pos_tol, rot_tol, w_dist):
    """IK seeds of one problem: the valid ones (within the success
    tolerances and collision free) in increasing pos_err + rot_err +
    w_dist |q - q0|, ties to the lower index.  With none valid, every seed
    in increasing cost.  A NaN key counts as +inf.  Returns (order, number
    valid)."""
    S = len(pos_err)
    valid = [pos_err[s] <= pos_tol and rot_err[s] <= rot_tol and clear[s] >= 0 for s in range(S)]
    if any(valid):
        key = {s: pos_err[s] + rot_err[s] + w_dist * float(np.linalg.norm(np.asarray(q[s]) - np.asarray(q0)))
               for s in range(S) if valid[s]}
    else:
        key = {s: cost[s] for s in range(S)}
    # a NaN key ranks last (the order stays total)
    key = {s: (math.inf if math.isnan(v) else v) for s, v in key.items()}
    order = sorted(key, key=lambda s: (key[s], s))
    return order, sum(valid)


def linear_seeds(q0, q_goal, T):
    """Waypoints t = 1..T on the line from q0 to q_goal: q0 + t/T (q_goal - q0)."""
    q0, q_goal = np.asarray(q0, dtype=np.float64), np.asarray(q_goal, dtype=np.float64)
    return np.array([q0 + (t / T) * (q_goal - q0) for t in range(1, T + 1)])


def traj_select(T, pos_err, rot_err, clear, cost, jerk, dt, pos_tol, rot_tol, w_jerk, w_time):
    """Trajectory seeds of one problem: among the valid ones (goal reached
    within the tolerances, collision free), the lowest pos_err + rot_err +
    w_jerk jerk + w_time T dt (the motion time: T intervals from the start
    at t = 0 to waypoint T), ties to the lower index; with none
    valid, the lowest cost.  Returns (seed, valid)."""
    S = len(pos_err)
    valid = [pos_err[s] <= pos_tol and rot_err[s] <= rot_tol and clear[s] >= 0 for s in range(S)]
    if any(valid):
        score = [pos_err[s] + rot_err[s] + w_jerk * jerk[s] + w_time * T * dt[s] if valid[s] else math.inf
                 for s in range(S)]
        return int(np.argmin(score)), True
    return int(np.argmin(cost)), False


def steer(r_eval, boxes, q_from, q_to, res, q_lo, q_hi):
    """Parallel steering of one edge (Alg.3): n = floor(max_j |g_j| / res) + 1
    steps of g / n from q_from toward q_to (g = q_to - q_from); samples
    l_i = q_from + (i / n) g, i = 0..n, are valid when within the joint
    limits and collision free (clearance >= 0 against the cuboids).  The
    edge keeps the last valid sample before the first invalid one: returns
    (h, l_h, |l_h - q_from|) with h = n when every sample is valid and
    h = -1 (no progress: q_from, 0) when q_from itself is invalid."""
    q_from, q_to = np.asarray(q_from, dtype=np.float64), np.asarray(q_to, dtype=np.float64)
    g = q_to - q_from
    n = int(math.floor(np.abs(g).max() / res)) + 1
    goal = np.array([[0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0]] * r_eval.robot.n_ee)
    h = n
    for i in range(n + 1):
        q = q_from + (i / n) * g
        inside = np.all(q >= q_lo) and np.all(q <= q_hi)
        clear = r_eval.traj_cost(boxes, q, goal, q[None], grad=False)[2]
        if not (inside and clear >= 0):
            h = i - 1
            break
    if h < 0:
        return -1, q_from.copy(), 0.0
    v = q_from + (h / n) * g
    return h, v, float(np.linalg.norm(v - q_from))
