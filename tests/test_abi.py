"""Host-side checks of the C ABI (no GPU needed): the library builds, loads,
exports every symbol include/mg.h declares, and rejects bad arguments before
touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2310_17274_amd import _lib, build
from paper_2310_17274_amd import workloads as wl

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mg.h")


@pytest.fixture(scope="module")
def L():
    if build.is_stale():
        build.build()
    return _lib.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("mg_cost_grad", "mg_lbfgs_step", "mg_linesearch", "mg_solve"):
        assert n in names
    assert sorted(_lib.EXPORTS) == names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_default_params_are_the_papers(L):
    import json
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
    p = _lib.Params()
    L.mg_default_params(C.byref(p))
    assert (p.a0, p.a1, p.a2, p.a3) == tuple(g["pose_weights"][k] for k in ("a0", "a1", "a2", "a3"))
    assert (p.a6, p.a7, p.a8, p.a9) == tuple(g["smooth_weights"][k] for k in ("a6", "a7", "a8", "a9"))
    assert p.w_bound == p.w_coll == g["soft_constraint_weight"]["w"]
    assert p.eta == pytest.approx(g["activation_distance"]["eta"])
    assert p.eta2 == pytest.approx(g["bound_band"]["eta2"])
    assert p.dt == pytest.approx(g["first_pass_dt"]["dt"])


def _desc(robot, keep):
    def fa(a):
        a = np.ascontiguousarray(a, dtype=np.float32); keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_float))

    def ia(a):
        a = np.ascontiguousarray(a, dtype=np.int32); keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_int))
    return _lib.RobotDesc(n_links=robot.n_links, dof=robot.dof, n_spheres=robot.n_spheres,
                          n_ee=robot.n_ee, parent=ia(robot.parent), joint=ia(robot.joint),
                          fixed_tf=fa(robot.fixed_tf), sphere_link=ia(robot.sphere_link),
                          sphere=fa(robot.sphere), ee_link=ia(robot.ee_link), ee_tf=fa(robot.ee_tf),
                          q_lo=fa(robot.q_lo), q_hi=fa(robot.q_hi))


@pytest.mark.parametrize("mutate,status", [
    (lambda r: setattr(r, "parent", np.array([-1, 5, 1, 2, 3, 4, 5], np.int32)), -1),
    (lambda r: setattr(r, "joint", np.array([0, 0, 1, 2, 3, 4, 5], np.int32)), -1),
    (lambda r: r.sphere.__setitem__((0, 3), -0.1), -1),
    (lambda r: setattr(r, "ee_link", np.array([9], np.int32)), -1),
    (lambda r: setattr(r, "q_lo", np.full(7, 3.0)), -1),
])
def test_create_rejects_bad_robots(L, mutate, status):
    robot = wl.make_arm(seed=0, n_spheres=10)
    mutate(robot)
    keep = []
    d = _desc(robot, keep)
    p = _lib.Params()
    L.mg_default_params(C.byref(p))
    h = C.c_void_p()
    assert L.mg_create(C.byref(d), C.byref(p), C.byref(h)) == status
    assert h.value is None
    assert len(L.mg_last_error()) > 0


def test_create_rejects_bad_params(L):
    robot = wl.make_arm(seed=0, n_spheres=10)
    keep = []
    d = _desc(robot, keep)
    p = _lib.Params()
    L.mg_default_params(C.byref(p))
    p.dt = 0.0
    h = C.c_void_p()
    assert L.mg_create(C.byref(d), C.byref(p), C.byref(h)) == -1
    assert L.mg_create(None, C.byref(p), C.byref(h)) == -1
