"""ctypes declarations of libmg.so (include/mg.h).

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmg.so")

_ip = C.POINTER(C.c_int)
_fp = C.POINTER(C.c_float)
_vp = C.c_void_p

MG_OK = 0
STATUS = {0: "MG_OK", -1: "MG_ERR_ARG", -2: "MG_ERR_SHAPE", -3: "MG_ERR_HIP",
          -4: "MG_ERR_OOM", -5: "MG_ERR_UNSUPPORTED", -6: "MG_ERR_STATE"}

# Every symbol include/mg.h declares.
EXPORTS = ("mg_default_params", "mg_create", "mg_destroy", "mg_set_params", "mg_set_worlds",
           "mg_batch_create", "mg_batch_destroy", "mg_batch_seeds", "mg_batch_rows",
           "mg_cost_grad", "mg_lbfgs_step", "mg_linesearch", "mg_linesearch_eval", "mg_linesearch_noalloc",
           "mg_solve",
           "mg_batch_reserve_particles", "mg_particles", "mg_particles_seeded", "mg_philox_normals",
           "mg_set_timing", "mg_eval_time", "mg_time_eval", "mg_autotune", "mg_batch_set_layout", "mg_batch_set_fusion", "mg_solve_fuses",
           "mg_ee_pose", "mg_set_self_collision", "mg_retime", "mg_solve_timestep", "mg_ik_seeds", "mg_traj_select", "mg_motion_gen",
           "mg_steer", "mg_plan", "mg_plan_batch", "mg_knn", "mg_last_error")


class RobotDesc(C.Structure):
    _fields_ = [("n_links", C.c_int), ("dof", C.c_int), ("n_spheres", C.c_int), ("n_ee", C.c_int),
                ("parent", _ip), ("joint", _ip), ("fixed_tf", _fp), ("sphere_link", _ip),
                ("sphere", _fp), ("ee_link", _ip), ("ee_tf", _fp), ("q_lo", _fp), ("q_hi", _fp)]


class Params(C.Structure):
    _fields_ = [("a0", C.c_float), ("a1", C.c_float), ("a2", C.c_float), ("a3", C.c_float),
                ("a6", C.c_float), ("a7", C.c_float), ("a8", C.c_float), ("a9", C.c_float),
                ("w_bound", C.c_float), ("eta2", C.c_float), ("w_coll", C.c_float),
                ("eta", C.c_float), ("dt", C.c_float), ("vel_all", C.c_int), ("swept", C.c_int),
                ("sweep_steps", C.c_int), ("ls_eta1", C.c_float), ("ls_eta_w", C.c_float),
                ("success_pos", C.c_float), ("success_rot", C.c_float), ("w_self", C.c_float), ("speed", C.c_int)]


class MgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_LIB = None


def lib():
    """Load libmg.so; raise if it is missing (build it first)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2310_17274_amd.build` (no fallback path exists)")
    L = C.CDLL(LIB_PATH)
    L.mg_default_params.argtypes = [C.POINTER(Params)]
    L.mg_default_params.restype = None
    L.mg_create.argtypes = [C.POINTER(RobotDesc), C.POINTER(Params), C.POINTER(_vp)]
    L.mg_destroy.argtypes = [_vp]
    L.mg_destroy.restype = None
    L.mg_set_params.argtypes = [_vp, C.POINTER(Params)]
    L.mg_set_worlds.argtypes = [_vp, C.c_int, _ip, _vp, _vp, _vp]
    L.mg_batch_create.argtypes = [_vp, C.c_int, _ip, _ip, _ip, C.c_int, C.c_int, C.POINTER(_vp)]
    L.mg_batch_destroy.argtypes = [_vp]
    L.mg_batch_destroy.restype = None
    L.mg_batch_seeds.argtypes = [_vp]
    L.mg_batch_rows.argtypes = [_vp]
    L.mg_cost_grad.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.mg_lbfgs_step.argtypes = [_vp, _vp, C.c_int, C.c_int, _vp, _vp, _vp, _vp]
    L.mg_linesearch.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int, _fp, C.c_int,
                                _vp, _vp, _vp, _vp, _vp, _vp]
    L.mg_linesearch_noalloc.argtypes = L.mg_linesearch.argtypes
    L.mg_linesearch_eval.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_int, _fp, _vp, _vp, _vp, _vp, _vp]
    L.mg_solve.argtypes = [_vp, _vp, _vp, _vp, _vp, C.c_int, C.c_int, C.c_int, _fp, C.c_int,
                           C.c_int, C.c_int, _vp, _vp, _vp, _vp]
    L.mg_batch_reserve_particles.argtypes = [_vp, C.c_int]
    L.mg_particles.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_int, C.c_int, _vp, C.c_float,
                               C.c_float, C.c_float, _vp, _vp]
    L.mg_particles_seeded.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_int, C.c_int, C.c_ulonglong, C.c_float,
                                      C.c_float, C.c_float, _vp, _vp]
    L.mg_philox_normals.argtypes = [C.c_ulonglong, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _vp, _vp]
    L.mg_set_timing.argtypes = [_vp, C.c_int]
    L.mg_time_eval.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_int, _fp, C.c_int,
                               C.POINTER(C.c_float), _vp]
    L.mg_batch_set_layout.argtypes = [_vp, C.c_int, C.c_int]
    L.mg_batch_set_fusion.argtypes = [_vp, C.c_int]
    L.mg_solve_fuses.argtypes = [_vp, _vp, C.c_int, C.c_int, _vp]
    L.mg_solve_fuses.restype = C.c_int
    L.mg_ee_pose.argtypes = [_vp, C.c_int, _vp, _vp, _vp]
    L.mg_set_self_collision.argtypes = [_vp, C.c_int, _ip]
    L.mg_autotune.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_int, _fp, C.c_int,
                              C.POINTER(C.c_int), _vp]
    L.mg_eval_time.argtypes = [_vp, C.POINTER(C.c_float), C.POINTER(C.c_int)]
    L.mg_retime.argtypes = [_vp, _vp, _vp, _vp, _fp, _fp, _fp, _vp, _vp, _vp]
    L.mg_plan.argtypes = [_vp, _vp, _fp, _fp, _fp, C.c_float, C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint,
                          C.c_int, _fp, C.POINTER(C.c_int), _vp]
    L.mg_plan_batch.argtypes = [_vp, _vp, C.c_int, _fp, _fp, _fp, C.c_float, C.c_int, C.c_int, C.c_int, C.c_int,
                                C.c_int, C.c_uint, C.c_int, _fp, _ip, _vp]
    L.mg_steer.argtypes = [_vp, _vp, C.c_int, _vp, _vp, C.c_float, C.c_int, _vp, _vp, _vp, _vp]
    L.mg_ik_seeds.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_float, _vp, _vp, _vp]
    L.mg_traj_select.argtypes = [_vp, _vp, _vp, _vp, _vp, _fp, _fp, _fp, C.c_float, C.c_float, _vp, _vp, _vp,
                                 _vp]
    L.mg_motion_gen.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                _fp, C.c_int, _fp, _fp, _fp, C.c_float, C.c_float, C.c_float, C.c_float, _vp, _vp,
                                _vp, _vp, _fp, _vp]
    L.mg_solve_timestep.argtypes = [_vp, _vp, _vp, _vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, _fp,
                                    C.c_int, C.c_int, C.c_int, _fp, _fp, _fp, C.c_float, _vp, _vp, _vp,
                                    _fp, _vp]
    L.mg_knn.argtypes = [C.c_int, C.c_int, _vp, C.c_int, _vp, C.c_int, _vp, _vp, _vp]
    L.mg_last_error.argtypes = []
    L.mg_last_error.restype = C.c_char_p
    for name in ("mg_create", "mg_set_params", "mg_set_worlds", "mg_batch_create", "mg_cost_grad",
                 "mg_lbfgs_step", "mg_linesearch", "mg_linesearch_eval", "mg_linesearch_noalloc", "mg_solve",
                 "mg_batch_seeds", "mg_batch_rows",
                 "mg_batch_reserve_particles", "mg_particles", "mg_particles_seeded", "mg_philox_normals",
                 "mg_set_timing", "mg_eval_time",
                 "mg_time_eval", "mg_autotune", "mg_batch_set_layout", "mg_batch_set_fusion", "mg_ee_pose",
                 "mg_set_self_collision", "mg_retime", "mg_solve_timestep", "mg_ik_seeds",
                 "mg_traj_select", "mg_motion_gen", "mg_steer", "mg_plan", "mg_plan_batch", "mg_knn"):
        getattr(L, name).restype = C.c_int
    _LIB = L
    return L


def check(status: int):
    if status != MG_OK:
        raise MgError(status, lib().mg_last_error().decode())
