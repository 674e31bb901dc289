"""ctypes binding of ``libostrich.so`` (the HIP library behind include/ostrich.h).

Argument marshalling only: every step of the method runs in the library's
kernels.  Device memory and streams come from PyTorch (ROCm build).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "_build", "libostrich.so")

c_int = ctypes.c_int32
c_dbl = ctypes.c_double
c_vp = ctypes.c_void_p
c_size = ctypes.c_size_t

E_ARG, E_HIP, E_WORKSPACE, E_UNSUPPORTED = -1, -2, -3, -4
ST_CONVERGED, ST_BUDGET, ST_NONFINITE, ST_REGULARIZED, ST_OVERFLOW = 1, 2, 4, 8, 16
ST_ADJ_INEXACT, ST_LOSS_BODY = 32, 64
FORWARD, BACKWARD, BOTH = 1, 2, 3
SCHED_FIXED, SCHED_BUCKETED = 0, 1


class OstrichBatch(ctypes.Structure):
    _fields_ = [("n_worlds", c_int), ("body_off", c_vp), ("body_mass", c_vp), ("body_inertia", c_vp),
                ("joint_off", c_vp), ("joint_body", c_vp), ("joint_frame", c_vp), ("joint_act", c_vp),
                ("joint_kp", c_vp), ("ctrl_off", c_vp), ("slot_off", c_vp), ("slot_int", c_vp),
                ("slot_real", c_vp), ("obs_off", c_vp), ("obs_box", c_vp), ("lam_off", c_vp),
                ("contact_cap", c_vp), ("world_hmap", c_vp), ("hmap_n", c_int), ("hmap_spacing", c_dbl),
                ("hmap_origin", c_vp), ("hmap_heights", c_vp), ("joint_kd", c_vp)]


class OstrichParams(ctypes.Structure):
    _fields_ = [("h", c_dbl), ("gravity", c_dbl * 3), ("tol", c_dbl), ("k_max", c_int), ("k_min", c_int),
                ("eps", c_dbl), ("delta_g", c_dbl), ("delta_reg", c_dbl), ("delta0", c_dbl),
                ("ls_max", c_int), ("refine", c_int), ("team", c_int), ("schedule", c_int),
                ("truncate", c_int), ("linear_solver", c_int), ("krylov_iters", c_int),
                ("tier_contacts", c_int), ("delta_reg_adj", c_dbl)]


class OstrichLoss(ctypes.Structure):
    _fields_ = [("w_pos", c_dbl), ("w_head", c_dbl), ("w_vel", c_dbl), ("w_ctrl", c_dbl), ("w_track", c_dbl),
                ("w_yaw", c_dbl), ("goal", c_vp), ("ref", c_vp)]


BATCH_ARRAYS = ("body_off", "body_mass", "body_inertia", "joint_off", "joint_body", "joint_frame", "joint_act",
                "joint_kp", "ctrl_off", "slot_off", "slot_int", "slot_real", "obs_off", "obs_box", "lam_off",
                "contact_cap", "world_hmap", "hmap_origin", "hmap_heights", "joint_kd")

_lib = None


class OstrichCopySeg(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("n", ctypes.c_int64)]


class OstrichError(RuntimeError):
    pass


def load() -> ctypes.CDLL:
    """Load the built library; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise OstrichError("libostrich.so is not built (run __graft_entry__.build()); no fallback exists")
    L = ctypes.CDLL(SO_PATH)
    L.ostrich_last_error.restype = ctypes.c_char_p
    L.ostrich_ctx_create.argtypes = [ctypes.POINTER(OstrichBatch), ctypes.POINTER(OstrichParams),
                                     ctypes.POINTER(c_vp)]
    L.ostrich_ctx_create.restype = c_int
    L.ostrich_ctx_destroy.argtypes = [c_vp]
    L.ostrich_ctx_destroy.restype = c_int
    L.ostrich_ctx_caps.argtypes = [c_vp, ctypes.POINTER(ctypes.c_int64)]
    L.ostrich_ctx_caps.restype = c_int
    L.ostrich_tape_bytes.argtypes = [c_vp]
    L.ostrich_tape_bytes.restype = c_size
    L.ostrich_ctx_device_bytes.argtypes = [c_vp]
    L.ostrich_ctx_device_bytes.restype = c_size
    L.ostrich_rollout_workspace_bytes.argtypes = [c_vp, c_int, c_int]
    L.ostrich_rollout_workspace_bytes.restype = c_size
    L.ostrich_step_forward.argtypes = [c_vp] + [c_vp] * 13 + [c_vp]
    L.ostrich_step_forward.restype = c_int
    L.ostrich_step_forward_noalloc.argtypes = [c_vp] + [c_vp] * 13 + [c_vp]
    L.ostrich_step_forward_noalloc.restype = c_int
    L.ostrich_step_adjoint.argtypes = [c_vp] + [c_vp] * 11 + [c_int, c_vp, c_vp]
    L.ostrich_step_adjoint.restype = c_int
    L.ostrich_step_adjoint_params.argtypes = [c_vp] + [c_vp] * 14 + [c_int, c_vp, c_vp]
    L.ostrich_step_adjoint_params.restype = c_int
    L.ostrich_rollout.argtypes = ([c_vp, c_int, c_vp, c_vp, c_vp, c_int, c_vp, c_int, c_int, c_vp, c_vp, c_vp,
                                   c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_size, c_vp, c_vp])
    L.ostrich_rollout.restype = c_int
    L.ostrich_rollout_shaped.argtypes = ([c_vp, c_int, c_vp, c_vp, c_vp, c_int, c_vp, c_int, c_int, c_vp,
                                          ctypes.POINTER(OstrichLoss), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                          c_vp, c_size, c_vp, c_vp])
    L.ostrich_rollout_shaped.restype = c_int
    L.ostrich_ctx_schedule.argtypes = [c_vp, c_vp, c_int]
    L.ostrich_ctx_schedule.restype = c_int
    L.ostrich_ctx_timing.argtypes = [c_vp, c_int, c_vp]
    L.ostrich_ctx_timing.restype = c_int
    L.ostrich_autotune.argtypes = [c_vp, c_vp, c_vp, c_vp, c_vp, c_int, c_vp]
    L.ostrich_autotune.restype = c_int
    L.ostrich_step_forward_list.argtypes = [c_vp, c_vp, c_int] + [c_vp] * 13 + [c_vp]
    L.ostrich_step_forward_list.restype = c_int
    L.ostrich_step_adjoint_list.argtypes = [c_vp, c_vp, c_int] + [c_vp] * 11 + [c_int, c_vp, c_vp]
    L.ostrich_step_adjoint_list.restype = c_int
    L.ostrich_step_forward_plain.argtypes = [c_vp] + [c_vp] * 13 + [c_vp]
    L.ostrich_step_forward_plain.restype = c_int
    L.ostrich_step_adjoint_plain.argtypes = [c_vp] + [c_vp] * 11 + [c_int, c_vp, c_vp]
    L.ostrich_step_adjoint_plain.restype = c_int
    L.ostrich_spline_controls.argtypes = [c_vp, c_vp, c_int, c_int, c_int, c_vp, c_vp]
    L.ostrich_spline_controls.restype = c_int
    L.ostrich_final_loss.argtypes = [c_vp, c_int, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]
    L.ostrich_final_loss.restype = c_int
    L.ostrich_knot_grad_accumulate.argtypes = [c_vp, c_vp, c_int, c_int, c_int, c_vp, c_vp]
    L.ostrich_knot_grad_accumulate.restype = c_int
    L.ostrich_adam.argtypes = [c_vp, c_vp, c_vp, c_vp, ctypes.c_int64, c_dbl, c_dbl, c_dbl, c_dbl, c_int, c_vp]
    L.ostrich_adam.restype = c_int
    L.ostrich_copy_segments.argtypes = [c_vp, c_int, c_vp]
    L.ostrich_copy_segments.restype = c_int
    L.ostrich_spline_basis.argtypes = [c_int, c_int, c_dbl, c_vp]
    L.ostrich_spline_basis.restype = c_int
    _lib = L
    return L


def check(rc: int, what: str):
    if rc != 0:
        msg = load().ostrich_last_error().decode(errors="replace")
        raise OstrichError(f"{what} failed ({rc}): {msg}")


def make_params(p: dict, team: int = 0, schedule: int = SCHED_BUCKETED) -> OstrichParams:
    cp = OstrichParams()
    cp.h = float(p["h"])
    for k in range(3):
        cp.gravity[k] = float(p["gravity"][k])
    cp.tol = float(p["tol"])
    cp.k_max = int(p["k_max"])
    cp.k_min = int(p["k_min"])
    cp.eps = float(p["eps"])
    cp.delta_g = float(p["delta_g"])
    cp.delta_reg = float(p["delta_reg"])
    cp.delta0 = float(p["delta0"])
    cp.ls_max = int(p.get("ls_max", 0))
    cp.refine = int(p.get("refine", 8))
    cp.team = int(team)
    cp.schedule = int(schedule)
    cp.truncate = int(p.get("truncate", 0))
    cp.linear_solver = int(p.get("linear_solver", 0))
    cp.krylov_iters = int(p.get("krylov_iters", 16))
    cp.tier_contacts = int(p.get("tier_contacts", 0))
    cp.delta_reg_adj = float(p.get("delta_reg_adj", p["delta_reg"]))
    return cp


def make_batch(n_worlds: int, ptrs: dict, hmap_n: int = 0, hmap_spacing: float = 0.0) -> OstrichBatch:
    cb = OstrichBatch()
    cb.n_worlds = int(n_worlds)
    for k in BATCH_ARRAYS:
        setattr(cb, k, ptrs.get(k))
    cb.hmap_n = int(hmap_n)
    cb.hmap_spacing = float(hmap_spacing)
    return cb
