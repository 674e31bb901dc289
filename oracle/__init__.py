"""CPU oracle (test infrastructure): ctypes binding of ``libostrich_ref.so``.

Only tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package.  It never imports the GPU package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "libostrich_ref.so")
_lib = None

c_int = ctypes.c_int32
c_dbl_p = ctypes.POINTER(ctypes.c_double)
c_int_p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (-O2, no fast-math)."""
    os.makedirs(os.path.join(_HERE, "_build"), exist_ok=True)
    src = os.path.join(_HERE, "ostrich_ref.cpp")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


class Batch(ctypes.Structure):
    _fields_ = [("n_worlds", c_int), ("body_off", c_int_p), ("body_mass", c_dbl_p),
                ("body_inertia", c_dbl_p), ("joint_off", c_int_p), ("joint_body", c_int_p),
                ("joint_frame", c_dbl_p), ("joint_act", c_int_p), ("joint_kp", c_dbl_p),
                ("ctrl_off", c_int_p), ("slot_off", c_int_p), ("slot_int", c_int_p),
                ("slot_real", c_dbl_p), ("obs_off", c_int_p), ("obs_box", c_dbl_p),
                ("lam_off", c_int_p), ("contact_cap", c_int_p), ("world_hmap", c_int_p),
                ("hmap_n", c_int), ("hmap_spacing", ctypes.c_double), ("hmap_origin", c_dbl_p),
                ("hmap_heights", c_dbl_p), ("joint_kd", c_dbl_p)]


class Params(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("gravity", ctypes.c_double * 3), ("tol", ctypes.c_double),
                ("k_max", c_int), ("k_min", c_int), ("eps", ctypes.c_double),
                ("delta_g", ctypes.c_double), ("delta_reg", ctypes.c_double),
                ("delta0", ctypes.c_double), ("sigma_mode", c_int), ("n_feat", c_int),
                ("newton_mode", c_int), ("ls_max", c_int), ("truncate", c_int),
                ("delta_reg_adj", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_SO)
        for name in ("ostrich_ref_step_forward", "ostrich_ref_step_adjoint", "ostrich_ref_step_adjoint_params",
                     "ostrich_ref_spline_basis",
                     "ostrich_ref_rollout", "ostrich_ref_rollout_shaped", "ostrich_ref_inspect"):
            getattr(_lib, name).restype = c_int
    return _lib


def _p(a, ct):
    if a is None:
        return ctypes.cast(None, ct)
    return a.ctypes.data_as(ct)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class _Handle:
    """Keeps the numpy arrays alive while the C structure points into them."""

    def __init__(self, batch, params: dict):
        b = batch
        self.arrays = dict(
            body_off=_i(b.body_off), body_mass=_d(b.body_mass), body_inertia=_d(b.body_inertia),
            joint_off=_i(b.joint_off), joint_body=_i(b.joint_body), joint_frame=_d(b.joint_frame),
            joint_act=_i(b.joint_act), joint_kp=_d(b.joint_kp), ctrl_off=_i(b.ctrl_off),
            slot_off=_i(b.slot_off), slot_int=_i(b.slot_int), slot_real=_d(b.slot_real),
            obs_off=_i(b.obs_off), obs_box=_d(b.obs_box), lam_off=_i(b.lam_off),
            contact_cap=_i(b.contact_cap), world_hmap=_i(b.world_hmap),
            hmap_origin=_d(b.hmap_origin), hmap_heights=_d(b.hmap_heights), joint_kd=_d(b.joint_kd))
        a = self.arrays
        self.cb = Batch()
        self.cb.n_worlds = b.n_worlds
        for k, v in a.items():
            setattr(self.cb, k, _p(v, c_int_p if v.dtype == np.int32 else c_dbl_p))
        self.cb.hmap_n = b.hmap_n
        self.cb.hmap_spacing = b.hmap_spacing
        self.cp = Params()
        self.cp.h = params["h"]
        for k in range(3):
            self.cp.gravity[k] = params["gravity"][k]
        for k in ("tol", "eps", "delta_g", "delta_reg", "delta0"):
            setattr(self.cp, k, float(params[k]))
        for k in ("k_max", "k_min", "sigma_mode", "n_feat"):
            setattr(self.cp, k, int(params[k]))
        self.cp.newton_mode = int(params.get("newton_mode", 0))
        self.cp.ls_max = int(params.get("ls_max", 0))
        self.cp.truncate = int(params.get("truncate", 0))
        self.cp.delta_reg_adj = float(params.get("delta_reg_adj", params["delta_reg"]))


def step_forward(batch, params, q, u, lam, ctrl):
    """One backward-Euler step of every world; returns a dict of outputs."""
    H = _Handle(batch, params)
    W = batch.n_worlds
    q, u, lam = _d(q), _d(u), _d(lam)
    ctrl = _d(ctrl if ctrl is not None else np.zeros(max(batch.n_ctrl, 1)))
    out = dict(q=np.zeros_like(q), u=np.zeros_like(u), lam=np.zeros_like(lam),
               act_slot=np.full(max(batch.n_slots, 1), -1, np.int32), n_act=np.zeros(W, np.int32),
               status=np.zeros(W, np.int32), iters=np.zeros(W, np.int32), resnorm=np.zeros(W))
    rc = lib().ostrich_ref_step_forward(
        ctypes.byref(H.cb), ctypes.byref(H.cp), _p(q, c_dbl_p), _p(u, c_dbl_p), _p(lam, c_dbl_p),
        _p(ctrl, c_dbl_p), _p(out["q"], c_dbl_p), _p(out["u"], c_dbl_p), _p(out["lam"], c_dbl_p),
        _p(out["act_slot"], c_int_p), _p(out["n_act"], c_int_p), _p(out["status"], c_int_p),
        _p(out["iters"], c_int_p), _p(out["resnorm"], c_dbl_p))
    if rc != 0:
        raise RuntimeError("oracle step_forward failed: %d" % rc)
    return out


def step_adjoint(batch, params, q, u, lam, ctrl, u_next, lam_next, gq_next, gu_next, mode=0):
    """Cotangents of (q-, u-, controls) from those of (q+, u+) through one step (Sec. III-D).
    mode 0: the exact implicit-function adjoint; 1: the paper's lagged Schur adjoint
    (Eqs. (18)-(19)); 2: the adjoint solved with the forward's own Newton matrix (the
    exact system without the geometric stiffness of J^T lambda)."""
    H = _Handle(batch, params)
    q, u, lam = _d(q), _d(u), _d(lam)
    ctrl = _d(ctrl if ctrl is not None else np.zeros(max(batch.n_ctrl, 1)))
    u_next, lam_next, gq_next, gu_next = _d(u_next), _d(lam_next), _d(gq_next), _d(gu_next)
    gq = np.zeros_like(q)
    gu = np.zeros_like(u)
    gc = np.zeros(max(batch.n_ctrl, 1))
    rc = lib().ostrich_ref_step_adjoint(
        ctypes.byref(H.cb), ctypes.byref(H.cp), _p(q, c_dbl_p), _p(u, c_dbl_p), _p(lam, c_dbl_p),
        _p(ctrl, c_dbl_p), _p(u_next, c_dbl_p), _p(lam_next, c_dbl_p), _p(gq_next, c_dbl_p),
        _p(gu_next, c_dbl_p), _p(gq, c_dbl_p), _p(gu, c_dbl_p), _p(gc, c_dbl_p), c_int(mode))
    if rc != 0:
        raise RuntimeError("oracle step_adjoint failed: %d" % rc)
    return gq, gu, gc[:batch.n_ctrl]


def step_adjoint_params(batch, params, q, u, ctrl, u_next, lam_next, gq_next, gu_next, mode=0):
    """The adjoint of step_adjoint and the cotangents of the body masses, the
    slots' friction coefficients and the joints' servo gains (Eq. (17) with a
    model parameter as xi)."""
    H = _Handle(batch, params)
    q, u = _d(q), _d(u)
    ctrl = _d(ctrl if ctrl is not None else np.zeros(max(batch.n_ctrl, 1)))
    u_next, lam_next, gq_next, gu_next = _d(u_next), _d(lam_next), _d(gq_next), _d(gu_next)
    gq, gu = np.zeros_like(q), np.zeros_like(u)
    gc = np.zeros(max(batch.n_ctrl, 1))
    gm = np.zeros(int(batch.body_off[-1]))
    gmu = np.zeros(max(int(batch.slot_off[-1]), 1))
    gkp = np.zeros(max(int(batch.joint_off[-1]), 1))
    rc = lib().ostrich_ref_step_adjoint_params(
        ctypes.byref(H.cb), ctypes.byref(H.cp), _p(q, c_dbl_p), _p(u, c_dbl_p), _p(ctrl, c_dbl_p),
        _p(u_next, c_dbl_p), _p(lam_next, c_dbl_p), _p(gq_next, c_dbl_p), _p(gu_next, c_dbl_p),
        _p(gq, c_dbl_p), _p(gu, c_dbl_p), _p(gc, c_dbl_p), _p(gm, c_dbl_p), _p(gmu, c_dbl_p), _p(gkp, c_dbl_p),
        c_int(mode))
    if rc != 0:
        raise RuntimeError("oracle step_adjoint_params failed: %d" % rc)
    return dict(gq=gq, gu=gu, gc=gc[:batch.n_ctrl], g_mass=gm, g_mu=gmu[:int(batch.slot_off[-1])],
                g_kp=gkp[:int(batch.joint_off[-1])])


def spline_basis(T, K, h):
    B = np.zeros((T, K))
    rc = lib().ostrich_ref_spline_basis(c_int(T), c_int(K), ctypes.c_double(h), _p(B, c_dbl_p))
    if rc != 0:
        raise RuntimeError("spline_basis failed")
    return B


def rollout(batch, params, q0, u0, knots, T, mode=0, grad=True):
    """T-step rollout, loss |xy - target|^2 and its gradient (per world)."""
    H = _Handle(batch, params)
    W = batch.n_worlds
    q0, u0 = _d(q0), _d(u0)
    knots = _d(knots) if knots is not None and knots.size else np.zeros((max(batch.n_ctrl, 1), 2))
    K = knots.shape[1] if knots.ndim == 2 else 0
    loss = np.zeros(W)
    qT, uT = np.zeros_like(q0), np.zeros_like(u0)
    gq0, gu0 = (np.zeros_like(q0), np.zeros_like(u0)) if grad else (None, None)
    gk = np.zeros_like(knots) if grad else None
    st = np.zeros(W, np.int32)
    rc = lib().ostrich_ref_rollout(
        ctypes.byref(H.cb), ctypes.byref(H.cp), _p(q0, c_dbl_p), _p(u0, c_dbl_p), _p(knots, c_dbl_p),
        c_int(K), c_int(T), _p(_i(batch.loss_body), c_int_p), _p(_d(batch.target), c_dbl_p),
        _p(loss, c_dbl_p), _p(qT, c_dbl_p), _p(uT, c_dbl_p), _p(gq0, c_dbl_p), _p(gu0, c_dbl_p),
        _p(gk, c_dbl_p), c_int(mode), _p(st, c_int_p))
    if rc != 0:
        raise RuntimeError("oracle rollout failed: %d" % rc)
    return dict(loss=loss, qT=qT, uT=uT, g_q0=gq0, g_u0=gu0, g_knots=gk, status=st)


LOSS_WEIGHTS = ("w_pos", "w_head", "w_vel", "w_ctrl", "w_track", "w_yaw")


class Loss(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in LOSS_WEIGHTS] + [("goal", c_dbl_p), ("ref", c_dbl_p)]


def rollout_shaped(batch, params, q0, u0, knots, T, weights, goal, ref=None, mode=0, grad=True):
    """T-step rollout with the shaped loss (final position, heading and velocity,
    control regulariser, per-step tracking and yaw alignment; weights by name,
    goal [W, 3], ref [T, W, 3]) and its gradient (per world)."""
    H = _Handle(batch, params)
    W = batch.n_worlds
    q0, u0 = _d(q0), _d(u0)
    knots = _d(knots) if knots is not None and knots.size else np.zeros((max(batch.n_ctrl, 1), 2))
    K = knots.shape[1] if knots.ndim == 2 else 0
    goal = _d(np.reshape(goal, (W, 3)))
    ref = _d(np.reshape(ref, (T, W, 3))) if ref is not None else None
    spec = Loss(*[float(weights.get(k, 0.0)) for k in LOSS_WEIGHTS])
    spec.goal = _p(goal, c_dbl_p)
    spec.ref = _p(ref, c_dbl_p)
    loss = np.zeros(W)
    qT, uT = np.zeros_like(q0), np.zeros_like(u0)
    gq0, gu0 = (np.zeros_like(q0), np.zeros_like(u0)) if grad else (None, None)
    gk = np.zeros_like(knots) if grad else None
    st = np.zeros(W, np.int32)
    rc = lib().ostrich_ref_rollout_shaped(
        ctypes.byref(H.cb), ctypes.byref(H.cp), _p(q0, c_dbl_p), _p(u0, c_dbl_p), _p(knots, c_dbl_p),
        c_int(K), c_int(T), _p(_i(batch.loss_body), c_int_p), ctypes.byref(spec),
        _p(loss, c_dbl_p), _p(qT, c_dbl_p), _p(uT, c_dbl_p), _p(gq0, c_dbl_p), _p(gu0, c_dbl_p),
        _p(gk, c_dbl_p), c_int(mode), _p(st, c_int_p))
    if rc != 0:
        raise RuntimeError("oracle rollout_shaped failed: %d" % rc)
    return dict(loss=loss, qT=qT, uT=uT, g_q0=gq0, g_u0=gu0, g_knots=gk, status=st)


def inspect(batch, params, world, q, u, ctrl, u_it=None, lam_it=None):
    """Residual, Jacobians and Newton system of one world at a given iterate."""
    H = _Handle(batch, params)
    q, u = _d(q), _d(u)
    ctrl = _d(ctrl if ctrl is not None else np.zeros(max(batch.n_ctrl, 1)))
    m = ctypes.c_int32()
    nu = ctypes.c_int32()
    act = np.full(max(batch.n_slots, 1), -1, np.int32)
    L = lib()
    rc = L.ostrich_ref_inspect(ctypes.byref(H.cb), ctypes.byref(H.cp), c_int(world), _p(q, c_dbl_p),
                               _p(u, c_dbl_p), _p(ctrl, c_dbl_p), None, None, ctypes.byref(m),
                               ctypes.byref(nu), None, None, None, None, None, None, None, None, None,
                               _p(act, c_int_p))
    if rc != 0:
        raise RuntimeError("inspect failed")
    m, nu = m.value, nu.value
    res = dict(m=m, nu=nu, act_slot=act[:max(0, int((act >= 0).sum()))])
    if u_it is None:
        return res
    u_it, lam_it = _d(u_it), _d(lam_it)
    n = nu + m
    out = dict(F=np.zeros(n), D=np.zeros(n), J=np.zeros((m, nu)), Gu=np.zeros((m, nu)), Gl=np.zeros((m, m)),
               A=np.zeros((m, m)), rhs=np.zeros(m), H=np.zeros((n, n)), sigma=np.zeros(m))
    rc = L.ostrich_ref_inspect(ctypes.byref(H.cb), ctypes.byref(H.cp), c_int(world), _p(q, c_dbl_p),
                               _p(u, c_dbl_p), _p(ctrl, c_dbl_p), _p(u_it, c_dbl_p), _p(lam_it, c_dbl_p),
                               ctypes.byref(ctypes.c_int32()), ctypes.byref(ctypes.c_int32()),
                               *[_p(out[k], c_dbl_p) for k in ("F", "J", "D", "Gu", "Gl", "A", "rhs", "H", "sigma")],
                               None)
    if rc != 0:
        raise RuntimeError("inspect failed")
    res.update(out)
    return res
