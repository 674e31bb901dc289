"""MI355X implementation of the batched backward-Euler contact step with
implicit differentiation (Ostrich, Sec. III).

The compute path is ``libostrich.so`` (HIP, gfx950) behind the C ABI of
``include/ostrich.h``; this package marshals PyTorch device tensors to it.
There is no CPU fallback: without the built library every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import _capi

__all__ = ["build", "Simulator", "GraphRollout", "spline_basis", "OstrichError"]

OstrichError = _capi.OstrichError
_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)

HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    """Compile libostrich.so for gfx950 in-tree (hipcc)."""
    out = _capi.SO_PATH
    os.makedirs(os.path.dirname(out), exist_ok=True)
    src = os.path.join(_HERE, "csrc", "ostrich.hip")
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["hipcc", *HIP_FLAGS, "-I", os.path.join(_ROOT, "include"), "-I", os.path.join(_HERE, "csrc"),
           "-o", tmp, src]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def spline_basis(T: int, K: int, h: float) -> np.ndarray:
    """Natural cubic spline basis [T, K] (host): control of step k = B[k] . knots."""
    L = _capi.load()
    B = np.zeros((T, K), dtype=np.float64)
    _capi.check(L.ostrich_spline_basis(T, K, float(h), B.ctypes.data), "ostrich_spline_basis")
    return B


def _torch():
    import torch
    return torch


class Simulator:
    """A batch of worlds resident on one GPU.

    ``batch`` is any object with the packed arrays of the scene description
    (see scenes.Batch): offsets and tables as numpy arrays.  All state tensors
    are float64 on the device; shapes: q [NB, 7], u [NB, 6], lam [NL],
    ctrl [NCTRL].
    """

    def __init__(self, batch, params: dict, device="cuda", team: int = 0, schedule: str = "bucketed"):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise OstrichError("a ROCm GPU is required (no CPU fallback)")
        self.lib = _capi.load()
        self.params = dict(params)
        self.W = int(batch.n_worlds)
        self.NB = int(batch.body_off[-1])
        self.NL = int(batch.lam_off[-1])
        self.NS = int(batch.slot_off[-1])
        self.NJ = int(batch.joint_off[-1])
        self.NCTRL = int(batch.ctrl_off[-1])
        self._dev = {}
        ptrs = {}
        for k in _capi.BATCH_ARRAYS:
            a = np.ascontiguousarray(getattr(batch, k))
            dt = torch.int32 if a.dtype == np.int32 else torch.float64
            t = torch.from_numpy(a.astype(np.int32 if a.dtype == np.int32 else np.float64).reshape(-1)).to(
                self.device, dtype=dt)
            if t.numel() == 0:
                t = torch.zeros(1, dtype=dt, device=self.device)
            self._dev[k] = t
            ptrs[k] = t.data_ptr()
        self.body_off = self._dev["body_off"]
        self._bodies = np.diff(np.asarray(batch.body_off, dtype=np.int64))
        self._cb = _capi.make_batch(self.W, ptrs, int(batch.hmap_n), float(batch.hmap_spacing))
        if schedule not in ("fixed", "bucketed"):
            raise OstrichError("schedule must be 'fixed' or 'bucketed'")
        self._cp = _capi.make_params(self.params, team,
                                     _capi.SCHED_FIXED if schedule == "fixed" else _capi.SCHED_BUCKETED)
        ctx = _capi.c_vp()
        torch.cuda.synchronize(self.device)
        _capi.check(self.lib.ostrich_ctx_create(self._cb, self._cp, ctx), "ostrich_ctx_create")
        self.ctx = ctx
        caps = (_capi.ctypes.c_int64 * 6)()
        _capi.check(self.lib.ostrich_ctx_caps(self.ctx, caps), "ostrich_ctx_caps")
        self.caps = dict(zip(("bodies", "joints", "slots", "contacts", "rows", "lds_bytes"), list(caps)))
        self.tape_bytes = int(self.lib.ostrich_tape_bytes(self.ctx))

    @property
    def device_bytes(self) -> int:
        """Device memory the library context holds (tables, off-chip scratch, counters)."""
        return int(self.lib.ostrich_ctx_device_bytes(self.ctx))

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.lib.ostrich_ctx_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def schedule(self):
        """Buckets of the launch schedule: list of dicts (rows, worlds, team, split, lds, tuned,
        tier_contacts, tier_lds)."""
        n = int(self.lib.ostrich_ctx_schedule(self.ctx, None, 0))
        buf = np.zeros(8 * max(n, 1), dtype=np.int32)
        self.lib.ostrich_ctx_schedule(self.ctx, buf.ctypes.data, n)
        keys = ("rows", "worlds", "team", "split", "lds", "tuned", "tier_contacts", "tier_lds")
        return [dict(zip(keys, map(int, buf[8 * i:8 * i + 8]))) for i in range(n)]

    def timing(self, mode: int):
        """Launch measurement: 1 start, 0 stop; 2 reads the forward steps (launches, total ms, algorithmic
        flops by the roofline count and by the finer count), 3 the adjoint steps (the same with bytes)."""
        out = np.zeros(4)
        _capi.check(self.lib.ostrich_ctx_timing(self.ctx, int(mode), out.ctypes.data), "ostrich_ctx_timing")
        if mode == 2:
            return {"launches": int(out[0]), "ms": float(out[1]), "flops": float(out[2]),
                    "flops_fine": float(out[3])}
        if mode == 3:
            return {"launches": int(out[0]), "ms": float(out[1]), "bytes": float(out[2]),
                    "bytes_fine": float(out[3])}
        return None

    def autotune(self, q, u, lam=None, ctrl=None, reps: int = 2, stream=None):
        """Pick each bucket's launch by timing forward steps from (q, u, lam, ctrl)."""
        q, u = self._f64(q, (self.NB, 7)), self._f64(u, (self.NB, 6))
        lam = self._lam(lam) if lam is not None else self.torch.zeros(max(self.NL, 1), dtype=self.torch.float64,
                                                                      device=self.device)
        ctrl = self._ctrl(ctrl)
        _capi.check(self.lib.ostrich_autotune(self.ctx, q.data_ptr(), u.data_ptr(), lam.data_ptr(),
                                              ctrl.data_ptr(), int(reps), self._stream(stream)),
                    "ostrich_autotune")
        return self.schedule()

    # ----------------------------------------------------------------- helpers
    def _stream(self, stream=None):
        torch = self.torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return s.cuda_stream

    def _f64(self, x, shape=None):
        torch = self.torch
        if x is None:
            return None
        if not torch.is_tensor(x):
            x = torch.as_tensor(np.asarray(x, dtype=np.float64), device=self.device)
        x = x.to(self.device, torch.float64).contiguous()
        if shape is not None:
            x = x.reshape(shape)
        return x

    @staticmethod
    def _p(t):
        return None if t is None else t.data_ptr()

    def empty_state(self):
        torch = self.torch
        return (torch.empty(self.NB, 7, dtype=torch.float64, device=self.device),
                torch.empty(self.NB, 6, dtype=torch.float64, device=self.device),
                torch.empty(max(self.NL, 1), dtype=torch.float64, device=self.device))

    def new_tape(self):
        return self.torch.empty((self.tape_bytes + 7) // 8, dtype=self.torch.float64, device=self.device)

    def _lam(self, lam):
        """Multipliers in slot layout [NL] (a one-entry placeholder when NL is 0)."""
        if self.NL == 0:
            return self.torch.zeros(1, dtype=self.torch.float64, device=self.device)
        return self._f64(lam, (self.NL,))

    def _status(self, st):
        """An optional per-world int32 device tensor of status bits."""
        if st is None:
            return None
        t = self.torch
        if (not t.is_tensor(st) or st.dtype != t.int32 or st.device != self.device or not st.is_contiguous()
                or st.numel() < self.W):
            raise OstrichError("adj_status must be a contiguous int32 device tensor of at least W entries")
        return st.data_ptr()

    def _tape(self, tape):
        """A tape must be a float64 device tensor of at least ostrich_tape_bytes."""
        if tape is None:
            return None
        t = self.torch
        if (not t.is_tensor(tape) or tape.dtype != t.float64 or tape.device != self.device
                or not tape.is_contiguous() or tape.numel() * 8 < self.tape_bytes):
            raise OstrichError("tape must be a contiguous float64 tensor on %s of at least %d bytes (new_tape())"
                               % (self.device, self.tape_bytes))
        return tape

    def check_loss_body(self, lb):
        """Host check of a loss-body array: one entry per world, each a body of that world."""
        lb = np.asarray(lb)
        if lb.shape != (self.W,):
            raise OstrichError("loss_body must have one entry per world (%d), got shape %s" % (self.W, lb.shape))
        if np.any(lb < 0) or np.any(lb >= self._bodies):
            w = int(np.argmax((lb < 0) | (lb >= self._bodies)))
            raise OstrichError("loss_body[%d] = %d is not a body of world %d (%d bodies)"
                               % (w, int(lb[w]), w, int(self._bodies[w])))
        return lb.astype(np.int32)

    def _loss_body(self, loss_body):
        """Device int32 [W].  Host arrays are checked value by value; a device tensor only by
        shape (reading it back would synchronise, which graph capture forbids)."""
        torch = self.torch
        if loss_body is None:
            raise OstrichError("loss_body is required: the loss body of every world")
        if torch.is_tensor(loss_body):
            if loss_body.shape != (self.W,):
                raise OstrichError("loss_body must have shape (%d,)" % self.W)
            return loss_body.to(self.device, torch.int32).contiguous()
        return torch.as_tensor(self.check_loss_body(loss_body), device=self.device).contiguous()

    def _check_out(self, out):
        torch = self.torch
        need = dict(q=(self.NB * 7, torch.float64), u=(self.NB * 6, torch.float64),
                    lam=(max(self.NL, 1), torch.float64), act_slot=(max(self.NS, 1), torch.int32),
                    n_act=(self.W, torch.int32), status=(self.W, torch.int32), iters=(self.W, torch.int32),
                    resnorm=(self.W, torch.float64))
        for k, (n, dt) in need.items():
            x = out.get(k)
            if (x is None or not torch.is_tensor(x) or x.dtype != dt or x.device != self.device
                    or not x.is_contiguous() or x.numel() < n):
                raise OstrichError("out[%r] must be a contiguous %s tensor on %s with at least %d entries"
                                   % (k, dt, self.device, n))

    def _ctrl(self, ctrl):
        if self.NCTRL == 0:
            return self.torch.zeros(1, dtype=self.torch.float64, device=self.device)
        return self._f64(ctrl, (self.NCTRL,))

    # ------------------------------------------------------------------- calls
    def step_forward(self, q, u, lam, ctrl=None, tape=None, out=None, stream=None, plain=False):
        """One backward-Euler step of every world; returns a dict of device tensors.
        plain=True runs the comparison baseline (one launch per world per Newton iteration)."""
        torch = self.torch
        q, u, lam = self._f64(q, (self.NB, 7)), self._f64(u, (self.NB, 6)), self._lam(lam)
        ctrl = self._ctrl(ctrl)
        tape = self._tape(tape)
        if out is not None:
            self._check_out(out)
        else:
            qn, un, ln = self.empty_state()
            out = dict(q=qn, u=un, lam=ln,
                       act_slot=torch.empty(max(self.NS, 1), dtype=torch.int32, device=self.device),
                       n_act=torch.empty(self.W, dtype=torch.int32, device=self.device),
                       status=torch.empty(self.W, dtype=torch.int32, device=self.device),
                       iters=torch.empty(self.W, dtype=torch.int32, device=self.device),
                       resnorm=torch.empty(self.W, dtype=torch.float64, device=self.device))
        fn = self.lib.ostrich_step_forward_plain if plain else self.lib.ostrich_step_forward
        rc = fn(
            self.ctx, q.data_ptr(), u.data_ptr(), lam.data_ptr(), ctrl.data_ptr(), out["q"].data_ptr(),
            out["u"].data_ptr(), out["lam"].data_ptr(), out["act_slot"].data_ptr(), out["n_act"].data_ptr(),
            out["status"].data_ptr(), out["iters"].data_ptr(), out["resnorm"].data_ptr(), self._p(tape),
            self._stream(stream))
        _capi.check(rc, "ostrich_step_forward")
        return out

    def step_adjoint(self, q, u, ctrl, u_next, lam_next, tape, gq_next, gu_next, refine=-1, stream=None,
                     plain=False, adj_status=None):
        """Cotangents of (q-, u-, ctrl) from those of (q+, u+); plain=True: one launch per world.
        adj_status: optional int32 [W] device tensor into which ST_ADJ_INEXACT is ORed for
        worlds whose Krylov solve ended above its stop."""
        torch = self.torch
        q, u = self._f64(q, (self.NB, 7)), self._f64(u, (self.NB, 6))
        ctrl = self._ctrl(ctrl)
        u_next, lam_next = self._f64(u_next, (self.NB, 6)), self._lam(lam_next)
        gq_next, gu_next = self._f64(gq_next, (self.NB, 7)), self._f64(gu_next, (self.NB, 6))
        if tape is None:
            raise OstrichError("the adjoint step needs the tape written by its forward step")
        tape = self._tape(tape)
        gq = torch.empty_like(q)
        gu = torch.empty_like(u)
        gc = torch.zeros(max(self.NCTRL, 1), dtype=torch.float64, device=self.device)
        fn = self.lib.ostrich_step_adjoint_plain if plain else self.lib.ostrich_step_adjoint
        rc = fn(
            self.ctx, q.data_ptr(), u.data_ptr(), ctrl.data_ptr(), u_next.data_ptr(), lam_next.data_ptr(),
            tape.data_ptr(), gq_next.data_ptr(), gu_next.data_ptr(), gq.data_ptr(), gu.data_ptr(), gc.data_ptr(),
            int(refine), self._status(adj_status), self._stream(stream))
        _capi.check(rc, "ostrich_step_adjoint")
        return gq, gu, gc[:self.NCTRL]

    def step_adjoint_params(self, q, u, ctrl, u_next, lam_next, tape, gq_next, gu_next, refine=-1, stream=None,
                            adj_status=None):
        """step_adjoint and the cotangents of every body's mass, every slot's friction
        coefficient and every joint's servo gain: (gq, gu, g_ctrl, g_mass, g_mu, g_kp)."""
        torch = self.torch
        q, u = self._f64(q, (self.NB, 7)), self._f64(u, (self.NB, 6))
        ctrl = self._ctrl(ctrl)
        u_next, lam_next = self._f64(u_next, (self.NB, 6)), self._lam(lam_next)
        gq_next, gu_next = self._f64(gq_next, (self.NB, 7)), self._f64(gu_next, (self.NB, 6))
        if tape is None:
            raise OstrichError("the adjoint step needs the tape written by its forward step")
        tape = self._tape(tape)
        f64 = dict(dtype=torch.float64, device=self.device)
        gq, gu = torch.empty_like(q), torch.empty_like(u)
        gc = torch.zeros(max(self.NCTRL, 1), **f64)
        gm = torch.empty(self.NB, **f64)
        gmu = torch.empty(max(self.NS, 1), **f64)
        gkp = torch.empty(max(self.NJ, 1), **f64)
        rc = self.lib.ostrich_step_adjoint_params(
            self.ctx, q.data_ptr(), u.data_ptr(), ctrl.data_ptr(), u_next.data_ptr(), lam_next.data_ptr(),
            tape.data_ptr(), gq_next.data_ptr(), gu_next.data_ptr(), gq.data_ptr(), gu.data_ptr(), gc.data_ptr(),
            gm.data_ptr(), gmu.data_ptr(), gkp.data_ptr(), int(refine), self._status(adj_status), self._stream(stream))
        _capi.check(rc, "ostrich_step_adjoint_params")
        return gq, gu, gc[:self.NCTRL], gm, gmu[:self.NS], gkp[:self.NJ]

    def workspace_bytes(self, T: int, ckpt_every: int) -> int:
        return int(self.lib.ostrich_rollout_workspace_bytes(self.ctx, int(T), int(ckpt_every)))

    def new_workspace(self, T: int, ckpt_every: int):
        n = self.workspace_bytes(T, ckpt_every)
        return self.torch.empty((n + 7) // 8, dtype=self.torch.float64, device=self.device)

    def rollout(self, q0, u0, knots, basis, T, ckpt_every=10, loss_body=None, target=None, phase=_capi.BOTH,
                workspace=None, grads=True, loss_grad=None, stream=None):
        """T-step rollout with the final-xy loss; FORWARD (1), BACKWARD (2) or both (3).
        Gradients are those of sum_w loss_grad[w] loss[w] (all ones by default)."""
        torch = self.torch
        q0, u0 = self._f64(q0, (self.NB, 7)), self._f64(u0, (self.NB, 6))
        K = 0
        if self.NCTRL > 0:
            knots = self._f64(knots)
            K = knots.numel() // self.NCTRL
            knots = knots.reshape(self.NCTRL, K)
            basis = self._f64(basis, (T, K))
        lb = self._loss_body(loss_body)
        tg = self._f64(target, (self.W, 2))
        lg = self._f64(loss_grad, (self.W,)) if loss_grad is not None else None
        ws = workspace if workspace is not None else self.new_workspace(T, ckpt_every)
        loss = torch.empty(self.W, dtype=torch.float64, device=self.device)
        qT, uT, _ = self.empty_state()
        st = torch.zeros(self.W, dtype=torch.int32, device=self.device)
        g_q0 = torch.empty_like(q0) if grads else None
        g_u0 = torch.empty_like(u0) if grads else None
        g_knots = torch.empty(self.NCTRL, max(K, 1), dtype=torch.float64, device=self.device) if grads else None
        rc = self.lib.ostrich_rollout(
            self.ctx, int(phase), q0.data_ptr(), u0.data_ptr(), self._p(knots) if self.NCTRL else None, int(K),
            self._p(basis) if self.NCTRL else None, int(T), int(ckpt_every), lb.data_ptr(), tg.data_ptr(),
            self._p(lg), loss.data_ptr(), qT.data_ptr(), uT.data_ptr(), self._p(g_q0), self._p(g_u0), self._p(g_knots),
            ws.data_ptr(), ws.numel() * 8, st.data_ptr(), self._stream(stream))
        _capi.check(rc, "ostrich_rollout")
        return dict(loss=loss, qT=qT, uT=uT, g_q0=g_q0, g_u0=g_u0, g_knots=g_knots, status=st, workspace=ws)

    def rollout_shaped(self, q0, u0, knots, basis, T, weights, goal, ref=None, ckpt_every=10, loss_body=None,
                       phase=_capi.BOTH, workspace=None, grads=True, loss_grad=None, stream=None):
        """T-step rollout with the shaped loss of ``ostrich_rollout_shaped``: ``weights``
        maps the names in LOSS_WEIGHTS to their values (missing: 0), ``goal`` is [W, 3]
        (x*, y*, psi*), ``ref`` [T, W, 3] the per-step reference (needed when w_track
        or w_yaw is not zero)."""
        torch = self.torch
        q0, u0 = self._f64(q0, (self.NB, 7)), self._f64(u0, (self.NB, 6))
        K = 0
        if self.NCTRL > 0:
            knots = self._f64(knots)
            K = knots.numel() // self.NCTRL
            knots = knots.reshape(self.NCTRL, K)
            basis = self._f64(basis, (T, K))
        lb = self._loss_body(loss_body)
        unknown = set(weights) - set(LOSS_WEIGHTS)
        if unknown:
            raise ValueError("unknown loss weights: %s" % sorted(unknown))
        gl = self._f64(goal, (self.W, 3))
        rf = self._f64(ref, (T, self.W, 3)) if ref is not None else None
        spec = _capi.OstrichLoss(*[float(weights.get(k, 0.0)) for k in LOSS_WEIGHTS])
        spec.goal = gl.data_ptr()
        spec.ref = rf.data_ptr() if rf is not None else None
        lg = self._f64(loss_grad, (self.W,)) if loss_grad is not None else None
        ws = workspace if workspace is not None else self.new_workspace(T, ckpt_every)
        loss = torch.empty(self.W, dtype=torch.float64, device=self.device)
        qT, uT, _ = self.empty_state()
        st = torch.zeros(self.W, dtype=torch.int32, device=self.device)
        g_q0 = torch.empty_like(q0) if grads else None
        g_u0 = torch.empty_like(u0) if grads else None
        g_knots = torch.empty(self.NCTRL, max(K, 1), dtype=torch.float64, device=self.device) if grads else None
        rc = self.lib.ostrich_rollout_shaped(
            self.ctx, int(phase), q0.data_ptr(), u0.data_ptr(), self._p(knots) if self.NCTRL else None, int(K),
            self._p(basis) if self.NCTRL else None, int(T), int(ckpt_every), lb.data_ptr(), ctypes.byref(spec),
            self._p(lg), loss.data_ptr(), qT.data_ptr(), uT.data_ptr(), self._p(g_q0), self._p(g_u0), self._p(g_knots),
            ws.data_ptr(), ws.numel() * 8, st.data_ptr(), self._stream(stream))
        _capi.check(rc, "ostrich_rollout_shaped")
        return dict(loss=loss, qT=qT, uT=uT, g_q0=g_q0, g_u0=g_u0, g_knots=g_knots, status=st, workspace=ws)


LOSS_WEIGHTS = ("w_pos", "w_head", "w_vel", "w_ctrl", "w_track", "w_yaw")


class GraphRollout:
    """A rollout with its adjoint (both phases of ``Simulator.rollout``) captured
    once into a HIP graph and replayed: one graph launch per rollout instead of
    one host launch per kernel.  Inputs live in static device tensors that
    ``replay`` overwrites; outputs are the same tensors on every replay.
    """

    def __init__(self, sim: "Simulator", q0, u0, knots, basis, T: int, ckpt_every: int, loss_body, target,
                 warmup: int = 1):
        torch = sim.torch
        self.sim = sim
        self.q0 = sim._f64(q0, (sim.NB, 7)).clone()
        self.u0 = sim._f64(u0, (sim.NB, 6)).clone()
        self.knots = sim._f64(knots).clone() if sim.NCTRL else None
        self.basis = sim._f64(basis).clone() if sim.NCTRL else None
        self.lb = torch.as_tensor(sim.check_loss_body(loss_body), device=sim.device).contiguous()
        self.tg = sim._f64(target, (sim.W, 2)).clone()
        self.ws = sim.new_workspace(T, ckpt_every)
        self.T, self.ck = int(T), int(ckpt_every)
        side = torch.cuda.Stream(device=sim.device)
        side.wait_stream(torch.cuda.current_stream(sim.device))
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self._run()
        torch.cuda.current_stream(sim.device).wait_stream(side)
        torch.cuda.synchronize(sim.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.out = self._run()

    def _run(self):
        return self.sim.rollout(self.q0, self.u0, self.knots, self.basis, self.T, ckpt_every=self.ck,
                                loss_body=self.lb, target=self.tg, phase=_capi.BOTH, workspace=self.ws)

    def replay(self, knots=None, q0=None, u0=None):
        if knots is not None:
            self.knots.copy_(self.sim._f64(knots).reshape(self.knots.shape))
        if q0 is not None:
            self.q0.copy_(self.sim._f64(q0, (self.sim.NB, 7)))
        if u0 is not None:
            self.u0.copy_(self.sim._f64(u0, (self.sim.NB, 6)))
        self.graph.replay()
        return self.out
