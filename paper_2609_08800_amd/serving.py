"""Serving system: continuous batching of trajectory-optimisation requests.

A request is a set of worlds (1..256 of one scene type), a horizon T and a
number of gradient iterations; one iteration is a T-step rollout, its final
position loss, the implicit adjoint back through every step (Sec. III-D) and an
Adam update of the spline knots (the optimisation loop of Sec. IV).

The engine owns a *pool* of world slots that all share one topology (the
template world), created once on the device.  A request admitted to the pool
gets a contiguous range of slots (its scene data are written into the pool's
batch arrays) and a device arena for its resident state: every state of the
rollout, every step's Schur factor (the tape), its knots, gradients and Adam
moments.  Admission needs free slots *and* room under the HBM budget.

The engine advances in ticks.  In one tick every request in its forward pass
advances one step and every request in its backward pass goes back one step:
the forward steps of all those requests run in ONE launch over the list of
their worlds, and so do the adjoint steps.  Requests that arrive while others
are in flight join at the next tick (continuous batching, not a queue).  Each
world's arithmetic does not depend on which other worlds share the launch, so
a request's results are the same alone and in the mix.

The device work goes through ``GpuBackend`` (the HIP library); the engine
talks to it through a small interface (admit, tick, end_forward,
end_iteration, release, mark / wait / seconds_between, to_host and the
clock), so the scheduler can also be driven by a host stand-in in tests.

The host does not wait for every tick: after issuing tick t it waits only for
the end of tick t - LOOKAHEAD, so its bookkeeping and the next launches
overlap the device's work.  An iteration's latency is measured on the device
stream, between a marker recorded when the iteration is issued and the marker
of its last tick.  Losses stay on the device until the engine returns.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import _capi

__all__ = ["Request", "ServingEngine", "GpuBackend", "poisson_arrivals", "percentile"]


@dataclasses.dataclass
class Request:
    rid: int
    batch: object            # packed worlds of the request (scenes.Batch), same topology as the pool template
    T: int
    iters: int = 10
    lr: float = 0.1
    arrival: float = 0.0     # seconds after the engine starts
    # filled by the engine
    slot0: int = -1
    admitted_at: float = math.nan
    finished_at: float = math.nan
    losses: List[np.ndarray] = dataclasses.field(default_factory=list)
    iter_latency: List[float] = dataclasses.field(default_factory=list)
    knots: Optional[np.ndarray] = None
    # progress
    it: int = 0
    phase: int = 0           # 0 forward, 1 backward
    k: int = 0
    iter_started: float = math.nan
    iter_mark: object = None
    iter_marks: list = dataclasses.field(default_factory=list)

    @property
    def n_worlds(self) -> int:
        return int(self.batch.n_worlds)

    @property
    def world_steps(self) -> int:
        return self.n_worlds * self.T * self.iters


def percentile(xs, p):
    xs = np.sort(np.asarray(xs, dtype=np.float64))
    if xs.size == 0:
        return math.nan
    return float(np.percentile(xs, p))


def poisson_arrivals(rate: float, duration: float, seed: int = 0) -> List[float]:
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        out.append(t)


class SlotAllocator:
    """First-fit allocator of contiguous world-slot ranges of the pool."""

    def __init__(self, capacity: int):
        self.capacity = capacity
        self.free = [(0, capacity)]  # sorted (start, length)

    def alloc(self, n: int) -> int:
        for i, (s, l) in enumerate(self.free):
            if l >= n:
                if l == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (s + n, l - n)
                return s
        return -1

    def release(self, s: int, n: int):
        self.free.append((s, n))
        self.free.sort()
        merged = []
        for a, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((a, l))
        self.free = merged

    @property
    def n_free(self) -> int:
        return sum(l for _, l in self.free)


class ServingEngine:
    """Admission, continuous batching and latency accounting over a backend."""

    LOOKAHEAD = 2  # ticks the host may issue before the device has finished them

    def __init__(self, backend, hbm_budget: float, clock: Callable[[], float] = time.perf_counter,
                 max_ticks: int = 10 ** 9):
        self.be = backend
        self.budget = float(hbm_budget)
        self.used = 0.0
        self.slots = SlotAllocator(backend.capacity)
        self.clock = clock
        self.max_ticks = max_ticks
        self.ticks = []          # per tick: (time, n_forward_worlds, n_backward_worlds, request ids)
        self.world_steps = 0     # forward world-steps (each with its adjoint step)

    def run(self, requests: List[Request], deadline: float = math.inf) -> Dict:
        """Serve the requests (arrival times relative to now).  With a deadline
        (seconds), stop when it passes: requests still pending or active are
        reported as unfinished and their device memory is released."""
        for r in requests:
            if r.n_worlds < 1 or r.T < 1 or r.iters < 1:
                raise ValueError(f"request {r.rid}: needs at least one world, one step and one iteration "
                                 f"({r.n_worlds} worlds, T = {r.T}, {r.iters} iterations)")
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        active: List[Request] = []
        done: List[Request] = []
        t0 = self.clock()
        tick = 0
        inflight = collections.deque()  # markers of the ticks issued but not yet waited for
        while (pending or active) and tick < self.max_ticks:
            now = self.clock() - t0
            if now > deadline:
                break
            if not active and pending and pending[0].arrival > now:
                self.be.idle(pending[0].arrival - now)
                now = self.clock() - t0
            # admission in arrival order (no overtaking): slots and HBM budget
            while pending and pending[0].arrival <= now:
                r = pending[0]
                need = self.be.request_bytes(r)
                if need > self.budget:
                    raise ValueError(f"request {r.rid} needs {need:.3g} B, more than the HBM budget")
                if self.used + need > self.budget or not self.be.can_admit(r):
                    break
                s = self.slots.alloc(r.n_worlds)
                if s < 0:
                    break
                pending.pop(0)
                r.slot0 = s
                r.admitted_at = now
                self.used += need
                self.be.admit(r)
                self.be.begin_iteration(r)
                r.iter_started = now
                r.iter_mark = self.be.mark()
                active.append(r)
            if not active:
                if pending and pending[0].arrival <= now:
                    # nothing runs, so no slot, budget or heightmap will be freed: the head
                    # request, which arrived and was not admitted, can never be
                    r = pending[0]
                    raise ValueError(f"request {r.rid} ({r.n_worlds} worlds) can never be admitted: the pool "
                                     f"holds {self.be.capacity} worlds, or it needs a resource the backend lacks")
                continue
            fw = [r for r in active if r.phase == 0]
            bw = [r for r in active if r.phase == 1]
            self.be.tick(fw, bw)
            mark = self.be.mark()
            inflight.append(mark)
            if len(inflight) > self.LOOKAHEAD:
                self.be.wait(inflight.popleft())
            self.world_steps += sum(r.n_worlds for r in fw)  # each forward step gets one adjoint step
            now = self.clock() - t0
            self.ticks.append((now, sum(r.n_worlds for r in fw), sum(r.n_worlds for r in bw),
                               tuple(sorted(r.rid for r in active))))
            tick += 1
            for r in list(active):
                if r.phase == 0:
                    r.k += 1
                    if r.k == r.T:
                        r.losses.append(self.be.end_forward(r))
                        r.phase, r.k = 1, r.T - 1
                else:
                    r.k -= 1
                    if r.k < 0:
                        self.be.end_iteration(r)
                        r.iter_marks.append((r.iter_mark, mark))
                        r.it += 1
                        if r.it == r.iters:
                            r.knots = self.be.release(r)
                            r.finished_at = now
                            self.used -= self.be.request_bytes(r)
                            self.slots.release(r.slot0, r.n_worlds)
                            active.remove(r)
                            done.append(r)
                            if not active:
                                self.used = 0.0  # no rounding residue once nothing is held
                        else:
                            self.be.begin_iteration(r)
                            r.phase, r.k = 0, 0
                            r.iter_started = now
                            r.iter_mark = self.be.mark()
        while inflight:
            self.be.wait(inflight.popleft())
        wall = self.clock() - t0
        for r in active:
            self.be.release(r)
            self.used -= self.be.request_bytes(r)
            self.slots.release(r.slot0, r.n_worlds)
        for r in done + active:  # device-side iteration latencies and losses, now that the device is done
            r.iter_latency = [self.be.seconds_between(a, b) for a, b in r.iter_marks]
            r.losses = [self.be.to_host(x) for x in r.losses]
        lat = [x for r in done + active for x in r.iter_latency]
        return {"requests": done, "unfinished": active + pending, "wall_s": wall, "ticks": len(self.ticks),
                "iterations": len(lat),
                "iter_latency_p50_s": percentile(lat, 50), "iter_latency_p99_s": percentile(lat, 99),
                "world_steps_per_s": self.world_steps / wall if wall > 0 else math.nan}


# --------------------------------------------------------------------------
# GPU backend (the HIP library)
# --------------------------------------------------------------------------
_SEG = {  # batch array -> (offset array, entries per item): per-world ranges copied on admission
    "body_mass": ("body_off", 1), "body_inertia": ("body_off", 3), "joint_body": ("joint_off", 2),
    "joint_frame": ("joint_off", 18), "joint_act": ("joint_off", 1), "joint_kp": ("joint_off", 1),
    "joint_kd": ("joint_off", 1),
    "slot_int": ("slot_off", 4), "slot_real": ("slot_off", 9), "obs_box": ("obs_off", 6),
}


class GpuBackend:
    """Pool of `capacity` worlds shaped like `template` on one GPU.

    `heightmap_slots` maps of the template's grid size are kept on the device;
    a request whose worlds use a heightmap gets one of them.
    """

    def __init__(self, template, capacity: int, params: dict, K: int, device="cuda:0", heightmaps=None,
                 heightmap_slots: int = 0, team: int = 0):
        import scenes
        from . import Simulator
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.capacity = int(capacity)
        self.K = int(K)
        self.P = dict(params)
        self.template = template
        hms = list(heightmaps or [])
        if heightmap_slots:
            base = hms[0] if hms else None
            assert base is not None, "heightmap slots need a template heightmap"
            hms = [base] * heightmap_slots
        self.pool = scenes.pack([template] * self.capacity, hms)
        self.sim = Simulator(self.pool, params, device=self.dev, team=team, schedule="fixed")
        self.L = _capi.load()
        self.hmap_free = list(range(len(hms)))
        S = self.sim
        f64 = dict(dtype=torch.float64, device=self.dev)
        i32 = dict(dtype=torch.int32, device=self.dev)
        NB, NL, NC, W = S.NB, max(S.NL, 1), max(S.NCTRL, 1), S.W
        self.nb_w = int(self.pool.body_off[1] - self.pool.body_off[0])
        self.nl_w = int(self.pool.lam_off[1] - self.pool.lam_off[0])
        self.nc_w = int(self.pool.ctrl_off[1] - self.pool.ctrl_off[0])
        self.tape_w = S.tape_bytes // 8 // W
        # pool-level working arrays: forward tick and adjoint tick
        self.q_cur, self.u_cur, self.l_cur = torch.zeros(NB, 7, **f64), torch.zeros(NB, 6, **f64), torch.zeros(NL, **f64)
        self.q_nxt, self.u_nxt, self.l_nxt = torch.zeros(NB, 7, **f64), torch.zeros(NB, 6, **f64), torch.zeros(NL, **f64)
        self.ctrl_f, self.ctrl_b = torch.zeros(NC, **f64), torch.zeros(NC, **f64)
        self.act, self.nact = torch.zeros(max(S.NS, 1), **i32), torch.zeros(W, **i32)
        self.st, self.its, self.res = torch.zeros(W, **i32), torch.zeros(W, **i32), torch.zeros(W, **f64)
        self.tape_f, self.tape_b = torch.zeros(S.tape_bytes // 8, **f64), torch.zeros(S.tape_bytes // 8, **f64)
        self.qp_b, self.up_b = torch.zeros(NB, 7, **f64), torch.zeros(NB, 6, **f64)
        self.un_b, self.ln_b = torch.zeros(NB, 6, **f64), torch.zeros(NL, **f64)
        self.gqn, self.gun = torch.zeros(NB, 7, **f64), torch.zeros(NB, 6, **f64)
        self.gqp, self.gup = torch.zeros(NB, 7, **f64), torch.zeros(NB, 6, **f64)
        self.gctrl = torch.zeros(NC, **f64)
        self.loss_buf = torch.zeros(W, **f64)
        self.state = {}
        self._wl_cache = {}
        self.stream = torch.cuda.current_stream(self.dev).cuda_stream

    # -- sizes
    def request_bytes(self, r: Request) -> float:
        n, T = r.n_worlds, r.T
        per_state = 7 * self.nb_w + 6 * self.nb_w + self.nl_w
        doubles = n * ((T + 1) * per_state + T * self.tape_w + T * self.nc_w + 6 * self.nc_w * self.K
                       + 2 * 13 * self.nb_w + 2) + T * self.K
        return 8.0 * doubles

    def idle(self, seconds: float):
        time.sleep(max(0.0, min(seconds, 0.05)))

    # -- device markers: events on the pool's stream
    def mark(self):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.torch.cuda.current_stream(self.dev))
        return ev

    def wait(self, marker):
        marker.synchronize()

    def seconds_between(self, a, b) -> float:
        return a.elapsed_time(b) * 1e-3

    def to_host(self, x):
        return x.cpu().numpy()

    def _copy(self, pairs):
        """One launch (per 32) for the listed (src, dst) tensor pairs: contiguous, float64, same size."""
        if not pairs:
            return
        segs = (_capi.OstrichCopySeg * len(pairs))()
        for i, (src, dst) in enumerate(pairs):
            segs[i].src, segs[i].dst, segs[i].n = src.data_ptr(), dst.data_ptr(), src.numel()
        _capi.check(self.L.ostrich_copy_segments(segs, len(pairs), self.stream), "ostrich_copy_segments")

    def _wlist(self, reqs):
        key = tuple(r.rid for r in reqs)
        wl = self._wl_cache.get(key)
        if wl is None:
            if len(self._wl_cache) > 64:
                self._wl_cache.clear()
            wl = self.torch.cat([self.state[r.rid]["wl"] for r in reqs])
            self._wl_cache[key] = wl
        return wl

    def can_admit(self, r: Request) -> bool:
        b = r.batch
        needs_map = b.hmap_heights.size and np.any(b.world_hmap >= 0)
        return bool(self.hmap_free) or not needs_map

    def _w(self, r):
        return slice(r.slot0, r.slot0 + r.n_worlds)

    def _b(self, r):
        return slice(r.slot0 * self.nb_w, (r.slot0 + r.n_worlds) * self.nb_w)

    def _l(self, r):
        return slice(r.slot0 * self.nl_w, (r.slot0 + r.n_worlds) * self.nl_w)

    def _c(self, r):
        return slice(r.slot0 * self.nc_w, (r.slot0 + r.n_worlds) * self.nc_w)

    def _t(self, r):
        return slice(r.slot0 * self.tape_w, (r.slot0 + r.n_worlds) * self.tape_w)

    # -- admission: scene data into the pool, resident arena
    def admit(self, r: Request):
        torch, b = self.torch, r.batch
        n = r.n_worlds
        for key in ("body_off", "joint_off", "slot_off", "obs_off", "ctrl_off", "lam_off"):
            d = np.diff(getattr(b, key))
            d0 = np.diff(getattr(self.pool, key))[:1]
            if not np.all(d == d0[0]):
                raise ValueError(f"request {r.rid}: worlds do not match the pool topology ({key})")
        lbh = np.asarray(b.loss_body)
        if lbh.shape != (n,) or np.any((lbh < 0) | (lbh >= self.nb_w)):
            raise ValueError(f"request {r.rid}: loss_body needs one body index in [0, {self.nb_w}) per world")
        for key, (off, per) in _SEG.items():
            src = np.asarray(getattr(b, key)).reshape(-1)
            if src.size == 0:
                continue
            o = getattr(self.pool, off)
            a, e = int(o[r.slot0]) * per, int(o[r.slot0 + n]) * per
            dst = self.sim._dev[key]
            dst[a:e].copy_(torch.as_tensor(src, device=self.dev, dtype=dst.dtype))
        self.sim._dev["contact_cap"][self._w(r)].copy_(torch.as_tensor(b.contact_cap, device=self.dev))
        hm = -np.ones(n, dtype=np.int32)
        if b.hmap_heights.size and np.any(b.world_hmap >= 0):
            if not self.hmap_free:
                raise ValueError("no free heightmap slot")
            h = self.hmap_free.pop(0)
            nn = self.pool.hmap_n
            self.sim._dev["hmap_heights"][h * nn * nn:(h + 1) * nn * nn].copy_(
                torch.as_tensor(b.hmap_heights[0].reshape(-1), device=self.dev))
            self.sim._dev["hmap_origin"][2 * h:2 * h + 2].copy_(torch.as_tensor(b.hmap_origin[0], device=self.dev))
            hm[:] = np.where(b.world_hmap >= 0, h, -1)
            r._hmap = h
        self.sim._dev["world_hmap"][self._w(r)].copy_(torch.as_tensor(hm, device=self.dev))
        f64 = dict(dtype=torch.float64, device=self.dev)
        T, nb, nl, nc = r.T, n * self.nb_w, n * self.nl_w, n * self.nc_w
        from . import spline_basis
        s = dict(
            q0=torch.as_tensor(b.q0, **f64).reshape(nb, 7), u0=torch.as_tensor(b.u0, **f64).reshape(nb, 6),
            hq=torch.zeros(T + 1, nb, 7, **f64), hu=torch.zeros(T + 1, nb, 6, **f64), hl=torch.zeros(T + 1, max(nl, 1), **f64),
            tapes=torch.zeros(T, n * self.tape_w, **f64), ctrl=torch.zeros(T, max(nc, 1), **f64),
            basis=torch.as_tensor(spline_basis(T, self.K, self.P["h"]), **f64),
            knots=torch.as_tensor(_knots_of(b, self.K), **f64).reshape(max(nc, 1), self.K),
            gk=torch.zeros(max(nc, 1), self.K, **f64), m=torch.zeros(max(nc, 1), self.K, **f64),
            v=torch.zeros(max(nc, 1), self.K, **f64), gq=torch.zeros(nb, 7, **f64), gu=torch.zeros(nb, 6, **f64),
            lb=torch.as_tensor(np.asarray(b.loss_body, dtype=np.int32), device=self.dev),
            tg=torch.as_tensor(b.target, **f64).reshape(n, 2), wl=torch.arange(r.slot0, r.slot0 + n, dtype=torch.int32,
                                                                                device=self.dev))
        self.state[r.rid] = s

    def release(self, r: Request) -> np.ndarray:
        s = self.state.pop(r.rid)
        self._wl_cache.clear()
        if getattr(r, "_hmap", None) is not None:
            self.hmap_free.append(r._hmap)
            self.hmap_free.sort()
        return s["knots"].cpu().numpy()

    # -- iteration boundaries
    def begin_iteration(self, r: Request):
        s = self.state[r.rid]
        s["hq"][0].copy_(s["q0"])
        s["hu"][0].copy_(s["u0"])
        s["hl"][0].zero_()
        self.q_cur[self._b(r)].copy_(s["q0"])
        self.u_cur[self._b(r)].copy_(s["u0"])
        self.l_cur[self._l(r)].zero_()
        if self.nc_w:
            _capi.check(self.L.ostrich_spline_controls(s["basis"].data_ptr(), s["knots"].data_ptr(), r.T, self.K,
                                                       r.n_worlds * self.nc_w, s["ctrl"].data_ptr(), self.stream),
                        "ostrich_spline_controls")
        s["gk"].zero_()

    def end_forward(self, r: Request) -> np.ndarray:
        s = self.state[r.rid]
        n = r.n_worlds
        bo = self.sim._dev["body_off"].data_ptr() + 4 * r.slot0
        self.gqn[self._b(r)].zero_()
        _capi.check(self.L.ostrich_final_loss(bo, n, self.q_cur.data_ptr(), s["lb"].data_ptr(), s["tg"].data_ptr(),
                                              None, self.loss_buf.data_ptr() + 8 * r.slot0, self.gqn.data_ptr(),
                                              self.stream), "ostrich_final_loss")
        s["gq"].copy_(self.gqn[self._b(r)])
        s["gu"].zero_()
        return self.loss_buf[self._w(r)].clone()

    def end_iteration(self, r: Request):
        s = self.state[r.rid]
        if self.nc_w:
            _capi.check(self.L.ostrich_adam(s["knots"].data_ptr(), s["gk"].data_ptr(), s["m"].data_ptr(),
                                            s["v"].data_ptr(), s["knots"].numel(), r.lr, 0.9, 0.999, 1e-8, r.it + 1,
                                            self.stream), "ostrich_adam")

    # -- one tick: forward step of `fw` requests and adjoint step of `bw` requests
    def tick(self, fw: List[Request], bw: List[Request]):
        """Issue one tick on the pool's stream without waiting for it.  The
        moves between request arenas and the working arrays are batched into
        segment-copy launches; the forward's current and next state arrays
        swap roles after the step instead of being copied (every world that
        reads the current state in a tick is one that the last forward step
        wrote, or one that begin_iteration has just set)."""
        if fw:
            if self.nc_w:
                self._copy([(self.state[r.rid]["ctrl"][r.k], self.ctrl_f[self._c(r)]) for r in fw])
            wl = self._wlist(fw)
            _capi.check(self.L.ostrich_step_forward_list(
                self.sim.ctx, wl.data_ptr(), wl.numel(), self.q_cur.data_ptr(), self.u_cur.data_ptr(),
                self.l_cur.data_ptr(), self.ctrl_f.data_ptr(), self.q_nxt.data_ptr(), self.u_nxt.data_ptr(),
                self.l_nxt.data_ptr(), self.act.data_ptr(), self.nact.data_ptr(), self.st.data_ptr(),
                self.its.data_ptr(), self.res.data_ptr(), self.tape_f.data_ptr(), self.stream),
                "ostrich_step_forward_list")
            pairs = []
            for r in fw:
                s = self.state[r.rid]
                b_, l_ = self._b(r), self._l(r)
                pairs += [(self.q_nxt[b_], s["hq"][r.k + 1]), (self.u_nxt[b_], s["hu"][r.k + 1]),
                          (self.l_nxt[l_], s["hl"][r.k + 1][:l_.stop - l_.start]),
                          (self.tape_f[self._t(r)], s["tapes"][r.k])]
            self._copy(pairs)
            self.q_cur, self.q_nxt = self.q_nxt, self.q_cur
            self.u_cur, self.u_nxt = self.u_nxt, self.u_cur
            self.l_cur, self.l_nxt = self.l_nxt, self.l_cur
        if bw:
            pairs = []
            for r in bw:
                s = self.state[r.rid]
                b_, l_, k = self._b(r), self._l(r), r.k
                pairs += [(s["hq"][k], self.qp_b[b_]), (s["hu"][k], self.up_b[b_]), (s["hu"][k + 1], self.un_b[b_]),
                          (s["hl"][k + 1][:l_.stop - l_.start], self.ln_b[l_]),
                          (s["tapes"][k], self.tape_b[self._t(r)]), (s["gq"], self.gqn[b_]), (s["gu"], self.gun[b_])]
                if self.nc_w:
                    pairs.append((s["ctrl"][k], self.ctrl_b[self._c(r)]))
            self._copy(pairs)
            wl = self._wlist(bw)
            _capi.check(self.L.ostrich_step_adjoint_list(
                self.sim.ctx, wl.data_ptr(), wl.numel(), self.qp_b.data_ptr(), self.up_b.data_ptr(),
                self.ctrl_b.data_ptr(), self.un_b.data_ptr(), self.ln_b.data_ptr(), self.tape_b.data_ptr(),
                self.gqn.data_ptr(), self.gun.data_ptr(), self.gqp.data_ptr(), self.gup.data_ptr(),
                self.gctrl.data_ptr(), -1, None, self.stream), "ostrich_step_adjoint_list")
            pairs = []
            for r in bw:
                s = self.state[r.rid]
                b_ = self._b(r)
                pairs += [(self.gqp[b_], s["gq"]), (self.gup[b_], s["gu"])]
            self._copy(pairs)
            if self.nc_w:
                for r in bw:
                    s = self.state[r.rid]
                    gc = self.gctrl[self._c(r)]
                    _capi.check(self.L.ostrich_knot_grad_accumulate(s["basis"].data_ptr(), gc.data_ptr(), r.k,
                                                                    self.K, gc.numel(), s["gk"].data_ptr(),
                                                                    self.stream), "ostrich_knot_grad_accumulate")


def _knots_of(b, K):
    out = np.zeros((max(int(b.ctrl_off[-1]), 1), K))
    for wi, w in enumerate(b.worlds):
        if w.n_ctrl and w.knots is not None:
            out[b.ctrl_off[wi]:b.ctrl_off[wi] + w.n_ctrl] = w.knots[:, :K]
    return out
