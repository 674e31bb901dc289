"""Host stand-in for the serving engine's device backend (test infrastructure):
the engine's scheduling, admission and latency accounting checked without a GPU."""
import numpy as np


class FakeBackend:
    """Deterministic stand-in with the GpuBackend interface: the 'rollout' of a
    world is a scalar walk x_{k+1} = x_k + knot-mean, so scheduling, admission
    and latency accounting can be checked on the host."""

    def __init__(self, capacity: int, bytes_per_world_step: float = 1.0, tick_seconds: float = 0.01):
        self.capacity = capacity
        self.bpws = bytes_per_world_step
        self.tick_seconds = tick_seconds
        self.state = {}
        self.log = []
        self.vtime = 0.0   # virtual clock: advanced by ticks and idling

    def clock(self):
        return self.vtime

    def request_bytes(self, r):
        return self.bpws * r.n_worlds * (r.T + 1)

    def can_admit(self, r):
        return True

    def idle(self, seconds):
        self.vtime += max(seconds, 0.0)

    # markers on the virtual clock (the device backend records events on its stream)
    def mark(self):
        return self.vtime

    def wait(self, marker):
        pass

    def seconds_between(self, a, b):
        return b - a

    def to_host(self, x):
        return x

    def admit(self, r):
        self.state[r.rid] = {"knots": np.full(r.n_worlds, 1.0), "x": np.zeros(r.n_worlds), "g": np.zeros(r.n_worlds)}

    def begin_iteration(self, r):
        self.state[r.rid]["x"][:] = 0.0

    def tick(self, fw, bw):
        self.log.append(([r.rid for r in fw], [r.rid for r in bw]))
        for r in fw:
            s = self.state[r.rid]
            s["x"] += s["knots"]
        for r in bw:
            s = self.state[r.rid]
            s["g"] = 2.0 * (s["x"] - 3.0) * r.T
        self.vtime += self.tick_seconds

    def end_forward(self, r):
        s = self.state[r.rid]
        return (s["x"] - 3.0) ** 2

    def end_iteration(self, r):
        s = self.state[r.rid]
        s["knots"] = s["knots"] - r.lr * np.sign(s["g"])

    def release(self, r):
        return self.state.pop(r.rid)["knots"]
