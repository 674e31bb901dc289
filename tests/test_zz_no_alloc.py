"""The allocation-free forward entry point (ostrich_step_forward_noalloc),
called through the C ABI, against ostrich_step_forward: the same bits on two
calls in a row, the second with a smaller batch, over robots (tiered launches,
whose deferral queue sits in the static scratch) and stacks up to 32 boxes
(worlds kept in device memory, whose slices sit there too)."""
import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _batch(n_robots, stacks, seed):
    worlds = list(scenes.robot_batch(n_robots, seed=seed).worlds)
    rng = scenes.world_rngs(seed + 1, len(stacks))
    worlds += [scenes.stack_world(r, n) for r, n in zip(rng, stacks)]
    return scenes.pack(worlds)


def _call(sim, fn, q, u, lam, ctrl, torch):
    from paper_2609_08800_amd import _capi
    out = dict(q=torch.empty_like(q), u=torch.empty_like(u), lam=torch.empty_like(lam),
               act_slot=torch.empty(max(sim.NS, 1), dtype=torch.int32, device=q.device),
               n_act=torch.empty(sim.W, dtype=torch.int32, device=q.device),
               status=torch.empty(sim.W, dtype=torch.int32, device=q.device),
               iters=torch.empty(sim.W, dtype=torch.int32, device=q.device),
               resnorm=torch.empty(sim.W, dtype=torch.float64, device=q.device))
    tape = torch.zeros(sim.tape_bytes // 8, dtype=torch.float64, device=q.device)  # entries off the band stay 0
    rc = fn(sim.ctx, q.data_ptr(), u.data_ptr(), lam.data_ptr(), ctrl.data_ptr(), out["q"].data_ptr(),
            out["u"].data_ptr(), out["lam"].data_ptr(), out["act_slot"].data_ptr(), out["n_act"].data_ptr(),
            out["status"].data_ptr(), out["iters"].data_ptr(), out["resnorm"].data_ptr(), tape.data_ptr(),
            torch.cuda.current_stream().cuda_stream)
    _capi.check(rc, "forward")
    out["tape"] = tape
    return out


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_forward_matches_forward(torch, order):
    from paper_2609_08800_amd import Simulator, spline_basis
    P = scenes.solver_params(tier_contacts=6)  # tiered robot buckets: their deferral queue and plan in the scratch
    dev = torch.device("cuda:0")
    for n_robots, stacks, seed in ((160, (32, 24, 9, 3), 11), (40, (30, 2), 12)):
        b = _batch(n_robots, stacks, seed)
        sim = Simulator(b, P, device=dev)
        sched = sim.schedule()
        assert any(x["split"] == 1 for x in sched) and any(x["tier_contacts"] > 0 for x in sched), sched
        ctrl = torch.as_tensor(scenes.knots_array(b, scenes.ROBOT_KNOTS) @
                               spline_basis(10, scenes.ROBOT_KNOTS, P["h"])[3], device=dev)
        q, u = torch.as_tensor(b.q0, device=dev), torch.as_tensor(b.u0, device=dev)
        lam = torch.zeros(max(b.n_lam, 1), dtype=torch.float64, device=dev)
        for _ in range(3):  # three steps, each output compared bit for bit
            want = _call(sim, sim.lib.ostrich_step_forward, q, u, lam, ctrl, torch)
            got = _call(sim, sim.lib.ostrich_step_forward_noalloc, q, u, lam, ctrl, torch)
            torch.cuda.synchronize()
            for k in want:
                assert torch.equal(got[k].view(torch.int8) if got[k].dtype == torch.float64 else got[k],
                                   want[k].view(torch.int8) if want[k].dtype == torch.float64 else want[k]), k
            q, u, lam = want["q"], want["u"], want["lam"]
        del sim
