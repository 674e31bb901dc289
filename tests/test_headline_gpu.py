"""The benchmark's own call at full size against the oracle: 8,192 wheeled
robots over the box obstacle, T = 100 steps at h = 0.1 s, checkpoints every 10
steps, Newton tolerance 1e-10 and budget 16 (the configuration the throughput
is quoted on).  Sixteen sampled worlds whose every step converged on the GPU
are rolled out alone by the oracle from their own initial state and knots; the
loss and the knot gradient of each are compared world by world.

Both sides stop at points inside the 1e-10 tolerance ball, and the bars are
the parity bars of the step (states 1e-9, gradients 1e-6), applied per world
(a world's loss, and its knot gradient of 32 entries against its own norm).
"""
import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu

LOSS_TOL = 1e-9   # relative, per world
GRAD_TOL = 1e-6   # relative, per world


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def test_full_size_rollout_sampled_worlds_match_oracle(torch):
    from paper_2609_08800_amd import Simulator, _capi, spline_basis
    W, T, K = 8192, 100, scenes.ROBOT_KNOTS
    b = scenes.robot_batch(W, seed=0)
    P = scenes.solver_params()
    dev = torch.device("cuda:0")
    sim = Simulator(b, P, device=dev)
    knots = scenes.knots_array(b, K)
    basis = spline_basis(T, K, P["h"])
    r = sim.rollout(torch.as_tensor(b.q0, device=dev), torch.as_tensor(b.u0, device=dev),
                    torch.as_tensor(knots, device=dev), torch.as_tensor(basis, device=dev), T, ckpt_every=10,
                    loss_body=b.loss_body, target=torch.as_tensor(b.target, device=dev))
    st = r["status"].cpu().numpy()
    loss, gk = r["loss"].cpu().numpy(), r["g_knots"].cpu().numpy()
    bad = _capi.ST_BUDGET | _capi.ST_NONFINITE | _capi.ST_ADJ_INEXACT | _capi.ST_OVERFLOW
    good = np.flatnonzero((st & bad) == 0)
    print("worlds whose every step converged:", len(good), "of", W, flush=True)
    assert len(good) >= W // 4
    rng = np.random.default_rng(0)
    compared, worst_l, worst_g = 0, 0.0, 0.0
    for w in rng.permutation(good):
        if compared == 16:
            break
        sub = scenes.pack([b.worlds[w]])
        c0, c1 = b.ctrl_off[w], b.ctrl_off[w + 1]
        ref = oracle.rollout(sub, P, sub.q0, sub.u0, knots[c0:c1], T)
        if ref["status"][0] & (_capi.ST_BUDGET | _capi.ST_NONFINITE):
            continue  # the oracle's root left the tolerance on some step: not comparable
        el = abs(loss[w] - ref["loss"][0]) / max(abs(ref["loss"][0]), 1e-12)
        eg = np.linalg.norm(gk[c0:c1] - ref["g_knots"]) / np.linalg.norm(ref["g_knots"])
        print("world %d: loss rel %.2e, knot gradient rel %.2e" % (w, el, eg), flush=True)
        worst_l, worst_g = max(worst_l, el), max(worst_g, eg)
        compared += 1
    print("worst over %d worlds: loss %.2e, gradient %.2e" % (compared, worst_l, worst_g))
    assert compared == 16
    assert worst_l <= LOSS_TOL and worst_g <= GRAD_TOL, (worst_l, worst_g)
