"""Differentiation system: torch.autograd over the HIP step and rollout.

Checked against the rollout entry point (same kernels), central finite
differences of the GPU forward, and the oracle's exact implicit-function
gradient.
"""
import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def setup(torch, n, seed, T, P=None):
    from paper_2609_08800_amd import Simulator, spline_basis
    b = scenes.robot_batch(n, seed=seed)
    P = P or scenes.solver_params(k_max=64)
    sim = Simulator(b, P, device="cuda:0")
    K = scenes.ROBOT_KNOTS
    dev = torch.device("cuda:0")
    knots = torch.as_tensor(scenes.knots_array(b, K), device=dev)
    basis = torch.as_tensor(spline_basis(T, K, P["h"]), device=dev)
    q0 = torch.as_tensor(b.q0, device=dev)
    u0 = torch.as_tensor(b.u0, device=dev)
    tg = torch.as_tensor(b.target, device=dev)
    return b, P, sim, knots, basis, q0, u0, tg


def relnorm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_rollout_function_matches_rollout_entry(torch):
    from paper_2609_08800_amd.autograd import rollout_loss
    T = 10
    b, P, sim, knots, basis, q0, u0, tg = setup(torch, 6, 11, T)
    ref = sim.rollout(q0, u0, knots, basis, T, ckpt_every=3, loss_body=b.loss_body, target=tg)
    k = knots.clone().requires_grad_(True)
    u = u0.clone().requires_grad_(True)
    q = q0.clone().requires_grad_(True)
    loss = rollout_loss(sim, k, q, u, basis, T, 3, b.loss_body, tg)
    assert torch.equal(loss.detach(), ref["loss"])
    loss.sum().backward()
    assert torch.equal(k.grad, ref["g_knots"].reshape(k.shape))
    assert torch.equal(u.grad, ref["g_u0"])
    assert torch.equal(q.grad, ref["g_q0"])


def test_rollout_function_weighted_cotangent(torch):
    """Upstream cotangents are per-world loss weights: the gradient of sum w_i L_i equals
    w_i times the world's own gradient."""
    from paper_2609_08800_amd.autograd import rollout_loss
    T = 8
    b, P, sim, knots, basis, q0, u0, tg = setup(torch, 5, 12, T)
    wts = torch.as_tensor(np.random.default_rng(0).uniform(-2, 2, b.n_worlds), device="cuda:0")
    k = knots.clone().requires_grad_(True)
    loss = rollout_loss(sim, k, q0, u0, basis, T, 0, b.loss_body, tg)
    (loss * wts).sum().backward()
    ref = sim.rollout(q0, u0, knots, basis, T, ckpt_every=0, loss_body=b.loss_body, target=tg)
    g = k.grad.cpu().numpy()
    r = ref["g_knots"].cpu().numpy()
    w = wts.cpu().numpy()
    for i in range(b.n_worlds):
        c = slice(b.ctrl_off[i], b.ctrl_off[i + 1])
        np.testing.assert_allclose(g[c], w[i] * r[c], rtol=1e-12, atol=1e-14)


def test_chained_step_function_matches_rollout(torch):
    """T differentiable steps chained by torch autograd (loss written in torch) against the
    rollout adjoint over the same steps."""
    from paper_2609_08800_amd.autograd import step
    T = 8
    b, P, sim, knots, basis, q0, u0, tg = setup(torch, 4, 13, T)
    k = knots.clone().requires_grad_(True)
    u = u0.clone().requires_grad_(True)
    q, uu = q0, u
    lam = torch.zeros(max(sim.NL, 1), dtype=torch.float64, device="cuda:0")
    for j in range(T):
        ctrl = k @ basis[j]
        q, uu, lam = step(sim, q, uu, lam, ctrl)
    lb = torch.as_tensor(b.body_off[:-1] + b.loss_body, device="cuda:0", dtype=torch.long)
    loss = ((q[lb, :2] - tg) ** 2).sum(dim=1)
    loss.sum().backward()
    ref = sim.rollout(q0, u0, knots, basis, T, ckpt_every=0, loss_body=b.loss_body, target=tg)
    np.testing.assert_allclose(loss.detach().cpu().numpy(), ref["loss"].cpu().numpy(), rtol=1e-9)
    assert relnorm(k.grad.cpu().numpy(), ref["g_knots"].cpu().numpy().reshape(k.shape)) <= 1e-9
    assert relnorm(u.grad.cpu().numpy(), ref["g_u0"].cpu().numpy()) <= 1e-9


def test_rollout_gradient_against_finite_differences(torch):
    """Central differences of the GPU forward at a tight tolerance (rel 1e-5)."""
    from paper_2609_08800_amd.autograd import rollout_loss
    T = 5
    P = scenes.solver_params(k_max=64, tol=1e-13)
    b, P, sim, knots, basis, q0, u0, tg = setup(torch, 2, 14, T, P)
    k = knots.clone().requires_grad_(True)
    loss = rollout_loss(sim, k, q0, u0, basis, T, 0, b.loss_body, tg)
    loss.sum().backward()
    g = k.grad.cpu().numpy()
    rng = np.random.default_rng(3)
    picks = [tuple(x) for x in rng.integers(0, [knots.shape[0], knots.shape[1]], size=(6, 2))]
    checked = 0
    for (c, j) in picks:
        hstep = 1e-6 * max(1.0, abs(float(knots[c, j])))
        vals, acts = [], []
        for s in (+1, -1):
            kk = knots.clone()
            kk[c, j] += s * hstep
            r = sim.rollout(q0, u0, kk, basis, T, ckpt_every=0, loss_body=b.loss_body, target=tg, grads=False,
                            phase=1)
            vals.append(float(r["loss"].sum()))
        fd = (vals[0] - vals[1]) / (2 * hstep)
        if abs(fd) < 1e-8:
            continue
        assert abs(g[c, j] - fd) <= 1e-5 * max(abs(fd), 1e-3), (c, j, g[c, j], fd)
        checked += 1
    assert checked >= 3


def test_rollout_function_against_oracle(torch):
    from paper_2609_08800_amd.autograd import rollout_loss
    T = 10
    b, P, sim, knots, basis, q0, u0, tg = setup(torch, 3, 15, T)
    k = knots.clone().requires_grad_(True)
    u = u0.clone().requires_grad_(True)
    loss = rollout_loss(sim, k, q0, u, basis, T, 5, b.loss_body, tg)
    loss.sum().backward()
    ref = oracle.rollout(b, P, b.q0, b.u0, scenes.knots_array(b, scenes.ROBOT_KNOTS), T)
    np.testing.assert_allclose(loss.detach().cpu().numpy(), ref["loss"], rtol=1e-9, atol=1e-12)
    assert relnorm(k.grad.cpu().numpy().reshape(-1), ref["g_knots"].reshape(-1)) <= 1e-6
    assert relnorm(u.grad.cpu().numpy().reshape(-1), ref["g_u0"].reshape(-1)) <= 1e-6
