"""The plain comparison path (one launch per world per Newton iteration) gives
the same bits as the fused batched kernels."""
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


@pytest.mark.parametrize("kind", ["robot", "terrain", "mixed"])
def test_plain_path_equals_fused(torch, kind):
    from paper_2609_08800_amd import Simulator, spline_basis
    b = {"robot": lambda: scenes.robot_batch(6, seed=21),
         "terrain": lambda: scenes.terrain_batch(3, seed=22, n_maps=2),
         "mixed": lambda: scenes.mixed_batch(4, 2, seed=23, max_boxes=6)}[kind]()
    P = scenes.solver_params()
    sim = Simulator(b, P, device="cuda:0")
    K = scenes.ROBOT_KNOTS
    kn = scenes.knots_array(b, K)
    B = spline_basis(10, K, P["h"])
    rng = np.random.default_rng(5)
    q, u, lam = b.q0.copy(), b.u0.copy(), np.zeros(b.n_lam)
    for k in range(3):
        c = kn @ B[k]
        t1, t2 = sim.new_tape(), sim.new_tape()
        f = sim.step_forward(q, u, lam, c, tape=t1)
        p = sim.step_forward(q, u, lam, c, tape=t2, plain=True)
        for key in ("q", "u", "lam", "act_slot", "n_act", "status", "iters", "resnorm"):
            assert torch.equal(f[key], p[key]), (k, key)
        gq_n, gu_n = rng.normal(size=q.shape), rng.normal(size=u.shape)
        ga = sim.step_adjoint(q, u, c, f["u"], f["lam"], t1, gq_n, gu_n)
        gb = sim.step_adjoint(q, u, c, p["u"], p["lam"], t2, gq_n, gu_n, plain=True)
        for x, y in zip(ga, gb):
            assert torch.equal(x, y), k
        q, u, lam = f["q"].cpu().numpy(), f["u"].cpu().numpy(), f["lam"].cpu().numpy()
