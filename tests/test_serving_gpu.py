"""Serving system on the GPU: a served request computes what the rollout
entry point and Adam compute, and its results are the same alone and in a mix
of requests of other sizes and horizons arriving while it runs."""
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


K = scenes.ROBOT_KNOTS


def engine(capacity=64, budget=8e9, P=None):
    from paper_2609_08800_amd.serving import GpuBackend, ServingEngine
    P = P or scenes.solver_params()
    tmpl = scenes.robot_batch(1, seed=0).worlds[0]
    be = GpuBackend(tmpl, capacity, P, K)
    return be, ServingEngine(be, budget)


def adam_ref(x, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    x = x - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return x, m, v


def test_served_request_matches_rollout_and_adam(torch):
    from paper_2609_08800_amd import Simulator, spline_basis
    from paper_2609_08800_amd.serving import Request
    b = scenes.robot_batch(3, seed=41)
    T, iters, lr = 8, 3, 0.1
    be, eng = engine(capacity=8)
    r = Request(0, b, T=T, iters=iters, lr=lr)
    out = eng.run([r])
    assert len(out["requests"]) == 1 and len(r.iter_latency) == iters
    P = scenes.solver_params()
    sim = Simulator(b, P, device="cuda:0")
    basis = spline_basis(T, K, P["h"])
    x = scenes.knots_array(b, K)
    m, v = np.zeros_like(x), np.zeros_like(x)
    for it in range(iters):
        ref = sim.rollout(b.q0, b.u0, x, basis, T, ckpt_every=0, loss_body=b.loss_body, target=b.target)
        np.testing.assert_allclose(r.losses[it], ref["loss"].cpu().numpy(), rtol=1e-12, atol=0)
        x, m, v = adam_ref(x, ref["g_knots"].cpu().numpy(), m, v, it + 1, lr)
    np.testing.assert_allclose(r.knots.reshape(x.shape), x, rtol=1e-12, atol=1e-14)


def test_results_same_alone_and_in_the_mix(torch):
    from paper_2609_08800_amd.serving import Request
    mine = scenes.robot_batch(5, seed=50)
    be, eng = engine(capacity=48)
    alone = Request(0, mine, T=10, iters=3)
    eng.run([alone])
    be2, eng2 = engine(capacity=48)
    mixed = Request(0, mine, T=10, iters=3, arrival=0.05)
    others = [Request(1 + i, scenes.robot_batch(n, seed=60 + i), T=t, iters=2, arrival=0.02 * i)
              for i, (n, t) in enumerate(((7, 6), (3, 14), (11, 9), (2, 5)))]
    out = eng2.run([mixed] + others)
    assert len(out["requests"]) == 5
    assert any(len(rids) >= 3 for _, _, _, rids in eng2.ticks), "requests never shared a launch"
    assert any(f and b_ for _, f, b_, _ in eng2.ticks), "no tick mixed forward and adjoint work"
    assert np.array_equal(alone.knots, mixed.knots)
    for a, c in zip(alone.losses, mixed.losses):
        assert np.array_equal(a, c)


def test_hbm_budget_serialises_requests(torch):
    from paper_2609_08800_amd.serving import Request
    be, eng = engine(capacity=32)
    reqs = [Request(i, scenes.robot_batch(4, seed=70 + i), T=6, iters=1) for i in range(3)]
    need = be.request_bytes(reqs[0])
    eng.budget = 1.5 * need
    out = eng.run(reqs)
    spans = sorted((r.admitted_at, r.finished_at) for r in out["requests"])
    for (a0, f0), (a1, f1) in zip(spans, spans[1:]):
        assert a1 >= f0


def test_terrain_requests_each_on_its_own_map(torch):
    """Requests on different terrains share the pool and the launches; each
    request's result equals serving it alone."""
    from paper_2609_08800_amd.serving import GpuBackend, Request, ServingEngine
    P = scenes.solver_params()
    base = scenes.value_noise_heightmap(10_000)
    tmpl = scenes.robot_terrain_world(None, base, 0)

    def make(rid, n, T, arrival):
        return Request(rid, scenes.terrain_request_batch(500 + rid, n), T=T, iters=2, arrival=arrival)

    be = GpuBackend(tmpl, 24, P, K, heightmaps=[base], heightmap_slots=4)
    alone = make(0, 3, 8, 0.0)
    ServingEngine(be, 8e9).run([alone])
    be2 = GpuBackend(tmpl, 24, P, K, heightmaps=[base], heightmap_slots=4)
    mix = [make(0, 3, 8, 0.03), make(1, 5, 6, 0.0), make(2, 2, 10, 0.01), make(3, 4, 7, 0.05)]
    eng = ServingEngine(be2, 8e9)
    out = eng.run(mix)
    assert len(out["requests"]) == 4
    assert any(len(rids) >= 3 for _, _, _, rids in eng.ticks)
    assert np.array_equal(alone.knots, mix[0].knots)
    for a, c in zip(alone.losses, mix[0].losses):
        assert np.array_equal(a, c)
    assert sorted(be2.hmap_free) == [0, 1, 2, 3]


def oracle_served(batch, P, T, iters, lr):
    """What a served request computes, from the oracle alone: per iteration a
    T-step rollout with the final-xy loss and its knot gradient, then Adam on
    the knots (a non-finite gradient entry counts as zero).  Returns the knots
    after `iters` iterations, each iteration's loss, and per world whether its
    every rollout converged at every step."""
    x = scenes.knots_array(batch, K)
    m, v = np.zeros_like(x), np.zeros_like(x)
    losses, ok = [], np.ones(batch.n_worlds, bool)
    for it in range(iters):
        ref = oracle.rollout(batch, P, batch.q0, batch.u0, x, T)
        losses.append(ref["loss"])
        ok &= (ref["status"] & 6) == 0
        g = np.where(np.isfinite(ref["g_knots"]), ref["g_knots"], 0.0)
        x, m, v = adam_ref(x, g, m, v, it + 1, lr)
    return x, losses, ok


def check_served_against_oracle(req, batch, P, T, iters, lr):
    x, losses, ok = oracle_served(batch, P, T, iters, lr)
    x0 = scenes.knots_array(batch, K)
    got = req.knots.reshape(x.shape)
    assert ok.sum() >= max(1, batch.n_worlds // 2), ok
    for w in np.flatnonzero(ok):
        c = slice(batch.ctrl_off[w], batch.ctrl_off[w + 1])
        step = np.linalg.norm(x[c] - x0[c])
        # the knot gradient passes through the q- cotangents of robots on four wheels, whose
        # spread between the two sides' roots is that of an indeterminate contact set
        assert np.linalg.norm(got[c] - x[c]) <= 1e-5 * step, (w, np.linalg.norm(got[c] - x[c]) / step)
        for it in range(iters):
            assert abs(req.losses[it][w] - losses[it][w]) <= 1e-9 * max(1.0, abs(losses[it][w])), (w, it)
    return int(ok.sum())


def test_served_knots_match_oracle_alone_and_in_a_terrain_mix(torch):
    """Two iterations (rollout, adjoint, Adam) of served requests against the
    oracle's rollouts and the Adam formula: a plane request served alone, and a
    terrain request served in a mix with three other terrain requests (their
    worlds in the same launches), world by world where the oracle converged at
    every step (tolerance 1e-12).  The terrain robots here have sphere wheels:
    with cylinder wheels (both rims, four mesh candidates each) most worlds
    have a landing step that exhausts 200 Newton iterations at tolerance
    1e-12, which leaves too few worlds to compare; the cylinder wheels' steps
    and adjoints are compared with the oracle in the terrain tests."""
    from paper_2609_08800_amd.serving import GpuBackend, Request, ServingEngine
    T, iters, lr = 8, 2, 0.1
    P = scenes.solver_params(k_max=64, tol=1e-12)
    mine = scenes.robot_batch(4, seed=43)
    be, eng = engine(capacity=8, P=P)
    r = Request(0, mine, T=T, iters=iters, lr=lr)
    eng.run([r])
    n_plane = check_served_against_oracle(r, mine, P, T, iters, lr)
    Pt = scenes.solver_params(k_max=200, tol=1e-12)
    base = scenes.value_noise_heightmap(10_000)
    tmpl = scenes.robot_terrain_world(None, base, 0, wheels="sphere")
    be2 = GpuBackend(tmpl, 24, Pt, K, heightmaps=[base], heightmap_slots=4)
    reqs = [Request(rid, scenes.terrain_request_batch(700 + rid, n, wheels="sphere"), T=t, iters=iters, lr=lr,
                    arrival=a)
            for rid, (n, t, a) in enumerate(((3, 8, 0.02), (5, 6, 0.0), (2, 10, 0.01), (4, 7, 0.04)))]
    eng2 = ServingEngine(be2, 8e9)
    out = eng2.run(reqs)
    assert len(out["requests"]) == 4
    assert any(len(rids) >= 3 for _, _, _, rids in eng2.ticks), "requests never shared a launch"
    n_terrain = sum(check_served_against_oracle(q, q.batch, Pt, q.T, iters, lr) for q in reqs)
    print("worlds compared: plane %d, terrain %d" % (n_plane, n_terrain))


def test_segment_copies_match_per_tensor_copies(torch):
    """The serving loop's batched copies: 70 segments of mixed lengths (empty
    ones among them, more than one launch's 32) land exactly where a copy per
    segment puts them, and nothing else in the destination changes."""
    from paper_2609_08800_amd import _capi
    L = _capi.load()
    rng = np.random.default_rng(0)
    src = torch.as_tensor(rng.normal(size=200_000), device="cuda:0")
    dst = torch.full((200_000,), -7.0, dtype=torch.float64, device="cuda:0")
    ref = dst.clone()
    lens = rng.integers(0, 3000, size=70)
    lens[[3, 40]] = 0
    segs = (_capi.OstrichCopySeg * len(lens))()
    o_src, o_dst = 0, 0
    for i, n in enumerate(lens):
        n = int(n)
        segs[i].src = src.data_ptr() + 8 * o_src
        segs[i].dst = dst.data_ptr() + 8 * o_dst
        segs[i].n = n
        ref[o_dst:o_dst + n] = src[o_src:o_src + n]
        o_src += n + 17
        o_dst += n + 5
    stream = torch.cuda.current_stream().cuda_stream
    assert L.ostrich_copy_segments(segs, len(lens), stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(dst, ref)
