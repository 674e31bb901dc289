#!/usr/bin/env python3
"""Benchmark: forward + adjoint world-steps/s of the batched backward-Euler
contact step (Ostrich) on one MI355X.

Workload (one benchmark "step"): 8,192 wheeled-robot worlds (5 bodies, 4
revolute wheel joints with spline-driven torques, ground plane and a
1.2 x 0.8 x 0.15 m box obstacle), a T = 100 rollout at h = 0.1 s with the
final-position loss, then its implicit adjoint with checkpoints every 10 steps
(segments recomputed).  That is 819,200 forward world-steps and as many adjoint
world-steps per benchmark step.  Inputs are seeded and synthetic and are
resident in HBM before the timed region.

Prints ONE JSON line (rank 0).  Extra fields: a roofline entry for the
dominant kernel (the fused forward step), measured with HIP events on the
launch stream, and the CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
HBM_PEAK_GBS = 8000.0


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the HIP sources, to tell whether recorded counters still describe the kernel."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2609_08800_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(key="hbm_bytes_per_launch"):
    """HBM bytes per k_forward launch (or, with key="adjoint_hbm_bytes_per_launch", per
    k_adjoint launch) from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by the copy calibration), or None when the kernel sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_forward_robot8192_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def _oracle_worker(args):
    seed, n, T = args
    import oracle
    import scenes
    b = scenes.robot_batch(n, seed=seed)
    P = scenes.solver_params()
    knots = scenes.knots_array(b, scenes.ROBOT_KNOTS)
    t0 = time.perf_counter()
    oracle.rollout(b, P, b.q0, b.u0, knots, T, grad=True)
    return time.perf_counter() - t0


def cpu_baseline(T=100, worlds_per_core=24):
    cores = max(1, min(16, os.cpu_count() or 1))
    jobs = [(1000 + i, worlds_per_core, T) for i in range(cores)]
    t0 = time.perf_counter()
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    ws = cores * worlds_per_core * T
    return {"value": ws / wall, "unit": "fwd+adj world-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores * worlds_per_core} robot worlds x T={T} (forward + exact adjoint), "
                      f"one process per core, {wall:.1f} s wall"}


def plain_path_measurement(n_worlds=64, T=5):
    """World-steps/s (forward + adjoint) of the plain path: one launch per world
    per Newton iteration, on a sample of the benchmark's robot worlds.  The
    plain path runs its worlds one after another, so its rate does not depend
    on how many worlds are sampled."""
    import torch
    import scenes
    from paper_2609_08800_amd import Simulator, spline_basis
    dev = torch.device("cuda:0")
    P = scenes.solver_params()
    b = scenes.robot_batch(n_worlds, seed=0)
    sim = Simulator(b, P, device=dev)
    K = scenes.ROBOT_KNOTS
    ctrl_all = torch.as_tensor(scenes.knots_array(b, K) @ spline_basis(T, K, P["h"]).T, device=dev).T.contiguous()
    q, u = torch.as_tensor(b.q0, device=dev), torch.as_tensor(b.u0, device=dev)
    lam = torch.zeros(max(sim.NL, 1), dtype=torch.float64, device=dev)
    gq = torch.zeros_like(q)
    gu = torch.zeros_like(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(T):
        tape = sim.new_tape()
        o = sim.step_forward(q, u, lam, ctrl_all[k], tape=tape, plain=True)
        sim.step_adjoint(q, u, ctrl_all[k], o["u"], o["lam"], tape, gq, gu, plain=True)
        q, u, lam = o["q"], o["u"], o["lam"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"world_steps_per_s": round(n_worlds * T / dt, 1), "sample": f"{n_worlds} robot worlds x {T} steps",
            "launches_per_world_step": P["k_max"] + 3}


def checkpoint_measurement(sim, q0, u0, knots, basis, T, loss_body, target, W):
    """One rollout with its adjoint at checkpoint interval 1 (every state kept, every
    step recomputed once) and with every step's factor kept (no recomputation):
    world-steps/s and peak HBM of each."""
    import torch
    dev = q0.device
    res = []
    for ck, what in ((1, "every state kept, each step recomputed"), (0, "every step's factor kept, no recomputation")):
        wsk = sim.new_workspace(T, ck)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats(dev)
        t0 = time.perf_counter()
        sim.rollout(q0, u0, knots, basis, T, ckpt_every=ck, loss_body=loss_body, target=target, workspace=wsk)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res.append({"ckpt_every": ck, "what": what, "world_steps_per_s": round(W * T / dt, 1),
                    "peak_hbm_gb": round(torch.cuda.max_memory_allocated(dev) / 1e9, 3)})
        del wsk
    return res


def uneven_measurement(n_stacks=2048, n_robots=2048, T=50, ckpt=10, seed=0):
    """The uneven batch (box stacks of 1..32 boxes with robots; Schur sizes 12..384): forward +
    adjoint world-steps/s of a checkpointed rollout under one fixed schedule and under the bucketed
    schedule after autotuning (the results are the same bits under both)."""
    import torch
    import scenes
    from paper_2609_08800_amd import Simulator, spline_basis
    dev = torch.device("cuda:0")
    P = scenes.solver_params()
    b = scenes.mixed_batch(n_stacks, n_robots, seed=seed, max_boxes=32)
    K = scenes.ROBOT_KNOTS
    knots = torch.as_tensor(scenes.knots_array(b, K), device=dev)
    basis = torch.as_tensor(spline_basis(T, K, P["h"]), device=dev)
    q0, u0 = torch.as_tensor(b.q0, device=dev), torch.as_tensor(b.u0, device=dev)
    tg = torch.as_tensor(b.target, device=dev)
    res = {"worlds": b.n_worlds, "T": T, "ckpt_every": ckpt,
           "rows_max": int(max(w.row_cap for w in b.worlds)), "rows_min": int(min(w.row_cap for w in b.worlds))}
    outs = {}
    for name in ("fixed", "autotuned"):
        sim = Simulator(b, P, device=dev, schedule="fixed" if name == "fixed" else "bucketed")
        if name == "autotuned":
            sim.autotune(q0, u0, None, basis[0] @ knots.t() if sim.NCTRL else None, reps=1)
        ws = sim.new_workspace(T, ckpt)
        run = lambda: sim.rollout(q0, u0, knots, basis, T, ckpt_every=ckpt, loss_body=b.loss_body, target=tg,
                                  workspace=ws)
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        outs[name] = torch.cat([o[k].reshape(-1) for k in ("loss", "g_knots", "g_q0", "g_u0")])
        res[name] = {"world_steps_per_s": round(b.n_worlds * T / dt, 1), "seconds": round(dt, 3),
                     "buckets": [(x["rows"], x["worlds"], x["team"], x["split"]) for x in sim.schedule()]}
    # bit patterns, so that worlds whose trajectory runs away to non-finite values compare too
    res["same_bits"] = bool(torch.equal(outs["fixed"].view(torch.int64), outs["autotuned"].view(torch.int64)))
    res["frac_worlds_nonfinite"] = round(float(((o["status"] & 4) > 0).double().mean()), 4)
    res["autotuned_over_fixed"] = round(res["autotuned"]["world_steps_per_s"] / res["fixed"]["world_steps_per_s"], 2)
    return res


# Weights of the shaped loss, and the learning rate, servo gain and initial guess of the
# control-synthesis task, chosen by small sweeps (lr 0.3 / 0.5 / 0.7 / 1 / 2 / 3, gain 0.5 / 2,
# several weight sets, knots from zero or from the nominal straight drive).  The knots are wheel
# speeds of 0.1 m wheels.
SHAPED_WEIGHTS = dict(w_pos=4.0, w_head=0.2, w_vel=4.0, w_ctrl=1e-3, w_track=0.05, w_yaw=0.0)
SYNTHESIS_LR = 0.5
SYNTHESIS_SERVO_KP = 2.0


# The pallet of the control-synthesis task: 1.2 x 0.8 m like the paper's, and low enough
# (0.02 m) for the synthetic robot's 0.1 m wheels to climb and its 0.025 m chassis
# clearance to pass (the paper's 0.35 m wheels climb a 0.144 m pallet).
SYNTHESIS_PALLET = (1.2, 0.8, 0.02)


def straight_line_ref(p0, goal, T):
    """Per-step reference of the control-synthesis task: the point moving from the start to
    the goal at constant speed, heading along the line; [T, W, 3]."""
    k = np.arange(1, T + 1)[:, None, None] / T
    xy = p0[None] + k * (goal[None, :, :2] - p0[None])
    d = goal[:, :2] - p0
    rho = np.broadcast_to(np.arctan2(d[:, 1], d[:, 0])[None, :, None], (T, len(p0), 1))
    return np.concatenate([xy, rho], axis=2)


def shaped_measurement(sim, q0, u0, knots, basis, T, batch, ckpt):
    """World-steps/s of the timed workload's rollout + adjoint with the shaped loss (final
    pose, heading and velocity, control regulariser, per-step straight-line tracking)."""
    import torch
    W = batch.n_worlds
    goal = np.concatenate([batch.target, np.zeros((W, 1))], axis=1)
    p0 = batch.q0[batch.body_off[:-1] + batch.loss_body, :2]
    ref = straight_line_ref(p0, goal, T)
    ws = sim.new_workspace(T, ckpt)
    run = lambda: sim.rollout_shaped(q0, u0, knots, basis, T, SHAPED_WEIGHTS, goal, ref, ckpt_every=ckpt,
                                     loss_body=batch.loss_body, workspace=ws)
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"world_steps_per_s": round(W * T / dt, 1), "weights": SHAPED_WEIGHTS}


def control_synthesis_measurement(trials=25, iters=50, lr=SYNTHESIS_LR, T=60, K=10, seed=0,
                                  servo_kp=SYNTHESIS_SERVO_KP, weights=None):
    """The control-synthesis task of Sec. IV-B on the robot over a pallet: open-loop
    wheel-velocity splines (K knots per wheel, velocity servos) starting from the nominal
    straight drive (every wheel at the speed that covers the distance to the goal in the
    horizon), the shaped loss towards a random goal at x = 3 m, 50 Adam iterations; per
    trial the iterate of least loss,
    success when its final position error is below 0.2 m and its terminal speed below
    0.3 m/s.  All trials run as one batch."""
    import torch
    import scenes
    from paper_2609_08800_amd import Simulator, spline_basis
    rng = np.random.default_rng(seed)
    wts = SHAPED_WEIGHTS if weights is None else weights
    worlds = [scenes.robot_world(rng, yaw=float(rng.normal(0, 0.1)), servo_kp=servo_kp, knots=np.zeros((4, K)),
                                 obstacle_size=SYNTHESIS_PALLET) for _ in range(trials)]
    b = scenes.pack(worlds)
    q0 = b.q0.copy()
    for w in range(trials):  # perturbed start
        q0[b.body_off[w]:b.body_off[w + 1], :2] += rng.normal(0, 0.05, 2)
    goal = np.stack([np.full(trials, 3.0), rng.uniform(-0.5, 0.5, trials), rng.uniform(-0.3, 0.3, trials)], axis=1)
    P = scenes.solver_params()
    dev = torch.device("cuda:0")
    sim = Simulator(b, P, device=dev)
    lb = b.body_off[:-1] + b.loss_body
    ref = straight_line_ref(q0[lb, :2], goal, T)
    basis = torch.as_tensor(spline_basis(T, K, P["h"]), device=dev)
    nominal = (goal[:, 0] - q0[lb, 0]) / (T * P["h"]) / scenes.WHEEL_R  # rad/s, per trial
    x0 = np.zeros((sim.NCTRL, K))
    for w in range(trials):
        x0[b.ctrl_off[w]:b.ctrl_off[w + 1]] = nominal[w]
    x = torch.as_tensor(x0, device=dev)
    m, v = torch.zeros_like(x), torch.zeros_like(x)
    ws = sim.new_workspace(T, 10)
    best = np.full(trials, np.inf)
    best_err, best_speed = np.zeros(trials), np.zeros(trials)
    t0 = time.perf_counter()
    for it in range(1, iters + 1):
        r = sim.rollout_shaped(q0, b.u0, x, basis, T, wts, goal, ref, ckpt_every=10,
                               loss_body=b.loss_body, workspace=ws)
        rc = sim.lib.ostrich_adam(x.data_ptr(), r["g_knots"].data_ptr(), m.data_ptr(), v.data_ptr(), x.numel(),
                                  lr, 0.9, 0.999, 1e-8, it, None)
        if rc != 0:
            raise RuntimeError("ostrich_adam failed: %d" % rc)
        loss = r["loss"].cpu().numpy()
        qT, uT = r["qT"].cpu().numpy(), r["uT"].cpu().numpy()
        err = np.hypot(qT[lb, 0] - goal[:, 0], qT[lb, 1] - goal[:, 1])
        speed = np.linalg.norm(uT[lb, :3], axis=1)
        better = np.isfinite(loss) & (loss < best)
        best[better], best_err[better], best_speed[better] = loss[better], err[better], speed[better]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = (best_err < 0.2) & (best_speed < 0.3)
    return {"trials": trials, "adam_iterations": iters, "lr": lr, "T": T, "knots_per_wheel": K,
            "success_rate": round(float(ok.mean()), 3), "median_final_position_error_m": round(float(np.median(best_err)), 4),
            "median_terminal_speed_m_s": round(float(np.median(best_speed)), 4),
            "median_best_loss": round(float(np.median(best)), 5), "seconds": round(dt, 2),
            "servo_kp": servo_kp, "weights": wts}


class _LazyRequestWorlds:
    """A request's packed worlds, built when first read.  Admission only ever looks at
    the head of the queue, so at high arrival rates the requests that never reach it
    within the window are never built; the seed, and so the worlds, are the same."""

    def __init__(self, seed, n_worlds):
        self.n_worlds = n_worlds
        self._seed = seed
        self._b = None

    def __getattr__(self, name):
        if self._b is None:
            import scenes
            self._b = scenes.terrain_request_batch(self._seed, self.n_worlds)
        return getattr(self._b, name)


def serving_measurement(rate, duration, drain, seed=0, capacity=4096, budget_gb=96.0, hmap_slots=64,
                        prebuilt=256):
    """Poisson arrivals of trajectory-optimisation requests (robots on their
    own value-noise terrain, 1..256 worlds, T in 20..100, 10 iterations of
    forward + adjoint + Adam) served with continuous batching; per-iteration
    latency percentiles and served world-steps/s."""
    import scenes
    from paper_2609_08800_amd.serving import GpuBackend, Request, ServingEngine, poisson_arrivals
    P = scenes.solver_params()
    base = scenes.value_noise_heightmap(10_000)
    tmpl = scenes.robot_terrain_world(None, base, 0)
    be = GpuBackend(tmpl, capacity, P, scenes.ROBOT_KNOTS, heightmaps=[base], heightmap_slots=hmap_slots)
    rng = np.random.default_rng(seed)
    arrivals = poisson_arrivals(rate, duration, seed)
    reqs = []
    for i, t in enumerate(arrivals):
        n = int(rng.integers(1, 257))
        # the first requests are built before the clock starts; later ones when they reach the queue's head
        worlds = (scenes.terrain_request_batch(1000 * seed + i, n) if i < prebuilt
                  else _LazyRequestWorlds(1000 * seed + i, n))
        reqs.append(Request(i, worlds, T=int(rng.integers(20, 101)), iters=10, lr=0.1, arrival=t))
    eng = ServingEngine(be, budget_gb * 1e9)
    out = eng.run(reqs, deadline=duration + drain)
    lat = [x for r in out["requests"] + [r for r in out["unfinished"] if r.slot0 >= 0] for x in r.iter_latency]
    admitted = sum(1 for r in reqs if r.slot0 >= 0)
    arrived = sum(1 for r in reqs if r.arrival <= out["wall_s"])
    # offered load: world-steps (forward and adjoint) per second that the arrivals ask for
    offered = rate * 128.5 * 60.0 * 10
    return {"rate_req_per_s": rate, "arrival_window_s": duration, "requests": len(reqs),
            "admitted": admitted, "queued_never_admitted": arrived - admitted,
            "offered_world_steps_per_s": round(offered, 1),
            "completed": len(out["requests"]), "iterations": len(lat),
            "iter_latency_p50_ms": round(1e3 * float(np.percentile(lat, 50)), 1) if lat else None,
            "iter_latency_p99_ms": round(1e3 * float(np.percentile(lat, 99)), 1) if lat else None,
            "served_world_steps_per_s": round(out["world_steps_per_s"], 1), "ticks": out["ticks"],
            "wall_s": round(out["wall_s"], 1), "pool_worlds": capacity}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--worlds", type=int, default=8192)
    ap.add_argument("--T", type=int, default=100)
    ap.add_argument("--ckpt", type=int, default=10)
    ap.add_argument("--team", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=10.0, help="request arrivals per second (0: skip serving)")
    ap.add_argument("--serve-seconds", type=float, default=20.0, help="arrival window of the serving run")
    ap.add_argument("--serve-drain", type=float, default=40.0, help="extra time to finish admitted requests")
    ap.add_argument("--uneven", type=int, default=1, help="also measure the uneven stacks + robots batch")
    ap.add_argument("--synthesis-trials", type=int, default=0,
                    help="trials of the control-synthesis task (0: skip; not part of the default line)")
    ap.add_argument("--serve-sweep", type=str, default="",
                    help="comma-separated arrival rates (req/s) of an additional serving sweep")
    ap.add_argument("--roofline-only", action="store_true",
                    help="one rollout (forward + adjoint, no warm-up) and the solver statistics pass, "
                         "none of the other legs (for hardware-counter runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of 1 GiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        y = x.clone()
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: it measures one GPU's share of worlds "
              "(worlds are independent, so N GPUs would each run 1/N of the batch)", file=sys.stderr)
        sys.exit(2)

    import torch
    import scenes
    from paper_2609_08800_amd import Simulator, spline_basis

    dev = torch.device("cuda:0")
    P = scenes.solver_params()
    W, T = args.worlds, args.T
    batch = scenes.robot_batch(W, seed=0)
    K = scenes.ROBOT_KNOTS
    knots = torch.as_tensor(scenes.knots_array(batch, K), device=dev)
    basis = torch.as_tensor(spline_basis(T, K, P["h"]), device=dev)
    sim = Simulator(batch, P, device=dev, team=args.team)
    q0 = torch.as_tensor(batch.q0, device=dev)
    u0 = torch.as_tensor(batch.u0, device=dev)
    lb = batch.loss_body
    tg = torch.as_tensor(batch.target, device=dev)
    ws = sim.new_workspace(T, args.ckpt)
    torch.cuda.synchronize()

    def one_step():
        return sim.rollout(q0, u0, knots, basis, T, ckpt_every=args.ckpt, loss_body=lb, target=tg,
                           phase=3, workspace=ws)

    if args.roofline_only:
        args.steps, args.warmup = 1, 0
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats(dev)
    # the dominant kernel's launches inside the timed region are bracketed by
    # HIP events on their stream and their algorithmic flops are counted on
    # the device from the kernels' own row and iteration counts
    sim.timing(1)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = one_step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sim.timing(0)
    fwd = sim.timing(2)
    adj = sim.timing(3)
    ms = dt / args.steps * 1e3
    world_steps = W * T * args.steps
    value = world_steps / dt
    peak_gb = (torch.cuda.max_memory_allocated(dev)) / 1e9
    progress(f"timed region done: {args.steps} steps in {dt:.2f} s")

    # Forward-only pass of the same trajectory (outside the timed region): solver statistics.
    q, u = q0.clone(), u0.clone()
    lam = torch.zeros(max(sim.NL, 1), dtype=torch.float64, device=dev)
    ctrl_all = basis @ knots.t()
    sim.timing(1)
    iters_all, m_all, st_all = [], [], []
    base_rows = np.array([5 * (batch.joint_off[w + 1] - batch.joint_off[w]) + batch.worlds[w].n_servo
                          for w in range(W)])
    for k in range(T):
        o = sim.step_forward(q, u, lam, ctrl_all[k])
        iters_all.append(o["iters"].cpu().numpy())
        m_all.append(base_rows + 3 * o["n_act"].cpu().numpy())
        st_all.append(o["status"].cpu().numpy())
        q, u, lam = o["q"], o["u"], o["lam"]
    sim.timing(0)
    fo = sim.timing(2)
    progress("solver statistics pass done")
    # One "launch" is one forward step of the whole batch: the contact count, the
    # launch plan and the tiered k_forward launches (first carve, full carve on
    # a side stream, deferred worlds), bracketed by one pair of events.  Its
    # work is the roofline count sum_k (m^3/3 + 14 m^2 + 170 m) over the worlds'
    # Newton iterations; the implementation's finer count is given beside it.
    avg_ms = fwd["ms"] / max(fwd["launches"], 1)
    flop_per_launch = fwd["flops"] / max(fwd["launches"], 1)
    achieved = flop_per_launch / (avg_ms * 1e-3) / 1e12
    fine = fwd["flops_fine"] / max(fwd["launches"], 1)
    traffic = recorded_traffic()
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 5),
                "traffic": traffic, "kernel": "k_forward (one forward step of the batch)",
                "launches_timed": fwd["launches"], "avg_launch_ms": round(avg_ms, 4),
                "flop_per_launch": flop_per_launch,
                "flop_formula": "sum over worlds and Newton iterations of m^3/3 + 14 m^2 + 170 m",
                "finer_count": {"flop_per_launch": fine,
                                "achieved": round(fine / (avg_ms * 1e-3) / 1e12, 4),
                                "frac": round(fine / (avg_ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 5)}}
    adjoint_roofline = None
    if adj["launches"]:
        a_ms = adj["ms"] / adj["launches"]
        a_bytes = adj["bytes"] / adj["launches"]
        a_fine = adj["bytes_fine"] / adj["launches"]
        a_gbs = a_bytes / (a_ms * 1e-3) / 1e9
        adjoint_roofline = {"bound": "hbm", "achieved": round(a_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(a_gbs / HBM_PEAK_GBS, 5),
                            "traffic": recorded_traffic("adjoint_hbm_bytes_per_launch"),
                            "kernel": "k_adjoint (one adjoint step of the batch)",
                            "launches_timed": adj["launches"], "avg_launch_ms": round(a_ms, 4),
                            "bytes_per_launch": a_bytes,
                            "byte_formula": "8 (26 n_b + multipliers + m (m + 1) / 2) per world",
                            "finer_count": {"bytes_per_launch": a_fine,
                                            "achieved": round(a_fine / (a_ms * 1e-3) / 1e9, 2)}}
    ckpt_modes = None
    if not args.roofline_only:
        ckpt_modes = checkpoint_measurement(sim, q0, u0, knots, basis, T, lb, tg, W)
        progress("checkpoint modes done")
    plain = None
    if not args.roofline_only:
        plain = plain_path_measurement()
        plain["batched_over_plain"] = round(value / plain["world_steps_per_s"], 1)
        progress("plain path done")
    shaped = synthesis = None
    if not args.roofline_only:
        shaped = shaped_measurement(sim, q0, u0, knots, basis, T, batch, args.ckpt)
        progress("shaped-loss rollout done")
        if args.synthesis_trials > 0:
            synthesis = control_synthesis_measurement(trials=args.synthesis_trials)
            progress("control synthesis done")
    uneven = None
    if args.uneven and not args.roofline_only:
        uneven = uneven_measurement()
        progress("uneven batch done")
    serving = None
    if args.serve_rate > 0 and not args.roofline_only:
        serving = serving_measurement(args.serve_rate, args.serve_seconds, args.serve_drain)
        progress("serving done")
    sweep = None
    if args.serve_sweep and not args.roofline_only:
        sweep = []
        for r in args.serve_sweep.split(","):
            sweep.append(serving_measurement(float(r), args.serve_seconds, args.serve_drain))
            progress(f"serving at {r} req/s done")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline()
        progress("cpu baseline done")
    iters_all = np.array(iters_all)
    status = np.array(st_all)
    line = {
        "metric": "fwd+adjoint world-steps/s at 8192 worlds (FP64); p50/p99 served iter latency",
        "value": round(value, 2),
        "unit": "world-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "robot_over_box_obstacle", "worlds": W, "T": T, "h": P["h"],
                   "ckpt_every": args.ckpt, "newton_k_max": P["k_max"], "tol": P["tol"],
                   "parallelism": "one workgroup per world"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": {"peak_hbm_gb": round(peak_gb, 3),
                  "forward_only_world_steps_per_s": round(W * fo["launches"] / (fo["ms"] * 1e-3), 1),
                  "mean_newton_iters": round(float(iters_all.mean()), 3),
                  "frac_converged": round(float(np.mean(status & 1)), 4),
                  "frac_budget": round(float(np.mean((status & 2) > 0)), 4),
                  "frac_worlds_nonfinite_at_T": round(float(np.mean((status[-1] & 4) > 0)), 4),
                  # the worlds whose state is still finite at T: their world-steps per second
                  # of the same timed region (the others leave Newton early and cost less)
                  "finite_worlds_world_steps_per_s": round(value * float(np.mean((status[-1] & 4) == 0)), 1),
                  "mean_rows": round(float(np.mean(m_all)), 2),
                  "adjoint_roofline": adjoint_roofline,
                  "checkpointing": ckpt_modes,
                  "plain_path": plain,
                  "shaped_loss_rollout": shaped,
                  "control_synthesis": synthesis,
                  "uneven_batch": uneven,
                  "serving": serving,
                  "serving_sweep": sweep},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
