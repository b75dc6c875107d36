"""Throughput of the batched drone step on one MI355X.

One bench step is one pass of the whole hot path over the uneven mixed batch
(2048 worlds, log-uniform 1..4000 drones each, half first-principles with the
attitude PID, half identified model, RK4 at dt = 2 ms):
  1. masked reset of every world to its initial state;
  2. 1000 held-command steps of all drones in one launch sequence (fused
     kernel, per-world tiles or the persistent work queue, autotuned);
  3. forward rollout (per-step commands, linear feedback, figure-eight
     tracking loss, checkpoints) and the hand-written adjoint on the seeded
     256-world subset, 1000 steps.
Part 3 is independent of parts 1-2 and runs on a second stream (default
priority) so that its latency-bound adjoint fills SIMD slots the forward leaves
idle. value = (D * T + D_sub * T) / wall time of the step (drone-steps/s),
inputs resident in HBM. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Algorithmic FP32 work per drone-step of the discrete map (add/sub/mul = 1,
# FMA = 2, each sqrt/rsqrt/sin-cos pair/atan2/asin = 1; no compensation or
# rotor-deviation bookkeeping), the smaller of two counts per path (an
# estimate from the equations and a line-by-line tally of them):
# first-principles RK4 at the rotor interface 596 + 1 rsqrt; with the attitude
# PID and allocation 806 + 4 sqrt + atan2 + asin; identified model RK4 293 + 12
# sin-cos; identified rollout with the 4x13 feedback and the tracking loss 413
# per step forward, and forward + checkpoint recompute + reverse 413 + 413 + 1000.
FLOPS_PER_DS = {"fp_rotor_rk4": 597.0, "fp_pid_rk4": 812.0, "id_rk4": 305.0,
                "id_rollout_fwd": 413.0, "id_rollout_fwd_bwd": 1826.0}
SPEC_FP32_VECTOR_TFLOPS = 157.3     # MI355X FP32 vector peak
# job steps timed per candidate when the launch choices are tuned inside the job
# (job steps vary by about 3 %; the median of 8 separates candidates 2 % apart)
TUNE_STEPS = 8
SPEC_HBM_GBS = 8000.0

# HBM bytes of one launch of the dominant kernel (the first-principles held-step
# work-queue kernel inside the job), FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (the
# factors a 256 MiB device copy gives) from two rocprofv3 --pmc runs, keyed by
# launch configuration "workqueue,tile,chunk,per_model"; summary in
# profiles/held_step_uneven_mixed_2048w_T1000.md. Valid only for the kernel
# sources it was measured on (SHA-256 below), reported as null otherwise.
PROFILED_TRAFFIC = {"sources_sha256": "c247793ad9bfb4d4c921b12a5793c93d669903915fbbb998d13e87b43f612cb7",
                    "by_launch": {"1,64,100,1": 134419568, "1,256,100,1": 115490200}}


def kernel_sources_sha256() -> str:
    """Hash of the sources that make up the held-step kernels and their launch."""
    import hashlib
    h = hashlib.sha256()
    for name in ("cf_api.hip", "cf_device.hpp", "cf_internal.hpp", "cf_layout.hpp", "cf_step.hip"):
        f = os.path.join(ROOT, "paper_2606_01478_amd", "csrc", name)
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--seed", type=int, default=1005)
    p.add_argument("--horizon", type=int, default=1000)
    p.add_argument("--ckpt", type=int, default=0,
                   help="checkpoint interval; 0 = tune among 1, 2, 5, 10, 50, 100 (alone, then in the job)")
    p.add_argument("--serial", action="store_true", help="run the subset adjoint after the forward")
    p.add_argument("--wq-waves", type=int, default=-1,
                   help="cap on the held step's resident work-queue waves per compute unit; -1 = tune in the job")
    p.add_argument("--no-standalone", action="store_true",
                   help="skip the standalone phase timings (profiler runs: every held-step dispatch is in the job)")
    p.add_argument("--graph", action="store_true",
                   help="time the job with the held steps replayed from a hipGraph (default: enqueued directly; "
                        "the other form is timed too and reported under graph_comparison)")
    p.add_argument("--autotune-ms", type=int, default=3000)
    p.add_argument("--launch", default="",
                   help="pin the held-step launch as 'workqueue,tile,chunk,per_model' (e.g. 1,64,100,1) "
                        "instead of autotuning it (profiler runs of one configuration)")
    p.add_argument("--adjoint-only", action="store_true",
                   help="only the forward rollout and adjoint of the 256-world subset, alone on the GPU "
                        "(profiler runs of the rollout kernels)")
    p.add_argument("--job-only", action="store_true",
                   help="only the timed job (for profiler runs): no comparators, configurations or baselines")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    p.add_argument("--no-comparators", action="store_true")
    p.add_argument("--no-workloads", action="store_true",
                   help="skip the per-configuration records (plain forward, closed loop, swarm, differentiable)")
    p.add_argument("--copy-probe", action="store_true", help="also run a 256 MiB device copy (profile scale)")
    p.add_argument("--no-hbm-sweep", action="store_true",
                   help="skip the plain and fused kernels on 2^20..2^24 single drones (HBM roofline)")
    p.add_argument("--no-mppi", action="store_true",
                   help="skip the sampled-rollout controller measurement (5 x 100k samples x 25 steps)")
    p.add_argument("--no-grad-bench", action="store_true",
                   help="skip the gradient-throughput measurement (2^20 worlds, 10 steps)")
    p.add_argument("--no-bptt", action="store_true",
                   help="skip the BPTT training-loop measurement (16 worlds, 40-step rollouts)")
    p.add_argument("--interfaces", action="store_true",
                   help="also time held steps behind each control interface (2^20 single-drone worlds)")
    a = p.parse_args()
    if a.job_only:
        a.no_cpu_baseline = a.no_comparators = a.no_workloads = a.no_hbm_sweep = True
        a.no_mppi = a.no_grad_bench = a.no_bptt = True
    return a


def stats(xs):
    xs = np.asarray(xs, np.float64)
    return {"mean": float(xs.mean()), "std": float(xs.std()), "median": float(np.median(xs)),
            "min": float(xs.min()), "max": float(xs.max()), "n": int(len(xs))}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; sharding across GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import workloads as W
    from paper_2606_01478_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    T = args.horizon
    w = W.uneven_mixed(seed=args.seed, steps=T)
    ws = W.uneven_mixed_adjoint(seed=args.seed, steps=T)
    D, Ds = w.n_drones_total, ws.n_drones_total
    t2d = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(dt)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    # the held-step handle: autotuned launch shape, per-launch timing events, and
    # (unless --no-graph) hipGraph replay of its launch sequence
    tune = B.Sim.from_workload(w)
    init = t2d(w.x0)
    state = init.clone()
    cmd = t2d(w.cmds)
    mask = torch.ones(w.n_worlds, dtype=torch.uint8, device=dev)
    if args.launch:
        wq_, tile_, chunk_, split_ = (int(v) for v in args.launch.split(","))
        tune.set_launch_config(wq_, tile_, chunk_, split_)
    elif args.autotune_ms > 0:
        tune.autotune(state, cmd, T, args.autotune_ms)
    cfg = tune.launch_config()
    tune.close()
    sim = B.Sim.from_workload(w, flags=B.F_GRAPH if args.graph else 0)
    sim.set_launch_config(cfg["workqueue"], cfg["tile"], cfg["chunk"], cfg["per_model_launches"])
    simO = B.Sim.from_workload(w, flags=0 if args.graph else B.F_GRAPH)   # the other form
    simO.set_launch_config(cfg["workqueue"], cfg["tile"], cfg["chunk"], cfg["per_model_launches"])
    # the same launches enqueued directly with an event pair around each kernel
    # launch, for the kernels' own durations (a graph replay is timed as a whole)
    simT = B.Sim.from_workload(w, flags=B.F_TIMING)
    simT.set_launch_config(cfg["workqueue"], cfg["tile"], cfg["chunk"], cfg["per_model_launches"])

    simA = B.Sim.from_workload(ws)
    x0s, cmds_s = t2d(ws.x0), t2d(ws.cmds)
    gain, off = t2d(ws.gain), t2d(ws.ref_offset)
    obj = B.Sim.objective(gain=gain, ref_amp=ws.ref_amp, ref_period=ws.ref_period, ref_offset=off, w_u=ws.w_u)
    dloss = t2d(ws.dloss)
    g_cmds, g_x0, g_gain = torch.empty_like(cmds_s), torch.empty_like(x0s), torch.empty_like(gain)
    loss = torch.empty(Ds, device=dev)
    loss_w = torch.empty(ws.n_worlds, device=dev)

    def adjoint_buffers(K):
        return simA.ckpt_buffer(T, K, device=dev)

    def adjoint(K, ckpt):
        simA.rollout(x0s, cmds_s, T, obj, K, ckpt=ckpt, loss=loss, loss_world=loss_w)
        simA.rollout_backward(x0s, cmds_s, T, obj, K, ckpt, dloss=dloss, g_cmds=g_cmds, g_x0=g_x0, g_gain=g_gain)

    if args.adjoint_only:
        # the subset's forward rollout and adjoint alone, checkpoint interval
        # --ckpt (default 1), `steps` timed repetitions
        Ka = max(args.ckpt, 1)
        ck = adjoint_buffers(Ka)
        for _ in range(max(args.warmup, 1)):
            adjoint(Ka, ck)
        torch.cuda.synchronize()
        recs = []
        for _ in range(args.steps):
            e = [ev() for _ in range(3)]
            e[0].record()
            simA.rollout(x0s, cmds_s, T, obj, Ka, ckpt=ck, loss=loss, loss_world=loss_w)
            e[1].record()
            simA.rollout_backward(x0s, cmds_s, T, obj, Ka, ck, dloss=dloss, g_cmds=g_cmds, g_x0=g_x0, g_gain=g_gain)
            e[2].record()
            recs.append(e)
        torch.cuda.synchronize()
        if simA.last_error() != 0:
            raise RuntimeError("device error in the adjoint run")
        fwd = [r[0].elapsed_time(r[1]) for r in recs]
        bwd = [r[1].elapsed_time(r[2]) for r in recs]
        ms = float(np.mean(fwd) + np.mean(bwd))
        print(json.dumps({"metric": "adjoint subset drone-steps/s (forward + backward)", "value": Ds * T / (ms * 1e-3),
                          "unit": "drone-steps/s", "ckpt_every": Ka, "drones": Ds, "horizon": T,
                          "forward_ms": stats(fwd), "backward_ms": stats(bwd)}))
        return

    side = torch.cuda.Stream(device=dev)   # default priority
    cur = {}                               # checkpoint interval and buffer of the job

    def one_step(record=None, sim=sim):
        K, ckpt = cur["K"], cur["ckpt"]
        e = [ev() for _ in range(7)]
        main = torch.cuda.current_stream()
        e[0].record(main)
        if args.serial:
            sim.reset(state, init, mask)
            e[1].record(main)
            sim.step_k(state, cmd, T)
            e[2].record(main)
            simA.rollout(x0s, cmds_s, T, obj, K, ckpt=ckpt, loss=loss, loss_world=loss_w)
            e[3].record(main)
            simA.rollout_backward(x0s, cmds_s, T, obj, K, ckpt, dloss=dloss, g_cmds=g_cmds, g_x0=g_x0,
                                  g_gain=g_gain)
            e[4].record(main)
            e[5].record(main)
        else:
            side.wait_event(e[0])
            with torch.cuda.stream(side):
                e[2].record(side)
                simA.rollout(x0s, cmds_s, T, obj, K, ckpt=ckpt, loss=loss, loss_world=loss_w)
                e[3].record(side)
                simA.rollout_backward(x0s, cmds_s, T, obj, K, ckpt, dloss=dloss, g_cmds=g_cmds, g_x0=g_x0,
                                      g_gain=g_gain)
                e[4].record(side)
            sim.reset(state, init, mask)
            if cur.get("fwd_first"):
                # the held steps start once the subset's forward rollout is done
                # (it then runs with the GPU to itself)
                main.wait_event(e[3])
            e[1].record(main)
            sim.step_k(state, cmd, T)
            e[5].record(main)
            main.wait_event(e[4])
        e[6].record(main)
        if record is not None:
            record.append(e)

    # checkpoint interval: the caller's choice; otherwise the candidates whose
    # adjoint alone is within 10 % of the fastest are tried inside the
    # overlapped job (median of TUNE_STEPS job steps) and the fastest job wins
    if args.ckpt > 0:
        cands = [args.ckpt]
    else:
        alone = []
        for Kc in (1, 2, 5, 10, 50, 100):
            ck = adjoint_buffers(Kc)
            adjoint(Kc, ck)
            a, b = ev(), ev()
            a.record()
            adjoint(Kc, ck)
            b.record()
            torch.cuda.synchronize()
            alone.append((Kc, a.elapsed_time(b)))
            del ck
        fastest = min(ms for _, ms in alone)
        cands = [Kc for Kc, ms in alone if ms <= 1.1 * fastest]
    K = cands[0]
    if len(cands) > 1:
        best = None
        for Kc in cands:
            cur["K"], cur["ckpt"] = Kc, adjoint_buffers(Kc)
            one_step()
            torch.cuda.synchronize()
            trial = []
            for _ in range(TUNE_STEPS):
                one_step(trial)
            torch.cuda.synchronize()
            med = float(np.median([r[0].elapsed_time(r[6]) for r in trial]))
            if best is None or med < best[1]:
                best = (Kc, med)
            del cur["ckpt"]
        K = best[0]
    cur["K"], cur["ckpt"] = K, adjoint_buffers(K)
    ckpt = cur["ckpt"]
    # tile size of the held step inside the job: on the held steps alone the
    # candidate tiles come out within a few per cent of each other, and the
    # overlap with the adjoint decides between them (median of TUNE_STEPS job steps each)
    if not args.serial and not args.launch:
        best_t = None
        for tl in sorted({64, 256, cfg["tile"]}):
            for h_ in (sim, simO, simT):
                h_.set_launch_config(cfg["workqueue"], tl, cfg["chunk"], cfg["per_model_launches"],
                                     max(args.wq_waves, 0))
            one_step()
            torch.cuda.synchronize()
            trial = []
            for _ in range(TUNE_STEPS):
                one_step(trial)
            torch.cuda.synchronize()
            med = float(np.median([r[0].elapsed_time(r[6]) for r in trial]))
            if best_t is None or med < best_t[1]:
                best_t = (tl, med)
        cfg["tile"] = best_t[0]
        for h_ in (sim, simO, simT):
            h_.set_launch_config(cfg["workqueue"], cfg["tile"], cfg["chunk"], cfg["per_model_launches"],
                                 max(args.wq_waves, 0))
    # resident work-queue waves per compute unit of the held step inside the job:
    # every wave that fits, or fewer so that the adjoint's waves, whose chain is
    # the job's critical path, find registers and issue slots on more SIMDs
    # (median of TUNE_STEPS job steps per candidate)
    wq_best = (max(args.wq_waves, 0), None)
    if cfg["workqueue"] and not args.serial and args.wq_waves < 0:
        for cap in (0, 8, 4, 2):
            for h_ in (sim, simO, simT):
                h_.set_launch_config(cfg["workqueue"], cfg["tile"], cfg["chunk"], cfg["per_model_launches"], cap)
            one_step()
            torch.cuda.synchronize()
            trial = []
            for _ in range(TUNE_STEPS):
                one_step(trial)
            torch.cuda.synchronize()
            med = float(np.median([r[0].elapsed_time(r[6]) for r in trial]))
            if wq_best[1] is None or med < wq_best[1]:
                wq_best = (cap, med)
    for h_ in (sim, simO, simT):
        h_.set_launch_config(cfg["workqueue"], cfg["tile"], cfg["chunk"], cfg["per_model_launches"], wq_best[0])
    # schedule inside the job: everything overlapped from the start, or the held
    # steps held back until the subset's forward rollout is done (median of TUNE_STEPS
    # job steps each)
    if not args.serial:
        sched = []
        for ff in (False, True):
            cur["fwd_first"] = ff
            one_step()
            torch.cuda.synchronize()
            trial = []
            for _ in range(TUNE_STEPS):
                one_step(trial)
            torch.cuda.synchronize()
            sched.append((float(np.median([r[0].elapsed_time(r[6]) for r in trial])), ff))
        cur["fwd_first"] = min(sched)[1]
    # standalone phases (nothing else on the GPU), HIP events on the same streams;
    # the held steps alone run with every work-queue wave that fits (the cap only
    # serves the overlap)
    standalone = {"adjoint_fwd_bwd": float("nan"), "forward": float("nan")}
    standalone_launch_ms = {"first_principles": [float("nan")], "identified": []}
    if not args.no_standalone:
        adjoint(K, ckpt)
        a, b = ev(), ev()
        a.record()
        adjoint(K, ckpt)
        b.record()
        for h_ in (sim, simT):
            h_.set_launch_config(cfg["workqueue"], cfg["tile"], cfg["chunk"], cfg["per_model_launches"], 0)
        sim.step_k(state, cmd, T)
        c = ev()
        c.record()
        torch.cuda.synchronize()
        standalone = {"adjoint_fwd_bwd": a.elapsed_time(b), "forward": b.elapsed_time(c)}
        simT.step_k(state, cmd, T)
        torch.cuda.synchronize()
        standalone_launch_ms = {"first_principles": simT.launch_times(0),
                                "identified": simT.launch_times(1) if cfg["per_model_launches"] else []}
        for h_ in (sim, simT):
            h_.set_launch_config(cfg["workqueue"], cfg["tile"], cfg["chunk"], cfg["per_model_launches"], wq_best[0])

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if sim.last_error() != 0 or simA.last_error() != 0:
        raise RuntimeError("device error during the timed region")
    # the same job with the held steps in the other form (graph replay or direct)
    for _ in range(args.warmup + 1):
        one_step(sim=simO)
    torch.cuda.synchronize()
    recsO = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(recsO, sim=simO)
    torch.cuda.synchronize()
    wallO = time.perf_counter() - t0
    jobO = np.array([r[0].elapsed_time(r[6]) for r in recsO])
    # the two forms alternated step by step (same conditions for both; the
    # blocks above run one after the other)
    alt = {"timed_form": [], "other_form": []}
    for i in range(2 * max(args.steps, 4)):
        rec = []
        one_step(rec, sim=sim if i % 2 == 0 else simO)
        torch.cuda.synchronize()
        alt["timed_form" if i % 2 == 0 else "other_form"].append(rec[0][0].elapsed_time(rec[0][6]))
    # per-launch durations of the held-step kernels inside the job: the same job
    # steps with the directly enqueued, event-timed handle (HIP events the
    # library records around each launch on the stream it is launched on)
    launch_ms = {"first_principles": [], "identified": []}
    for _ in range(max(3, args.steps)):
        one_step(sim=simT)
        torch.cuda.synchronize()
        launch_ms["first_principles"] += simT.launch_times(0)
        if cfg["per_model_launches"]:
            launch_ms["identified"] += simT.launch_times(1)
    # per-phase durations from the events (ms); with overlap the forward is
    # e[1]->e[5] on the main stream and the adjoint e[2]->e[4] on the side stream
    if args.serial:
        ph = np.array([[r[0].elapsed_time(r[1]), r[1].elapsed_time(r[2]), r[2].elapsed_time(r[3]),
                        r[3].elapsed_time(r[4])] for r in recs])
    else:
        ph = np.array([[r[0].elapsed_time(r[1]), r[1].elapsed_time(r[5]), r[2].elapsed_time(r[3]),
                        r[3].elapsed_time(r[4])] for r in recs])
    step_ms = wall * 1e3 / args.steps
    job = np.array([r[0].elapsed_time(r[6]) for r in recs])
    fwd_ms = float(ph[:, 1].mean())
    rf_ms, rb_ms = float(ph[:, 2].mean()), float(ph[:, 3].mean())

    # the dominant kernel: the first-principles held-step kernel (attitude PID,
    # RK4) over its tiles, one launch per `chunk` steps
    world = np.repeat(np.arange(w.n_worlds), w.drones_per_world)
    n_fp = int((w.model_per_world[world] == W.MODEL_FP).sum())
    n_id = D - n_fp
    steps_per_launch = T if cfg["chunk"] <= 0 else min(cfg["chunk"], T)
    n_chunks = -(-T // steps_per_launch)
    flops_fp_launch = n_fp * FLOPS_PER_DS["fp_pid_rk4"] * steps_per_launch
    flops_id_launch = n_id * FLOPS_PER_DS["id_rk4"] * steps_per_launch
    bytes_fp_launch = n_fp * (2 * W.S_FP_PID * 4 + 16)
    fp_ms = float(np.mean(launch_ms["first_principles"]))
    fp_ms_alone = float(np.mean(standalone_launch_ms["first_principles"]))
    achieved = flops_fp_launch / (fp_ms * 1e-3) / 1e12
    flops_phase = (n_fp * FLOPS_PER_DS["fp_pid_rk4"] + n_id * FLOPS_PER_DS["id_rk4"]) * T
    value = (D * T + Ds * T) / (step_ms * 1e-3)
    traffic = None
    if kernel_sources_sha256() == PROFILED_TRAFFIC["sources_sha256"]:
        traffic = PROFILED_TRAFFIC["by_launch"].get(
            "%d,%d,%d,%d" % (cfg["workqueue"], cfg["tile"], cfg["chunk"], cfg["per_model_launches"]))
    out = {
        "metric": "drone-steps/s fwd & fwd+bwd on 1 MI355X vs plain kernel; % of VALU/HBM roofline",
        "value": value, "unit": "drone-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded Philox, Crazyflie-class parameters)",
        "config": {"workload": "uneven_mixed_2048w_logu1-4000_T1000_plus_adjoint_256w",
                   "worlds": w.n_worlds, "drones": D, "horizon": T, "adjoint_worlds": ws.n_worlds,
                   "adjoint_drones": Ds, "ckpt_every": K, "integrator": "rk4", "dt": w.dt,
                   "launch": dict(cfg, wq_waves_per_cu=wq_best[0]), "hipgraph": bool(args.graph),
                   "held_steps_after_subset_forward": bool(cur.get("fwd_first", False)),
                   "adjoint_overlapped": not args.serial},
        "fwd_drone_steps_per_s": D * T / (fwd_ms * 1e-3),
        "fwdbwd_drone_steps_per_s": Ds * T / ((rf_ms + rb_ms) * 1e-3),
        "step_ms_stats": stats(job),
        "graph_comparison": {"held_steps_replayed_from_hipgraph": not args.graph,
                             "ms_per_step": wallO * 1e3 / args.steps, "step_ms_stats": stats(jobO),
                             "value": (D * T + Ds * T) / (wallO / args.steps),
                             "alternating_step_ms": {k: stats(v) for k, v in alt.items()}},
        "phase_ms": {"reset": float(ph[:, 0].mean()), "forward": fwd_ms, "rollout_fwd": rf_ms,
                     "rollout_bwd": rb_ms, "forward_std": float(ph[:, 1].std())},
        "standalone_ms": standalone,
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": SPEC_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / SPEC_FP32_VECTOR_TFLOPS, "traffic": traffic,
            "kernel": "k_step_wq<first-principles, attitude PID, RK4> (held-command steps of the "
                      "first-principles worlds, %d launches of %d steps per job step)" % (n_chunks, steps_per_launch),
            "flops_per_launch": flops_fp_launch, "flops_per_drone_step": FLOPS_PER_DS["fp_pid_rk4"],
            "drone_steps_per_launch": n_fp * steps_per_launch,
            "algorithmic_bytes_per_launch": bytes_fp_launch,
            "launch_ms_in_job": fp_ms, "launch_ms_in_job_stats": stats(launch_ms["first_principles"]),
            "launch_ms_standalone": fp_ms_alone,
            "achieved_standalone": flops_fp_launch / (fp_ms_alone * 1e-3) / 1e12,
            "frac_standalone": flops_fp_launch / (fp_ms_alone * 1e-3) / 1e12 / SPEC_FP32_VECTOR_TFLOPS,
            "identified_kernel": {
                "launch_ms_in_job": float(np.mean(launch_ms["identified"])) if launch_ms["identified"] else None,
                "flops_per_launch": flops_id_launch,
                "achieved_in_job": (flops_id_launch / (np.mean(launch_ms["identified"]) * 1e-3) / 1e12
                                    if launch_ms["identified"] else None)},
            "phase": {"flops": flops_phase, "ms_in_job": fwd_ms, "ms_standalone": standalone["forward"],
                      "achieved_in_job": flops_phase / (fwd_ms * 1e-3) / 1e12,
                      "achieved_standalone": flops_phase / (standalone["forward"] * 1e-3) / 1e12},
            "note": "achieved: the kernel's average launch duration inside the job (HIP events the library "
                    "records around each launch on its stream, in job steps identical to the timed ones but "
                    "enqueued directly instead of replayed from the graph; the job overlaps the adjoint); "
                    "standalone: the same launches with nothing else on the GPU"},
    }

    if not args.no_comparators:
        # plain single-step kernel over the whole batch (one launch per step)
        simP = B.Sim.from_workload(w, flags=B.F_PLAIN_KERNEL | B.F_NO_AUTOTUNE_CACHE)
        xs = init.clone()
        n_plain = 50
        simP.step_k(xs, cmd, 5)
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        simP.step_k(xs, cmd, n_plain)
        b.record()
        torch.cuda.synchronize()
        plain_ms = a.elapsed_time(b) / n_plain
        out["plain_kernel_drone_steps_per_s"] = D / (plain_ms * 1e-3)
        # algorithmic bytes per drone-step: state in + out + held command
        plain_bytes = n_fp * (2 * W.S_FP_PID * 4 + 16) + n_id * (2 * W.S_ID * 4 + 16)
        out["plain_kernel_bytes_per_step"] = plain_bytes
        out["plain_kernel_gbs"] = plain_bytes / (plain_ms * 1e-3) / 1e9
        simP.close()
        # per-world loop of plain launches (one handle per world), a few steps
        handles = []
        offs = w.world_offsets()
        for i in range(w.n_worlds):
            sub = W.subset(w, [i])
            h = B.Sim.from_workload(sub, flags=B.F_PLAIN_KERNEL | B.F_NO_AUTOTUNE_CACHE)
            handles.append((h, state[:h.S, offs[i]:offs[i + 1]].clone(), cmd[:, offs[i]:offs[i + 1]].contiguous()))
        n_loop = 5
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        for h, xs_i, u_i in handles:
            h.step_k(xs_i, u_i, n_loop)
        b.record()
        torch.cuda.synchronize()
        out["per_world_loop_drone_steps_per_s"] = D * n_loop / (a.elapsed_time(b) * 1e-3)
        for h, _, _ in handles:
            h.close()

    if not args.job_only:
        pk = measured_peaks(B, dev, ev)
        out["peaks_measured"] = pk
        out["roofline"]["frac_of_measured_fma_peak"] = out["roofline"]["achieved"] / pk["fp32_fma_tflops"]
        out["roofline"]["frac_standalone_of_measured_fma_peak"] = (out["roofline"]["achieved_standalone"]
                                                                  / pk["fp32_fma_tflops"])
    if not args.no_workloads:
        out["other_workloads"] = workload_records(B, W, dev, t2d, ev)
    if not args.no_grad_bench:
        out["gradient_benchmark"] = gradient_benchmark(B, W, dev, t2d, ev)
    if not args.no_mppi:
        out["mppi"] = mppi_benchmark(B, W, dev, t2d, ev)
    if not args.no_bptt:
        out["bptt"] = bptt_benchmark(B, W, dev, t2d, ev)
    if not args.no_hbm_sweep:
        out["hbm_sweep"] = hbm_sweep(B, W, dev, t2d, ev)
    if args.interfaces:
        out["interfaces"] = interface_benchmark(B, W, dev, t2d, ev)

    if args.copy_probe:
        src = torch.empty(64 * 1024 * 1024, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        out["cpu_baseline_1_thread"] = cpu_baseline(w, args.cpu_seconds, threads=1)
    print(json.dumps(out), flush=True)


def _time(fn, reps, ev):
    """Per-call milliseconds of fn() over `reps` calls (one warm-up), HIP events on
    the current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = ev(), ev()
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return stats(ts)


def workload_records(B, W, dev, t2d, ev):
    """The other four configurations, each at its full size: drone-steps/s of the
    plain single-step kernel and of the fused / batched forms on the same GPU,
    and the ALU roofline fraction of the fused forms."""
    import torch
    peak = SPEC_FP32_VECTOR_TFLOPS
    out = {}

    # 1: plain forward, first-principles rotor interface, 16 x 1, 500 steps, per-step commands
    w = W.fp_rotor_open_loop()
    T, D = w.steps, w.n_drones_total
    x0, cmds = t2d(w.x0), t2d(w.cmds)
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    xT = torch.empty_like(x0)
    fused = _time(lambda: sim.rollout(x0, cmds, T, None, T, x_T=xT), 10, ev)
    simP = B.Sim.from_workload(w, flags=B.F_PLAIN_KERNEL | B.F_NO_AUTOTUNE_CACHE)
    x = x0.clone()
    steps_cmd = [cmds[t] for t in range(T)]

    def plain():
        for t in range(T):
            simP.step_k(x, steps_cmd[t], 1)
    pl = _time(plain, 3, ev)
    fl = FLOPS_PER_DS["fp_rotor_rk4"] * D * T
    out["fp_rotor_16x1_T500"] = {
        "drones": D, "steps": T, "fused_rollout_ms": fused, "plain_ms": pl,
        "fused_drone_steps_per_s": D * T / (fused["mean"] * 1e-3),
        "plain_drone_steps_per_s": D * T / (pl["mean"] * 1e-3),
        "fused_frac_alu": fl / (fused["mean"] * 1e-3) / 1e12 / peak, "waves": 1,
        "note": "one wave of 16 lanes: latency-bound; the plain form is 500 launches of one step"}
    sim.close()
    simP.close()

    # 2: closed loop 4096 x 1, 1000 steps, attitude PID
    w = W.fp_pid_closed_loop()
    T, D = w.steps, w.n_drones_total
    x0, u = t2d(w.x0), t2d(w.cmds)
    sim = B.Sim.from_workload(w)
    x = x0.clone()
    sim.autotune(x, u, T, 500)
    fused = _time(lambda: sim.step_k(x, u, T), 5, ev)
    simP = B.Sim.from_workload(w, flags=B.F_PLAIN_KERNEL | B.F_NO_AUTOTUNE_CACHE)
    pl = _time(lambda: simP.step_k(x, u, T), 3, ev)
    fl = FLOPS_PER_DS["fp_pid_rk4"] * D * T
    out["fp_pid_4096x1_T1000"] = {
        "drones": D, "steps": T, "fused_ms": fused, "plain_ms": pl, "launch": sim.launch_config(),
        "fused_drone_steps_per_s": D * T / (fused["mean"] * 1e-3),
        "plain_drone_steps_per_s": D * T / (pl["mean"] * 1e-3),
        "plain_gbs": D * T * (2 * W.S_FP_PID * 4 + 16) / (pl["mean"] * 1e-3) / 1e9,
        "fused_frac_alu": fl / (fused["mean"] * 1e-3) / 1e12 / peak, "waves": D // 64}
    sim.close()
    simP.close()

    # 3: swarm 64 x 4000, identified model, 1000 steps: plain and fused K = 1, 10, 100
    w = W.id_swarm()
    T, D = w.steps, w.n_drones_total
    x0, u = t2d(w.x0), t2d(w.cmds)
    rec = {"drones": D, "steps": T, "waves": D // 64}
    fl = FLOPS_PER_DS["id_rk4"] * D * T
    simP = B.Sim.from_workload(w, flags=B.F_PLAIN_KERNEL | B.F_NO_AUTOTUNE_CACHE)
    x = x0.clone()
    pl = _time(lambda: simP.step_k(x, u, T), 3, ev)
    rec["plain_ms"] = pl
    rec["plain_drone_steps_per_s"] = D * T / (pl["mean"] * 1e-3)
    rec["plain_gbs"] = D * T * (2 * W.S_ID * 4 + 16) / (pl["mean"] * 1e-3) / 1e9
    simP.close()
    sim = B.Sim.from_workload(w)
    for k in (1, 10, 100):
        sim.set_launch_config(0, 64, k, 1)
        t = _time(lambda: sim.step_k(x, u, T), 3, ev)
        rec[f"fused_k{k}_ms"] = t
        rec[f"fused_k{k}_drone_steps_per_s"] = D * T / (t["mean"] * 1e-3)
        rec[f"fused_k{k}_frac_alu"] = fl / (t["mean"] * 1e-3) / 1e12 / peak
    sim.autotune(x, u, T, 500)
    t = _time(lambda: sim.step_k(x, u, T), 3, ev)
    rec["autotuned"] = {"launch": sim.launch_config(), "ms": t, "drone_steps_per_s": D * T / (t["mean"] * 1e-3),
                        "frac_alu": fl / (t["mean"] * 1e-3) / 1e12 / peak}
    out["id_swarm_64x4000_T1000"] = rec
    sim.close()

    # 4: differentiable rollout 1024 x 1, 500 steps, identified model, feedback, K = 25, 50, 100,
    # and K = 1: every state kept by the forward (computed for all drones in parallel), so the
    # reverse sweep recomputes nothing
    w = W.id_rollout_grad()
    T, D = w.steps, w.n_drones_total
    x0, cmds, gain = t2d(w.x0), t2d(w.cmds), t2d(w.gain)
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    obj4 = B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u)
    loss = torch.empty(D, device=dev)
    g = (torch.empty_like(cmds), torch.empty_like(x0), torch.empty_like(gain))
    rec = {"drones": D, "steps": T, "waves": D // 64}
    for K in (1, 25, 50, 100):
        ck = sim.ckpt_buffer(T, K, device=dev)
        f = _time(lambda: sim.rollout(x0, cmds, T, obj4, K, ckpt=ck, loss=loss), 10, ev)
        bw = _time(lambda: sim.rollout_backward(x0, cmds, T, obj4, K, ck, g_cmds=g[0], g_x0=g[1], g_gain=g[2]),
                   10, ev)
        ms = f["mean"] + bw["mean"]
        rec[f"k{K}"] = {"forward_ms": f, "backward_ms": bw,
                        "fwd_drone_steps_per_s": D * T / (f["mean"] * 1e-3),
                        "fwdbwd_drone_steps_per_s": D * T / (ms * 1e-3),
                        "roofline": {"bound": "alu", "flops_per_drone_step": FLOPS_PER_DS["id_rollout_fwd_bwd"],
                                     "achieved_tflops": FLOPS_PER_DS["id_rollout_fwd_bwd"] * D * T / (ms * 1e-3) / 1e12,
                                     "frac": FLOPS_PER_DS["id_rollout_fwd_bwd"] * D * T / (ms * 1e-3) / 1e12 / peak}}
        del ck
    rec["note"] = "16 waves on 1024 SIMDs: one chain per drone, latency-bound"
    out["id_adjoint_1024x1_T500"] = rec
    sim.close()
    return out


def measured_peaks(B, dev, ev):
    """Achievable peaks on this device: FP32 FMA rate of the library's probe
    (8 independent chains per lane, 8 waves per SIMD) and device-to-device copy
    bandwidth of a 1 GiB buffer (read + write bytes)."""
    import torch
    n_blocks, iters = 256 * 8, 20000
    out = torch.empty(n_blocks * 256, device=dev)
    rates = []
    for form in (0, 1):
        B.probe_fma(out, n_blocks, 100, form)
        best = 1e30
        for _ in range(5):
            a, b = ev(), ev()
            a.record()
            B.probe_fma(out, n_blocks, iters, form)
            b.record()
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b))
        rates.append(n_blocks * 256 * 16.0 * iters / (best * 1e-3) / 1e12)
    tflops = max(rates)
    src = torch.empty(256 * 1024 * 1024, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    cb = 1e30
    for _ in range(5):
        a, b = ev(), ev()
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        cb = min(cb, a.elapsed_time(b))
    gbs = 2 * src.numel() * 4 / (cb * 1e-3) / 1e9
    del src, dst, out
    return {"fp32_fma_tflops": tflops, "fp32_fma_tflops_three_operand": rates[0],
            "fp32_fma_tflops_accumulate_form": rates[1], "copy_gbs": gbs,
            "fma_probe": f"{n_blocks} x 256 lanes, 8 chains x {iters} FMA, best of 5 per form",
            "copy": "1 GiB device-to-device, read + write bytes, best of 5"}


def gradient_benchmark(B, W, dev, t2d, ev, reps=10):
    """Gradients of a 10-step goal-distance loss w.r.t. the per-step commands and
    the initial state for 2^20 single-drone closed-loop worlds: forward with one
    checkpoint, then the adjoint; gradients/s = worlds / (forward + backward)."""
    import torch
    wg = W.gradient_goal()
    T = wg.steps
    sim = B.Sim.from_workload(wg)
    x0, cmds, goal = t2d(wg.x0), t2d(wg.cmds), t2d(wg.ref_offset)
    obj = B.Sim.objective(ref_amp=wg.ref_amp, ref_period=wg.ref_period, ref_offset=goal, w_u=wg.w_u)
    ckpt = sim.ckpt_buffer(T, T, device=dev)
    loss = torch.empty(sim.D, device=dev)
    g_cmds, g_x0 = torch.empty_like(cmds), torch.empty_like(x0)

    def once():
        sim.rollout(x0, cmds, T, obj, T, ckpt=ckpt, loss=loss)
        sim.rollout_backward(x0, cmds, T, obj, T, ckpt, g_cmds=g_cmds, g_x0=g_x0)

    once()
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record()
    for _ in range(reps):
        once()
    b.record()
    torch.cuda.synchronize()
    if sim.last_error() != 0:
        raise RuntimeError("device error in the gradient benchmark")
    ms = a.elapsed_time(b) / reps
    sim.close()
    return {"workload": "fp_pid_goal_gradient_2^20w_T10", "worlds": wg.n_worlds, "steps": T,
            "ms_fwd_bwd": ms, "gradients_per_s": wg.n_worlds / (ms * 1e-3),
            "drone_steps_per_s": wg.n_worlds * T / (ms * 1e-3), "reps": reps,
            "paper_context": "9e6 gradients/s at 1e6 environments x 10 steps (other hardware)"}


def interface_benchmark(B, W, dev, t2d, ev, n=1 << 20, T=100, reps=5):
    """Held-command RK4 steps of the first-principles model behind each control
    interface, and with the attitude controller at a fifth of the physics rate:
    2^20 single-drone worlds, T steps per call, each handle with the launch shape
    the autotuner picks for it."""
    import dataclasses

    import torch
    pid = W.fp_pid_closed_loop(n_worlds=n, steps=T)
    cases = [("rotor_speeds", W.fp_rotor_open_loop(n_worlds=n, steps=1)),
             ("attitude_pid", pid),
             ("attitude_pid_ctrl_every_5", dataclasses.replace(pid, ctrl_every=5)),
             ("thrust_torques", W.fp_torque(n_worlds=n)),
             ("position", W.fp_position(n_worlds=n))]
    rows = []
    for name, w in cases:
        sim = B.Sim.from_workload(w)
        x0 = t2d(w.x0)
        cmd = t2d(w.cmds[0] if w.cmds.ndim == 3 else w.cmds)
        st = x0.clone()
        sim.autotune(st, cmd, T, 500)
        sim.step_k(st, cmd, T)
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        for _ in range(reps):
            sim.step_k(st, cmd, T)
        b.record()
        torch.cuda.synchronize()
        if sim.last_error() != 0:
            raise RuntimeError(f"device error in the interface benchmark ({name})")
        ms = a.elapsed_time(b) / (reps * T)
        rows.append({"interface": name, "drones": w.n_drones_total, "state_dim": sim.S,
                     "ctrl_every": w.ctrl_every, "ms_per_step": ms,
                     "drone_steps_per_s": w.n_drones_total / (ms * 1e-3), "launch": sim.launch_config()})
        sim.close()
    return rows


def hbm_sweep(B, W, dev, t2d, ev):
    """Plain single-step kernel (one launch per step: state in + out + held command
    per drone-step through HBM) and the fused kernel (K steps per launch) on
    2^20, 2^22 and 2^24 drones of the rotor-interface and identified models."""
    import torch
    rows = []
    for model, name in ((W.MODEL_FP, "fp_rotor_rk4"), (W.MODEL_ID, "id_rk4")):
        for lg in (20, 22, 24):
            w = W.hbm_sweep(model, 1 << lg)
            D = w.n_drones_total
            S = w.x0.shape[0]
            x, u = t2d(w.x0), t2d(w.cmds)
            row = {"model": name, "drones": D, "bytes_per_drone_step_plain": 2 * S * 4 + 16}
            for label, flags, k, reps in (("plain", B.F_PLAIN_KERNEL, 20, 1), ("fused_k10", 0, 10, 3),
                                          ("fused_k100", 0, 100, 1)):
                sim = B.Sim.from_workload(w, flags=flags | B.F_NO_AUTOTUNE_CACHE)
                sim.step_k(x, u, 2)
                torch.cuda.synchronize()
                a, b = ev(), ev()
                a.record()
                for _ in range(reps):
                    sim.step_k(x, u, k)
                b.record()
                torch.cuda.synchronize()
                if sim.last_error() != 0:
                    raise RuntimeError("device error in the bandwidth sweep")
                ms = a.elapsed_time(b) / (reps * k)
                row[f"{label}_ms_per_step"] = ms
                row[f"{label}_drone_steps_per_s"] = D / (ms * 1e-3)
                if label == "plain":
                    row["plain_gbs"] = (2 * S * 4 + 16) * D / (ms * 1e-3) / 1e9
                sim.close()
            rows.append(row)
            del x, u
    return rows


def mppi_benchmark(B, W, dev, t2d, ev, reps=20):
    """Control steps of 5 sampled-rollout controllers x 100 000 samples x 25 steps
    of the closed-loop first-principles model at 50 Hz (dt = 20 ms): sampling,
    rollouts, costs, elite selection, weighted means and the command, with the
    warm start shifted by one step per call."""
    import torch
    w, P, mean0 = W.mppi_task()
    sim = B.Sim.from_workload(w)
    mp = B.Mppi(sim, P)
    x_now, mean = t2d(w.x0[:, 0]), t2d(mean0)
    u = torch.empty(4, device=dev)
    best = torch.empty(1, dtype=torch.int32, device=dev)
    mp.step(x_now, mean, 0, 0, u_apply=u, best=best)
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record()
    for it in range(reps):
        mp.step(x_now, mean, 1, it + 1, u_apply=u, best=best)
    b.record()
    torch.cuda.synchronize()
    if sim.last_error() != 0:
        raise RuntimeError("device error in the sampled-rollout controller")
    ms = a.elapsed_time(b) / reps
    n = P["n_controllers"] * P["n_samples"]
    steps = n * P["horizon"] * P["substeps"]
    mp.close()
    sim.close()
    return {"workload": "mppi_5x100k_H25_fp_pid_50Hz", "controllers": P["n_controllers"],
            "samples": n, "horizon": P["horizon"], "elites_per_controller": P["n_elite"],
            "ms_per_control_step": ms, "sim_steps_per_s": steps / (ms * 1e-3),
            "max_rate_hz": 1e3 / ms, "reps": reps,
            "paper_context": "500k samples x 25 steps at 50 Hz, > 0.5e9 steps/s (other hardware)"}


def bptt_benchmark(B, W, dev, t2d, ev, timesteps=100_000, eval_steps=500):
    """Back-propagation through time at the paper's BPTT scale: 16 environments,
    40-step rollouts at 50 Hz, starts spread along a 10 s figure-eight, the
    paper's reward weights (on normalised actions) and learning rate, Adam until
    100 000 environment steps have been simulated (157 iterations), each iteration
    a forward rollout, the adjoint and the update (identified model). Rollouts
    chain along the trajectory in episodes of 12 rollouts; gradients are clipped
    to norm 10. Two policies: the linear 4x13 feedback and the small-MLP policy
    (width 16), both squashed onto the command ranges. Tracking quality: the RMS
    distance to the reference over `eval_steps` steps (10 s) from the 16 starts,
    before and after training."""
    import torch
    from paper_2606_01478_amd.bptt import tracking_rms, train_policy
    out = {"workload": "id_figure_eight_10s_16env_T40_50Hz_paper_reward", "envs": 16, "steps_per_rollout": 40,
           "eval_steps": eval_steps,
           "paper_context": "100 000 timesteps (16 envs x 40 steps, same reward) trained end to end in 1.56 s "
                            "on a CPU (other hardware); 8.7 mm tracking error on the real drone (not comparable "
                            "with a simulated error)"}
    for name, H in (("linear_policy", 0), ("mlp_policy_w16", 16)):
        w = W.bptt_tracking(hidden=H)
        sim = B.Sim.from_workload(w)
        iters = -(-timesteps // (w.n_worlds * w.steps))
        x0, ubar, theta0 = t2d(w.x0), t2d(w.cmds), t2d(w.gain)
        evk = dict(ref_amp=w.ref_amp, ref_period=w.ref_period, policy_hidden=H,
                   ref_time_shift=t2d(w.ref_time_shift), policy_scale=w.policy_scale)
        hover = ubar[:1].expand(eval_steps, 4, w.n_worlds).contiguous()
        rms0 = tracking_rms(sim, x0, hover, eval_steps, theta0, **evk)
        kw = dict(evk, reward=w.reward, w_u=0.0)
        tkw = dict(lr=4.6e-2, ckpt_every=10, obj_kw=kw, chain=True, reset_every=12, clip_grad_norm=10.0)
        train_policy(sim, x0, ubar, w.steps, theta0, iters=3, **tkw)   # warm-up
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        res = train_policy(sim, x0, ubar, w.steps, theta0, iters=iters, **tkw)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        rms1 = tracking_rms(sim, x0, hover, eval_steps, res["gain"], **evk)
        losses = res["losses"].cpu().numpy()
        out["iterations"] = iters
        out["env_steps"] = iters * w.n_worlds * w.steps
        out[name] = {"ms_total": ms, "ms_per_iteration": ms / iters,
                     "objective_first_last": [float(losses[0]), float(losses[-1])],
                     "tracking_rms_m_before_after": [rms0, rms1]}
        if sim.last_error() != 0:
            raise RuntimeError("device error in the BPTT benchmark")
        sim.close()
    return out


def cpu_baseline(w, seconds, threads=None):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    every 16th world (every 128th with one thread) for as many steps as fit in
    about ``seconds``, on all host threads or on ``threads``."""
    import torch

    import oracle as O
    import workloads as W
    prev = torch.get_num_threads()
    if threads:
        torch.set_num_threads(threads)
    pick = np.arange(0, w.n_worlds, 128 if threads == 1 else 16)
    sub = W.subset(w, pick)
    b = O.Batch.from_workload(sub)
    x = O.t64(sub.x0)
    u = O.t64(sub.cmds)
    threads = torch.get_num_threads()
    n = 0
    t0 = time.perf_counter()
    with torch.no_grad():
        while time.perf_counter() - t0 < seconds and n < w.steps:
            x = b.step(x, u)
            n += 1
    el = time.perf_counter() - t0
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    torch.set_num_threads(prev)
    return {"value": sub.n_drones_total * n / el, "unit": "drone-steps/s", "cores": threads, "kind": "oracle",
            "host": {"cpu_model": cpu_model, "logical_cpus": os.cpu_count()},
            "sample": f"worlds 0,16,32,... ({len(pick)} worlds, {sub.n_drones_total} drones), {n} steps, "
                      f"FP64 PyTorch CPU, {el:.1f} s"}


if __name__ == "__main__":
    main()
