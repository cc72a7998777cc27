"""Throughput of the rollout planner on one MI355X.

One step = one full planning call (Step 5 of Alg. 1, Sect. II-E) at the full-scale workload:
N = 65536 parameter samples of an 8-32-32-2 tanh controller (1410 parameters), horizon T = 50,
3000 obstacle points (2000 static + 20 moving obstacles x 50 points), every sample rolled over
the whole horizon with the rectangle test (eq. (2)) and the nearest distance at every step,
then the argmin and the winner's outputs. Ten synthetic scenes (seeds 0..9) stay resident in
device memory and the steps cycle through them.

The obstacle pass skips groups of points that cannot change a sample's minima (same results bit
for bit as testing every point). The roofline's `achieved` counts the method's whole work (every
point tested, the fixed per-rollout-step figure); `point_groups_tested` is the measured share of
the point tests the kernel executed and `frac_executed` the FP32 rate of the work it did.

Prints one JSON line: rollout-steps/s = N * T * steps / wall time of the timed steps, the
rollout kernel's roofline figures (device time from HIP events recorded around that kernel on
its stream), and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_SAMPLES, HORIZON, N_SCENES = 65536, 50, 10
PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector peak (vendor figure, packed FP32)
FLOPS_PER_POINT_TEST = 11         # translate 2, rotate 6, squared distance 3
FLOPS_STEP_OVERHEAD = 75          # features, control map, model, effort (transcendentals = 0)
MINMAX_PER_POINT_TEST = 3         # max(|xi'|, |eta'|) and the two running minima


def mlp_flops(widths) -> int:
    macs = sum(widths[l] * widths[l + 1] for l in range(len(widths) - 1))
    biases = sum(widths[1:])
    return 2 * macs + biases


def algorithmic_flops(N: int, T: int, P: int, widths) -> float:
    """FP32 flops of one rollout launch: N * [(T+1) * P * 11 + T * (MLP + overhead)]."""
    return float(N) * ((T + 1) * P * FLOPS_PER_POINT_TEST + T * (mlp_flops(widths)
                                                                + FLOPS_STEP_OVERHEAD))


def executed_flops(N: int, T: int, P: int, widths, tested: float) -> float:
    """The flops of one rollout launch that the kernel executes when a share `tested` of the
    point tests is carried out (the rest skipped as unable to change any minimum)."""
    return float(N) * ((T + 1) * P * FLOPS_PER_POINT_TEST * tested
                       + T * (mlp_flops(widths) + FLOPS_STEP_OVERHEAD))


def point_groups_tested(pl, probs) -> float:
    """Share of the point groups the obstacle pass tested, over one plan of every scene (after
    the timed region; the counter is off while timing)."""
    import torch
    pl.set_cull_stats(True)
    pl.cull_stats(reset=True)
    for pr, _, res in probs:
        pl.plan_async(pr, res)
    torch.cuda.synchronize()
    tested, total = pl.cull_stats(reset=True)
    pl.set_cull_stats(False)
    return tested / max(total, 1)


def algorithmic_ops_with_minmax(N: int, T: int, P: int, widths) -> float:
    """The same work with the point test's min/max operations counted as well (14 per test)."""
    return algorithmic_flops(N, T, P, widths) + float(N) * (T + 1) * P * MINMAX_PER_POINT_TEST


def source_hash() -> str:
    """Hash of the rollout kernels' code (csrc/nnplan.hip, rollout.hpp, philox.hpp) with comments
    and blank lines removed, so that edits to comments leave it unchanged."""
    h = hashlib.sha256()
    for f in ("nnplan.hip", "rollout.hpp", "philox.hpp"):
        with open(os.path.join(ROOT, "paper_1904_06680_amd", "csrc", f), encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", " ", fh.read(), flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def traffic_record(kernel_hash: str):
    """HBM bytes per rollout launch from the committed rocprofv3 counter summary, or None when
    the summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "rollout_c1_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_hash:
        return None
    return rec.get("bytes_per_launch")


def oracle_c0_plan() -> dict:
    """The FP64 oracle's whole plan on the small configuration (N = 1024, T = 20, 200 points,
    6-16-2 controller, scene 0), timed on the host cores."""
    import oracle
    from paper_1904_06680_amd import scenes
    sc = scenes.scene_c0(0)
    m = oracle.make_model(scenes.C0)
    ob = oracle.SceneBuf(sc.z0, sc.goal, sc.a_prev_or_idle(scenes.C0), sc.points, sc.T)
    oracle.plan(m, ob, 1024, seed=0)
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        oracle.plan(m, ob, 1024, seed=0)
    el = (time.perf_counter() - t0) / reps
    return {"workload": "C0 plan: N=1024, T=20, P=200, MLP 6-16-2, scene 0", "ms": round(el * 1e3, 3),
            "value": 1024 * sc.T / el, "unit": "rollout-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle"}


def per_scene_kernel_ms(pl, probs, reps: int = 5) -> list:
    """Rollout-kernel device time of every scene (mean of `reps` plans each, after the timed
    region), for the median and the worst scene."""
    import torch
    out = []
    for pr, _, res in probs:
        pl.kernel_time(reset=True)
        for _ in range(reps):
            pl.plan_async(pr, res)
        torch.cuda.synchronize()
        ms, n = pl.kernel_time(reset=True)
        out.append(ms / max(n, 1))
    return out


def cpu_baseline(scene, preset, target_s: float) -> dict:
    import numpy as np

    import oracle
    m = oracle.make_model(preset)
    ob = oracle.SceneBuf(scene.z0, scene.goal, scene.a_prev_or_idle(preset), scene.points,
                         scene.T)
    cal = 64
    t0 = time.perf_counter()
    oracle.rollout_samples(m, ob, 0, 0, np.arange(cal), want_traj=False, want_controls=False)
    dt = time.perf_counter() - t0
    n = int(min(N_SAMPLES, max(cal, cal * target_s / max(dt, 1e-6))))
    t0 = time.perf_counter()
    oracle.rollout_samples(m, ob, 0, 0, np.arange(n), want_traj=False, want_controls=False)
    el = time.perf_counter() - t0
    return {"value": n * scene.T / el, "unit": "rollout-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"samples 0..{n - 1} of scene 0 (full T={scene.T}, P={scene.P}), FP64, "
                      f"{el:.1f} s"}


_T_START = time.perf_counter()


def progress(msg: str) -> None:
    """One progress line on stderr (stdout carries only the result line)."""
    print(f"[bench {time.perf_counter() - _T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched, learned-proposal and served legs")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="instead of planning, run a plain device copy of this many MiB "
                         "(reference kernel for scaling HBM counter readings)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the planner's "
              "multi-GPU sharding is a design note, not a measured path.", file=sys.stderr)
        return 2

    import torch

    from paper_1904_06680_amd import scenes
    from paper_1904_06680_amd.nnplan import Planner

    dev = torch.device("cuda", 0)
    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize(dev)
        print(json.dumps({"copy_mib": args.copy_mib, "launches": args.steps}), flush=True)
        return 0
    preset = scenes.C1
    pl = Planner(preset, device=0)
    scs = [scenes.scene_c1(s) for s in range(N_SCENES)]
    probs = []
    for sc in scs:
        pr, keep = pl.problem(sc, N_SAMPLES, seed=0)
        probs.append((pr, keep, pl.alloc_result(sc.T)))
    P = scs[0].P
    assert all(sc.P == P and sc.T == HORIZON for sc in scs)
    stream = torch.cuda.current_stream(dev)

    for k in range(args.warmup):
        pr, _, out = probs[k % N_SCENES]
        pl.plan_async(pr, out)
    torch.cuda.synchronize(dev)

    pl.set_timing(True)
    pl.kernel_time(reset=True)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for k in range(args.steps):
        pr, _, out = probs[k % N_SCENES]
        pl.plan_async(pr, out)
    torch.cuda.synchronize(dev)
    elapsed = time.perf_counter() - t0
    progress(f"timed region: {args.steps} plans, {elapsed / args.steps * 1e3:.3f} ms each")
    kern_ms, launches = pl.kernel_time(reset=True)
    scene_ms = per_scene_kernel_ms(pl, probs)
    pl.set_timing(False)
    tested = point_groups_tested(pl, probs)
    costs = [float(probs[k][2]["cost"].item()) for k in range(min(N_SCENES, args.steps))]

    value = N_SAMPLES * HORIZON * args.steps / elapsed
    flops = algorithmic_flops(N_SAMPLES, HORIZON, P, preset["widths"])
    avg_s = kern_ms / max(launches, 1) / 1e3
    achieved = flops / avg_s / 1e12
    khash = source_hash()
    ops_mm = algorithmic_ops_with_minmax(N_SAMPLES, HORIZON, P, preset["widths"])
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": traffic_record(khash), "kernel": "rollout_kernel<8-32-32-2, K=8>",
            "kernel_ms": round(avg_s * 1e3, 4), "flops_per_launch": flops,
            "frac_with_minmax": round(ops_mm / avg_s / 1e12 / PEAK_FP32_TFLOPS, 4),
            "ops_with_minmax_per_launch": ops_mm, "source_hash": khash,
            "point_groups_tested": round(tested, 4),
            "executed_flops_per_launch": executed_flops(N_SAMPLES, HORIZON, P, preset["widths"],
                                                        tested)}
    roof["frac_executed"] = round(roof["executed_flops_per_launch"] / avg_s / 1e12
                                  / PEAK_FP32_TFLOPS, 4)
    order = sorted(range(len(scene_ms)), key=lambda i: scene_ms[i])
    med, worst = order[len(order) // 2], order[-1]
    per_scene = {"kernel_ms": [round(v, 4) for v in scene_ms],
                 "median": {"scene": med, "kernel_ms": round(scene_ms[med], 4),
                            "rollout_steps_per_s": N_SAMPLES * HORIZON / (scene_ms[med] / 1e3)},
                 "worst": {"scene": worst, "kernel_ms": round(scene_ms[worst], 4),
                           "rollout_steps_per_s": N_SAMPLES * HORIZON / (scene_ms[worst] / 1e3)}}
    line = {
        "metric": "rollout-steps/s (N=65536,T=50)",
        "value": value, "unit": "rollout-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain planner, full scale: N=65536 samples, T=50, MLP 8-32-32-2 "
                               "(1410 params), 2000 static + 20x50 moving obstacle points, "
                               "10 seeded scenes",
                   "N": N_SAMPLES, "T": HORIZON, "P": P, "mlp": "8-32-32-2",
                   "scenes": N_SCENES, "parallelism": "single GPU"},
        "roofline": roof,
        "per_scene": per_scene,
        "best_costs_first_scenes": [round(c, 4) for c in costs[:3]],
    }
    if not args.no_extra:
        progress("points-scaling leg")
        line["points_scaling"] = bench_points_scaling(pl)
        progress("batched leg")
        line["batched_uneven"] = bench_batch(pl)
        progress("learned-proposal leg")
        prop_res, prop = bench_proposal(pl)
        line["proposal"] = prop_res
        progress("served leg")
        line["served"] = bench_served(pl, prop)
        prop.close()
        progress("paper-context leg")
        line["paper_context"] = bench_paper_context()
    if not args.no_cpu:
        progress("CPU baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(scs[0], preset, args.cpu_seconds)
        line["cpu_baseline_c0"] = oracle_c0_plan()
    progress("done")
    pl.close()
    print(json.dumps(line), flush=True)
    return 0


def bench_points_scaling(pl, reps: int = 5) -> dict:
    """The C1 plan (scene 0's recipe, N = 65536, T = 50) with 1x, 4x and 16x its obstacle points
    in the same box: rollout kernel time with the group skipping and with every point tested
    (all_points), and the share of groups tested."""
    import torch

    from paper_1904_06680_amd import scenes
    from paper_1904_06680_amd.nnplan import Planner
    full = Planner(scenes.C1, device=pl.device, all_points=True)
    rows = []
    for mult in (1, 4, 16):
        sc = scenes.scene_c1(0, n_static=2000 * mult, n_dyn=20 * mult)
        row = {"P": sc.P}
        for name, p in (("culled", pl), ("all_points", full)):
            pr, keep = p.problem(sc, N_SAMPLES, seed=0)
            res = p.alloc_result(sc.T)
            p.plan_async(pr, res)
            torch.cuda.synchronize()
            p.set_timing(True)
            p.kernel_time(reset=True)
            for _ in range(reps):
                p.plan_async(pr, res)
            torch.cuda.synchronize()
            ms, n = p.kernel_time(reset=True)
            p.set_timing(False)
            row[f"{name}_kernel_ms"] = round(ms / max(n, 1), 4)
            if name == "culled":
                row["point_groups_tested"] = round(point_groups_tested(p, [(pr, keep, res)]), 4)
            del keep
        row["speedup"] = round(row["all_points_kernel_ms"] / row["culled_kernel_ms"], 2)
        rows.append(row)
    full.close()
    return {"workload": "C1 scene 0 recipe with 1x, 4x, 16x the points (same 130 m box), "
                        "N=65536, T=50", "rows": rows}


def bench_batch(pl) -> dict:
    """256 uneven problems (N, P, T spread) in one nnp_plan_batch call; launch shape from the
    autotuner. Rollout-steps/s over the wall time of the call (mean of 3 after the tuning runs)."""
    from paper_1904_06680_amd import autotune, scenes
    scs, Ns, seeds = scenes.batch_c2(0)
    tune = autotune.tune_batch(scenes.C1, scs, Ns, seeds, reps=3)
    steps = sum(N * sc.T for sc, N in zip(scs, Ns))
    flops = sum(algorithmic_flops(N, sc.T, sc.P, scenes.C1["widths"]) for sc, N in zip(scs, Ns))
    achieved = flops / (tune["ms"] / 1e3) / 1e12
    return {"workload": "256 problems, N log-uniform 4096-65536, P log-uniform 100-5000, "
                        "T in {20,40,60,80}, MLP 8-32-32-2",
            "rollout_steps": steps, "ms": round(tune["ms"], 3),
            "value": steps / (tune["ms"] / 1e3), "unit": "rollout-steps/s",
            "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                         "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                         "flops_per_call": flops,
                         "note": "the method's flops (every point tested) over the whole call's "
                                 "wall time"},
            "lanes_per_sample": tune["lanes_per_sample"],
            "block_threads": tune["block_threads"], "tile_pairs": tune["tile_pairs"],
            "timings_ms": {k: round(v, 3) for k, v in tune["timings_ms"].items()}}


def bench_proposal(pl):
    """Reduced learned-proposal run (4096 training scenes labelled at 16384 uniform samples, 64
    held-out scenes), plus the training step's MFMA throughput at a batch of 4096."""
    import torch

    from paper_1904_06680_amd import learn, scenes
    from paper_1904_06680_amd.proposal import Proposal
    nt = pl.n_theta
    dev = pl._dev()
    prop = Proposal(scenes.C1, nt, 4096)
    lab = learn.Labeller(pl, prop)
    enc, th, cost = lab.label(4096, 16384, scene_seed=1)
    ok = torch.isfinite(cost)
    learn.train(prop, enc[ok].contiguous(), th[ok].contiguous(), epochs=30, batch=512)
    ev = learn.evaluate(lab, 64, scene_seed=2, budgets=(1024, 4096, 16384, 65536))
    # training-step throughput (forward + NLL + backward + Adam) at B = 4096
    B = 4096
    X = torch.randn(B, 72, device=dev)
    T = torch.rand(B, nt, device=dev) * 2 - 1
    loss = torch.empty(1, device=dev)
    snap = prop.get_params()
    for _ in range(3):
        prop.train_step(X, T, 1e-6, loss)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        prop.train_step(X, T, 1e-6, loss)
    e1.record()
    torch.cuda.synchronize(dev)
    ms = e0.elapsed_time(e1) / 20
    prop.set_params(snap)
    lin = 72 * 256 + 256 * 256 + 256 * 2 * nt
    flops = 2.0 * B * (2 * lin + (256 * 256 + 256 * 2 * nt))
    res = {"workload": "reduced: 4096 labelled C1-style scenes (16384 uniform samples each), "
                       "64 held-out scenes; uniform reference 65536 samples",
           "feasible_labels": int(ok.sum()), "samples_to_matched_cost": ev["samples_to_matched_cost"],
           "ratio": ev["ratio"], "fixed_8192_vs_65536": ev["fixed"],
           "median_diff_by_budget": {n: round(ev["proposal"][n]["median_diff"], 4)
                                     for n in ev["proposal"]},
           "uniform_median_diff_by_budget": {n: round(ev["uniform"][n]["median_diff"], 4)
                                             for n in ev["uniform"]},
           "train_roofline": {"bound": "mfma", "batch": B, "ms": round(ms, 4),
                              "achieved": round(flops / ms / 1e9, 3), "peak": 2500.0,
                              "unit": "TFLOP/s", "frac": round(flops / ms / 1e9 / 2500.0, 5),
                              "dtype": "bf16 products, f32 accumulate"}}
    return res, prop


def bench_served(pl, prop) -> dict:
    """Closed loop served: 64 vehicles (waypoint missions and reverse parking) x 200 steps, each
    plan 8192 proposal + 8192 uniform samples over T = 50, with the served preset's cost (terminal
    heading and speed terms; the parking vehicles with their own weights) and plan-based waypoint
    switching."""
    from paper_1904_06680_amd import serve
    from paper_1904_06680_amd.scenes import C4
    vs, kinds = serve.c4_vehicles(64, device=pl._dev(), goal_weights=serve.SERVED_GOAL_WEIGHTS)
    p4 = serve.tuned_planner(C4, vs, 50, 16384, device=pl.device)
    shape = [p4.model.lanes_per_sample, p4.model.block_threads, p4.model.tile_pairs]
    r = serve.run(p4, vs, kinds, 200, 50, 8192, 8192, proposal=prop)
    p4.close()
    return {"workload": "64 vehicles x 200 replans, 8192 proposal + 8192 uniform samples, T=50, "
                        "cost with terminal heading/speed terms (2, 0.1; parking 2, 0.5), "
                        "plan-based waypoint switching",
            "latency_ms_p50": round(r["latency_ms"]["p50"], 3),
            "latency_ms_p99": round(r["latency_ms"]["p99"], 3),
            "rollout_steps_per_s": r["rollout_steps_per_s"],
            "missions_completed": r["missions_completed"],
            "vehicles_per_kind": r["vehicles_per_kind"],
            "mean_waypoints_reached": r["mean_waypoints_reached"],
            "launch_shape": shape}


# The paper's own figures (Table III and Sect. III): average computation time of one planning
# step on an Intel i7-7700K with one NVIDIA Titan V, TSHC with 15 restarts of n = 20480 samples
# over H = 200, host-GPU transfers included. Context, not a target: the sampler, the sample count
# (taken here as 15 x 20480) and the hardware differ.
PAPER_SAMPLES = 15 * 20480
PAPER_FIGURES = [
    ("Experiment 5 (parking): NN-[5,2,2], the 20 printed points", (5, 2, 2), "exp5", 0.088),
    ("Experiment 2: NN-[5,2,2], no points, goal 50 m", (5, 2, 2), "exp2", 0.036),
    ("Experiment 2: NN-[5,10,2], no points, goal 50 m", (5, 10, 2), "exp2", 0.047),
    ("Experiment 2: NN-[5,10,10,2], no points, goal 50 m", (5, 10, 10, 2), "exp2", 0.130),
]


def bench_paper_context(reps: int = 5) -> dict:
    """The paper preset (its vehicle, rate limit, features and networks) on the paper's workloads
    at 15 x 20480 samples and H = 200: wall time of one plan (inputs resident on the device) and
    rollout-steps/s, beside the paper's figure for the same experiment and network."""
    import numpy as np
    import torch

    from paper_1904_06680_amd import scenes
    from paper_1904_06680_amd.nnplan import Planner
    rows = []
    for name, widths, kind, paper_s in PAPER_FIGURES:
        preset = dict(scenes.PAPER, widths=widths)
        if kind == "exp5":
            sc = scenes.scene_exp5_parking(T=200)
        else:
            sc = scenes.Scene([0, 0, 0, 0], [50, 0, 0, 0], np.zeros((0, 4)), 200, name="exp2")
        pl = Planner(preset, device=0)
        pr, keep = pl.problem(sc, PAPER_SAMPLES, seed=0)
        res = pl.alloc_result(sc.T)
        pl.plan_async(pr, res)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pl.plan_async(pr, res)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        del keep
        pl.close()
        rows.append({"workload": name, "ms_per_plan": round(ms, 3),
                     "rollout_steps_per_s": PAPER_SAMPLES * sc.T / (ms / 1e3),
                     "paper_ms": paper_s * 1e3})
    return {"samples": PAPER_SAMPLES, "H": 200,
            "paper_hardware": "Intel i7-7700K + NVIDIA Titan V, TSHC, host-GPU transfers "
                              "included (Table III, Sect. III)",
            "rows": rows}


if __name__ == "__main__":
    sys.exit(main())
