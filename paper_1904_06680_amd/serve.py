"""Served closed-loop runs (Alg. 1 for a fleet of vehicles) with latency and throughput figures.

Workload: n vehicles split between the waypoint mission (after Experiment 4: four static setpoints,
alternating forward and reverse driving at full steering, no obstacles) and reverse parking into a
2.5 x 5.5 m slot between two parked rectangles sampled as 400 points, each vehicle with its own
random rigid placement. Every step plans with n_prop proposal draws plus n_uniform uniform draws
over the horizon T, warm-started with the previous best parameters. The cost carries the terminal
heading and speed terms of the served preset (scenes.C4), and intermediate waypoints are passed
once the last plan reached them over its horizon (NNP_SWITCH_PLAN, the recursive goal-setpoint
logic of Sect. II-D); the mission completes when the vehicle itself reaches the last waypoint. Reported: per-step latency
(host wall time of one fleet step: encoding, proposal network, batched plan, status copy; p50,
p99, mean), rollout throughput (planned samples x T per second of step time), missions completed.

Command line (one GPU): ``python -m paper_1904_06680_amd.serve --vehicles 64 --steps 200``.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import learn, scenes
from .fleet import SWITCH_PLAN, SWITCH_STATE, Fleet
from .nnplan import Planner
from .proposal import Proposal


# The served workload's per-kind goal weights: parking plans with (2, 0.5), a stronger speed term
# than the preset's (2, 0.1) that waypoint missions use (sweeps of the 64-vehicle workload on
# three fleet layouts, one kind's weights at a time).
SERVED_GOAL_WEIGHTS = {"parking": (2.0, 0.5)}


def c4_vehicles(n: int, seed: int = 0, device=None, goal_weights=None):
    """n vehicles, alternating waypoint missions and parking slots. goal_weights maps a mission
    kind ("waypoints", "parking") to that kind's own (heading, speed) goal weights; kinds it does
    not name plan with the planner model's."""
    import torch
    vs, kinds = [], []
    gw = goal_weights or {}
    for i in range(n):
        if i % 2 == 0:
            z0, wps = scenes.mission_waypoints(1000 * seed + i)
            vs.append(dict(z0=z0, waypoints=wps, points=None, goal_weights=gw.get("waypoints")))
            kinds.append("waypoints")
        else:
            z0, wps, pts = scenes.parking_slot(1000 * seed + i)
            vs.append(dict(z0=z0, waypoints=wps, points=torch.from_numpy(pts).to(device),
                           goal_weights=gw.get("parking")))
            kinds.append("parking")
    return vs, kinds


def tuned_planner(preset: dict, vehicles, T: int, n_samples: int, device: int = 0) -> Planner:
    """A planner in the launch shape the autotuner picks for this fleet's batch (every vehicle's
    first plan: start state, first waypoint, obstacles; all shapes give the same results)."""
    from . import autotune
    scs = []
    for v in vehicles:
        pts = v.get("points")
        pts = np.zeros((0, 4), np.float32) if pts is None else pts.cpu().numpy()
        scs.append(scenes.Scene(np.asarray(v["z0"], np.float32),
                                np.asarray(v["waypoints"][0], np.float32), pts, T,
                                goal_weights=v.get("goal_weights")))
    res = autotune.tune_batch(preset, scs, [n_samples] * len(scs), list(range(len(scs))),
                              reps=2, device=device)
    return Planner(preset, device=device, lanes_per_sample=res["lanes_per_sample"],
                   block_threads=res["block_threads"], tile_pairs=res["tile_pairs"])


def run(planner: Planner, vehicles, kinds, steps: int, T: int, n_uniform: int, n_prop: int,
        proposal=None, seed: int = 0, warmup: int = 3, tolerances=None, log=None,
        switch_rule: int = SWITCH_PLAN) -> dict:
    """Serve `steps` sampling times; the first `warmup` steps are excluded from the latency
    statistics (workspace growth, clock ramp)."""
    fl = Fleet(planner, vehicles, T=T, n_uniform=n_uniform, n_prop=n_prop, proposal=proposal,
               seed=seed, tolerances=tolerances, switch_rule=switch_rule)
    lat, work = [], []
    t0 = time.perf_counter()
    for t in range(steps):
        ms, na = fl.step()
        if na == 0:
            break
        if t >= warmup:
            lat.append(ms)
            work.append(na * (n_uniform + n_prop) * T)
        if log and t % 50 == 0:
            log(f"step {t}: {na} active, {ms:.2f} ms")
    wall = time.perf_counter() - t0
    st = fl.state()
    fl.close()
    lat = np.array(lat)
    done = {k: sum(1 for s, kk in zip(st, kinds) if kk == k and s["done"]) for k in set(kinds)}
    total = {k: kinds.count(k) for k in set(kinds)}
    reached = {k: float(np.mean([s["waypoint"] for s, kk in zip(st, kinds) if kk == k]))
               for k in set(kinds)}
    return {
        "vehicles": len(vehicles), "steps": steps, "T": T, "samples_per_plan": n_uniform + n_prop,
        "n_prop": n_prop, "latency_ms": {"p50": float(np.percentile(lat, 50)),
                                         "p99": float(np.percentile(lat, 99)),
                                         "mean": float(lat.mean()), "max": float(lat.max())},
        "rollout_steps_per_s": float(np.sum(work) / (np.sum(lat) / 1e3)),
        "wall_s": wall, "missions_completed": done, "vehicles_per_kind": total,
        "mean_waypoints_reached": reached,
        "infeasible_plans": int(sum(s["infeasible_steps"] for s in st)),
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--vehicles", type=int, default=64)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--T", type=int, default=50)
    ap.add_argument("--uniform", type=int, default=8192)
    ap.add_argument("--prop", type=int, default=8192)
    ap.add_argument("--labels", type=int, default=16384, help="training scenes for the proposal")
    ap.add_argument("--label-samples", type=int, default=16384)
    ap.add_argument("--position-only", action="store_true",
                    help="switch waypoints on position (eps_xi, eps_eta) alone")
    ap.add_argument("--goal-terms", type=float, nargs=2, default=None, metavar=("W_PHI", "W_V"),
                    help="weights of the terminal heading / speed terms of the cost (default: "
                         "the served preset's 2.0 and 0.1; 0 0 gives the plain cost)")
    ap.add_argument("--parking-terms", type=float, nargs=2,
                    default=list(SERVED_GOAL_WEIGHTS["parking"]), metavar=("W_PHI", "W_V"),
                    help="the parking vehicles' own goal weights (default: 2.0 0.5)")
    ap.add_argument("--waypoint-terms", type=float, nargs=2, default=None,
                    metavar=("W_PHI", "W_V"),
                    help="the waypoint vehicles' own goal weights (default: the preset's)")
    ap.add_argument("--switch", choices=("plan", "state"), default="plan",
                    help="pass intermediate waypoints once the last plan reached them over its "
                         "horizon (plan, NNP_SWITCH_PLAN) or once the vehicle is within the "
                         "tolerances (state)")
    ap.add_argument("--fleet-seed", type=int, default=0, help="seed of the vehicles' layouts")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    import torch
    t0 = time.time()

    def log(*a):
        print(f"[{time.time() - t0:7.1f}s]", *a, flush=True)

    preset = dict(scenes.C4)
    if args.goal_terms:
        preset.update(goal_heading_weight=args.goal_terms[0], goal_speed_weight=args.goal_terms[1])
    nt = scenes.n_theta(preset["widths"])
    pl = Planner(preset)
    prop = None
    if args.prop > 0:
        prop = Proposal(preset, nt, max(1024, args.vehicles))
        lab = learn.Labeller(pl, prop)
        enc, th, cost = lab.label(args.labels, args.label_samples, scene_seed=1, log=log)
        ok = torch.isfinite(cost)
        learn.train(prop, enc[ok].contiguous(), th[ok].contiguous(), epochs=20, log=log)
    gw = {}
    if args.parking_terms:
        gw["parking"] = tuple(args.parking_terms)
    if args.waypoint_terms:
        gw["waypoints"] = tuple(args.waypoint_terms)
    vs, kinds = c4_vehicles(args.vehicles, args.fleet_seed, device=pl._dev(), goal_weights=gw)
    tol = dict(eps_phi=4.0, eps_v=1e3) if args.position_only else None
    pl.close()                  # the labelling planner; the fleet gets the tuned launch shape
    pl = tuned_planner(preset, vs, args.T, args.uniform + args.prop)
    log(f"launch shape: {pl.model.lanes_per_sample}/{pl.model.block_threads}/{pl.model.tile_pairs}")
    res = run(pl, vs, kinds, args.steps, args.T, args.uniform, args.prop, proposal=prop,
              tolerances=tol, log=log,
              switch_rule=SWITCH_PLAN if args.switch == "plan" else SWITCH_STATE)
    res["switch_rule"] = args.switch
    res["tolerances"] = "position only" if args.position_only else "Table II"
    res["goal_terms"] = [preset["goal_heading_weight"], preset["goal_speed_weight"]]
    res["goal_terms_per_kind"] = {k: list(v) for k, v in gw.items()}
    print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
