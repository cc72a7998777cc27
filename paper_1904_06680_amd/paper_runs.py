"""Paper-preset closed-loop runs: the setups of the paper's experiments with its own vehicle and
controller (Table I vehicle with l_f = 1.1 m, l_r = 1.4 m, steering limit 40 deg and rate limit
20 deg/s, asymmetric acceleration bounds, NN-[5,2,2] with the five features of eq. (3), horizon
H = 200, T_s = 0.1 s), run through the fleet runtime with one vehicle per random seed.

Experiment 5 (Sect. III-E): start [0, 2, 0, 0], the 20 printed parking-lot points, and either the
three waypoints "1", the auxiliary [0, 0, pi/2, 0] and "2", or only the auxiliary one and "2".
The run reports, per the paper's quantities, missions solved, the computation time per sampling
time (here: one batched plan for all seeds, and its share per vehicle), the speed range in km/h
and the driven path length. The paper's numbers come from TSHC on a Titan V and are context, not a
parity target (its seeds and samples are unpublished). ``--goal-terms`` adds the optional
terminal heading and speed terms to the cost (the setpoints prescribe heading and speed).

Command line (one GPU): ``python -m paper_1904_06680_amd.paper_runs``.
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

from . import scenes
from .fleet import SWITCH_PLAN, SWITCH_STATE, Fleet
from .nnplan import Planner

EXP5_POINTS = np.array([[-6.5, -2], [-5.5, -2], [-4.5, -2], [-3.5, -2], [-2.5, -2], [-2.5, -7],
                        [-1.25, -7], [0, -7], [1.25, -7], [2.5, -7], [2.5, -2], [3.5, -2],
                        [4.5, -2], [5.5, -2], [6.5, -2], [-4, 6], [-2, 6], [0, 6], [2, 6], [4, 6]],
                       np.float32)
EXP5_WAYPOINTS = {
    3: np.array([[5.0, 2.0, 0.0, 0.0], [0.0, 0.0, math.pi / 2, 0.0], [0.0, -5.0, math.pi / 2, 0.0]],
                np.float32),
    2: np.array([[0.0, 0.0, math.pi / 2, 0.0], [0.0, -5.0, math.pi / 2, 0.0]], np.float32),
}
PAPER_EXP5 = {3: dict(tau_a_s=0.088, v_kmh=(-17.3, -1.2, 16.2), path_m=(13.8, 14.3, 15.2)),
              2: dict(tau_a_s=0.088, v_kmh=(-16.4, -1.5, 19.1), path_m=(12.5, 15.7, 17.8))}


def exp5(planner: Planner, n_waypoints: int, seeds: int = 10, N: int = 65536, H: int = 200,
         max_steps: int = 600, seed: int = 0, switch_rule: int = SWITCH_PLAN) -> dict:
    """One Experiment 5 mission for `seeds` vehicles (one per seed) until all are done or
    max_steps sampling times have passed. switch_rule: when an intermediate waypoint is passed
    (nnfleet.h; the plan rule by default)."""
    import torch
    pts = np.zeros((len(EXP5_POINTS), 4), np.float32)
    pts[:, :2] = EXP5_POINTS
    dev_pts = torch.from_numpy(pts).to(planner._dev())
    z0 = np.array([0.0, 2.0, 0.0, 0.0], np.float32)
    vs = [dict(z0=z0, waypoints=EXP5_WAYPOINTS[n_waypoints], points=dev_pts)
          for _ in range(seeds)]
    fl = Fleet(planner, vs, T=H, n_uniform=N, seed=seed, switch_rule=switch_rule)
    states = [[z0.copy()] for _ in range(seeds)]
    lat = []
    for t in range(max_steps):
        ms, na = fl.step()
        if na == 0:
            break
        lat.append((ms, na))
        for i, s in enumerate(fl.state()):
            if s["steps"] == len(states[i]):          # stepped this time
                states[i].append(s["z"].copy())
    st = fl.state()
    fl.close()
    v_all = np.concatenate([np.asarray(s)[:, 3] for s in states]) * 3.6
    paths = [float(np.sum(np.hypot(*np.diff(np.asarray(s)[:, :2], axis=0).T))) for s in states]
    lat = np.array(lat)
    return {
        "waypoints": n_waypoints, "seeds": seeds, "samples": N, "H": H,
        "solved": int(sum(s["done"] for s in st)),
        "steps_to_solve": [s["steps"] if s["done"] else None for s in st],
        "step_ms_all_seeds": float(lat[:, 0].mean()),
        "step_ms_per_vehicle": float(np.mean(lat[:, 0] / lat[:, 1])),
        "v_kmh_min_mean_max": [float(v_all.min()), float(v_all.mean()), float(v_all.max())],
        "path_m_min_mean_max": [min(paths), float(np.mean(paths)), max(paths)],
        "infeasible_plans": int(sum(s["infeasible_steps"] for s in st)),
        "goal_heading_weight": float(planner.preset.get("goal_heading_weight", 0.0)),
        "goal_speed_weight": float(planner.preset.get("goal_speed_weight", 0.0)),
        "switch_rule": "plan" if switch_rule == SWITCH_PLAN else "state",
        "paper": PAPER_EXP5[n_waypoints],
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--samples", type=int, default=65536)
    ap.add_argument("--seeds", type=int, default=10)
    ap.add_argument("--max-steps", type=int, default=600)
    ap.add_argument("--goal-terms", type=float, nargs=2, default=None, metavar=("W_PHI", "W_V"),
                    help="add the optional terminal heading / speed terms to the cost")
    ap.add_argument("--switch", choices=("plan", "state"), default="plan",
                    help="intermediate waypoints passed once the last plan reached them (plan) or "
                         "once the vehicle is within the tolerances (state)")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    preset = dict(scenes.PAPER)
    if args.goal_terms:
        preset.update(goal_heading_weight=args.goal_terms[0], goal_speed_weight=args.goal_terms[1])
    pl = Planner(preset)
    rule = SWITCH_PLAN if args.switch == "plan" else SWITCH_STATE
    res = [exp5(pl, w, args.seeds, args.samples, max_steps=args.max_steps, switch_rule=rule)
           for w in (3, 2)]
    for r in res:
        print(json.dumps(r), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh, indent=1)
    pl.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
