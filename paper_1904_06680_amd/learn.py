"""Training and evaluation of the learned proposal (the proposal network of nnproposal.h).

Labels come from the plain planner itself: for every training scene the batched planner (uniform
Philox draws) returns its best parameter vector theta*, and the proposal network learns a Gaussian
over theta given the scene's encoding (Gaussian NLL, Adam). Evaluation compares plans that draw
from the proposal with plans that draw uniformly, on held-out scenes, at matched numbers of
samples. Every computation runs in the library's HIP kernels (encoding, batched planning,
forward/backward/Adam); this module only moves tensors between the calls.

Command line (one GPU): ``python -m paper_1904_06680_amd.learn --labels 100000``.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import scenes
from .nnplan import Planner
from .proposal import Proposal


def init_params(n_theta: int, seed: int, enc: int = 72, hidden: int = 256) -> np.ndarray:
    """Seeded starting parameters in the flat layout of nnproposal.h: uniform weights in
    +-1/sqrt(fan_in) (output layer scaled by 0.1), zero hidden biases, mu biases 0 and log-sigma
    biases log(1/sqrt(3)) (the standard deviation of the uniform draws)."""
    rng = np.random.default_rng([int(seed), 0x9A0])
    u = lambda shape, fan: rng.uniform(-1.0, 1.0, shape) / math.sqrt(fan)  # noqa: E731
    parts = [u((hidden, enc), enc), np.zeros(hidden), u((hidden, hidden), hidden), np.zeros(hidden),
             u((2 * n_theta, hidden), hidden) * 0.1,
             np.concatenate([np.zeros(n_theta), np.full(n_theta, math.log(1.0 / math.sqrt(3.0)))])]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


class Labeller:
    """Plain-planner labels (encoding, theta*, best cost) for C1-style scenes."""

    def __init__(self, planner: Planner, proposal: Proposal, T: int = 50):
        self.pl, self.prop, self.T = planner, proposal, T
        self.torch = planner.torch

    def plan(self, z0, goal, pts_dev, Ns, seeds, proposal=None, a_prev=None, keys=("theta", "cost")):
        probs, keep = self.pl.array_problems(z0, goal, pts_dev, self.T, Ns, seeds, a_prev=a_prev,
                                             proposal=proposal)
        out = self.pl.alloc_batch(len(z0), self.T, keys)
        self.pl.plan_batch_into(probs, out)
        return probs, out, keep

    def encode(self, probs):
        return self.prop.encode_problems(probs)

    def label(self, count: int, N: int, scene_seed: int, chunk: int = 1024, log=None):
        torch = self.torch
        dev = self.pl._dev()
        z0, goal, pts = scenes.c1_arrays(scene_seed, count)
        encs, ths, costs = [], [], []
        for c0 in range(0, count, chunk):
            n = min(chunk, count - c0)
            pd = torch.from_numpy(pts[c0:c0 + n]).to(dev)
            probs, out, keep = self.plan(z0[c0:c0 + n], goal[c0:c0 + n], pd, [N] * n,
                                         np.arange(c0, c0 + n) + 1_000_003 * scene_seed)
            encs.append(self.encode(probs))
            ths.append(out["theta"])
            costs.append(out["cost"])
            torch.cuda.synchronize(dev)
            del keep, pd
            if log and (c0 // chunk) % 8 == 0:
                log(f"labels {c0 + n}/{count}")
        return torch.cat(encs), torch.cat(ths), torch.cat(costs)


def train(prop: Proposal, enc, theta, epochs: int, batch: int = 1024, lr: float = 1e-3,
          seed: int = 0, log=None, checkpoint: str = "", resume: bool = False,
          stop_after: int = 0) -> list:
    """Adam on the Gaussian NLL over (enc, theta) pairs; lr drops to 0.3 lr for the last 30% of
    the epochs. Returns the mean loss per epoch.

    checkpoint: a file written after every epoch with the network's training state (parameters,
    Adam moments and step), the shuffling generator's state, the epoch count and the loss history.
    resume: continue from that file when it exists; the run then ends bit for bit where an
    uninterrupted run would have (same data, batch, lr, seed and epochs, which are checked).
    stop_after: end this call after that many epochs (0: none), e.g. to split a run into
    time-boxed sessions that resume from the checkpoint."""
    torch = prop.torch
    dev = prop._dev()
    n = enc.shape[0]
    batch = min(batch, n, prop.max_batch)
    loss = torch.empty(1, device=dev)
    acc = torch.zeros(1, device=dev)
    gen = torch.Generator(device="cpu").manual_seed(int(seed))
    hist = []
    start = 0
    run = dict(n=int(n), batch=int(batch), lr=float(lr), seed=int(seed), epochs=int(epochs))
    if resume and checkpoint and os.path.exists(checkpoint):
        ck = torch.load(checkpoint, map_location="cpu", weights_only=True)
        if ck["run"] != run:
            raise ValueError(f"checkpoint {checkpoint} is of another run: {ck['run']} vs {run}")
        prop.set_state(ck["state"])
        gen.set_state(ck["generator"])
        start, hist = int(ck["epoch"]), [float(x) for x in ck["hist"]]
        if log:
            log(f"resumed from {checkpoint} at epoch {start}")
    else:
        prop.set_params(torch.from_numpy(init_params(prop.n_theta, seed)).to(dev))
    end = epochs if stop_after <= 0 else min(epochs, start + stop_after)
    for ep in range(start, end):
        perm = torch.randperm(n, generator=gen).to(dev)
        acc.zero_()
        steps = 0
        rate = lr if ep < 0.7 * epochs else 0.3 * lr
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            prop.train_step(enc[idx].contiguous(), theta[idx].contiguous(), rate, loss)
            acc += loss
            steps += 1
        hist.append(float(acc.item()) / max(steps, 1))
        if log and (ep % 5 == 0 or ep == epochs - 1):
            log(f"epoch {ep}: loss {hist[-1]:.2f}")
        if checkpoint:
            st = {k: (v.cpu() if hasattr(v, "cpu") else v) for k, v in prop.get_state().items()}
            tmp = checkpoint + ".tmp"
            torch.save(dict(run=run, state=st, generator=gen.get_state(), epoch=ep + 1,
                            hist=hist), tmp)
            os.replace(tmp, checkpoint)
    return hist


def _diff(a, b):
    with np.errstate(invalid="ignore"):      # inf - inf: both infeasible, counted as equal
        d = a - b
    d[np.isinf(a) & np.isinf(b)] = 0.0
    return d


def evaluate(lab: Labeller, count: int, scene_seed: int, n_ref: int = 65536,
             budgets=(1024, 2048, 4096, 8192, 16384, 32768, 65536), tau: float = 1.0,
             fixed=(8192, 65536), log=None) -> dict:
    """Held-out comparison on `count` scenes. b_U = best cost of n_ref uniform draws; for every
    budget n, b_P(n) = best cost of n proposal draws (sampling width scaled by tau) and, for
    reference, the best of n uniform draws; both as the median and the win rate of b(n) - b_U over
    the scenes where b_U is finite. samples_to_matched_cost is the smallest budget whose median
    difference is <= 0 (ratio = n_ref / that budget). The fixed comparison pits fixed[0] proposal
    draws against fixed[1] uniform draws, with the uniform plan as the fallback when the
    proposal's best is worse."""
    torch = lab.torch
    dev = lab.pl._dev()
    z0, goal, pts = scenes.c1_arrays(scene_seed, count)
    pd = torch.from_numpy(pts).to(dev)
    seeds = np.arange(count) + 7_777_777
    probs, out, keep = lab.plan(z0, goal, pd, [n_ref] * count, seeds)
    enc = lab.encode(probs)
    mu, ls = lab.prop.forward(enc)
    ls = (ls + math.log(tau)).contiguous()
    bU = out["cost"].cpu().numpy()
    feas = np.isfinite(bU)
    res = {"scenes": count, "feasible": int(feas.sum()), "n_ref": n_ref, "tau": tau,
           "uniform": {}, "proposal": {}}

    def stats(b):
        d = _diff(b, bU)[feas]
        return {"median_diff": float(np.median(d)), "win_rate": float(np.mean(d <= 0)),
                "infeasible": float(np.mean(np.isinf(b[feas])))}

    for n in budgets:
        _, o, k = lab.plan(z0, goal, pd, [n] * count, seeds)
        res["uniform"][n] = stats(o["cost"].cpu().numpy())
        _, o, k = lab.plan(z0, goal, pd, [n] * count, seeds, proposal=(mu, ls, n))
        res["proposal"][n] = stats(o["cost"].cpu().numpy())
        if log:
            log(f"N={n}: uniform {res['uniform'][n]}  proposal {res['proposal'][n]}")
    matched = [n for n in budgets if res["proposal"][n]["median_diff"] <= 0.0]
    res["samples_to_matched_cost"] = matched[0] if matched else None
    res["ratio"] = n_ref / matched[0] if matched else None
    # fixed comparison: fixed[0] proposal draws against fixed[1] uniform draws, with the uniform
    # plan as fallback whenever the proposal's best is worse
    n_p, n_u = fixed
    _, o, k = lab.plan(z0, goal, pd, [n_p] * count, seeds, proposal=(mu, ls, n_p))
    bP = o["cost"].cpu().numpy()
    d = _diff(bP, bU)[feas]
    res["fixed"] = {"proposal_samples": n_p, "uniform_samples": n_u,
                    "proposal_not_worse": float(np.mean(d <= 0)),
                    "median_diff": float(np.median(d)),
                    "with_fallback_median_diff": float(np.median(np.minimum(d, 0.0)))}
    del keep, k, pd
    return res


def canonical(theta: np.ndarray, widths=(8, 32, 32, 2)) -> np.ndarray:
    """The same networks in a canonical form (rows [n][n_theta], float64): tanh is odd, so the
    sign of a hidden unit's incoming weights and bias can be flipped together with its outgoing
    weights, and hidden units can be permuted with their outgoing weights, without changing the
    function. Every hidden unit is made to have a non-negative bias, then the units of a layer are
    sorted by bias. Two hidden layers (the 8-32-32-2 layout of nnplan.h) only."""
    n0, n1, n2, n3 = widths
    th = np.array(theta, np.float64)
    n = th.shape[0]
    o = 0
    w1 = th[:, o:o + n1 * n0].reshape(n, n1, n0); o += n1 * n0
    b1 = th[:, o:o + n1]; o += n1
    w2 = th[:, o:o + n2 * n1].reshape(n, n2, n1); o += n2 * n1
    b2 = th[:, o:o + n2]; o += n2
    wo = th[:, o:o + n3 * n2].reshape(n, n3, n2); o += n3 * n2
    bo = th[:, o:o + n3]
    s = np.where(b1 < 0, -1.0, 1.0)
    w1, b1, w2 = w1 * s[:, :, None], b1 * s, w2 * s[:, None, :]
    k = np.argsort(b1, 1)
    w1 = np.take_along_axis(w1, k[:, :, None], 1)
    b1 = np.take_along_axis(b1, k, 1)
    w2 = np.take_along_axis(w2, k[:, None, :], 2)
    s = np.where(b2 < 0, -1.0, 1.0)
    w2, b2, wo = w2 * s[:, :, None], b2 * s, wo * s[:, None, :]
    k = np.argsort(b2, 1)
    w2 = np.take_along_axis(w2, k[:, :, None], 1)
    b2 = np.take_along_axis(b2, k, 1)
    wo = np.take_along_axis(wo, k[:, None, :], 2)
    return np.concatenate([w1.reshape(n, -1), b1, w2.reshape(n, -1), b2, wo.reshape(n, -1), bo], 1)


def elite_gaussian_bound(pl: Planner, count: int, scene_seed: int = 7, n_ref: int = 65536,
                         n_prop: int = 16384, elites: int = 64, seed: int = 0, log=None) -> dict:
    """What a Gaussian proposal could reach at best: per held-out C1-style scene, the `elites`
    best of `n_ref` uniform draws (the plain planner's own samples) are put in canonical form and
    three Gaussians are fitted to them: diagonal, and the elites' own covariance (rank elites - 1)
    plus a small diagonal, at temperature 1 and 0.5. `n_prop` draws from each (numpy, on the
    host) are rolled out by the planner (explicit parameters) and their best cost is compared with
    the best of the `n_ref` uniform draws, next to uniform draws of n_prop and 2 n_prop. These
    are the Gaussians a proposal trained on the planner's good samples can at best learn to
    predict from the scene, which sees neither the n_ref draws nor the scene's one best sample.
    Returns, per variant, the median excess over the reference and the share of scenes that
    match it."""
    torch = pl.torch
    dev = pl._dev()
    rng = np.random.default_rng([seed, 0xE7])
    z0, goal, pts = scenes.c1_arrays(scene_seed, count)
    names = ("uniform_n", "uniform_2n", "diagonal", "elite_covariance", "elite_covariance_t0.5")
    diff = {k: [] for k in names}
    for i in range(count):
        sc = scenes.Scene(z0[i], goal[i], pts[i], 50)
        cu = pl.rollout(sc, n_ref, seed=100 + i, want_traj=False,
                        want_controls=False)["cost"].cpu().numpy()
        bU = float(cu.min())
        if not np.isfinite(bU):
            continue
        diff["uniform_n"].append(float(cu[:n_prop].min()) - bU)
        diff["uniform_2n"].append(float(cu[:2 * n_prop].min()) - bU)
        top = np.argsort(cu, kind="stable")[:min(elites, int(np.isfinite(cu).sum()))]
        th = pl.sample_theta(n_ref, seed=100 + i)[torch.from_numpy(top).to(dev)].cpu().numpy()
        E = canonical(th)
        mu, sd = E.mean(0), E.std(0)
        L = (E - mu).T / math.sqrt(max(len(E) - 1, 1))
        for name in names[2:]:
            if name == "diagonal":
                draw = mu + sd * rng.standard_normal((n_prop, E.shape[1]))
            else:
                tau = 0.5 if name.endswith("t0.5") else 1.0
                draw = (mu + tau * rng.standard_normal((n_prop, len(E))) @ L.T +
                        0.05 * sd * rng.standard_normal((n_prop, E.shape[1])))
            c = pl.rollout(sc, n_prop, theta=torch.from_numpy(draw.astype(np.float32)),
                           want_traj=False, want_controls=False)["cost"].cpu().numpy()
            diff[name].append(float(c.min()) - bU)
        if log and i % 16 == 0:
            log(f"scene {i}: " + ", ".join(f"{k} {np.median(v):.3f}" for k, v in diff.items()
                                           if v))
    return {"scenes": count, "feasible": len(diff["uniform_n"]), "n_ref": n_ref,
            "n_prop": n_prop, "elites": elites,
            "variants": {k: {"median_excess": float(np.median(v)),
                             "matched_share": float(np.mean(np.asarray(v) <= 0))}
                         for k, v in diff.items()}}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--labels", type=int, default=100000)
    ap.add_argument("--label-samples", type=int, default=65536)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-scenes", type=int, default=256)
    ap.add_argument("--tau", type=float, default=1.0)
    ap.add_argument("--out", default="")
    ap.add_argument("--checkpoint", default="", help="training state file, written every epoch")
    ap.add_argument("--resume", action="store_true", help="continue from --checkpoint")
    ap.add_argument("--elite-bound", type=int, default=0, metavar="SCENES",
                    help="instead of training: the best a Gaussian fitted to each scene's elite "
                         "uniform draws reaches (elite_gaussian_bound) on this many scenes")
    args = ap.parse_args(argv)
    import torch
    t0 = time.time()

    def log(*a):
        print(f"[{time.time() - t0:7.1f}s]", *a, flush=True)

    if args.elite_bound:
        res = elite_gaussian_bound(Planner(scenes.C1), args.elite_bound, log=log)
        print(json.dumps(res), flush=True)
        if args.out:
            with open(args.out, "w") as fh:
                json.dump(res, fh, indent=1)
        return 0

    preset = scenes.C1
    nt = scenes.n_theta(preset["widths"])
    pl = Planner(preset)
    prop = Proposal(preset, nt, max(args.batch, args.eval_scenes))
    lab = Labeller(pl, prop)
    enc, th, cost = lab.label(args.labels, args.label_samples, scene_seed=1, log=log)
    keep = torch.isfinite(cost)
    enc, th = enc[keep].contiguous(), th[keep].contiguous()
    log(f"labels: {int(keep.sum())} feasible of {args.labels}")
    hist = train(prop, enc, th, args.epochs, args.batch, args.lr, log=log,
                 checkpoint=args.checkpoint, resume=args.resume)
    res = evaluate(lab, args.eval_scenes, scene_seed=2, tau=args.tau, log=log)
    res.update(labels=args.labels, label_samples=args.label_samples, feasible_labels=int(keep.sum()),
               epochs=args.epochs, final_loss=hist[-1])
    print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
