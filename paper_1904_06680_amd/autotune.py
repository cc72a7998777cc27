"""Autotuner for the launch shape of batched planning.

The rollout kernel is compiled in several launch shapes for one network: K lanes per sample (4, 8
or 16 for the 8-32-32-2 controller), workgroup size (threads, hence samples per work item and
wavefronts per CU) and LDS tile size (point pairs per buffer, hence barriers per step for large
point sets). All shapes give bit-identical results, so the choice is purely a matter of speed on
the given batch; this module times every compiled candidate on the caller's batch and returns the
fastest, optionally caching the answer per device and batch signature.
"""
from __future__ import annotations

import json
import os
import time

from .nnplan import NnpError, Planner

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "nnplan", "autotune.json")


def signature(preset: dict, scenes_, Ns) -> str:
    """Coarse key of a batch shape: network, count, and size buckets of N, P and T."""
    b = lambda v: int(round(v)).bit_length()  # noqa: E731
    tot = sum(N * (sc.T + 1) * max(sc.P, 1) for sc, N in zip(scenes_, Ns))
    return "w{}-c{}-w{}".format("x".join(map(str, preset["widths"])), len(Ns), b(tot))


# Launch shapes (lanes per sample, workgroup threads, tile pairs; 0 = the layout's default) the
# library compiles for the 8-32-32-2 network; a shape the library does not offer is skipped.
SHAPES = ((8, 0, 0), (4, 0, 0), (16, 0, 0), (8, 512, 4096), (8, 512, 2048))


def _shape(c):
    return tuple(c) + (0,) * (3 - len(c)) if isinstance(c, (tuple, list)) else (int(c), 0, 0)


def _name(c) -> str:
    K, rb, tp = c
    return str(K) if rb == 0 and tp == 0 else f"{K}/{rb}/{tp}"


def tune_batch(preset: dict, scenes_, Ns, seeds, candidates=SHAPES, reps: int = 3,
               device: int = 0, cache: str | None = None) -> dict:
    """Times every candidate shape (an int K or a tuple (K, block_threads, tile_pairs)) on the
    batch; returns the fastest with all timings."""
    import torch
    dev = torch.device("cuda", device)
    key = f"{torch.cuda.get_device_name(dev)}|{signature(preset, scenes_, Ns)}"
    if cache and os.path.exists(cache):
        try:
            with open(cache) as fh:
                known = json.load(fh)
            if key in known:
                return dict(known[key], cached=True)
        except (OSError, ValueError):
            pass
    timings = {}
    for c in map(_shape, candidates):
        try:
            pl = Planner(preset, device=device, lanes_per_sample=c[0], block_threads=c[1],
                         tile_pairs=c[2])
        except NnpError:
            continue
        probs, keep = pl.batch_problems(scenes_, Ns, seeds)
        outs = [pl.alloc_result(sc.T) for sc in scenes_]
        pl.plan_batch_async(probs, outs)          # warm-up (sizes the workspace)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(reps):
            pl.plan_batch_async(probs, outs)
        torch.cuda.synchronize(dev)
        timings[c] = (time.perf_counter() - t0) / reps * 1e3
        del keep
        pl.close()
    best = min(timings, key=timings.get)
    res = {"lanes_per_sample": best[0], "block_threads": best[1], "tile_pairs": best[2],
           "ms": timings[best], "timings_ms": {_name(k): v for k, v in timings.items()},
           "key": key}
    if cache:
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            known = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    known = json.load(fh)
            known[key] = res
            with open(cache, "w") as fh:
                json.dump(known, fh, indent=1)
        except (OSError, ValueError):
            pass
    return dict(res, cached=False)


def main(argv=None) -> int:
    """Tune the launch shape on the seeded 256-problem uneven batch (`scenes.batch_c2`) and print
    the timings; `--plans n` then plans that batch n more times with the chosen shape (the
    command a kernel trace of the batched path runs)."""
    import argparse

    import torch

    from . import scenes
    ap = argparse.ArgumentParser(description="launch-shape autotuner on the uneven C2 batch")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--plans", type=int, default=0)
    ap.add_argument("--cache", default="")
    args = ap.parse_args(argv)
    scs, Ns, seeds = scenes.batch_c2(args.seed)
    res = tune_batch(scenes.C1, scs, Ns, seeds, cache=args.cache or None)
    print(json.dumps(res), flush=True)
    if args.plans > 0:
        pl = Planner(scenes.C1, lanes_per_sample=res["lanes_per_sample"],
                     block_threads=res["block_threads"], tile_pairs=res["tile_pairs"])
        probs, keep = pl.batch_problems(scs, Ns, seeds)
        outs = [pl.alloc_result(sc.T) for sc in scs]
        for i in range(args.plans):
            pl.plan_batch_async(probs, outs)
            torch.cuda.synchronize(pl._dev())
            print(json.dumps({"plan": i}), flush=True)
        del keep
        pl.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
