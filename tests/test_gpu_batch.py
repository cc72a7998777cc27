"""GPU tests of batched planning (many independent problems in one persistent launch).

Every problem of a batch must come out bit-identical to a single nnp_plan call on it (which the
parity tests pin to the oracle), for every lane layout, with the winners gathered from records
or re-simulated, and when the batch is captured into a HIP graph and replayed. A few small C0 problems of a batch are also checked against the oracle's
plan directly.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1904_06680_amd import scenes
from parity import check_argmin, oracle_scene

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1904_06680_amd.nnplan import NNP_EINVAL, NnpError, Planner  # noqa: E402

KEYS = ("theta", "controls", "controls_phys", "traj", "cost", "best_index", "status",
        "goal_reached")


def say(*a):
    print(*a, flush=True)


def np_out(d):
    return {k: d[k].cpu().numpy() for k in KEYS}


def mixed_batch(seed=0):
    """Uneven problems: empty and multi-tile point sets, N below and above one tile, T = 1..60,
    explicit and idle previous controls."""
    rng = np.random.default_rng([seed, 0xBA7C])
    shapes = [(0, 64, 20), (1, 1, 1), (17, 333, 7), (3000, 2500, 50), (5000, 700, 13),
              (1537, 1200, 40), (2048, 256, 60), (120, 4096, 20), (2049, 97, 5),
              (400, 5000, 33), (3000, 65, 50), (999, 1023, 2), (9000, 300, 6)]
    scs, Ns, seeds = [], [], []
    for i, (P, N, T) in enumerate(shapes):
        sc = scenes.scene_mixed(rng, P, T, name=f"mixed-{i}")
        if i % 3 == 1:
            sc.a_prev = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1)], np.float32)
        scs.append(sc)
        Ns.append(N)
        seeds.append(1000 + 17 * i)
    return scs, Ns, seeds


def singles(pl, scs, Ns, seeds):
    return [np_out(pl.plan(sc, N, seed=s)) for sc, N, s in zip(scs, Ns, seeds)]


def bits(x):
    """The array's bit patterns (floats compared bit for bit: the sign of zero included)."""
    return x.view(np.uint32) if x.dtype == np.float32 else x


def assert_same(a, b, where):
    for k in KEYS:
        assert np.array_equal(bits(a[k]), bits(b[k])), (where, k)


@pytest.fixture(scope="module")
def c1_planner():
    pl = Planner(scenes.C1)
    yield pl
    pl.close()


def test_batch_equals_single_plans(c1_planner):
    scs, Ns, seeds = mixed_batch(0)
    say(f"batch vs single plans: C1, {len(scs)} problems, "
        f"P={[s.P for s in scs]}, N={Ns}, T={[s.T for s in scs]}")
    ref = singles(c1_planner, scs, Ns, seeds)
    for rep in range(2):
        got = [np_out(o) for o in c1_planner.plan_batch(scs, Ns, seeds)]
        for i in range(len(scs)):
            assert_same(ref[i], got[i], (rep, i))


def test_batch_records_equal_winner_replay(c1_planner):
    """The batch's winners gathered from the per-sample records (when every problem's records
    fit the handle's limit) and re-simulated (record limit 0) give the same outputs, bit for
    bit."""
    scs, Ns, seeds = mixed_batch(2)
    say(f"batch records vs replay: C1, {len(scs)} problems")
    c1_planner.set_record_limit(1 << 32)
    rec = [np_out(o) for o in c1_planner.plan_batch(scs, Ns, seeds)]
    c1_planner.set_record_limit(0)
    rep = [np_out(o) for o in c1_planner.plan_batch(scs, Ns, seeds)]
    c1_planner.set_record_limit(1 << 32)
    for i in range(len(scs)):
        assert_same(rec[i], rep[i], i)


def test_batch_launch_shapes_bit_identical(c1_planner):
    """Every compiled launch shape of the 8-32-32-2 network (lanes per sample, workgroup
    threads, LDS tile pairs) gives the same batch results, bit for bit; the mixed batch has
    point sets of one, two and more tiles for every tile size."""
    from paper_1904_06680_amd.autotune import SHAPES
    scs, Ns, seeds = mixed_batch(1)
    say(f"batch launch shapes {SHAPES}: C1, {len(scs)} problems")
    ref = [np_out(o) for o in c1_planner.plan_batch(scs, Ns, seeds)]
    for K, rb, tp in SHAPES[1:]:
        pl = Planner(scenes.C1, lanes_per_sample=K, block_threads=rb, tile_pairs=tp)
        got = [np_out(o) for o in pl.plan_batch(scs, Ns, seeds)]
        pl.close()
        for i in range(len(scs)):
            assert_same(ref[i], got[i], (K, rb, tp, i))


def test_batch_c0_against_oracle():
    """Small C0 problems of one batch against the oracle's plan (argmin rule and cost)."""
    rng = np.random.default_rng(11)
    scs = [scenes.scene_c0(s, T=T, P=P) for s, (T, P) in
           enumerate([(20, 200), (7, 50), (20, 0), (13, 333), (1, 10)])]
    Ns = [1024, 300, 64, 700, 5]
    seeds = [int(x) for x in rng.integers(0, 2**40, len(scs))]
    say(f"C0 batch vs oracle: {len(scs)} problems, N={Ns}")
    pl = Planner(scenes.C0)
    got = [np_out(o) for o in pl.plan_batch(scs, Ns, seeds)]
    pl.close()
    for sc, N, seed, g in zip(scs, Ns, seeds, got):
        m, ob = oracle_scene(scenes.C0, sc)
        ref = oracle.plan(m, ob, N, seed=seed)
        best = int(g["best_index"][0])
        say("  ", sc.name, "best", best, "oracle", ref["best"], check_argmin(ref["cost"], best))
        assert np.array_equal(g["theta"].astype(np.float64),
                              oracle.theta(seed, 0, best, 1, scenes.n_theta(scenes.C0["widths"]))[0])


def test_batch_graph_capture_replay():
    """Capture one batch into a HIP graph; replay it several times with eager GPU work and
    synchronisations in between, zeroing the outputs before each replay; every replay must
    equal the eager batch."""
    scs, Ns, seeds = mixed_batch(2)
    say(f"batch graph capture: C1, {len(scs)} problems, 4 replays")
    pl = Planner(scenes.C1)
    other = Planner(scenes.C1)
    dev = torch.device("cuda", 0)
    probs, keep = pl.batch_problems(scs, Ns, seeds)
    outs = [pl.alloc_result(sc.T) for sc in scs]
    s = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s):
        pl.plan_batch_async(probs, outs)          # sizes the workspace
    torch.cuda.synchronize(dev)
    eager = [np_out(o) for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pl.plan_batch_async(probs, outs)
    for rep in range(4):
        for o in outs:
            for t in o.values():
                t.zero_()
        # unrelated eager work on the device between replays, including another planner
        other.plan(scs[rep], Ns[rep], seed=seeds[rep] + 1)
        x = torch.randn(1 << 20, device=dev)
        (x * 2).sum().item()
        torch.cuda.synchronize(dev)
        g.replay()
        torch.cuda.synchronize(dev)
        got = [np_out(o) for o in outs]
        for i in range(len(scs)):
            assert_same(eager[i], got[i], (rep, i))
    del g, keep
    pl.close()
    other.close()


def test_batch_capture_requires_sized_workspace():
    scs, Ns, seeds = mixed_batch(3)
    pl = Planner(scenes.C1)
    probs, keep = pl.batch_problems(scs[:3], Ns[:3], seeds[:3])
    outs = [pl.alloc_result(sc.T) for sc in scs[:3]]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(NnpError) as ei:
        with torch.cuda.graph(g, stream=s):
            pl.plan_batch_async(probs, outs)
    assert ei.value.rc == NNP_EINVAL
    del keep
    pl.close()


def test_batch_rejects_invalid_problem(c1_planner):
    scs, Ns, seeds = mixed_batch(4)
    Ns = list(Ns)
    Ns[5] = 0
    with pytest.raises(NnpError) as ei:
        c1_planner.plan_batch(scs, Ns, seeds)
    assert ei.value.rc == NNP_EINVAL
    assert "problem 5" in str(ei.value)


def test_c2_workload_sampled(c1_planner):
    """The 256-problem uneven batch: 24 sampled problems equal single plans bit for bit; every
    problem has a finite cost or the infeasible status."""
    scs, Ns, seeds = scenes.batch_c2(0)
    say(f"C2 batch: {len(scs)} problems, sum N = {sum(Ns)}")
    got = c1_planner.plan_batch(scs, Ns, seeds)
    rng = np.random.default_rng(5)
    for i in sorted(rng.choice(len(scs), 24, replace=False)):
        ref = np_out(c1_planner.plan(scs[i], Ns[i], seed=seeds[i]))
        assert_same(ref, np_out(got[i]), i)
    for o in got:
        st = int(o["status"].item())
        assert st in (0, 1)
        assert (st == 0) == math.isfinite(o["cost"].item())


def test_problem_goal_weights():
    """A problem's own goal heading / speed weights plan exactly as a model that carries them
    (the served preset is C1 with its goal weights); in a batch, problems with their own weights
    and with the model's equal their single plans; invalid weights are rejected."""
    rng = np.random.default_rng([3, 0x60A1])
    sc = scenes.scene_mixed(rng, 800, 30, name="weights")
    model_w = Planner(scenes.C4)
    own_w = Planner(scenes.C1)
    sw = scenes.Scene(sc.z0, sc.goal, sc.points, sc.T, goal_weights=(
        scenes.C4["goal_heading_weight"], scenes.C4["goal_speed_weight"]))
    a = np_out(model_w.plan(sc, 4096, seed=2))
    b = np_out(own_w.plan(sw, 4096, seed=2))
    assert_same(a, b, "own weights = model weights")
    plain = np_out(own_w.plan(sc, 4096, seed=2))
    assert plain["cost"][0] != b["cost"][0]
    scs = [scenes.scene_mixed(rng, P, T, name=f"w{i}") for i, (P, T) in
           enumerate([(300, 20), (0, 15), (1200, 40), (64, 8)])]
    for i, w in enumerate([(2.0, 0.5), None, (0.0, 3.0), (5.0, 0.0)]):
        scs[i].goal_weights = w
    Ns, seeds = [2000, 777, 3000, 64], [11, 12, 13, 14]
    got = own_w.plan_batch(scs, Ns, seeds)
    for i in range(len(scs)):
        assert_same(np_out(got[i]), np_out(own_w.plan(scs[i], Ns[i], seed=seeds[i])), ("batch", i))
    for bad in ((-1.0, 0.5), (float("nan"), 0.0), (1.0, float("inf"))):
        with pytest.raises(NnpError) as e:
            own_w.plan(scenes.Scene(sc.z0, sc.goal, sc.points, sc.T, goal_weights=bad), 64)
        assert e.value.rc == NNP_EINVAL
    model_w.close()
    own_w.close()
