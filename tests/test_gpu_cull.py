"""GPU tests of the obstacle pass's group skipping (nnp_model.all_points = 0, the default).

A wavefront skips a group of points (16 or 32 consecutive pairs in spatial order, by launch
shape) at a step when the group's bounding box lies farther than
the cull radius (the rectangle's corner distance and, for the distance features, d_cap) from
every one of its samples; such points cannot change a collision flag, a margin below 1 or the
capped nearest distance. The results must therefore be the same bits as with every point tested
(all_points = 1): checked here on the benchmark scenes at full size, for every compiled launch
shape of the 8-32-32-2 network, the small networks (one, two and four lanes per sample), the
paper's parking scene, point counts around the group, tile and spatial-order limits, scenes where
every group or no group is skipped, batches, and per-sample rollouts.
"""
import math

import numpy as np
import pytest

from paper_1904_06680_amd import autotune, scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1904_06680_amd.nnplan import Planner  # noqa: E402

KEYS = ("theta", "controls", "controls_phys", "traj", "cost", "best_index", "status",
        "goal_reached")
ROLL = ("cost", "collided", "first_collision", "traj", "controls")


def say(*a):
    print(*a, flush=True)


def np_out(d, keys=KEYS):
    return {k: d[k].cpu().numpy() for k in keys if k in d}


def bits(x):
    """The array's bit patterns (floats compared bit for bit: the sign of zero and NaN payloads
    included)."""
    return x.view(np.uint32) if x.dtype == np.float32 else x


def assert_same(a, b, where):
    for k in a:
        assert np.array_equal(bits(a[k]), bits(b[k])), (where, k)


def pair(preset, **kw):
    return Planner(preset, **kw), Planner(preset, all_points=True, **kw)


@pytest.mark.parametrize("seed", [4, 1])
def test_c1_full_size_plan_identical(seed):
    """The benchmark workload (N = 65536, T = 50, P = 3000): same winner, parameters, controls,
    states and cost with and without skipping."""
    sc = scenes.scene_c1(seed)
    say(f"cull: C1 scene {seed} N=65536 T={sc.T} P={sc.P}")
    cu, al = pair(scenes.C1)
    assert_same(np_out(cu.plan(sc, 65536, seed=0)), np_out(al.plan(sc, 65536, seed=0)),
                f"c1 scene {seed}")
    cu.close()
    al.close()


@pytest.mark.parametrize("mult", [4, 16])
def test_dense_scenes_identical(mult):
    """The benchmark scene's recipe with 4 and 16 times its points in the same box (12000 and
    48000 points, the densities of the bench's points-scaling leg): skipping equals the
    exhaustive pass."""
    sc = scenes.scene_c1(0, n_static=2000 * mult, n_dyn=20 * mult)
    say(f"cull: C1 scene 0 x{mult} points N=8192 T={sc.T} P={sc.P}")
    cu, al = pair(scenes.C1)
    assert_same(np_out(cu.plan(sc, 8192, seed=2)), np_out(al.plan(sc, 8192, seed=2)), mult)
    cu.close()
    al.close()


@pytest.mark.parametrize("shape", autotune.SHAPES)
def test_c1_launch_shapes_identical(shape):
    """Every compiled launch shape (lanes per sample, workgroup size, tile) with skipping equals
    the default shape with every point tested."""
    K, rb, tp = shape
    sc = scenes.scene_c1(2)
    say(f"cull: C1 scene 2 N=8192 shape K={K} RB={rb} TP={tp}")
    cu = Planner(scenes.C1, lanes_per_sample=K, block_threads=rb, tile_pairs=tp)
    al = Planner(scenes.C1, all_points=True)
    assert_same(np_out(cu.plan(sc, 8192, seed=3)), np_out(al.plan(sc, 8192, seed=3)), shape)
    cu.close()
    al.close()


@pytest.mark.parametrize("K", [1, 2, 4])
def test_small_network_point_counts(K):
    """6-16-2 at one, two and four lanes per sample, on point counts at the edges of a group (64
    points) and of a tile (2048 points at one or two lanes per sample, 4096 at four) (the spatial
    order's limit is covered by test_beyond_the_spatial_order)."""
    rng = np.random.default_rng([K, 0xC011])
    cu, al = pair(scenes.C0, lanes_per_sample=K)
    for P in (1, 63, 64, 65, 200, 2047, 2049, 4095, 4097, 16384, 16385):
        sc = scenes.random_scene(rng, P, 20, box=40.0)
        say(f"cull: C0 K={K} P={P} N=2048")
        assert_same(np_out(cu.plan(sc, 2048, seed=P)), np_out(al.plan(sc, 2048, seed=P)),
                    (K, P))
    cu.close()
    al.close()


def test_beyond_the_spatial_order():
    """Point sets at the spatial order's limit (2^20 points, ordered) and just beyond it (the
    caller's order, no displacement bound: the radius alone), both equal to the exhaustive pass."""
    rng = np.random.default_rng(99)
    cu, al = pair(scenes.C0, lanes_per_sample=4)
    for P in ((1 << 20), (1 << 20) + 1):
        sc = scenes.random_scene(rng, P, 3, box=400.0, vmax=3.0)
        say(f"cull: C0 K=4 P={P} N=256 T=3")
        assert_same(np_out(cu.plan(sc, 256, seed=5)), np_out(al.plan(sc, 256, seed=5)), P)
    cu.close()
    al.close()


def test_paper_network_parking_scene():
    """NN-[5,2,2] (no distance feature: the cull radius is the corner distance alone) on the
    Experiment 5 parking lot, T = 200."""
    preset = scenes.PAPER
    sc = scenes.scene_exp5_parking()
    say(f"cull: paper network, parking scene T={sc.T} P={sc.P}")
    cu, al = pair(preset)
    for seed in range(3):
        assert_same(np_out(cu.plan(sc, 4096, seed=seed)), np_out(al.plan(sc, 4096, seed=seed)),
                    ("parking", seed))
    cu.close()
    al.close()


def test_everything_or_nothing_skipped():
    """Every point far beyond the cull radius (every group skipped at every step: the distance
    feature saturates at d_cap), and every point inside a 3 m disc around the start (no group
    skipped); both equal the exhaustive pass."""
    rng = np.random.default_rng(7)
    far = np.zeros((3000, 4))
    ang = rng.uniform(-math.pi, math.pi, 3000)
    far[:, 0], far[:, 1] = 400 * np.cos(ang), 400 * np.sin(ang)
    near = np.zeros((3000, 4))
    r, ang = 3 * np.sqrt(rng.uniform(0, 1, 3000)), rng.uniform(-math.pi, math.pi, 3000)
    near[:, 0], near[:, 1] = r * np.cos(ang), r * np.sin(ang)
    cu, al = pair(scenes.C1)
    for name, pts in (("far", far), ("near", near)):
        sc = scenes.Scene([0, 0, 0.3, 5], [40, 10, 0, 0], pts, 50, name=name)
        say(f"cull: {name} points, C1 N=16384")
        assert_same(np_out(cu.plan(sc, 16384, seed=1)), np_out(al.plan(sc, 16384, seed=1)), name)
    cu.close()
    al.close()


def test_fast_points_and_fast_vehicle():
    """The bound on a step's nearest distance uses how far the points (up to 42 m/s here) and the
    sample (up to 25 m/s) can move in one step; both at their extremes still give the exhaustive
    result, for the centred (C1) and the offset (paper) rectangle."""
    rng = np.random.default_rng(21)
    for preset in (scenes.C1, dict(scenes.C1, front=2.6, rear=1.9, v_max=25.0)):
        cu, al = pair(preset)
        for k in range(3):
            sc = scenes.random_scene(rng, 3000, 50, box=60.0, vmax=30.0)
            sc.z0[3] = 20.0
            say(f"cull: fast points, scene {k}, N=16384, front={preset['front']}")
            assert_same(np_out(cu.plan(sc, 16384, seed=k)), np_out(al.plan(sc, 16384, seed=k)),
                        ("fast", k))
        cu.close()
        al.close()


def test_rollout_outputs_identical():
    """Per-sample rollout outputs without the margin (skipping on) equal the exhaustive ones; a
    rollout that asks for the margin tests every point and returns the exhaustive margin."""
    sc = scenes.scene_c1(3)
    say("cull: C1 scene 3 rollout N=4096")
    cu, al = pair(scenes.C1)
    a = cu.rollout(sc, 4096, seed=5, want_margin=False)
    b = al.rollout(sc, 4096, seed=5)
    assert_same(np_out(a, ROLL), np_out(b, ROLL), "rollout")
    c = cu.rollout(sc, 4096, seed=5)
    assert np.array_equal(c["min_margin"].cpu().numpy(), b["min_margin"].cpu().numpy())
    cu.close()
    al.close()


def test_batch_identical():
    """A batch of uneven problems (no points, one point, multi-tile sets, a set beyond the spatial
    order's limit: 2^20 + 1 points) equals the exhaustive batch."""
    rng = np.random.default_rng(11)
    shapes = [(0, 64, 20), (1, 100, 5), (3000, 2500, 50), (5000, 700, 13), (20000, 300, 6),
              ((1 << 20) + 1, 64, 2), (120, 4096, 20), (2049, 97, 5)]
    scs = [scenes.scene_mixed(rng, P, T, name=f"b{i}") if P <= 20000 else
           scenes.random_scene(rng, P, T, box=300.0) for i, (P, N, T) in enumerate(shapes)]
    Ns = [N for _, N, _ in shapes]
    seeds = list(range(len(shapes)))
    say(f"cull: batch of {len(shapes)} problems")
    cu, al = pair(scenes.C1)
    got, ref = cu.plan_batch(scs, Ns, seeds), al.plan_batch(scs, Ns, seeds)
    for i in range(len(shapes)):
        assert_same(np_out(got[i]), np_out(ref[i]), ("batch", shapes[i]))
    cu.close()
    al.close()


def test_work_counter():
    """The counter of tested groups: every group counted once per wavefront and step, the tested
    ones no more than all; with every point tested (all_points) they are equal. Counting does not
    change the results."""
    sc = scenes.scene_c1(4)
    N = 8192
    cu, al = pair(scenes.C1)
    ref = np_out(cu.plan(sc, N, seed=1))
    for pl in (cu, al):
        pl.set_cull_stats(True)
        out = np_out(pl.plan(sc, N, seed=1))
        assert_same(out, ref, "counting")
        tested, total = pl.cull_stats(reset=True)
        waves = N * 8 // 64              # eight lanes per sample: 64 wavefronts per 512 samples
        # points padded to a multiple of 64, in groups of 32 or 64 (the launch shape's)
        per_step = total // (waves * (sc.T + 1))
        assert total == waves * (sc.T + 1) * per_step, (total, waves)
        assert per_step in (-(-sc.P // 64), 2 * -(-sc.P // 64)), per_step
        say(f"cull counter: {tested} of {total} groups tested ({tested / total:.3f})",
            "all points" if pl is al else "")
        if pl is al:
            assert tested == total
        else:
            assert 0 < tested < total
        assert pl.cull_stats() == (0, 0)
    cu.close()
    al.close()
