"""nnp_plan_noalloc, the variant of nnp_plan for callers that cannot allocate device memory,
against nnp_plan through the C-ABI: every output bit for bit, on two calls in a row (the second
smaller), a third call on another handle of the same GPU, and a problem too large for its fixed
scratch array rejected with NNP_EINVAL and the sizes in the message."""
import numpy as np
import pytest

from paper_1904_06680_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1904_06680_amd.nnplan import NNP_EINVAL, NnpError, Planner  # noqa: E402


def say(*a):
    print(*a, flush=True)


def np_out(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), (what, k)


def test_noalloc_equals_plan():
    sc_big = scenes.scene_c1(4)                       # 3000 points, T = 50
    sc0 = scenes.scene_c1(6)
    sc_small = scenes.Scene(sc0.z0, sc0.goal, sc0.points[:500], 20)
    pl = Planner(scenes.C1)                           # fresh handle: no workspace grown yet
    got = []
    for sc, N, seed in ((sc_big, 65536, 3), (sc_small, 1000, 5)):
        say(f"noalloc: C1 N={N} T={sc.T} P={sc.P} seed={seed}")
        got.append(np_out(pl.plan(sc, N, seed=seed, noalloc=True)))
    for (sc, N, seed), g in zip(((sc_big, 65536, 3), (sc_small, 1000, 5)), got):
        ref = np_out(pl.plan(sc, N, seed=seed))
        same(ref, g, f"N={N}")
        say("   best", int(g["best_index"][0]), "cost", float(g["cost"][0]), "status",
            int(g["status"][0]))
    # another handle (another network) on the same GPU shares the array; calls are sequential
    pc = Planner(scenes.C0)
    sc = scenes.scene_c0(2)
    say("noalloc: C0 N=1024 on a second handle")
    g = np_out(pc.plan(sc, 1024, seed=2, noalloc=True))
    same(np_out(pc.plan(sc, 1024, seed=2)), g, "C0")
    # an infeasible start: status and outputs of sample 0, as nnp_plan
    pts = np.concatenate([sc_big.points, [[0.5, 0.2, 0.0, 0.0]]]).astype(np.float32)
    sc_inf = scenes.Scene(sc_big.z0, sc_big.goal, pts, sc_big.T)
    say("noalloc: infeasible start")
    same(np_out(pl.plan(sc_inf, 2000, seed=1)), np_out(pl.plan(sc_inf, 2000, seed=1, noalloc=True)),
         "infeasible")
    pc.close()
    pl.close()


def test_noalloc_rejects_problems_beyond_its_scratch():
    pl = Planner(scenes.C1)
    rng = np.random.default_rng(0)
    pts = np.zeros((20000, 4), np.float32)
    pts[:, :2] = rng.uniform(-300, 300, (20000, 2))
    sc = scenes.Scene(np.zeros(4, np.float32), np.array([30, 0, 0, 0], np.float32), pts, 50)
    with pytest.raises(NnpError) as e:
        pl.plan(sc, 256, seed=0, noalloc=True)
    say("rejected:", str(e.value))
    assert e.value.rc == NNP_EINVAL and "NNP_NOALLOC_SCRATCH_BYTES" in str(e.value)
    # the same problem still plans through nnp_plan, and a fitting one through the variant
    pl.plan(sc, 256, seed=0)
    small = scenes.Scene(sc.z0, sc.goal, pts[:1000], 50)
    same(np_out(pl.plan(small, 256, seed=0)), np_out(pl.plan(small, 256, seed=0, noalloc=True)),
         "after rejection")
    pl.close()
