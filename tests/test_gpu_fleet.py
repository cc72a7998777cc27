"""GPU tests of the served closed loop (include/nnfleet.h): every fleet step must equal an
independent nnp_plan call on the same inputs (current state, current waypoint, previous controls,
warm start with the previous best parameters, Philox key = seed + vehicle index and instance =
step index, obstacles moved by their velocities), bit for bit; waypoint switching and mission completion follow the tolerances.
"""
import numpy as np
import pytest

from paper_1904_06680_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1904_06680_amd import learn  # noqa: E402
from paper_1904_06680_amd.fleet import Fleet  # noqa: E402
from paper_1904_06680_amd.nnplan import Planner, nnp_problem  # noqa: E402
from paper_1904_06680_amd.proposal import Proposal  # noqa: E402

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)


def vehicles_for_test():
    z0a, wa = scenes.mission_waypoints(1)
    z0b, wb, pb = scenes.parking_slot(2)
    rng = np.random.default_rng(3)
    pc = np.zeros((300, 4), np.float32)
    pc[:, :2] = rng.uniform(-30, 30, (300, 2))
    pc[:, 2:] = rng.integers(-1, 2, (300, 2))          # velocities in {-1, 0, 1}: exact motion
    z0c = np.array([0.0, 0.0, 0.3, 2.0], np.float32)
    wc = np.array([[25.0, 10.0, 0.0, 0.0]], np.float32)
    return [dict(z0=z0a, waypoints=wa, points=None),
            dict(z0=z0b, waypoints=wb, points=pb),
            dict(z0=z0c, waypoints=wc, points=pc)]


def replicate(pl, vehicles, steps, T, N, seed, proposal=None, n_prop=0):
    """Per-vehicle nnp_plan calls that mirror the fleet (no waypoint is reached in these runs)."""
    dt = np.float32(scenes.C1["dt"])
    out = []
    for iv, v in enumerate(vehicles):
        z = np.asarray(v["z0"], np.float32)
        a_prev = None
        warm = None
        pts = None if v["points"] is None else np.array(v["points"], np.float32)
        traj = []
        for t in range(steps):
            sc = scenes.Scene(z, v["waypoints"][0], np.zeros((0, 4), np.float32) if pts is None
                              else pts, T, a_prev=a_prev)
            prop = None
            if proposal is not None:
                pr, keep = pl.problem(sc, N, seed + iv, inst=t)
                arr = (nnp_problem * 1)(pr)
                enc = proposal.encode_problems(arr)
                mu, ls = proposal.forward(enc)
                prop = (mu[0].contiguous(), ls[0].contiguous(), n_prop)
            res = pl.plan(sc, N, seed=seed + iv, inst=t, warm_theta=warm, proposal=prop)
            z = res["traj"][1].cpu().numpy()
            a_prev = res["controls"][0].cpu().numpy()
            warm = res["theta"].clone()
            traj.append((z.copy(), a_prev.copy(), float(res["cost"].item())))
            if pts is not None:
                pts[:, 0] = pts[:, 0] + dt * pts[:, 2]
                pts[:, 1] = pts[:, 1] + dt * pts[:, 3]
        out.append(traj)
    return out


def dev_points(vs):
    return [dict(v, points=None if v["points"] is None else torch.from_numpy(v["points"]).to(DEV))
            for v in vs]


def test_fleet_steps_equal_independent_plans():
    vs = vehicles_for_test()
    T, N, seed, steps = 20, 700, 5, 3
    pl = Planner(scenes.C1)
    fl = Fleet(pl, dev_points(vs), T=T, n_uniform=N, seed=seed)
    got = []
    for t in range(steps):
        ms, na = fl.step()
        assert na == len(vs)
        got.append(fl.state())
    say(f"fleet: {len(vs)} vehicles, {steps} steps; last latency {ms:.2f} ms")
    ref = replicate(pl, vs, steps, T, N, seed)
    for t in range(steps):
        for i in range(len(vs)):
            z, a, cost = ref[i][t]
            s = got[t][i]
            assert np.array_equal(s["z"], z), (t, i, s["z"], z)
            assert np.array_equal(s["a"], a), (t, i)
            assert s["cost"] == np.float32(cost) or (np.isinf(s["cost"]) and np.isinf(cost))
            assert s["steps"] == t + 1 and s["waypoint"] == 0 and not s["done"]
    fl.close()
    pl.close()


def test_fleet_with_proposal_equals_independent_plans():
    vs = vehicles_for_test()[:2]
    T, N, n_prop, seed, steps = 20, 300, 200, 9, 2
    nt = scenes.n_theta(scenes.C1["widths"])
    pl = Planner(scenes.C1)
    prop = Proposal(scenes.C1, nt, 64)
    prop.set_params(torch.from_numpy(learn.init_params(nt, 3)).to(DEV))
    fl = Fleet(pl, dev_points(vs), T=T, n_uniform=N, n_prop=n_prop, proposal=prop, seed=seed)
    got = []
    for t in range(steps):
        fl.step()
        got.append(fl.state())
    ref = replicate(pl, vs, steps, T, N + n_prop, seed, proposal=prop, n_prop=n_prop)
    for t in range(steps):
        for i in range(len(vs)):
            z, a, _ = ref[i][t]
            assert np.array_equal(got[t][i]["z"], z), (t, i)
            assert np.array_equal(got[t][i]["a"], a), (t, i)
    fl.close()
    prop.close()
    pl.close()


def test_fleet_waypoint_switching_and_completion():
    """A mission whose waypoints are the start state: reached after the first step (the vehicle
    moves a few millimetres), so the mission completes after one step per waypoint and the
    vehicle leaves the active set."""
    z0 = np.array([1.0, 2.0, 0.5, 0.0], np.float32)
    vs = [dict(z0=z0, waypoints=np.stack([z0, z0]), points=None),
          dict(z0=np.zeros(4, np.float32), waypoints=np.array([[30.0, 0, 0, 0]], np.float32),
               points=None)]
    pl = Planner(scenes.C1)
    fl = Fleet(pl, vs, T=20, n_uniform=512, seed=1)
    _, na1 = fl.step()
    s1 = fl.state()
    _, na2 = fl.step()
    s2 = fl.state()
    _, na3 = fl.step()
    s3 = fl.state()
    assert (na1, na2, na3) == (2, 2, 1)
    assert s1[0]["waypoint"] == 1 and not s1[0]["done"]
    assert s2[0]["waypoint"] == 2 and s2[0]["done"]
    assert s3[0]["steps"] == 2 and np.array_equal(s3[0]["z"], s2[0]["z"])
    assert s3[1]["steps"] == 3 and not s3[1]["done"]
    fl.close()
    pl.close()
