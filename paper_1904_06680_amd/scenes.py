"""Model presets and seeded synthetic planning scenes.

This module only produces inputs: vehicle/controller constants and obstacle layouts. It holds
none of the planner's arithmetic, so the GPU library and the CPU oracle can both be fed from it.

Presets
  ``PAPER``  Table I vehicle (l_f = 1.1, l_r = 1.4, chassis (l_f+0.7+l_r+0.6) x 2 m), steering
             limit 40 deg with a 20 deg/s rate limit, asymmetric acceleration bounds, no speed
             clamp, NN-[5,2,2] with the five features of eq. (3), Table II constants.
  ``C0``     single plan at CPU scale: 2.7 m wheelbase with the CoG at mid-wheelbase, centred
             4.5 x 1.8 m rectangle, steering +-0.6 rad, acceleration +-3 m/s^2, speed clamp
             [-3, 15] m/s, MLP 6-16-2 (six features), N = 1024, T = 20, 200 points.
  ``C1``     the same vehicle with MLP 8-32-32-2 (eight features), N = 65536, T = 50,
             2000 static points + 20 moving obstacles x 50 points.

Scenes are drawn with numpy's PCG64 generator from the scene seed; the recipes are below.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32

TABLE_II = dict(norm_xi=30.0, norm_eta=3.5, norm_phi=2.0 * math.pi, norm_v=120.0 / 3.6,
                eps_xi=1.0, eps_eta=0.25, eps_phi=10.0 * math.pi / 180.0, eps_v=5.0 / 3.6)

FEAT_PAPER, FEAT_SIX, FEAT_EIGHT = 0, 1, 2

PAPER = dict(
    dt=0.1, lf=1.1, lr=1.4, front=1.1 + 0.7, rear=1.4 + 0.6, half_width=1.0,
    delta_max=40.0 * math.pi / 180.0, delta_rate_max=20.0 * math.pi / 180.0,
    u_min=-100.0 / (3.8 * 3.6), u_max=100.0 / (7.4 * 3.6),
    v_min=-math.inf, v_max=math.inf,
    widths=(5, 2, 2), feature_set=FEAT_PAPER, d_cap=20.0, effort_weight=0.1, **TABLE_II)

C0 = dict(
    dt=0.1, lf=1.35, lr=1.35, front=2.25, rear=2.25, half_width=0.9,
    delta_max=0.6, delta_rate_max=0.0, u_min=-3.0, u_max=3.0, v_min=-3.0, v_max=15.0,
    widths=(6, 16, 2), feature_set=FEAT_SIX, d_cap=20.0, effort_weight=0.1, **TABLE_II)

C1 = dict(C0, widths=(8, 32, 32, 2), feature_set=FEAT_EIGHT)

# The served closed loop: the C1 vehicle and network with the optional terminal heading and
# speed terms (2 m per rad, 0.1 s per m/s), because its missions prescribe a heading and a stop
# at every waypoint; chosen by sweeps of the 64-vehicle workload (plain sampler, 200 steps,
# three fleet layouts).
C4 = dict(C1, goal_heading_weight=2.0, goal_speed_weight=0.1)

PRESETS = {"paper": PAPER, "c0": C0, "c1": C1, "c4": C4}


def with_net(preset: dict, widths, feature_set=None) -> dict:
    """A copy of ``preset`` with another MLP (e.g. the Table III sizes [5,10,2], [5,10,10,2])."""
    d = dict(preset, widths=tuple(widths))
    if feature_set is not None:
        d["feature_set"] = feature_set
    return d


def n_theta(widths) -> int:
    """Weights plus biases of an MLP, the count Table III reports."""
    return sum(widths[l + 1] * widths[l] + widths[l + 1] for l in range(len(widths) - 1))


def a_idle(preset: dict) -> np.ndarray:
    """Initial controls [0, a_idle[1]] with zero acceleration (Sect. III, first paragraph)."""
    a1 = -1.0 - 2.0 * preset["u_min"] / (preset["u_max"] - preset["u_min"])
    return np.array([0.0, a1], F32)


class Scene:
    """One planning problem: start state, goal setpoint, previous controls, obstacle points
    (float32 rows x, y, vx, vy) and the horizon."""

    def __init__(self, z0, goal, points, T, a_prev=None, name="", goal_weights=None):
        self.z0 = np.asarray(z0, F32).reshape(4)
        self.goal = np.asarray(goal, F32).reshape(4)
        self.points = np.ascontiguousarray(np.asarray(points, F32).reshape(-1, 4))
        self.T = int(T)
        self.a_prev = None if a_prev is None else np.asarray(a_prev, F32).reshape(2)
        self.name = name
        # optional (heading, speed) weights of the goal terms for this problem alone; None: the
        # planner model's
        self.goal_weights = None if goal_weights is None else tuple(float(w) for w in goal_weights)

    @property
    def P(self) -> int:
        return len(self.points)

    def a_prev_or_idle(self, preset: dict) -> np.ndarray:
        return a_idle(preset) if self.a_prev is None else self.a_prev


def _in_start_footprint(px, py, z0, preset, dilate):
    c, s = math.cos(z0[2]), math.sin(z0[2])
    dx, dy = px - z0[0], py - z0[1]
    xi = c * dx + s * dy
    eta = -s * dx + c * dy
    return ((xi < preset["front"] + dilate) & (xi > -preset["rear"] - dilate)
            & (np.abs(eta) < preset["half_width"] + dilate))


def _wrap(a):
    return (a + math.pi) % (2.0 * math.pi) - math.pi


def scene_c0(seed: int, T: int = 20, P: int = 200) -> Scene:
    """Start at rest at the origin heading +x; goal 25 m away on a random bearing psi, goal
    heading psi, speed 0; P static points uniform in a 40 x 40 m box centred on the start-goal
    midpoint, redrawn while inside the start footprint dilated by 0.5 m."""
    rng = np.random.default_rng([int(seed), 0xC0])
    psi = rng.uniform(-math.pi, math.pi)
    z0 = np.array([0.0, 0.0, 0.0, 0.0])
    goal = np.array([25.0 * math.cos(psi), 25.0 * math.sin(psi), _wrap(psi), 0.0])
    cx, cy = 0.5 * goal[0], 0.5 * goal[1]
    pts = np.zeros((P, 4))
    filled = 0
    while filled < P:
        x = rng.uniform(cx - 20.0, cx + 20.0, P - filled)
        y = rng.uniform(cy - 20.0, cy + 20.0, P - filled)
        ok = ~_in_start_footprint(x, y, z0, C0, 0.5)
        k = int(ok.sum())
        pts[filled:filled + k, 0] = x[ok]
        pts[filled:filled + k, 1] = y[ok]
        filled += k
    return Scene(z0, goal, pts, T, name=f"c0-seed{seed}")


def rectangle_outline(cx, cy, yaw, length, width, n):
    """n points evenly spaced along the perimeter of a length x width rectangle."""
    per = 2.0 * (length + width)
    s = (np.arange(n) + 0.5) * per / n
    hl, hw = 0.5 * length, 0.5 * width
    out = np.zeros((n, 2))
    for i, d in enumerate(s):
        if d < length:
            px, py = -hl + d, -hw
        elif d < length + width:
            px, py = hl, -hw + (d - length)
        elif d < 2 * length + width:
            px, py = hl - (d - length - width), hw
        else:
            px, py = -hl, hw - (d - 2 * length - width)
        out[i] = (px, py)
    c, s_ = math.cos(yaw), math.sin(yaw)
    return np.stack([cx + c * out[:, 0] - s_ * out[:, 1], cy + s_ * out[:, 0] + c * out[:, 1]], 1)


def scene_c1(seed: int, T: int = 50, n_static: int = 2000, n_dyn: int = 20,
             pts_per_dyn: int = 50, box: float = 65.0) -> Scene:
    """Start at the origin with random heading in [-pi, pi) and speed in [-3, 15] m/s; goal at a
    distance in [20, 60] m on a random bearing (behind the vehicle means reversing), random goal
    heading, goal speed 0. n_static points uniform in [-box, box]^2; n_dyn moving obstacles, each
    pts_per_dyn points evenly on the perimeter of a 4.5 x 1.8 m rectangle with random centre in
    the box and random yaw, all its points sharing one velocity uniform in [-5, 5]^2 m/s. Points
    (and whole moving obstacles) inside the start footprint dilated by 0.5 m are redrawn."""
    rng = np.random.default_rng([int(seed), 0xC1])
    z0 = np.array([0.0, 0.0, rng.uniform(-math.pi, math.pi), rng.uniform(-3.0, 15.0)])
    dist = rng.uniform(20.0, 60.0)
    bearing = rng.uniform(-math.pi, math.pi)
    goal = np.array([dist * math.cos(bearing), dist * math.sin(bearing),
                     rng.uniform(-math.pi, math.pi), 0.0])
    stat = np.zeros((n_static, 4))
    filled = 0
    while filled < n_static:
        x = rng.uniform(-box, box, n_static - filled)
        y = rng.uniform(-box, box, n_static - filled)
        ok = ~_in_start_footprint(x, y, z0, C1, 0.5)
        k = int(ok.sum())
        stat[filled:filled + k, 0] = x[ok]
        stat[filled:filled + k, 1] = y[ok]
        filled += k
    dyn = []
    while len(dyn) < n_dyn:
        cx, cy = rng.uniform(-box, box, 2)
        yaw = rng.uniform(-math.pi, math.pi)
        v = rng.uniform(-5.0, 5.0, 2)
        xy = rectangle_outline(cx, cy, yaw, 4.5, 1.8, pts_per_dyn)
        if _in_start_footprint(xy[:, 0], xy[:, 1], z0, C1, 0.5).any():
            continue
        blk = np.zeros((pts_per_dyn, 4))
        blk[:, :2] = xy
        blk[:, 2:] = v
        dyn.append(blk)
    pts = np.concatenate([stat] + dyn, 0) if dyn else stat
    return Scene(z0, goal, pts, T, name=f"c1-seed{seed}")


def scene_exp5_parking(T: int = 200) -> Scene:
    """Experiment 5 (Sect. III-E): start [0, 2, 0, 0], the 20 printed static parking-lot points,
    first waypoint "1" at (5, 2) heading 0."""
    pts = np.array([[-6.5, -2], [-5.5, -2], [-4.5, -2], [-3.5, -2], [-2.5, -2], [-2.5, -7],
                    [-1.25, -7], [0, -7], [1.25, -7], [2.5, -7], [2.5, -2], [3.5, -2],
                    [4.5, -2], [5.5, -2], [6.5, -2], [-4, 6], [-2, 6], [0, 6], [2, 6], [4, 6]],
                   float)
    full = np.zeros((len(pts), 4))
    full[:, :2] = pts
    return Scene([0, 2, 0, 0], [5, 2, 0, 0], full, T, name="exp5-parking")


def random_scene(rng: np.random.Generator, P: int, T: int, box: float = 30.0,
                 vmax: float = 3.0) -> Scene:
    """A generic small scene for parity sweeps: random start/goal, P points uniform in
    [-box, box]^2 with velocities uniform in [-vmax, vmax]^2."""
    z0 = np.array([rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(-math.pi, math.pi),
                   rng.uniform(-3, 10)])
    goal = np.array([rng.uniform(-30, 30), rng.uniform(-30, 30), rng.uniform(-math.pi, math.pi),
                     rng.uniform(0, 5)])
    pts = np.zeros((P, 4))
    pts[:, :2] = rng.uniform(-box, box, (P, 2))
    pts[:, 2:] = rng.uniform(-vmax, vmax, (P, 2))
    return Scene(z0, goal, pts, T, name="random")


def scene_mixed(rng: np.random.Generator, P: int, T: int, box: float = 65.0,
                name: str = "mixed") -> Scene:
    """A C1-style scene with P points: a third of them (rounded to whole obstacles) on moving
    4.5 x 1.8 m rectangles of 50 points, the rest static, all in [-box, box]^2."""
    z0 = np.array([0.0, 0.0, rng.uniform(-math.pi, math.pi), rng.uniform(-3.0, 15.0)])
    dist, bearing = rng.uniform(20.0, 60.0), rng.uniform(-math.pi, math.pi)
    goal = np.array([dist * math.cos(bearing), dist * math.sin(bearing),
                     rng.uniform(-math.pi, math.pi), 0.0])
    n_dyn = int(round(P / 3 / 50))
    n_static = P - 50 * n_dyn
    pts = []
    while len(pts) < n_static:
        x, y = rng.uniform(-box, box, 2)
        if not _in_start_footprint(np.array([x]), np.array([y]), z0, C1, 0.5)[0]:
            pts.append([x, y, 0.0, 0.0])
    blocks = [np.array(pts, float).reshape(-1, 4)]
    while len(blocks) < n_dyn + 1:
        cx, cy = rng.uniform(-box, box, 2)
        xy = rectangle_outline(cx, cy, rng.uniform(-math.pi, math.pi), 4.5, 1.8, 50)
        if _in_start_footprint(xy[:, 0], xy[:, 1], z0, C1, 0.5).any():
            continue
        blk = np.zeros((50, 4))
        blk[:, :2] = xy
        blk[:, 2:] = rng.uniform(-5.0, 5.0, 2)
        blocks.append(blk)
    return Scene(z0, goal, np.concatenate(blocks, 0), T, name=name)


def batch_c2(seed: int = 0, count: int = 256, n_range=(4096, 65536), p_range=(100, 5000),
             horizons=(20, 40, 60, 80)):
    """The batched, uneven workload: `count` independent problems with N log-uniform in
    n_range, P log-uniform in p_range and T uniform in `horizons`, each a scene_mixed layout.
    Returns (scenes, Ns, seeds)."""
    rng = np.random.default_rng([int(seed), 0xC2])
    scs, Ns, seeds = [], [], []
    for i in range(count):
        N = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        P = int(round(math.exp(rng.uniform(math.log(p_range[0]), math.log(p_range[1])))))
        T = int(horizons[rng.integers(len(horizons))])
        scs.append(scene_mixed(rng, P, T, name=f"c2-{seed}-{i}"))
        Ns.append(N)
        seeds.append(1000 * seed + i)
    return scs, Ns, seeds


def c1_arrays(seed: int, count: int, n_static: int = 2000, n_dyn: int = 20,
              pts_per_dyn: int = 50, box: float = 65.0):
    """`count` scenes of the scene_c1 recipe, drawn vectorised (another stream than scene_c1, so
    the scenes differ from scene_c1(seed)): returns z0 [count, 4], goal [count, 4] and points
    [count, n_static + n_dyn * pts_per_dyn, 4] as float32 arrays. Used for the proposal's
    training and held-out sets."""
    rng = np.random.default_rng([int(seed), 0xC3])
    z0 = np.zeros((count, 4))
    z0[:, 2] = rng.uniform(-math.pi, math.pi, count)
    z0[:, 3] = rng.uniform(-3.0, 15.0, count)
    dist = rng.uniform(20.0, 60.0, count)
    bearing = rng.uniform(-math.pi, math.pi, count)
    goal = np.stack([dist * np.cos(bearing), dist * np.sin(bearing),
                     rng.uniform(-math.pi, math.pi, count), np.zeros(count)], 1)
    c, s = np.cos(z0[:, 2])[:, None], np.sin(z0[:, 2])[:, None]

    def inside(x, y, dilate=0.5):
        xi = c * x + s * y
        eta = -s * x + c * y
        return ((xi < C1["front"] + dilate) & (xi > -C1["rear"] - dilate)
                & (np.abs(eta) < C1["half_width"] + dilate))

    sx = rng.uniform(-box, box, (count, n_static))
    sy = rng.uniform(-box, box, (count, n_static))
    bad = inside(sx, sy)
    while bad.any():
        k = int(bad.sum())
        sx[bad] = rng.uniform(-box, box, k)
        sy[bad] = rng.uniform(-box, box, k)
        bad = inside(sx, sy)
    # moving rectangles: unit perimeter offsets, then yaw / centre per obstacle
    per = 2.0 * (4.5 + 1.8)
    d = (np.arange(pts_per_dyn) + 0.5) * per / pts_per_dyn
    hl, hw = 2.25, 0.9
    ox = np.where(d < 4.5, -hl + d, np.where(d < 6.3, hl, np.where(d < 10.8, hl - (d - 6.3), -hl)))
    oy = np.where(d < 4.5, -hw, np.where(d < 6.3, -hw + (d - 4.5),
                                         np.where(d < 10.8, hw, hw - (d - 10.8))))
    cx = rng.uniform(-box, box, (count, n_dyn))
    cy = rng.uniform(-box, box, (count, n_dyn))
    yaw = rng.uniform(-math.pi, math.pi, (count, n_dyn))
    vel = rng.uniform(-5.0, 5.0, (count, n_dyn, 2))

    def outline():
        cyw, syw = np.cos(yaw)[..., None], np.sin(yaw)[..., None]
        return cx[..., None] + cyw * ox - syw * oy, cy[..., None] + syw * ox + cyw * oy

    dx, dy = outline()
    bad = inside(dx.reshape(count, -1), dy.reshape(count, -1)).reshape(count, n_dyn, -1).any(2)
    while bad.any():
        k = int(bad.sum())
        cx[bad] = rng.uniform(-box, box, k)
        cy[bad] = rng.uniform(-box, box, k)
        yaw[bad] = rng.uniform(-math.pi, math.pi, k)
        dx, dy = outline()
        bad = inside(dx.reshape(count, -1), dy.reshape(count, -1)).reshape(count, n_dyn, -1).any(2)
    P = n_static + n_dyn * pts_per_dyn
    pts = np.zeros((count, P, 4), np.float32)
    pts[:, :n_static, 0], pts[:, :n_static, 1] = sx, sy
    pts[:, n_static:, 0] = dx.reshape(count, -1)
    pts[:, n_static:, 1] = dy.reshape(count, -1)
    pts[:, n_static:, 2] = np.repeat(vel[..., 0], pts_per_dyn, 1)
    pts[:, n_static:, 3] = np.repeat(vel[..., 1], pts_per_dyn, 1)
    return z0.astype(np.float32), goal.astype(np.float32), pts


def _rigid(rng, xy_box=20.0):
    a = rng.uniform(-math.pi, math.pi)
    return a, rng.uniform(-xy_box, xy_box), rng.uniform(-xy_box, xy_box)


def _apply(a, tx, ty, z):
    """Rigid motion (rotation a, translation tx, ty) of states [n][4] or points [n][4]
    (x, y, heading-or-vx, v-or-vy)."""
    c, s = math.cos(a), math.sin(a)
    z = np.asarray(z, np.float64).reshape(-1, 4).copy()
    x, y = z[:, 0].copy(), z[:, 1].copy()
    z[:, 0] = c * x - s * y + tx
    z[:, 1] = s * x + c * y + ty
    return z


def mission_waypoints(seed: int):
    """Waypoint mission after Experiment 4 (Sect. III): from rest, four static setpoints with
    position and heading that need alternating forward and reverse driving and full steering,
    moved by a random rigid motion. Returns (z0, waypoints [4][4])."""
    rng = np.random.default_rng([int(seed), 0xE4])
    z0 = np.array([[0.0, 0.0, 0.0, 0.0]])
    wps = np.array([[10.0, 5.0, math.pi / 2, 0.0],      # forward, left turn
                    [10.0, -3.0, math.pi / 2, 0.0],     # straight back in reverse
                    [2.0, -8.0, math.pi, 0.0],          # forward, left turn
                    [10.0, -8.0, math.pi, 0.0]])        # straight back in reverse
    a, tx, ty = _rigid(rng)
    z0 = _apply(a, tx, ty, z0)
    wps = _apply(a, tx, ty, wps)
    z0[:, 2] = _wrap(z0[:, 2] + a)
    wps[:, 2] = _wrap(wps[:, 2] + a)
    return z0[0].astype(np.float32), wps.astype(np.float32)


def parking_slot(seed: int, n_points: int = 400):
    """Reverse parking: a 2.5 m wide, 5.5 m deep slot between two parked 1.8 x 4.5 m rectangles
    (n_points/2 points evenly on each perimeter); the vehicle starts at rest in the aisle 6 m in
    front of the slot, heading along the aisle, with an auxiliary waypoint past the slot and the
    final waypoint in the slot facing out. Moved by a random rigid motion. Returns (z0,
    waypoints [2][4], points [n_points][4] with zero velocity)."""
    rng = np.random.default_rng([int(seed), 0x9A4])
    half = n_points // 2
    cars = []
    for cx in (-(1.25 + 0.9), 1.25 + 0.9):
        xy = rectangle_outline(cx, 0.0, math.pi / 2, 4.5, 1.8, half)
        cars.append(np.column_stack([xy, np.zeros((half, 2))]))
    pts = np.concatenate(cars, 0)
    z0 = np.array([[-8.0 + rng.uniform(-1, 1), 6.0 + rng.uniform(-0.3, 0.3), 0.0, 0.0]])
    wps = np.array([[3.5, 6.5, 0.0, 0.0],                 # auxiliary: past the slot
                    [0.0, 0.25, math.pi / 2, 0.0]])       # in the slot, facing out
    a, tx, ty = _rigid(rng)
    z0 = _apply(a, tx, ty, z0)
    wps = _apply(a, tx, ty, wps)
    pts = _apply(a, tx, ty, pts)
    z0[:, 2] = _wrap(z0[:, 2] + a)
    wps[:, 2] = _wrap(wps[:, 2] + a)
    return z0[0].astype(np.float32), wps.astype(np.float32), pts.astype(np.float32)
