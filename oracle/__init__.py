"""ctypes access to the FP64 CPU oracle (``oracle/nnp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle checks the HIP planner. Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this module. It imports
nothing from the product package; model constants and scenes reach it as plain numbers.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnnp_oracle.so")
SRC_PATH = os.path.join(_HERE, "nnp_oracle.c")

MAX_LAYERS = 3
FEAT_PAPER, FEAT_SIX, FEAT_EIGHT = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, OpenMP, no fused multiply-add contraction)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


SANITIZE_SRC = os.path.join(_HERE, "sanitize_check.c")


def build_sanitized(out_path: str) -> str:
    """Compile the oracle with its host driver (sanitize_check.c) under AddressSanitizer and
    UndefinedBehaviorSanitizer into the executable out_path (no OpenMP: one thread, so the
    sanitizers see every access of the plain code)."""
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wno-unknown-pragmas", "-o", out_path, SANITIZE_SRC,
           SRC_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


class Model(C.Structure):
    _fields_ = [
        ("dt", C.c_double), ("lf", C.c_double), ("lr", C.c_double),
        ("front", C.c_double), ("rear", C.c_double), ("half_width", C.c_double),
        ("delta_max", C.c_double), ("delta_rate_max", C.c_double),
        ("u_min", C.c_double), ("u_max", C.c_double), ("v_min", C.c_double), ("v_max", C.c_double),
        ("n_layers", C.c_int), ("widths", C.c_int * (MAX_LAYERS + 1)), ("feature_set", C.c_int),
        ("norm_xi", C.c_double), ("norm_eta", C.c_double), ("norm_phi", C.c_double),
        ("norm_v", C.c_double), ("d_cap", C.c_double), ("effort_weight", C.c_double),
        ("eps_xi", C.c_double), ("eps_eta", C.c_double), ("eps_phi", C.c_double),
        ("eps_v", C.c_double), ("goal_heading_weight", C.c_double),
        ("goal_speed_weight", C.c_double),
    ]


class Scene(C.Structure):
    _fields_ = [
        ("z0", C.c_double * 4), ("goal", C.c_double * 4), ("a_prev", C.c_double * 2),
        ("points", C.POINTER(C.c_double)), ("P", C.c_int), ("T", C.c_int),
    ]


class Record(C.Structure):
    _fields_ = [
        ("traj", C.POINTER(C.c_double)), ("controls", C.POINTER(C.c_double)),
        ("d_near", C.POINTER(C.c_double)), ("step_flags", C.POINTER(C.c_int)),
        ("cost", C.c_double), ("collided", C.c_int), ("first_collision", C.c_int),
        ("min_margin", C.c_double), ("min_abs_face", C.c_double), ("goal_reached", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        D, I, U32, U64 = C.c_double, C.c_int, C.c_uint32, C.c_uint64
        PD, PI, PU32 = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_uint32)
        PM, PS = C.POINTER(Model), C.POINTER(Scene)
        sig = {
            "orc_n_theta": (I, [PM]),
            "orc_num_threads": (I, []),
            "orc_philox4x32_10": (None, [PU32, PU32, PU32]),
            "orc_theta_value": (D, [U64, U32, U32, U32, U32]),
            "orc_draw_theta": (None, [U64, U32, U32, U32, U32, PD]),
            "orc_wrap_angle": (D, [D]),
            "orc_mlp": (None, [PM, PD, PD, PD]),
            "orc_features": (None, [PM, PD, PD, D, PD, PD]),
            "orc_limit_rate": (None, [PM, PD, PD, PD]),
            "orc_control_map": (None, [PM, PD, PD, PD]),
            "orc_vehicle_step": (None, [PM, PD, D, D, PD]),
            "orc_extrapolate": (None, [PD, D, PD]),
            "orc_point_inside": (I, [PM, PD, PD]),
            "orc_face_distance": (D, [PM, PD, PD]),
            "orc_margin": (D, [PM, PD, PD]),
            "orc_rollout": (None, [PM, PS, PD, I, C.POINTER(Record)]),
            "orc_rollout_samples": (None, [PM, PS, U64, U32, PU32, I, I, PD, PD, PD, PD, PI, PI,
                                           PD, PD]),
            "orc_argmin": (I, [PD, I, PI]),
            "orc_plan": (I, [PM, PS, I, U64, U32, PD, PI, PD, PD, PD, PI]),
            "orc_flags_at_poses": (None, [PM, PD, I, D, PD, PI, I, D, PI]),
            "orc_step_at_states": (None, [PM, PS, PD, PD, PD, PI, I, PD, PD, PD]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _pd(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _pi(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int))


def f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def make_model(p: dict) -> Model:
    """Build the oracle's model from a mapping of constants. Values are widened from float32 so
    the oracle sees exactly the numbers the GPU library receives."""
    m = Model()
    w = lambda k: float(np.float32(p[k]))  # noqa: E731
    for k in ("dt", "lf", "lr", "front", "rear", "half_width", "delta_max", "delta_rate_max",
              "u_min", "u_max", "v_min", "v_max", "norm_xi", "norm_eta", "norm_phi", "norm_v",
              "d_cap", "effort_weight", "eps_xi", "eps_eta", "eps_phi", "eps_v"):
        setattr(m, k, w(k))
    widths = list(p["widths"])
    m.n_layers = len(widths) - 1
    for i in range(MAX_LAYERS + 1):
        m.widths[i] = widths[i] if i < len(widths) else 0
    m.feature_set = int(p["feature_set"])
    m.goal_heading_weight = float(np.float32(p.get("goal_heading_weight", 0.0)))
    m.goal_speed_weight = float(np.float32(p.get("goal_speed_weight", 0.0)))
    return m


class SceneBuf:
    """An oracle scene plus the buffers it points into (kept alive together)."""

    def __init__(self, z0, goal, a_prev, points, T):
        self.points = f64(np.asarray(points, dtype=np.float32).reshape(-1, 4))
        self.s = Scene()
        for i in range(4):
            self.s.z0[i] = float(np.float32(z0[i]))
            self.s.goal[i] = float(np.float32(goal[i]))
        for i in range(2):
            self.s.a_prev[i] = float(np.float32(a_prev[i]))
        self.s.points = _pd(self.points) if len(self.points) else None
        self.s.P = len(self.points)
        self.s.T = int(T)


def n_theta(m: Model) -> int:
    return lib().orc_n_theta(C.byref(m))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def theta(seed: int, inst: int, i0: int, n: int, nt: int) -> np.ndarray:
    out = np.empty((n, nt), np.float64)
    lib().orc_draw_theta(seed, inst, i0, n, nt, _pd(out))
    return out


def mlp(m: Model, th, s) -> np.ndarray:
    a = np.empty(2, np.float64)
    lib().orc_mlp(C.byref(m), _pd(f64(th)), _pd(f64(s)), _pd(a))
    return a


def features(m: Model, z, goal, d_near, a_prev) -> np.ndarray:
    s = np.empty(m.widths[0], np.float64)
    lib().orc_features(C.byref(m), _pd(f64(z)), _pd(f64(goal)), float(d_near), _pd(f64(a_prev)),
                       _pd(s))
    return s


def limit_rate(m: Model, a_raw, a_prev) -> np.ndarray:
    a = np.empty(2, np.float64)
    lib().orc_limit_rate(C.byref(m), _pd(f64(a_raw)), _pd(f64(a_prev)), _pd(a))
    return a


def control_map(m: Model, a):
    d, u = C.c_double(), C.c_double()
    lib().orc_control_map(C.byref(m), _pd(f64(a)), C.byref(d), C.byref(u))
    return d.value, u.value


def vehicle_step(m: Model, z, delta, u) -> np.ndarray:
    zn = np.empty(4, np.float64)
    lib().orc_vehicle_step(C.byref(m), _pd(f64(z)), float(delta), float(u), _pd(zn))
    return zn


def extrapolate(point, t) -> np.ndarray:
    o = np.empty(2, np.float64)
    lib().orc_extrapolate(_pd(f64(point)), float(t), _pd(o))
    return o


def point_inside(m: Model, pose, p) -> int:
    return lib().orc_point_inside(C.byref(m), _pd(f64(pose)), _pd(f64(p)))


def face_distance(m: Model, pose, p) -> float:
    return lib().orc_face_distance(C.byref(m), _pd(f64(pose)), _pd(f64(p)))


def margin(m: Model, pose, p) -> float:
    return lib().orc_margin(C.byref(m), _pd(f64(pose)), _pd(f64(p)))


def wrap_angle(a: float) -> float:
    return lib().orc_wrap_angle(float(a))


def rollout(m: Model, sc: SceneBuf, th, fp32_state: int = 0) -> dict:
    T = sc.s.T
    traj = np.empty((T + 1, 4), np.float64)
    ctrl = np.empty((T, 2), np.float64)
    dn = np.empty(T + 1, np.float64)
    flags = np.empty(T + 1, np.int32)
    r = Record()
    r.traj, r.controls, r.d_near, r.step_flags = _pd(traj), _pd(ctrl), _pd(dn), _pi(flags)
    lib().orc_rollout(C.byref(m), C.byref(sc.s), _pd(f64(th)), int(fp32_state), C.byref(r))
    return dict(traj=traj, controls=ctrl, d_near=dn, step_flags=flags, cost=r.cost,
                collided=r.collided, first_collision=r.first_collision,
                min_margin=r.min_margin, min_abs_face=r.min_abs_face,
                goal_reached=r.goal_reached)


def rollout_samples(m: Model, sc: SceneBuf, seed: int, inst: int, idx, fp32_state=0,
                    want_traj=True, want_controls=True, want_dnear=False) -> dict:
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint32))
    n, T = len(idx), sc.s.T
    traj = np.empty((n, T + 1, 4), np.float64) if want_traj else None
    ctrl = np.empty((n, T, 2), np.float64) if want_controls else None
    dn = np.empty((n, T + 1), np.float64) if want_dnear else None
    cost = np.empty(n, np.float64)
    coll = np.empty(n, np.int32)
    first = np.empty(n, np.int32)
    mm = np.empty(n, np.float64)
    maf = np.empty(n, np.float64)
    lib().orc_rollout_samples(C.byref(m), C.byref(sc.s), seed, inst,
                              idx.ctypes.data_as(C.POINTER(C.c_uint32)), n, int(fp32_state),
                              _pd(traj), _pd(ctrl), _pd(dn), _pd(cost), _pi(coll), _pi(first),
                              _pd(mm), _pd(maf))
    return dict(traj=traj, controls=ctrl, d_near=dn, cost=cost, collided=coll,
                first_collision=first, min_margin=mm, min_abs_face=maf)


def argmin(cost) -> tuple[int, int]:
    c = f64(cost)
    b = C.c_int()
    st = lib().orc_argmin(_pd(c), len(c), C.byref(b))
    return b.value, st


def plan(m: Model, sc: SceneBuf, N: int, seed: int, inst: int = 0) -> dict:
    nt = n_theta(m)
    T = sc.s.T
    cost = np.empty(N, np.float64)
    best = C.c_int()
    th = np.empty(nt, np.float64)
    traj = np.empty((T + 1, 4), np.float64)
    ctrl = np.empty((T, 2), np.float64)
    gr = C.c_int()
    st = lib().orc_plan(C.byref(m), C.byref(sc.s), N, seed, inst, _pd(cost), C.byref(best),
                        _pd(th), _pd(traj), _pd(ctrl), C.byref(gr))
    return dict(cost=cost, best=best.value, status=st, theta=th, traj=traj, controls=ctrl,
                goal_reached=gr.value)


def flags_at_poses(m: Model, sc: SceneBuf, poses, steps, eps: float) -> np.ndarray:
    poses = f64(poses).reshape(-1, 3)
    steps = np.ascontiguousarray(np.asarray(steps, dtype=np.int32))
    out = np.empty(len(poses), np.int32)
    lib().orc_flags_at_poses(C.byref(m), sc.s.points if sc.s.P else None, sc.s.P, m.dt,
                             _pd(poses), _pi(steps), len(poses), float(eps), _pi(out))
    return out


def step_at_states(m: Model, sc: SceneBuf, th, states, a_prev, steps) -> dict:
    states = f64(states).reshape(-1, 4)
    a_prev = f64(a_prev).reshape(-1, 2)
    steps = np.ascontiguousarray(np.asarray(steps, dtype=np.int32))
    M = len(states)
    a = np.empty((M, 2), np.float64)
    zn = np.empty((M, 4), np.float64)
    dn = np.empty(M, np.float64)
    lib().orc_step_at_states(C.byref(m), C.byref(sc.s), _pd(f64(th)), _pd(states), _pd(a_prev),
                             _pi(steps), M, _pd(a), _pd(zn), _pd(dn))
    return dict(a=a, z_next=zn, d_near=dn)


def num_threads() -> int:
    return lib().orc_num_threads()
