"""Python binding of the C-ABI in ``include/nnfleet.h`` (ctypes; argument marshalling only).

``Fleet`` serves Alg. 1 for many vehicles: every ``step()`` is one sampling time for every vehicle
whose mission is not complete, computed by the library (proposal network, batched plan, status
kernel, obstacle motion) and synchronised before it returns.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .nnplan import NNP_OK, NnpError, load_library

EXPORTED = ("nnp_fleet_create", "nnp_fleet_step", "nnp_fleet_state", "nnp_fleet_destroy",
            "nnp_fleet_last_error")


class nnp_fleet_config(C.Structure):
    _fields_ = [("n_vehicles", C.c_int32), ("T", C.c_int32), ("n_uniform", C.c_int32),
                ("n_prop", C.c_int32), ("seed", C.c_uint64), ("warm_start", C.c_int32),
                ("dt", C.c_float), ("eps_xi", C.c_float), ("eps_eta", C.c_float),
                ("eps_phi", C.c_float), ("eps_v", C.c_float), ("switch_rule", C.c_int32)]


SWITCH_STATE, SWITCH_PLAN = 0, 1


class nnp_vehicle_spec(C.Structure):
    _fields_ = [("z0", C.c_float * 4), ("waypoints", C.POINTER(C.c_float)),
                ("n_waypoints", C.c_int32), ("obst", C.c_void_p), ("P", C.c_int32),
                ("own_goal_weights", C.c_int32), ("goal_heading_weight", C.c_float),
                ("goal_speed_weight", C.c_float)]


class nnp_vehicle_state(C.Structure):
    _fields_ = [("z", C.c_float * 4), ("a", C.c_float * 2), ("cost", C.c_float),
                ("waypoint", C.c_int32), ("steps", C.c_int32), ("done", C.c_int32),
                ("infeasible_steps", C.c_int32)]


_bound = None


def lib():
    global _bound
    if _bound is not None:
        return _bound
    L = load_library()
    H, V = C.c_void_p, C.c_void_p
    sig = {
        "nnp_fleet_create": (C.c_int, [C.POINTER(H), H, H, C.POINTER(nnp_fleet_config),
                                       C.POINTER(nnp_vehicle_spec)]),
        "nnp_fleet_step": (C.c_int, [H, V, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
        "nnp_fleet_state": (C.c_int, [H, C.POINTER(nnp_vehicle_state)]),
        "nnp_fleet_destroy": (None, [H]),
        "nnp_fleet_last_error": (C.c_char_p, [H]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _bound = L
    return L


class Fleet:
    """Vehicles: list of dicts with z0 [4], waypoints [[x, y, phi, v], ...] and points (a device
    float32 tensor [P][4] or None). Waypoint tolerances default to the planner preset's (Table
    II); `tolerances` overrides any of eps_xi, eps_eta, eps_phi, eps_v."""

    def __init__(self, planner, vehicles, T: int, n_uniform: int, n_prop: int = 0,
                 proposal=None, seed: int = 0, warm_start: bool = True, tolerances=None,
                 switch_rule: int = SWITCH_STATE):
        import torch
        self.torch = torch
        self.planner = planner
        self.proposal = proposal
        p = planner.preset
        c = nnp_fleet_config()
        c.n_vehicles, c.T, c.n_uniform, c.n_prop = len(vehicles), T, n_uniform, n_prop
        c.seed, c.warm_start, c.dt = seed, int(warm_start), float(p["dt"])
        tol = dict(p, **(tolerances or {}))
        c.eps_xi, c.eps_eta, c.eps_phi, c.eps_v = (float(tol[k]) for k in
                                                   ("eps_xi", "eps_eta", "eps_phi", "eps_v"))
        c.switch_rule = int(switch_rule)
        specs = (nnp_vehicle_spec * len(vehicles))()
        self._keep = []
        for i, v in enumerate(vehicles):
            for k in range(4):
                specs[i].z0[k] = float(v["z0"][k])
            wp = np.ascontiguousarray(np.asarray(v["waypoints"], np.float32).reshape(-1, 4))
            self._keep.append(wp)
            specs[i].waypoints = wp.ctypes.data_as(C.POINTER(C.c_float))
            specs[i].n_waypoints = len(wp)
            pts = v.get("points")
            specs[i].P = 0 if pts is None else int(pts.shape[0])
            specs[i].obst = None if pts is None or pts.shape[0] == 0 else pts.data_ptr()
            gw = v.get("goal_weights")
            if gw is not None:         # this vehicle's own goal heading / speed weights
                specs[i].own_goal_weights = 1
                specs[i].goal_heading_weight = float(np.float32(gw[0]))
                specs[i].goal_speed_weight = float(np.float32(gw[1]))
        self.n = len(vehicles)
        self.h = C.c_void_p()
        rc = lib().nnp_fleet_create(C.byref(self.h), planner.h,
                                    proposal.h if proposal is not None else None, C.byref(c),
                                    specs)
        if rc != NNP_OK:
            raise NnpError(rc, lib().nnp_fleet_last_error(None).decode())

    def close(self):
        if self.h:
            lib().nnp_fleet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self):
        """One sampling time; returns (latency_ms, vehicles planned)."""
        ms, na = C.c_double(), C.c_int32()
        stream = self.torch.cuda.current_stream(self.planner._dev()).cuda_stream
        rc = lib().nnp_fleet_step(self.h, C.c_void_p(stream), C.byref(ms), C.byref(na))
        if rc < 0:
            raise NnpError(rc, lib().nnp_fleet_last_error(self.h).decode())
        return ms.value, na.value

    def state(self) -> list:
        arr = (nnp_vehicle_state * self.n)()
        lib().nnp_fleet_state(self.h, arr)
        return [dict(z=np.array(s.z[:], np.float32), a=np.array(s.a[:], np.float32),
                     cost=s.cost, waypoint=s.waypoint, steps=s.steps, done=bool(s.done),
                     infeasible_steps=s.infeasible_steps) for s in arr]
