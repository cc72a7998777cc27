"""Python binding of the C-ABI in ``include/nnplan.h`` (ctypes; argument marshalling only).

The raw entry points keep their C names (``nnp_create``, ``nnp_plan``, ``nnp_rollout``,
``nnp_sample_theta``, ...). ``Planner`` wraps a handle and marshals torch device tensors into the
C structs; every step of the planner runs in the HIP kernels of ``libnnplan.so``. There is no
CPU fallback: importing this module fails when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB

MAX_LAYERS = 3
NNP_OK, NNP_INFEASIBLE = 0, 1
NNP_EINVAL, NNP_ENOMEM, NNP_EDEVICE, NNP_EUNSUPPORTED = -1, -2, -3, -4
FEAT_PAPER, FEAT_SIX, FEAT_EIGHT = 0, 1, 2

EXPORTED = ("nnp_create", "nnp_destroy", "nnp_n_theta", "nnp_plan", "nnp_plan_noalloc",
            "nnp_plan_batch", "nnp_rollout",
            "nnp_sample_theta", "nnp_sample_gauss", "nnp_last_error", "nnp_set_timing", "nnp_kernel_time",
            "nnp_set_cull_stats", "nnp_cull_stats",
            "nnp_set_record_limit", "nnp_set_workspace_limit", "nnp_version")


class nnp_model(C.Structure):
    _fields_ = [
        ("dt", C.c_float), ("lf", C.c_float), ("lr", C.c_float),
        ("front", C.c_float), ("rear", C.c_float), ("half_width", C.c_float),
        ("delta_max", C.c_float), ("delta_rate_max", C.c_float),
        ("u_min", C.c_float), ("u_max", C.c_float), ("v_min", C.c_float), ("v_max", C.c_float),
        ("n_layers", C.c_int32), ("widths", C.c_int32 * (MAX_LAYERS + 1)),
        ("feature_set", C.c_int32),
        ("norm_xi", C.c_float), ("norm_eta", C.c_float), ("norm_phi", C.c_float),
        ("norm_v", C.c_float), ("d_cap", C.c_float), ("effort_weight", C.c_float),
        ("eps_xi", C.c_float), ("eps_eta", C.c_float), ("eps_phi", C.c_float),
        ("eps_v", C.c_float), ("lanes_per_sample", C.c_int32),
        ("goal_heading_weight", C.c_float), ("goal_speed_weight", C.c_float),
        ("block_threads", C.c_int32), ("tile_pairs", C.c_int32), ("all_points", C.c_int32),
    ]


class nnp_problem(C.Structure):
    _fields_ = [
        ("z0", C.c_float * 4), ("goal", C.c_float * 4), ("a_prev", C.POINTER(C.c_float)),
        ("obst", C.c_void_p), ("P", C.c_int32), ("N", C.c_int32), ("T", C.c_int32),
        ("inst", C.c_uint32), ("seed", C.c_uint64), ("warm_theta", C.c_void_p),
        ("n_prop", C.c_int32), ("prop_mu", C.c_void_p), ("prop_log_sigma", C.c_void_p),
        ("own_goal_weights", C.c_int32), ("goal_heading_weight", C.c_float),
        ("goal_speed_weight", C.c_float),
    ]


class nnp_result(C.Structure):
    _fields_ = [
        ("theta", C.c_void_p), ("controls", C.c_void_p), ("controls_phys", C.c_void_p),
        ("traj", C.c_void_p), ("cost", C.c_void_p), ("best_index", C.c_void_p),
        ("status", C.c_void_p), ("goal_reached", C.c_void_p),
    ]


class nnp_rollout_out(C.Structure):
    _fields_ = [
        ("cost", C.c_void_p), ("collided", C.c_void_p), ("first_collision", C.c_void_p),
        ("min_margin", C.c_void_p), ("traj", C.c_void_p), ("controls", C.c_void_p),
    ]


_lib = None


def load_library(path: str = LIB):
    """Load libnnplan.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -m paper_1904_06680_amd.build` "
                          "(or __graft_entry__.build())")
    # torch brings its own HIP runtime; it has to be in the process first so that the library
    # binds to that same runtime (two runtimes in one process do not share the device).
    import torch  # noqa: F401
    L = C.CDLL(path)
    H = C.c_void_p
    sig = {
        "nnp_create": (C.c_int, [C.POINTER(H), C.POINTER(nnp_model), C.c_int]),
        "nnp_destroy": (None, [H]),
        "nnp_n_theta": (C.c_int, [H]),
        "nnp_plan": (C.c_int, [H, C.POINTER(nnp_problem), C.POINTER(nnp_result), C.c_void_p]),
        "nnp_plan_noalloc": (C.c_int, [H, C.POINTER(nnp_problem), C.POINTER(nnp_result),
                                       C.c_void_p]),
        "nnp_plan_batch": (C.c_int, [H, C.POINTER(nnp_problem), C.c_int, C.POINTER(nnp_result),
                                     C.c_void_p]),
        "nnp_rollout": (C.c_int, [H, C.POINTER(nnp_problem), C.c_void_p,
                                  C.POINTER(nnp_rollout_out), C.c_void_p]),
        "nnp_sample_theta": (C.c_int, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                       C.c_uint32, C.c_void_p, C.c_void_p]),
        "nnp_sample_gauss": (C.c_int, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                       C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
        "nnp_last_error": (C.c_char_p, [H]),
        "nnp_set_timing": (C.c_int, [H, C.c_int]),
        "nnp_set_cull_stats": (C.c_int, [H, C.c_int]),
        "nnp_cull_stats": (C.c_int, [H, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.c_int]),
        "nnp_set_record_limit": (C.c_int, [H, C.c_uint64]),
        "nnp_set_workspace_limit": (C.c_int, [H, C.c_uint64]),
        "nnp_kernel_time": (C.c_int, [H, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]),
        "nnp_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


# Raw C entry points under their C names.
def nnp_create(model: nnp_model, device: int = 0):
    h = C.c_void_p()
    rc = load_library().nnp_create(C.byref(h), C.byref(model), device)
    return rc, h


def nnp_destroy(h):
    load_library().nnp_destroy(h)


def nnp_n_theta(h) -> int:
    return load_library().nnp_n_theta(h)


def nnp_plan(h, problem: nnp_problem, result: nnp_result, stream: int = 0) -> int:
    return load_library().nnp_plan(h, C.byref(problem), C.byref(result), C.c_void_p(stream))


def nnp_plan_noalloc(h, problem: nnp_problem, result: nnp_result, stream: int = 0) -> int:
    return load_library().nnp_plan_noalloc(h, C.byref(problem), C.byref(result),
                                           C.c_void_p(stream))


def nnp_plan_batch(h, problems, results, stream: int = 0) -> int:
    """problems: ctypes array of nnp_problem; results: ctypes array of nnp_result (same length)."""
    return load_library().nnp_plan_batch(h, problems, len(problems), results, C.c_void_p(stream))


def nnp_rollout(h, problem: nnp_problem, theta_ptr, out: nnp_rollout_out, stream: int = 0) -> int:
    return load_library().nnp_rollout(h, C.byref(problem), C.c_void_p(theta_ptr), C.byref(out),
                                      C.c_void_p(stream))


def nnp_sample_theta(seed: int, inst: int, i0: int, N: int, n_theta: int, out_ptr: int,
                     stream: int = 0) -> int:
    return load_library().nnp_sample_theta(seed, inst, i0, N, n_theta, C.c_void_p(out_ptr),
                                           C.c_void_p(stream))


def nnp_sample_gauss(seed: int, inst: int, i0: int, N: int, n_theta: int, mu_ptr: int,
                     log_sigma_ptr: int, out_ptr: int, stream: int = 0) -> int:
    return load_library().nnp_sample_gauss(seed, inst, i0, N, n_theta, C.c_void_p(mu_ptr),
                                           C.c_void_p(log_sigma_ptr), C.c_void_p(out_ptr),
                                           C.c_void_p(stream))


def nnp_last_error(h=None) -> str:
    return load_library().nnp_last_error(h).decode()


def nnp_set_timing(h, enable: bool) -> int:
    return load_library().nnp_set_timing(h, int(enable))


def nnp_set_record_limit(h, nbytes: int) -> int:
    return load_library().nnp_set_record_limit(h, int(nbytes))


def nnp_set_workspace_limit(h, nbytes: int) -> int:
    return load_library().nnp_set_workspace_limit(h, int(nbytes))


def nnp_kernel_time(h, reset: bool = False):
    ms, n = C.c_double(), C.c_int64()
    rc = load_library().nnp_kernel_time(h, C.byref(ms), C.byref(n), int(reset))
    return rc, ms.value, n.value


def nnp_set_cull_stats(h, enable: bool) -> int:
    return load_library().nnp_set_cull_stats(h, int(enable))


def nnp_cull_stats(h, reset: bool = False):
    tested, total = C.c_uint64(), C.c_uint64()
    rc = load_library().nnp_cull_stats(h, C.byref(tested), C.byref(total), int(reset))
    return rc, tested.value, total.value


def nnp_version() -> str:
    return load_library().nnp_version().decode()


# --------------------------------------------------------------------------------------------
# Marshalling helpers
# --------------------------------------------------------------------------------------------
def make_model(p: dict, lanes_per_sample: int = 0, block_threads: int = 0,
               tile_pairs: int = 0, all_points: bool = False) -> nnp_model:
    m = nnp_model()
    for k in ("dt", "lf", "lr", "front", "rear", "half_width", "delta_max", "delta_rate_max",
              "u_min", "u_max", "v_min", "v_max", "norm_xi", "norm_eta", "norm_phi", "norm_v",
              "d_cap", "effort_weight", "eps_xi", "eps_eta", "eps_phi", "eps_v"):
        setattr(m, k, float(np.float32(p[k])))
    widths = list(p["widths"])
    m.n_layers = len(widths) - 1
    for i in range(MAX_LAYERS + 1):
        m.widths[i] = widths[i] if i < len(widths) else 0
    m.feature_set = int(p["feature_set"])
    m.lanes_per_sample = int(lanes_per_sample)
    m.block_threads = int(block_threads)
    m.tile_pairs = int(tile_pairs)
    m.all_points = int(bool(all_points))
    m.goal_heading_weight = float(np.float32(p.get("goal_heading_weight", 0.0)))
    m.goal_speed_weight = float(np.float32(p.get("goal_speed_weight", 0.0)))
    return m


class NnpError(RuntimeError):
    def __init__(self, rc: int, msg: str):
        super().__init__(f"nnplan error {rc}: {msg}")
        self.rc = rc


def _check(rc: int, h=None):
    if rc < 0:
        raise NnpError(rc, nnp_last_error(h))
    return rc


class Planner:
    """A planner handle for one model on one device, fed with torch tensors."""

    def __init__(self, preset: dict, device: int = 0, lanes_per_sample: int = 0,
                 block_threads: int = 0, tile_pairs: int = 0, all_points: bool = False):
        import torch
        self.torch = torch
        self.preset = dict(preset)
        self.model = make_model(preset, lanes_per_sample, block_threads, tile_pairs, all_points)
        self.device = device
        rc, self.h = nnp_create(self.model, device)
        if rc != NNP_OK:
            raise NnpError(rc, nnp_last_error(None))
        self.n_theta = nnp_n_theta(self.h)

    def close(self):
        if self.h:
            nnp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self):
        return self.torch.device("cuda", self.device)

    def _stream(self):
        return self.torch.cuda.current_stream(self._dev()).cuda_stream

    def problem(self, scene, N: int, seed: int = 0, inst: int = 0, obst=None,
                warm_theta=None, proposal=None) -> tuple:
        """nnp_problem for a scene; returns (problem, keep-alive tuple). `proposal` = (mu,
        log_sigma, n_prop) draws samples 0..n_prop-1 from that Gaussian (device tensors)."""
        torch = self.torch
        pr = nnp_problem()
        for i in range(4):
            pr.z0[i] = float(scene.z0[i])
            pr.goal[i] = float(scene.goal[i])
        keep = []
        if scene.a_prev is not None:
            ap = (C.c_float * 2)(float(scene.a_prev[0]), float(scene.a_prev[1]))
            keep.append(ap)
            pr.a_prev = C.cast(ap, C.POINTER(C.c_float))
        else:
            pr.a_prev = None
        if obst is None and scene.P > 0:
            obst = torch.from_numpy(scene.points).to(self._dev())
        if obst is not None:
            keep.append(obst)
            pr.obst = obst.data_ptr()
        pr.P = scene.P
        pr.N = int(N)
        pr.T = scene.T
        pr.inst = int(inst)
        pr.seed = int(seed)
        if warm_theta is not None:
            keep.append(warm_theta)
            pr.warm_theta = warm_theta.data_ptr()
        if proposal is not None:
            mu, ls, n_prop = proposal
            keep += [mu, ls]
            pr.prop_mu = mu.data_ptr()
            pr.prop_log_sigma = ls.data_ptr()
            pr.n_prop = int(n_prop)
        gw = getattr(scene, "goal_weights", None)
        if gw is not None:             # this problem's own goal heading / speed weights
            pr.own_goal_weights = 1
            pr.goal_heading_weight = float(np.float32(gw[0]))
            pr.goal_speed_weight = float(np.float32(gw[1]))
        return pr, keep

    def plan_async(self, pr: nnp_problem, out: dict, stream=None, noalloc: bool = False):
        """nnp_plan, or nnp_plan_noalloc when noalloc is set, into the tensors of `out`."""
        res = nnp_result()
        for k in ("theta", "controls", "controls_phys", "traj", "cost", "best_index", "status",
                  "goal_reached"):
            t = out.get(k)
            setattr(res, k, t.data_ptr() if t is not None else None)
        entry = nnp_plan_noalloc if noalloc else nnp_plan
        _check(entry(self.h, pr, res, self._stream() if stream is None else stream), self.h)

    def alloc_result(self, T: int) -> dict:
        torch, d = self.torch, self._dev()
        return dict(theta=torch.empty(self.n_theta, dtype=torch.float32, device=d),
                    controls=torch.empty(T, 2, dtype=torch.float32, device=d),
                    controls_phys=torch.empty(T, 2, dtype=torch.float32, device=d),
                    traj=torch.empty(T + 1, 4, dtype=torch.float32, device=d),
                    cost=torch.empty(1, dtype=torch.float32, device=d),
                    best_index=torch.empty(1, dtype=torch.int32, device=d),
                    status=torch.empty(1, dtype=torch.int32, device=d),
                    goal_reached=torch.empty(1, dtype=torch.int32, device=d))

    def plan(self, scene, N: int, seed: int = 0, inst: int = 0, warm_theta=None,
             proposal=None, noalloc: bool = False) -> dict:
        pr, keep = self.problem(scene, N, seed, inst, warm_theta=warm_theta, proposal=proposal)
        out = self.alloc_result(scene.T)
        self.plan_async(pr, out, noalloc=noalloc)
        self.torch.cuda.synchronize(self._dev())
        del keep
        return out

    def batch_problems(self, scenes_, Ns, seeds, insts=None):
        """ctypes arrays (problems, results) and keep-alive objects for a batch of scenes."""
        n = len(scenes_)
        probs = (nnp_problem * n)()
        keep = []
        for i, sc in enumerate(scenes_):
            pr, k = self.problem(sc, int(Ns[i]), int(seeds[i]), 0 if insts is None else insts[i])
            probs[i] = pr
            keep.append(k)
        return probs, keep

    def plan_batch_async(self, probs, outs: list, stream=None):
        res = (nnp_result * len(outs))()
        for i, out in enumerate(outs):
            for k in ("theta", "controls", "controls_phys", "traj", "cost", "best_index",
                      "status", "goal_reached"):
                t = out.get(k)
                setattr(res[i], k, t.data_ptr() if t is not None else None)
        _check(nnp_plan_batch(self.h, probs, res, self._stream() if stream is None else stream),
               self.h)
        return res

    def array_problems(self, z0, goal, pts, T: int, Ns, seeds, a_prev=None, proposal=None,
                       warm_theta=None, insts=None):
        """ctypes array of problems for n scenes held as arrays: z0, goal host float [n][4];
        pts a device float32 tensor [n][P][4] (or None for no obstacles); a_prev host [n][2] or
        None (idle); proposal = (mu, log_sigma, n_prop) with device tensors [n][n_theta] and an
        int or per-problem counts; warm_theta a device tensor [n][n_theta] or None. The caller
        keeps every tensor alive until the work has run. Returns (problems, host keep-alive)."""
        n = len(z0)
        probs = (nnp_problem * n)()
        P = 0 if pts is None else int(pts.shape[1])
        ap_all = None
        if a_prev is not None:
            ap_all = (C.c_float * (2 * n))(*np.asarray(a_prev, np.float32).ravel().tolist())
        base = C.addressof(ap_all) if ap_all is not None else 0
        for i in range(n):
            pr = probs[i]
            for k in range(4):
                pr.z0[k] = float(z0[i][k])
                pr.goal[k] = float(goal[i][k])
            if ap_all is not None:
                pr.a_prev = C.cast(base + 8 * i, C.POINTER(C.c_float))
            pr.P = P
            pr.obst = pts[i].data_ptr() if P else None
            pr.N = int(Ns[i])
            pr.T = int(T)
            pr.seed = int(seeds[i])
            pr.inst = 0 if insts is None else int(insts[i])
            if warm_theta is not None:
                pr.warm_theta = warm_theta[i].data_ptr()
            if proposal is not None:
                mu, ls, n_prop = proposal
                pr.prop_mu = mu[i].data_ptr()
                pr.prop_log_sigma = ls[i].data_ptr()
                pr.n_prop = int(n_prop if np.isscalar(n_prop) else n_prop[i])
        return probs, ap_all

    def alloc_batch(self, n: int, T: int, keys=("theta", "cost", "best_index", "status")) -> dict:
        """Batched output tensors (row i is problem i's result)."""
        torch, d = self.torch, self._dev()
        shapes = dict(theta=((n, self.n_theta), torch.float32), controls=((n, T, 2), torch.float32),
                      controls_phys=((n, T, 2), torch.float32),
                      traj=((n, T + 1, 4), torch.float32), cost=((n,), torch.float32),
                      best_index=((n,), torch.int32), status=((n,), torch.int32),
                      goal_reached=((n,), torch.int32))
        return {k: torch.empty(*shapes[k][0], dtype=shapes[k][1], device=d) for k in keys}

    def plan_batch_into(self, probs, out: dict, stream=None):
        """nnp_plan_batch with problem i's outputs written to row i of the tensors in `out`."""
        n = len(probs)
        res = (nnp_result * n)()
        for k, t in out.items():
            stride = t.stride(0) * t.element_size()
            base = t.data_ptr()
            for i in range(n):
                setattr(res[i], k, base + i * stride)
        _check(nnp_plan_batch(self.h, probs, res, self._stream() if stream is None else stream),
               self.h)

    def plan_batch(self, scenes_, Ns, seeds) -> list:
        probs, keep = self.batch_problems(scenes_, Ns, seeds)
        outs = [self.alloc_result(sc.T) for sc in scenes_]
        self.plan_batch_async(probs, outs)
        self.torch.cuda.synchronize(self._dev())
        del keep
        return outs

    def rollout(self, scene, N: int, seed: int = 0, inst: int = 0, theta=None,
                want_traj: bool = True, want_controls: bool = True, proposal=None,
                want_margin: bool = True) -> dict:
        """Per-sample outputs of nnp_rollout. The minimum margin is a minimum over every point,
        so requesting it (want_margin) makes the call test every point."""
        torch, d = self.torch, self._dev()
        pr, keep = self.problem(scene, N, seed, inst, proposal=proposal)
        T = scene.T
        out = dict(cost=torch.empty(N, dtype=torch.float32, device=d),
                   collided=torch.empty(N, dtype=torch.int32, device=d),
                   first_collision=torch.empty(N, dtype=torch.int32, device=d))
        if want_margin:
            out["min_margin"] = torch.empty(N, dtype=torch.float32, device=d)
        if want_traj:
            out["traj"] = torch.empty(N, T + 1, 4, dtype=torch.float32, device=d)
        if want_controls:
            out["controls"] = torch.empty(N, T, 2, dtype=torch.float32, device=d)
        o = nnp_rollout_out()
        for k in ("cost", "collided", "first_collision", "min_margin", "traj", "controls"):
            t = out.get(k)
            setattr(o, k, t.data_ptr() if t is not None else None)
        th = 0
        if theta is not None:
            theta = theta.to(device=d, dtype=torch.float32).contiguous()
            assert theta.shape == (N, self.n_theta)
            keep.append(theta)
            th = theta.data_ptr()
        _check(nnp_rollout(self.h, pr, th, o, self._stream()), self.h)
        torch.cuda.synchronize(d)
        del keep
        return out

    def sample_theta(self, N: int, seed: int = 0, inst: int = 0, i0: int = 0):
        torch = self.torch
        out = torch.empty(N, self.n_theta, dtype=torch.float32, device=self._dev())
        _check(nnp_sample_theta(seed, inst, i0, N, self.n_theta, out.data_ptr(), self._stream()))
        torch.cuda.synchronize(self._dev())
        return out

    def sample_gauss(self, mu, log_sigma, N: int, seed: int = 0, inst: int = 0, i0: int = 0):
        torch = self.torch
        out = torch.empty(N, self.n_theta, dtype=torch.float32, device=self._dev())
        _check(nnp_sample_gauss(seed, inst, i0, N, self.n_theta, mu.data_ptr(),
                                log_sigma.data_ptr(), out.data_ptr(), self._stream()))
        return out

    def set_timing(self, enable: bool = True):
        _check(nnp_set_timing(self.h, enable), self.h)

    def set_record_limit(self, nbytes: int):
        """Largest per-sample record workspace of plan() and plan_batch(); 0 re-simulates every
        winner."""
        _check(nnp_set_record_limit(self.h, nbytes), self.h)

    def set_workspace_limit(self, nbytes: int):
        """Cap on the handle's grown device workspace; calls needing more raise (NNP_ENOMEM)."""
        _check(nnp_set_workspace_limit(self.h, nbytes), self.h)

    def set_cull_stats(self, enable: bool = True):
        """Count the point groups the obstacle pass tests (see cull_stats)."""
        _check(nnp_set_cull_stats(self.h, enable), self.h)

    def cull_stats(self, reset: bool = False):
        """(tested, total) point groups over wavefront-steps since the last reset."""
        rc, tested, total = nnp_cull_stats(self.h, reset)
        _check(rc, self.h)
        return tested, total

    def kernel_time(self, reset: bool = False):
        rc, ms, n = nnp_kernel_time(self.h, reset)
        _check(rc, self.h)
        return ms, n

