"""Python binding of the C-ABI in ``include/nnproposal.h`` (ctypes; argument marshalling only).

The raw entry points keep their C names (``nnp_proposal_create``, ``nnp_proposal_train_step``,
``nnp_gemm_bf16``, ...). ``Proposal`` wraps a handle and passes torch device tensors; every
computation runs in the HIP kernels of ``libnnplan.so``.
"""
from __future__ import annotations

import ctypes as C

from .nnplan import NNP_OK, NnpError, load_library

EXPORTED = ("nnp_proposal_create", "nnp_proposal_destroy", "nnp_proposal_n_params",
            "nnp_proposal_set_params", "nnp_proposal_get_params", "nnp_proposal_get_state",
            "nnp_proposal_set_state", "nnp_proposal_encode",
            "nnp_proposal_forward", "nnp_proposal_gradients", "nnp_proposal_train_step",
            "nnp_gemm_bf16", "nnp_proposal_last_error")

ENC, HIDDEN, NEAR = 72, 256, 16


class nnp_proposal_config(C.Structure):
    _fields_ = [("n_theta", C.c_int32), ("max_batch", C.c_int32), ("norm_xi", C.c_float),
                ("norm_eta", C.c_float), ("norm_phi", C.c_float), ("norm_v", C.c_float),
                ("d_cap", C.c_float), ("u_min", C.c_float), ("u_max", C.c_float)]


_bound = None


def lib():
    global _bound
    if _bound is not None:
        return _bound
    L = load_library()
    H, V, I, F = C.c_void_p, C.c_void_p, C.c_int, C.c_float
    sig = {
        "nnp_proposal_create": (I, [C.POINTER(H), C.POINTER(nnp_proposal_config), I]),
        "nnp_proposal_destroy": (None, [H]),
        "nnp_proposal_n_params": (I, [H]),
        "nnp_proposal_set_params": (I, [H, V, V]),
        "nnp_proposal_get_params": (I, [H, V, V]),
        "nnp_proposal_get_state": (I, [H, V, V, V, C.POINTER(C.c_int64), V]),
        "nnp_proposal_set_state": (I, [H, V, V, V, C.c_int64, V]),
        "nnp_proposal_encode": (I, [H, V, I, V, V]),
        "nnp_proposal_forward": (I, [H, V, I, V, V, V]),
        "nnp_proposal_gradients": (I, [H, V, V, I, V, V, V]),
        "nnp_proposal_train_step": (I, [H, V, V, I, F, V, V]),
        "nnp_gemm_bf16": (I, [I, I, I, I, I, V, I, V, I, I, V, V, I, V, I, V, I, V]),
        "nnp_proposal_last_error": (C.c_char_p, [H]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _bound = L
    return L


def _p(t):
    return None if t is None else t.data_ptr()


def nnp_proposal_last_error(q=None) -> str:
    return lib().nnp_proposal_last_error(q).decode()


def nnp_gemm_bf16(a_layout, b_layout, M, N, K, A, lda, B, ldb, epilogue=0, bias=None, mask=None,
                  ldm=0, Cout=None, ldc=0, Cq=None, ldcq=0, stream=0) -> int:
    """Tensors in, raw return code out (bfloat16 operands as int16/uint16/bfloat16 tensors)."""
    return lib().nnp_gemm_bf16(a_layout, b_layout, M, N, K, _p(A), lda, _p(B), ldb, epilogue,
                               _p(bias), _p(mask), ldm, _p(Cout), ldc, _p(Cq), ldcq,
                               C.c_void_p(stream))


def config(preset: dict, n_theta: int, max_batch: int) -> nnp_proposal_config:
    c = nnp_proposal_config()
    c.n_theta, c.max_batch = n_theta, max_batch
    for k in ("norm_xi", "norm_eta", "norm_phi", "norm_v", "d_cap", "u_min", "u_max"):
        setattr(c, k, float(preset[k]))
    return c


class Proposal:
    """A proposal network handle on one device, fed with torch tensors."""

    def __init__(self, preset: dict, n_theta: int, max_batch: int, device: int = 0):
        import torch
        self.torch = torch
        self.device = device
        self.n_theta = n_theta
        self.max_batch = max_batch
        self.cfg = config(preset, n_theta, max_batch)
        self.h = C.c_void_p()
        rc = lib().nnp_proposal_create(C.byref(self.h), C.byref(self.cfg), device)
        if rc != NNP_OK:
            raise NnpError(rc, nnp_proposal_last_error(None))
        self.n_params = lib().nnp_proposal_n_params(self.h)

    def close(self):
        if self.h:
            lib().nnp_proposal_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self):
        return self.torch.device("cuda", self.device)

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self._dev()).cuda_stream)

    def _check(self, rc):
        if rc < 0:
            raise NnpError(rc, nnp_proposal_last_error(self.h))

    def set_params(self, params):
        self._check(lib().nnp_proposal_set_params(self.h, _p(params), self._stream()))

    def get_params(self):
        out = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self._dev())
        self._check(lib().nnp_proposal_get_params(self.h, _p(out), self._stream()))
        return out

    def get_state(self) -> dict:
        """Training state: parameters, Adam moments m and v (device tensors) and the step count."""
        t = self.torch
        params, m, v = (t.empty(self.n_params, dtype=t.float32, device=self._dev())
                        for _ in range(3))
        step = C.c_int64()
        self._check(lib().nnp_proposal_get_state(self.h, _p(params), _p(m), _p(v),
                                                  C.byref(step), self._stream()))
        return dict(params=params, m=m, v=v, step=int(step.value))

    def set_state(self, state: dict):
        """Load a state from get_state (tensors on any device; copied to this one)."""
        d = self._dev()
        ts = [state[k].to(d, self.torch.float32).contiguous() for k in ("params", "m", "v")]
        self._check(lib().nnp_proposal_set_state(self.h, *(_p(x) for x in ts), int(state["step"]),
                                                  self._stream()))
        self.torch.cuda.synchronize(d)

    def encode_problems(self, probs):
        """probs: ctypes array of nnplan.nnp_problem (obstacles on this device)."""
        out = self.torch.empty(len(probs), ENC, dtype=self.torch.float32, device=self._dev())
        self._check(lib().nnp_proposal_encode(self.h, probs, len(probs), _p(out), self._stream()))
        return out

    def forward(self, enc):
        B = enc.shape[0]
        mu = self.torch.empty(B, self.n_theta, dtype=self.torch.float32, device=self._dev())
        ls = self.torch.empty_like(mu)
        self._check(lib().nnp_proposal_forward(self.h, _p(enc), B, _p(mu), _p(ls),
                                               self._stream()))
        return mu, ls

    def gradients(self, enc, theta_star):
        g = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self._dev())
        loss = self.torch.empty(1, dtype=self.torch.float32, device=self._dev())
        self._check(lib().nnp_proposal_gradients(self.h, _p(enc), _p(theta_star), enc.shape[0],
                                                 _p(g), _p(loss), self._stream()))
        return g, loss

    def train_step(self, enc, theta_star, lr: float, loss=None):
        self._check(lib().nnp_proposal_train_step(self.h, _p(enc), _p(theta_star), enc.shape[0],
                                                  float(lr), _p(loss), self._stream()))
