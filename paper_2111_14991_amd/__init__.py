"""Python binding of the gfx950 BO-step library (libbo_mi355x.so).

Thin ctypes marshalling over the C ABI declared in include/bo.h: every
function named ``bo_*`` here calls the C function of the same name; the
``Session`` class bundles a session handle with a torch-allocated device
workspace and the current torch stream.  Torch provides device memory and
streams only; every step of the computation runs in the library's kernels.
There is no fallback: without the built library (or without a GPU) the calls
raise.

The seeded synthetic inputs live in ``paper_2111_14991_amd.workloads`` and do
not load the library.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbo_mi355x.so")

BO_OK, BO_E_INVALID_ARG, BO_E_NOT_PD, BO_E_NO_CANDIDATE, BO_E_WORKSPACE, BO_E_HIP, BO_E_STATE, \
    BO_E_BUDGET, BO_E_NUMERIC = range(9)
BO_FP64, BO_FP32, BO_BF16X3 = 0, 1, 2
BO_EI, BO_POI, BO_LCB = 1, 2, 4
PRECISIONS = {"fp64": BO_FP64, "fp32": BO_FP32, "bf16x3": BO_BF16X3}


class bo_problem(C.Structure):
    _fields_ = [("N", C.c_int64), ("d", C.c_int32), ("n_max", C.c_int32), ("precision", C.c_int32),
                ("reserved", C.c_int32)]


class bo_gp_params(C.Structure):
    _fields_ = [("nu2", C.c_int32), ("jitter_tries", C.c_int32), ("lengthscale", C.c_double),
                ("amp", C.c_double), ("noise", C.c_double)]


class bo_acq_params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("acq_bits", C.c_uint32), ("lambda_const", C.c_double),
                ("mu_s", C.c_double), ("var_s_mean", C.c_double)]


class bo_acq_result(C.Structure):
    _fields_ = [("idx", C.c_int64 * 3), ("score", C.c_double * 3), ("lambda_", C.c_double),
                ("var_mean", C.c_double), ("jitter", C.c_double), ("f_best", C.c_double),
                ("mean_y", C.c_double), ("n_unmasked", C.c_int64), ("status", C.c_int32),
                ("n_obs", C.c_int32)]


class bo_fit_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("n", C.c_int32), ("attempt", C.c_int32), ("reserved", C.c_int32),
                ("jitter", C.c_double), ("mean_y", C.c_double), ("f_best", C.c_double)]


class BOError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


_lib = None
_VP, _I64P, _DP, _I32P, _U8P = C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p

# name -> (restype, argtypes)
_SIGS = {
    "bo_version": (C.c_char_p, []),
    "bo_last_error": (C.c_char_p, []),
    "bo_workspace_query": (C.c_int, [C.POINTER(bo_problem), C.POINTER(C.c_size_t)]),
    "bo_session_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(bo_problem), C.POINTER(bo_gp_params),
                                    _VP, C.c_size_t, _VP]),
    "bo_session_destroy": (None, [_VP]),
    "bo_session_set_stream": (C.c_int, [_VP, _VP]),
    "bo_set_grid": (C.c_int, [_VP, _I32P, _I64P, _U8P, C.POINTER(C.c_int64)]),
    "bo_set_candidates": (C.c_int, [_VP, _VP, C.c_int32, _U8P, C.POINTER(C.c_int64)]),
    "bo_gp_fit": (C.c_int, [_VP, _I64P, _DP, C.c_int32]),
    "bo_fit_read": (C.c_int, [_VP, C.POINTER(bo_fit_info), _DP, _DP]),
    "bo_posterior": (C.c_int, [_VP, _U8P, _DP, _DP, C.POINTER(C.c_double)]),
    "bo_acquire": (C.c_int, [_VP, _U8P, C.POINTER(bo_acq_params), C.POINTER(bo_acq_result)]),
    "bo_acquire_async": (C.c_int, [_VP, _U8P, C.POINTER(bo_acq_params), _VP]),
    "bo_set_timing": (C.c_int, [_VP, C.c_int32]),
    "bo_get_timing": (C.c_int, [_VP, C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_float)]),
}


def exported_symbols() -> list:
    return list(_SIGS)


def lib():
    """Load libbo_mi355x.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2111_14991_amd/build.py "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().bo_last_error().decode()


def _check(rc: int, where: str) -> int:
    if rc != BO_OK:
        raise BOError(rc, where, last_error())
    return rc


# ---- thin same-name wrappers ------------------------------------------------

def bo_version() -> str:
    return lib().bo_version().decode()


def bo_workspace_query(N: int, d: int, n_max: int, precision: int) -> int:
    p = bo_problem(N, d, n_max, precision, 0)
    out = C.c_size_t()
    _check(lib().bo_workspace_query(C.byref(p), C.byref(out)), "bo_workspace_query")
    return out.value


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the BO-step library runs only on an MI355X (gfx950)")
    return torch


def _dev(x, dtype, torch, device):
    """Host array or tensor -> contiguous device tensor of `dtype`."""
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=device, dtype=dtype).contiguous()


@dataclass
class GpParams:
    nu2: int = 5
    lengthscale: float = 1.0
    amp: float = 1.0
    noise: float = 1e-6
    jitter_tries: int = 7

    def c(self) -> bo_gp_params:
        return bo_gp_params(self.nu2, self.jitter_tries, self.lengthscale, self.amp, self.noise)


@dataclass
class AcqParams:
    mode: int = 1
    lambda_const: float = 0.01
    mu_s: float = 0.0
    var_s_mean: float = 0.0
    acq_bits: int = 0

    def c(self) -> bo_acq_params:
        return bo_acq_params(self.mode, self.acq_bits, self.lambda_const, self.mu_s, self.var_s_mean)


@dataclass
class StepResult:
    idx: np.ndarray
    score: np.ndarray
    lam: float
    var_mean: float
    jitter: float
    f_best: float
    mean_y: float
    n_unmasked: int
    status: int
    n_obs: int


def _result(r: bo_acq_result) -> StepResult:
    return StepResult(np.array(r.idx[:], dtype=np.int64), np.array(r.score[:]), r.lambda_, r.var_mean,
                      r.jitter, r.f_best, r.mean_y, r.n_unmasked, r.status, r.n_obs)


def result_from_bytes(buf: bytes) -> StepResult:
    return _result(bo_acq_result.from_buffer_copy(buf))


RESULT_BYTES = C.sizeof(bo_acq_result)


class Session:
    """One tuning session: a C session handle over a torch device workspace."""

    def __init__(self, N: int, d: int, n_max: int, precision="fp64", gp: Optional[GpParams] = None,
                 device=None, stream=None):
        torch = _torch()
        self.torch = torch
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.N, self.d, self.n_max = int(N), int(d), int(n_max)
        nbytes = bo_workspace_query(self.N, self.d, self.n_max, self.precision)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        self.gp = gp or GpParams()
        h = C.c_void_p()
        prob = bo_problem(self.N, self.d, self.n_max, self.precision, 0)
        g = self.gp.c()
        _check(lib().bo_session_create(C.byref(h), C.byref(prob), C.byref(g), self._ws_ptr, nbytes,
                                       self.stream.cuda_stream), "bo_session_create")
        self.h = h
        self.n_valid = None
        self._keep = []

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().bo_session_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _d(self, x, dtype):
        return _dev(x, dtype, self.torch, self.device)

    def set_grid(self, levels: Sequence[int], cand=None, invalid=None) -> int:
        torch = self.torch
        lv = (C.c_int32 * self.d)(*[int(k) for k in levels])
        cd = self._d(cand, torch.int64)
        inv = self._d(invalid, torch.uint8)
        nv = C.c_int64()
        _check(lib().bo_set_grid(self.h, lv, _ptr(cd), _ptr(inv), C.byref(nv)), "bo_set_grid")
        self.n_valid = nv.value
        return nv.value

    def set_candidates(self, X, invalid=None) -> int:
        torch = self.torch
        if isinstance(X, torch.Tensor) and X.dtype == torch.float32:
            Xd, f32 = X.to(self.device).contiguous(), 1
        else:
            Xd, f32 = self._d(X, torch.float64), 0
        inv = self._d(invalid, torch.uint8)
        nv = C.c_int64()
        _check(lib().bo_set_candidates(self.h, _ptr(Xd), f32, _ptr(inv), C.byref(nv)), "bo_set_candidates")
        self.n_valid = nv.value
        return nv.value

    def fit(self, obs_idx, y):
        torch = self.torch
        oi = self._d(obs_idx, torch.int64)
        yy = self._d(y, torch.float64)
        self._keep = [oi, yy]  # alive until the next synchronizing call
        _check(lib().bo_gp_fit(self.h, _ptr(oi), _ptr(yy), int(oi.shape[0])), "bo_gp_fit")

    def fit_read(self, want_alpha=True, want_linv=False):
        info = bo_fit_info()
        n = int(self._keep[0].shape[0]) if self._keep else 0
        alpha = np.zeros(n) if want_alpha else None
        Linv = np.zeros((n, n)) if want_linv else None
        rc = lib().bo_fit_read(self.h, C.byref(info), None if alpha is None else alpha.ctypes.data,
                               None if Linv is None else Linv.ctypes.data)
        return rc, info, alpha, Linv

    def posterior(self, visited=None, arrays=True):
        torch = self.torch
        vis = self._d(visited, torch.uint8)
        mu = torch.empty(self.N, dtype=torch.float64, device=self.device) if arrays else None
        var = torch.empty(self.N, dtype=torch.float64, device=self.device) if arrays else None
        vm = C.c_double()
        _check(lib().bo_posterior(self.h, _ptr(vis), _ptr(mu), _ptr(var), C.byref(vm)), "bo_posterior")
        return mu, var, vm.value

    def acquire(self, visited=None, acq: Optional[AcqParams] = None, check=True) -> StepResult:
        torch = self.torch
        vis = self._d(visited, torch.uint8)
        a = (acq or AcqParams(mode=0)).c()
        r = bo_acq_result()
        rc = lib().bo_acquire(self.h, _ptr(vis), C.byref(a), C.byref(r))
        if check and rc not in (BO_OK,):
            raise BOError(rc, "bo_acquire", last_error())
        return _result(r)

    def set_timing(self, enable: bool = True):
        _check(lib().bo_set_timing(self.h, 1 if enable else 0), "bo_set_timing")

    def timing(self):
        """(fit, posterior, acquire) durations in ms of the latest phases."""
        f, p, a = C.c_float(), C.c_float(), C.c_float()
        _check(lib().bo_get_timing(self.h, C.byref(f), C.byref(p), C.byref(a)), "bo_get_timing")
        return f.value, p.value, a.value

    def posterior_async(self, visited=None):
        """Enqueue only the posterior (no outputs, no synchronization)."""
        _check(lib().bo_posterior(self.h, _ptr(visited), None, None, None), "bo_posterior")

    def acquire_async(self, out_dev, visited=None, acq: Optional[AcqParams] = None):
        """Enqueue a step writing its result record into `out_dev` (a device
        uint8 tensor of RESULT_BYTES bytes).  `visited` must stay alive until
        the stream has run the step."""
        a = (acq or AcqParams(mode=0)).c()
        _check(lib().bo_acquire_async(self.h, _ptr(visited), C.byref(a), out_dev.data_ptr()),
               "bo_acquire_async")
