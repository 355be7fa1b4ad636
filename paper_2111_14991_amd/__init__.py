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


class bo_batch_config(C.Structure):
    _fields_ = [("post_order", C.c_int32), ("acq_chunk", C.c_int32), ("fit_order", C.c_int32),
                ("reserved", C.c_int32)]


class bo_server_config(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_batch", C.c_int32), ("streams", C.c_int32),
                ("tiles", bo_batch_config)]


class bo_server_info(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("launches", C.c_int64), ("sessions_resident", C.c_int64),
                ("sessions_waiting", C.c_int64), ("pending", C.c_int64), ("bytes_in_use", C.c_size_t),
                ("mean_batch", C.c_double), ("sessions_setting_up", C.c_int64),
                ("mean_wait_us", C.c_double), ("mean_launch_us", C.c_double), ("mean_gpu_us", C.c_double)]


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
    "bo_gp_append": (C.c_int, [_VP, _I64P, _DP, C.c_int32]),
    "bo_observe": (C.c_int, [_VP, C.c_int64, C.c_double, C.c_int32]),
    "bo_fit_read": (C.c_int, [_VP, C.POINTER(bo_fit_info), _DP, _DP]),
    "bo_posterior": (C.c_int, [_VP, _U8P, _DP, _DP, C.POINTER(C.c_double)]),
    "bo_acquire": (C.c_int, [_VP, _U8P, C.POINTER(bo_acq_params), C.POINTER(bo_acq_result)]),
    "bo_acquire_values": (C.c_int, [_VP, _U8P, C.POINTER(bo_acq_params), _DP, _DP, _DP,
                                    C.POINTER(bo_acq_result)]),
    "bo_acquire_async": (C.c_int, [_VP, _U8P, C.POINTER(bo_acq_params), _VP]),
    "bo_step_noalloc": (C.c_int, [C.POINTER(bo_problem), C.POINTER(bo_gp_params), _VP, C.c_int32, _U8P, _U8P,
                                  _I64P, _DP, C.c_int32, C.POINTER(bo_acq_params), C.POINTER(bo_acq_result), _VP]),
    "bo_set_timing": (C.c_int, [_VP, C.c_int32]),
    "bo_get_timing": (C.c_int, [_VP, C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "bo_batch_workspace_query": (C.c_int, [C.c_int32, C.POINTER(C.c_size_t)]),
    "bo_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32, _VP, C.c_size_t,
                                  _VP]),
    "bo_batch_destroy": (None, [_VP]),
    "bo_batch_set_config": (C.c_int, [_VP, C.POINTER(bo_batch_config)]),
    "bo_batch_get_config": (C.c_int, [_VP, C.POINTER(bo_batch_config)]),
    "bo_batch_set_timing": (C.c_int, [_VP, C.c_int32]),
    "bo_batch_step": (C.c_int, [_VP, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_int32),
                                C.POINTER(C.c_void_p), C.POINTER(bo_acq_params), C.POINTER(bo_acq_result),
                                C.POINTER(C.c_float)]),
    "bo_batch_tune": (C.c_int, [_VP, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_int32),
                                C.POINTER(C.c_void_p), C.POINTER(bo_acq_params), C.c_int32,
                                C.POINTER(bo_batch_config), C.POINTER(bo_acq_result)]),
    "bo_server_session_bytes": (C.c_int, [C.POINTER(bo_problem), C.POINTER(C.c_size_t)]),
    "bo_server_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(bo_server_config)]),
    "bo_server_destroy": (None, [_VP]),
    "bo_server_open": (C.c_int, [_VP, C.POINTER(bo_problem), C.POINTER(bo_gp_params), _VP, _VP, _VP, _VP, _VP,
                                 C.c_int32, C.POINTER(C.c_int32)]),
    "bo_server_close": (C.c_int, [_VP, C.c_int32]),
    "bo_server_submit": (C.c_int, [_VP, C.c_int32, C.c_int64, C.c_double, C.c_int32, C.POINTER(bo_acq_params),
                                   C.POINTER(C.c_uint64)]),
    "bo_server_poll": (C.c_int, [_VP, C.c_uint64, C.POINTER(C.c_int32)]),
    "bo_server_wait": (C.c_int, [_VP, C.c_uint64, C.POINTER(bo_acq_result), C.POINTER(C.c_double)]),
    "bo_server_wait_any": (C.c_int, [_VP, C.c_int32, C.c_int32, C.POINTER(C.c_uint64), C.POINTER(bo_acq_result),
                                     C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "bo_server_stats": (C.c_int, [_VP, C.POINTER(bo_server_info)]),
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
        self.n_fit = 0
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
        self.n_fit = 0
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
        self.n_fit = 0
        return nv.value

    def fit(self, obs_idx, y):
        torch = self.torch
        oi = self._d(obs_idx, torch.int64)
        yy = self._d(y, torch.float64)
        self._keep = [oi, yy]  # alive until the next synchronizing call
        _check(lib().bo_gp_fit(self.h, _ptr(oi), _ptr(yy), int(oi.shape[0])), "bo_gp_fit")
        self.n_fit = int(oi.shape[0])

    def append(self, obs_idx, y):
        """Refit after one new observation: obs_idx / y hold the current fit's
        observations followed by the new one (bo_gp_append)."""
        torch = self.torch
        oi = self._d(obs_idx, torch.int64)
        yy = self._d(y, torch.float64)
        self._keep = [oi, yy]
        _check(lib().bo_gp_append(self.h, _ptr(oi), _ptr(yy), int(oi.shape[0])), "bo_gp_append")
        self.n_fit = int(oi.shape[0])

    def observe(self, idx: int, y: float = 0.0, valid: bool = True):
        """Record one evaluation (bo_observe): candidate `idx` is marked
        evaluated; a valid one is appended to the fit, which is refit."""
        _check(lib().bo_observe(self.h, int(idx), float(y), 1 if valid else 0), "bo_observe")
        if valid:
            self.n_fit += 1

    def fit_read(self, want_alpha=True, want_linv=False):
        info = bo_fit_info()
        n = self.n_fit
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

    def acquire_values(self, visited=None, acq: Optional[AcqParams] = None, check=True):
        """bo_acquire_values: the step result and the EI, PI, LCB arrays over the
        caller's enumeration (device float64 tensors, NaN where excluded)."""
        torch = self.torch
        vis = self._d(visited, torch.uint8)
        a = (acq or AcqParams(mode=0)).c()
        vals = [torch.empty(self.N, dtype=torch.float64, device=self.device) for _ in range(3)]
        r = bo_acq_result()
        rc = lib().bo_acquire_values(self.h, _ptr(vis), C.byref(a), *[_ptr(v) for v in vals], C.byref(r))
        if check and rc != BO_OK:
            raise BOError(rc, "bo_acquire_values", last_error())
        return _result(r), vals

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


def bo_step_noalloc(X, obs_idx, y, precision="fp64", invalid=None, visited=None, gp: Optional[GpParams] = None,
                    acq: Optional[AcqParams] = None, n_max: Optional[int] = None, stream=None, check=True):
    """One whole step with no session and no workspace (bo_step_noalloc): X is
    an N x d device tensor of normalized coordinates (float64, or float32),
    invalid / visited device uint8[N] or None, obs_idx / y the observations.
    Runs on the current torch stream of X's device unless `stream` is given."""
    torch = _torch()
    dev = X.device
    f32 = 1 if X.dtype == torch.float32 else 0
    Xd = X.contiguous() if f32 else X.to(torch.float64).contiguous()
    oi = _dev(obs_idx, torch.int64, torch, dev)
    yy = _dev(y, torch.float64, torch, dev)
    inv = _dev(invalid, torch.uint8, torch, dev)
    vis = _dev(visited, torch.uint8, torch, dev)
    n = int(oi.shape[0])
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    prob = bo_problem(int(Xd.shape[0]), int(Xd.shape[1]), int(n_max or n), prec, 0)
    g = (gp or GpParams()).c()
    a = (acq or AcqParams(mode=0)).c()
    st = torch.cuda.current_stream(dev) if stream is None else stream
    r = bo_acq_result()
    rc = lib().bo_step_noalloc(C.byref(prob), C.byref(g), _ptr(Xd), f32, _ptr(inv), _ptr(vis), _ptr(oi), _ptr(yy),
                               n, C.byref(a), C.byref(r), st.cuda_stream)
    if check and rc != BO_OK:
        raise BOError(rc, "bo_step_noalloc", last_error())
    return _result(r)


class Batch:
    """Many sessions stepped together by one captured graph of kernels
    (bo_batch_*).  The sessions must outlive the batch."""

    def __init__(self, sessions: Sequence[Session], device=None, stream=None):
        torch = _torch()
        self.torch = torch
        self.sessions = list(sessions)
        self.count = len(self.sessions)
        self.device = self.sessions[0].device if device is None else torch.device(device)
        nb = C.c_size_t()
        _check(lib().bo_batch_workspace_query(self.count, C.byref(nb)), "bo_batch_workspace_query")
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        ws = (self.workspace.data_ptr() + 255) // 256 * 256
        hs = (C.c_void_p * self.count)(*[s.h.value for s in self.sessions])
        st = None if stream is None else stream.cuda_stream
        h = C.c_void_p()
        _check(lib().bo_batch_create(C.byref(h), hs, self.count, ws, nb.value, st), "bo_batch_create")
        self.h = h
        self._keep = []

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().bo_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _args(self, obs, ys, visited, acqs):
        torch = self.torch
        k = self.count
        oi = [_dev(o, torch.int64, torch, self.device) for o in obs]
        yy = [_dev(v, torch.float64, torch, self.device) for v in ys]
        vis = [None if v is None else _dev(v, torch.uint8, torch, self.device) for v in (visited or [None] * k)]
        self._keep = [oi, yy, vis]
        P = C.c_void_p * k
        po = P(*[t.data_ptr() for t in oi])
        py = P(*[t.data_ptr() for t in yy])
        pv = P(*[0 if t is None else t.data_ptr() for t in vis])
        pn = (C.c_int32 * k)(*[int(t.shape[0]) for t in oi])
        acqs = acqs if isinstance(acqs, (list, tuple)) else [acqs or AcqParams(mode=0)] * k
        pa = (bo_acq_params * k)(*[a.c() for a in acqs])
        return po, py, pn, pv, pa

    def set_config(self, post_order=0, acq_chunk=8192, fit_order=1):
        c = bo_batch_config(post_order, acq_chunk, fit_order, 0)
        _check(lib().bo_batch_set_config(self.h, C.byref(c)), "bo_batch_set_config")

    def config(self):
        c = bo_batch_config()
        _check(lib().bo_batch_get_config(self.h, C.byref(c)), "bo_batch_get_config")
        return {"post_order": c.post_order, "acq_chunk": c.acq_chunk, "fit_order": c.fit_order}

    def set_timing(self, enable: bool = True):
        _check(lib().bo_batch_set_timing(self.h, 1 if enable else 0), "bo_batch_set_timing")

    def step(self, obs, ys, visited=None, acqs=None):
        """One step of every session; returns ([StepResult], graph_ms)."""
        po, py, pn, pv, pa = self._args(obs, ys, visited, acqs)
        out = (bo_acq_result * self.count)()
        ms = C.c_float(-1.0)
        _check(lib().bo_batch_step(self.h, po, py, pn, pv, pa, out, C.byref(ms)), "bo_batch_step")
        return [_result(r) for r in out], ms.value

    def tune(self, obs, ys, visited=None, acqs=None, reps=3):
        """Autotune tile shapes on these inputs; returns the chosen config."""
        po, py, pn, pv, pa = self._args(obs, ys, visited, acqs)
        out = (bo_acq_result * self.count)()
        c = bo_batch_config()
        _check(lib().bo_batch_tune(self.h, po, py, pn, pv, pa, int(reps), C.byref(c), out), "bo_batch_tune")
        return {"post_order": c.post_order, "acq_chunk": c.acq_chunk, "fit_order": c.fit_order}


def server_session_bytes(N: int, d: int, n_max: int, precision="fp32") -> int:
    p = bo_problem(int(N), int(d), int(n_max), PRECISIONS[precision] if isinstance(precision, str) else precision, 0)
    out = C.c_size_t()
    _check(lib().bo_server_session_bytes(C.byref(p), C.byref(out)), "bo_server_session_bytes")
    return out.value


class Server:
    """Serving runtime (bo_server_*): sessions live on the device, step
    requests are batched continuously by the library's scheduler thread."""

    def __init__(self, hbm_budget: int = 64 << 30, max_batch: int = 256, streams: int = 2,
                 post_order: int = 0, acq_chunk: int = 2048, fit_order: int = 1):
        _torch()
        cfg = bo_server_config(int(hbm_budget), int(max_batch), int(streams),
                               bo_batch_config(post_order, acq_chunk, fit_order, 0))
        h = C.c_void_p()
        _check(lib().bo_server_create(C.byref(h), C.byref(cfg)), "bo_server_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().bo_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def open(self, levels, obs_idx, y, N=None, cand=None, invalid=None, n_max=220, precision="fp32",
             gp: Optional[GpParams] = None) -> int:
        lv = np.ascontiguousarray(levels, dtype=np.int32)
        d = lv.shape[0]
        if N is None:
            N = int(np.prod(lv.astype(np.int64))) if cand is None else len(cand)
        cd = None if cand is None else np.ascontiguousarray(cand, dtype=np.int64)
        inv = None if invalid is None else np.ascontiguousarray(invalid, dtype=np.uint8)
        oi = np.ascontiguousarray(obs_idx, dtype=np.int64)
        yy = np.ascontiguousarray(y, dtype=np.float64)
        prob = bo_problem(int(N), d, int(n_max), PRECISIONS[precision] if isinstance(precision, str) else precision,
                          0)
        g = (gp or GpParams()).c()
        sid = C.c_int32()
        _check(lib().bo_server_open(self.h, C.byref(prob), C.byref(g), lv.ctypes.data,
                                    None if cd is None else cd.ctypes.data, None if inv is None else inv.ctypes.data,
                                    oi.ctypes.data, yy.ctypes.data, int(oi.shape[0]), C.byref(sid)),
               "bo_server_open")
        return sid.value

    def close_session(self, sid: int):
        _check(lib().bo_server_close(self.h, int(sid)), "bo_server_close")

    def submit(self, sid: int, idx: int, y: float, valid: bool = True, acq=None) -> int:
        """acq: AcqParams, or its C form (AcqParams.c()) to convert once for
        many requests."""
        a = acq if isinstance(acq, bo_acq_params) else (acq or AcqParams(mode=0)).c()
        t = C.c_uint64()
        _check(lib().bo_server_submit(self.h, int(sid), int(idx), float(y), 1 if valid else 0, C.byref(a),
                                      C.byref(t)), "bo_server_submit")
        return t.value

    def poll(self, ticket: int) -> bool:
        d = C.c_int32()
        _check(lib().bo_server_poll(self.h, C.c_uint64(ticket), C.byref(d)), "bo_server_poll")
        return bool(d.value)

    def wait(self, ticket: int):
        """Returns (StepResult, latency_ms)."""
        r = bo_acq_result()
        ms = C.c_double()
        _check(lib().bo_server_wait(self.h, C.c_uint64(ticket), C.byref(r), C.byref(ms)), "bo_server_wait")
        return _result(r), ms.value

    def wait_any(self, max_count: int = 256, timeout_us: int = 1000, raw: bool = False) -> list:
        """Finished requests not yet returned, in completion order (waits up
        to timeout_us for the first): [(ticket, StepResult, latency_ms)].
        raw: the results as bo_acq_result structures that stay valid until
        the next wait_any call (no conversion)."""
        if getattr(self, "_cq", None) is None or self._cq[0] < max_count:
            self._cq = (max_count, (C.c_uint64 * max_count)(), (bo_acq_result * max_count)(),
                        (C.c_double * max_count)())
        _, t, r, ms = self._cq
        k = C.c_int32()
        _check(lib().bo_server_wait_any(self.h, int(max_count), int(timeout_us), t, r, ms, C.byref(k)),
               "bo_server_wait_any")
        conv = (lambda x: x) if raw else _result
        return [(t[i], conv(r[i]), ms[i]) for i in range(k.value)]

    def stats(self) -> dict:
        i = bo_server_info()
        _check(lib().bo_server_stats(self.h, C.byref(i)), "bo_server_stats")
        return {k: getattr(i, k) for k, _ in bo_server_info._fields_}
