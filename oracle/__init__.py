"""FP64 CPU oracle for the BO surrogate step (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (plain C,
OpenMP over candidates) built from ``oracle.c`` and shares nothing with the
GPU library.  See ``oracle.h`` for the definitions each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVALID_ARG, E_NOT_PD, E_NO_CANDIDATE, E_STATE, E_NUMERIC = 0, 1, 2, 3, 6, 8


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (IEEE double, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class _Gp(C.Structure):
    _fields_ = [("nu2", C.c_int32), ("lengthscale", C.c_double), ("amp", C.c_double),
                ("noise", C.c_double), ("jitter_tries", C.c_int32)]


class _Acq(C.Structure):
    _fields_ = [("mode", C.c_int32), ("lambda_const", C.c_double), ("mu_s", C.c_double),
                ("var_s_mean", C.c_double)]


class _Res(C.Structure):
    _fields_ = [("idx", C.c_int64 * 3), ("score", C.c_double * 3), ("lambda_", C.c_double),
                ("var_mean", C.c_double), ("jitter", C.c_double), ("f_best", C.c_double),
                ("mean_y", C.c_double), ("n_unmasked", C.c_int64), ("status", C.c_int32),
                ("nan_seen", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_normalize_grid.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.c_int64, C.c_void_p, dp]
        L.orc_matern.argtypes = [C.c_int32, C.c_double, C.c_double]
        L.orc_matern.restype = C.c_double
        L.orc_fit.argtypes = [C.c_int32, C.c_int32, dp, dp, C.POINTER(_Gp), dp, dp, dp, dp, dp]
        L.orc_predict.argtypes = [C.c_int64, C.c_int32, dp, C.c_int32, dp, dp, dp, C.c_double,
                                  C.POINTER(_Gp), dp, dp]
        L.orc_acquisitions.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc_acquisitions_all.argtypes = [C.c_int64, dp, dp, C.c_void_p, C.c_double, C.c_double, dp]
        L.orc_step.argtypes = [C.c_int64, C.c_int32, dp, C.c_void_p, C.c_void_p, C.c_int32,
                               C.c_void_p, dp, C.POINTER(_Gp), C.POINTER(_Acq), C.c_void_p,
                               C.c_void_p, C.POINTER(_Res)]
        L.orc_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class GP:
    nu2: int = 5
    lengthscale: float = 1.0
    amp: float = 1.0
    noise: float = 1e-6
    jitter_tries: int = 7

    def c(self) -> _Gp:
        return _Gp(self.nu2, self.lengthscale, self.amp, self.noise, self.jitter_tries)


@dataclass
class Acq:
    mode: int = 1
    lambda_const: float = 0.01
    mu_s: float = 0.0
    var_s_mean: float = 0.0

    def c(self) -> _Acq:
        return _Acq(self.mode, self.lambda_const, self.mu_s, self.var_s_mean)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def threads() -> int:
    return int(lib().orc_threads())


def normalize_grid(levels: Sequence[int], cand: Optional[np.ndarray] = None, N: Optional[int] = None) -> np.ndarray:
    lv = np.ascontiguousarray(levels, dtype=np.int32)
    if cand is not None:
        cand = np.ascontiguousarray(cand, dtype=np.int64)
        N = cand.shape[0]
    elif N is None:
        N = int(np.prod(lv.astype(np.int64)))
    X = np.empty((N, lv.shape[0]), dtype=np.float64)
    rc = lib().orc_normalize_grid(lv.shape[0], lv.ctypes.data_as(C.POINTER(C.c_int32)), N,
                                  None if cand is None else cand.ctypes.data, _dp(X))
    if rc != OK:
        raise OracleError(rc, "normalize_grid")
    return X


def matern(nu2: int, r, l: float) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    f = lib().orc_matern
    return np.vectorize(lambda x: f(nu2, float(x), float(l)), otypes=[np.float64])(r)


@dataclass
class Fit:
    L: np.ndarray
    alpha: np.ndarray
    mean_y: float
    f_best: float
    jitter: float
    Xo: np.ndarray
    gp: GP


def fit(Xo: np.ndarray, y: np.ndarray, gp: GP = GP()) -> Fit:
    Xo = np.ascontiguousarray(Xo, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n, d = Xo.shape
    L = np.zeros((n, n))
    alpha = np.zeros(n)
    m, fb, jit = C.c_double(), C.c_double(), C.c_double()
    g = gp.c()
    rc = lib().orc_fit(n, d, _dp(Xo), _dp(y), C.byref(g), _dp(L), _dp(alpha), C.byref(m), C.byref(fb), C.byref(jit))
    if rc != OK:
        raise OracleError(rc, "fit")
    return Fit(L, alpha, m.value, fb.value, jit.value, Xo, gp)


def predict(f: Fit, P: np.ndarray):
    P = np.ascontiguousarray(P, dtype=np.float64)
    M, d = P.shape
    mu = np.empty(M)
    var = np.empty(M)
    g = f.gp.c()
    lib().orc_predict(M, d, _dp(P), f.Xo.shape[0], _dp(f.Xo), _dp(f.L), _dp(f.alpha), f.mean_y,
                      C.byref(g), _dp(mu), _dp(var))
    return mu, var


def acquisitions(mu: float, var: float, f_best: float, lam: float) -> np.ndarray:
    out = np.empty(3)
    lib().orc_acquisitions(float(mu), float(var), float(f_best), float(lam), _dp(out))
    return out


def acquisition_arrays(mu: np.ndarray, var: np.ndarray, mask: np.ndarray, f_best: float, lam: float) -> np.ndarray:
    """EI, PI, LCB (columns) of every candidate with mask == 0; NaN rows elsewhere."""
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    var = np.ascontiguousarray(var, dtype=np.float64)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    out = np.empty((mu.shape[0], 3))
    lib().orc_acquisitions_all(mu.shape[0], _dp(mu), _dp(var), m.ctypes.data, float(f_best), float(lam), _dp(out))
    return out


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
    nan_seen: bool
    mu: Optional[np.ndarray] = None
    var: Optional[np.ndarray] = None


def step(X: np.ndarray, invalid: np.ndarray, visited: np.ndarray, obs_idx: np.ndarray, y: np.ndarray,
         gp: GP = GP(), acq: Acq = Acq(), want_posterior: bool = False, check: bool = True) -> StepResult:
    X = np.ascontiguousarray(X, dtype=np.float64)
    N, d = X.shape
    inv = np.ascontiguousarray(invalid, dtype=np.uint8)
    vis = np.ascontiguousarray(visited, dtype=np.uint8)
    oi = np.ascontiguousarray(obs_idx, dtype=np.int64)
    yy = np.ascontiguousarray(y, dtype=np.float64)
    mu = np.empty(N) if want_posterior else None
    var = np.empty(N) if want_posterior else None
    r = _Res()
    g, a = gp.c(), acq.c()
    rc = lib().orc_step(N, d, _dp(X), inv.ctypes.data, vis.ctypes.data, oi.shape[0], oi.ctypes.data, _dp(yy),
                        C.byref(g), C.byref(a), None if mu is None else mu.ctypes.data,
                        None if var is None else var.ctypes.data, C.byref(r))
    res = StepResult(np.array(r.idx[:], dtype=np.int64), np.array(r.score[:]), r.lambda_, r.var_mean, r.jitter,
                     r.f_best, r.mean_y, r.n_unmasked, r.status, bool(r.nan_seen), mu, var)
    if check and rc not in (OK,):
        raise OracleError(rc, "step")
    return res


def initial_acq(X: np.ndarray, invalid: np.ndarray, obs_idx: np.ndarray, y: np.ndarray, n_init: int,
                gp: GP = GP()) -> Acq:
    """Contextual-variance constants of Section III-F for a session whose first
    `n_init` observations are the initial sample: mu_s is their mean and
    var_s_mean the mean posterior variance of the step taken right after it."""
    n_init = min(n_init, obs_idx.shape[0])
    vis = np.zeros(X.shape[0], dtype=np.uint8)
    vis[obs_idx[:n_init]] = 1
    r = step(X, invalid, vis, obs_idx[:n_init], y[:n_init], gp, Acq(mode=0))
    return Acq(mode=1, mu_s=float(np.mean(y[:n_init])), var_s_mean=r.var_mean)
