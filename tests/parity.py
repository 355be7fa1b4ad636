"""Comparison rules between the GPU library and the FP64 oracle.

Values: |q_gpu - q_ref| <= tol * max(|q_ref|, S_q), with the scale floors
S_mu = S_LCB = max|y|, S_var = amp, S_EI = sqrt(amp), S_PI = 1; the scalars
lambda and the mean variance use plain relative tolerance.
Indices: the GPU's choice g equals the oracle's o, or g is a candidate the
oracle also predicts whose reference acquisition is within the same tolerance
of the reference optimum (EI and PI maximized, LCB minimized).
"""
from __future__ import annotations

import numpy as np

import oracle


def normwise_err(got, ref, scale):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.maximum(np.abs(ref), scale)
    return float(np.max(np.abs(got - ref) / den)) if ref.size else 0.0


def acq_arrays(mu, var, f_best, lam, mask):
    """Reference acquisitions of every predicted candidate (oracle formulas)."""
    return oracle.acquisition_arrays(np.nan_to_num(mu), np.nan_to_num(var), mask, f_best, lam)


def index_ok(g, o, A_ref, q, mask, tol, scale):
    """R18: exact, or within tolerance of the reference optimum."""
    if g == o:
        return True
    if g < 0 or o < 0 or mask[g]:
        return False
    a = A_ref[:, q] if q < 2 else -A_ref[:, q]
    return bool(a[g] >= a[o] - tol * max(abs(a[o]), scale))


def check_step(gpu, ref, mu_g, var_g, mu_r, var_r, mask, y, amp, tol):
    """Element-by-element parity of one step; returns the error report."""
    assert gpu.status == ref.status == 0, (gpu.status, ref.status)
    assert gpu.n_unmasked == ref.n_unmasked
    ymax = float(np.max(np.abs(y)))
    # masks: exactly the excluded candidates are NaN on both sides
    np.testing.assert_array_equal(np.isnan(mu_g), mask)
    np.testing.assert_array_equal(np.isnan(var_g), mask)
    keep = ~mask
    rep = {
        "mu": normwise_err(mu_g[keep], mu_r[keep], ymax),
        "var": normwise_err(var_g[keep], var_r[keep], amp),
        "lambda": abs(gpu.lam - ref.lam) / abs(ref.lam) if ref.lam != 0 else abs(gpu.lam),
        "var_mean": abs(gpu.var_mean - ref.var_mean) / abs(ref.var_mean),
    }
    A_g = acq_arrays(mu_g, var_g, gpu.f_best, gpu.lam, mask)
    A_r = acq_arrays(mu_r, var_r, ref.f_best, ref.lam, mask)
    rep["ei"] = normwise_err(A_g[keep, 0], A_r[keep, 0], np.sqrt(amp))
    rep["pi"] = normwise_err(A_g[keep, 1], A_r[keep, 1], 1.0)
    rep["lcb"] = normwise_err(A_g[keep, 2], A_r[keep, 2], ymax)
    scales = (np.sqrt(amp), 1.0, ymax)
    for q in range(3):
        assert index_ok(int(gpu.idx[q]), int(ref.idx[q]), A_r, q, mask, tol, scales[q]), \
            (q, gpu.idx, ref.idx, gpu.score, ref.score)
        assert not mask[gpu.idx[q]]
    # reported scores are the acquisition at the reported index
    for q in range(3):
        rep[f"score{q}"] = abs(gpu.score[q] - A_r[gpu.idx[q], q]) / max(abs(A_r[gpu.idx[q], q]), scales[q])
    rep["f_best"] = abs(gpu.f_best - ref.f_best)
    rep["mean_y"] = abs(gpu.mean_y - ref.mean_y) / abs(ref.mean_y)
    rep["jitter_equal"] = gpu.jitter == ref.jitter
    return rep
