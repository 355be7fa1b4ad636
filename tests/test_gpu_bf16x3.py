"""BF16X3 precision mode against the FP64 oracle.

The cross-covariance and L^-1 enter the matrix cores as bfloat16 high and low
parts (16 significant bits each value) and three products are accumulated in
FP32, so each contraction term carries a relative error of about 2^-16 and the
posterior variance an absolute error of a few 1e-5.  The tolerance TOL_B =
2e-4 (normwise, same scale floors as the FP64/FP32 modes) is derived from that
arithmetic; the measured errors are printed as the mode's error report.  The
full-size step is also run in the FP64 mode against the same oracle step, at
the 1e-6 bar of the FP64 and FP32 modes.
"""
import numpy as np
import pytest

import oracle
from paper_2111_14991_amd import workloads as W
from tests import parity as PR

pytestmark = pytest.mark.gpu

TOL_B = 2e-4
TOL = 1e-6


@pytest.fixture(scope="module")
def bo():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2111_14991_amd as bo
    bo.lib()
    return bo


def _report(name, err):
    q = np.quantile(err, [0.5, 0.99, 1.0]) if err.size else np.zeros(3)
    print(f"{name}: median {q[0]:.2e} p99 {q[1]:.2e} max {q[2]:.2e}")
    return q[2]


def bf16x3_parity(bo, s, gp=None, acq_mode=1):
    """One BF16X3 step against the oracle: mean and variance of every
    candidate, the mean variance, lambda and the chosen indices within TOL_B.
    Contextual mode takes the step as the first after the initial sample."""
    n = s.n
    gpp = gp or bo.GpParams()
    ogp = oracle.GP(gpp.nu2, gpp.lengthscale, gpp.amp, gpp.noise, gpp.jitter_tries)
    S = bo.Session(s.N, s.d, s.n, "bf16x3", gp=gpp)
    S.set_grid(s.levels, None, s.invalid)
    S.fit(s.obs_idx, s.y)
    mu_s = float(np.mean(s.y[:s.n_init]))
    r = S.acquire(s.visited(), bo.AcqParams(mode=acq_mode, mu_s=mu_s))
    mu, var, vm = S.posterior(s.visited())
    mu, var = mu.cpu().numpy(), var.cpu().numpy()
    X = oracle.normalize_grid(s.levels)
    ref = oracle.step(X, s.invalid, s.visited(), s.obs_idx, s.y, ogp, oracle.Acq(mode=acq_mode, mu_s=mu_s),
                      want_posterior=True)
    mask = (s.invalid | s.visited()).astype(bool)
    keep = ~mask
    np.testing.assert_array_equal(np.isnan(mu), mask)
    ymax = np.abs(s.y).max()
    e_mu = _report(f"n={n} mu", np.abs(mu[keep] - ref.mu[keep]) / np.maximum(np.abs(ref.mu[keep]), ymax))
    e_var = _report(f"n={n} var", np.abs(var[keep] - ref.var[keep]))
    assert e_mu <= TOL_B and e_var <= TOL_B
    # the mean variance carries the variance's absolute error (floor amp = 1)
    assert abs(r.var_mean - ref.var_mean) <= TOL_B * max(ref.var_mean, 1.0)
    assert abs(r.lam - ref.lam) <= TOL_B * ref.lam
    A_r = PR.acq_arrays(ref.mu, ref.var, ref.f_best, ref.lam, mask)
    A_g = PR.acq_arrays(mu, var, r.f_best, r.lam, mask)
    scales = (1.0, 1.0, ymax)
    for q, name in enumerate(("ei", "pi", "lcb")):
        e = np.abs(A_g[keep, q] - A_r[keep, q]) / np.maximum(np.abs(A_r[keep, q]), scales[q])
        _report(f"n={n} {name}", e)
        assert PR.index_ok(int(r.idx[q]), int(ref.idx[q]), A_r, q, mask, TOL_B, scales[q]), (q, r.idx, ref.idx)
    S.close()


@pytest.mark.parametrize("n", [1, 37, 100, 300, 1000])
def test_bf16x3_mid_size_parity(bo, n):
    bf16x3_parity(bo, W.make_session(20 + n, (6, 6, 6, 6, 6), n, invalid_frac=0.3))


@pytest.mark.parametrize("d,n", [(12, 150), (14, 200), (16, 70)])
def test_bf16x3_wide_parity(bo, d, n):
    # d + 4 > 16 takes the distance products over two k-steps (d = 14, 16);
    # d = 12 is the widest space with one
    bf16x3_parity(bo, W.make_session(90 + d, (2,) * d, n, invalid_frac=0.2))


def test_bf16x3_full_size(bo):
    """The 1M-candidate step (4^10 grid, 30% invalid, n = 1000) in the launch
    configuration the benchmark times, against one whole FP64 oracle step:
    mean, variance and the kernel's own EI, PI and LCB of every one of the
    ~738k predicted candidates, the mean variance, lambda in its contextual
    form after the initial sample (so it depends on both mean variances), and
    each chosen index against the oracle's full acquisition arrays."""
    s = W.config_c3(0)
    S = bo.Session(s.N, s.d, s.n, "bf16x3")
    S.set_grid(s.levels, None, s.invalid)
    X = oracle.normalize_grid(s.levels)
    n0 = s.n_init
    vis0 = np.zeros(s.N, np.uint8)
    vis0[s.obs_idx[:n0]] = 1
    S.fit(s.obs_idx[:n0], s.y[:n0])
    var_s_g = S.acquire(vis0, bo.AcqParams(mode=0)).var_mean
    var_s_o = oracle.step(X, s.invalid, vis0, s.obs_idx[:n0], s.y[:n0], oracle.GP(), oracle.Acq(mode=0)).var_mean
    assert abs(var_s_g - var_s_o) <= TOL_B * max(var_s_o, 1.0)
    mu_s = float(np.mean(s.y[:n0]))
    vis = s.visited()
    S.fit(s.obs_idx, s.y)
    r, vals = S.acquire_values(vis, bo.AcqParams(mode=1, mu_s=mu_s, var_s_mean=var_s_g))
    assert r.status == 0
    mu, var, vm = S.posterior(vis)
    mu, var = mu.cpu().numpy(), var.cpu().numpy()
    A_g = np.stack([v.cpu().numpy() for v in vals], axis=1)
    ref = oracle.step(X, s.invalid, vis, s.obs_idx, s.y, oracle.GP(),
                      oracle.Acq(mode=1, mu_s=mu_s, var_s_mean=var_s_o), want_posterior=True)
    mask = (s.invalid | vis).astype(bool)
    keep = ~mask
    assert r.n_unmasked == ref.n_unmasked == int(keep.sum())
    for arr in (mu, var, A_g[:, 0], A_g[:, 1], A_g[:, 2]):
        np.testing.assert_array_equal(np.isnan(arr), mask)
    ymax = np.abs(s.y).max()
    e_mu = _report("c3 mu", np.abs(mu[keep] - ref.mu[keep]) / np.maximum(np.abs(ref.mu[keep]), ymax))
    e_var = _report("c3 var", np.abs(var[keep] - ref.var[keep]))
    assert e_mu <= TOL_B and e_var <= TOL_B
    assert abs(r.var_mean - ref.var_mean) <= TOL_B * max(ref.var_mean, 1.0)
    assert abs(vm - r.var_mean) <= 1e-12 * r.var_mean
    # contextual lambda = (var_mean / (mu_s / f_best)) / var_s_mean: both mean variances enter
    assert abs(r.lam - ref.lam) <= TOL_B * ref.lam
    assert abs(r.lam - r.f_best / mu_s) > 1e-3 * r.lam
    A_r = PR.acq_arrays(ref.mu, ref.var, ref.f_best, ref.lam, mask)
    scales = (1.0, 1.0, ymax)
    for q, name in enumerate(("ei", "pi", "lcb")):
        e = np.abs(A_g[keep, q] - A_r[keep, q]) / np.maximum(np.abs(A_r[keep, q]), scales[q])
        assert _report(f"c3 {name}", e) <= TOL_B, name
        assert PR.index_ok(int(r.idx[q]), int(ref.idx[q]), A_r, q, mask, TOL_B, scales[q]), (q, r.idx, ref.idx)
        # the reported score is the kernel's own value at the chosen index
        assert r.score[q] == A_g[r.idx[q], q]
    print(f"c3 chosen {list(r.idx)} oracle {list(ref.idx)}; agreement "
          f"{[int(a == b) for a, b in zip(r.idx, ref.idx)]}")
    S.close()
    # the same step in the FP64 mode (register-resident posterior in column
    # passes) against the same oracle step, at the 1e-6 bar
    T = bo.Session(s.N, s.d, s.n, "fp64")
    T.set_grid(s.levels, None, s.invalid)
    T.fit(s.obs_idx[:n0], s.y[:n0])
    var_s_64 = T.acquire(vis0, bo.AcqParams(mode=0)).var_mean
    assert abs(var_s_64 - var_s_o) <= TOL * var_s_o
    T.fit(s.obs_idx, s.y)
    r64, vals64 = T.acquire_values(vis, bo.AcqParams(mode=1, mu_s=mu_s, var_s_mean=var_s_64))
    assert r64.status == 0 and r64.n_unmasked == ref.n_unmasked
    mu64, var64, _ = T.posterior(vis)
    mu64, var64 = mu64.cpu().numpy(), var64.cpu().numpy()
    A_64 = np.stack([v.cpu().numpy() for v in vals64], axis=1)
    e_mu = _report("c3 fp64 mu", np.abs(mu64[keep] - ref.mu[keep]) / np.maximum(np.abs(ref.mu[keep]), ymax))
    e_var = _report("c3 fp64 var", np.abs(var64[keep] - ref.var[keep]))
    assert e_mu <= TOL and e_var <= TOL
    assert abs(r64.var_mean - ref.var_mean) <= TOL * ref.var_mean
    assert abs(r64.lam - ref.lam) <= TOL * ref.lam
    for q, name in enumerate(("ei", "pi", "lcb")):
        e = np.abs(A_64[keep, q] - A_r[keep, q]) / np.maximum(np.abs(A_r[keep, q]), scales[q])
        assert _report(f"c3 fp64 {name}", e) <= TOL, name
        assert PR.index_ok(int(r64.idx[q]), int(ref.idx[q]), A_r, q, mask, TOL, scales[q]), (q, r64.idx, ref.idx)
    print(f"c3 fp64 chosen {list(r64.idx)} oracle {list(ref.idx)}")
    T.close()
