"""GPU parity on paths and edge cases beyond the configurations' own steps:

- the kernel's per-candidate EI, PI and LCB (bo_acquire_values) against the
  oracle's, element by element (Section III-C);
- both modes above 256 observations (the register-resident posterior in
  column passes) at n = 300 and 1000;
- the sigma = 0 limits of the acquisitions (candidates that duplicate observed
  points, zero noise) and the far lower tail of EI and PI;
- bo_observe: one evaluation per call, failures marked and never fitted
  (Section III-D.2), valid ones appended (Section III-B), against bo_gp_fit on
  the same history with an explicit mask, and against the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2111_14991_amd import workloads as W
from tests import parity as PR
from tests.test_gpu_parity import _parity

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def bo():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2111_14991_amd as bo
    bo.lib()
    return bo


def _values_vs_oracle(bo, S, X, invalid, vis, obs, y, ga, oa, ogp, tol, ymax):
    """bo_acquire_values against the oracle step on the same inputs: masks,
    every EI / PI / LCB value, the chosen indices; returns (result, arrays, ref)."""
    r, vals = S.acquire_values(vis, ga)
    A_g = np.stack([v.cpu().numpy() for v in vals], axis=1)
    ref = oracle.step(X, invalid, vis, obs, y, ogp, oa, want_posterior=True)
    mask = (invalid.astype(bool) | vis.astype(bool))
    keep = ~mask
    assert r.status == ref.status == 0
    for q in range(3):
        np.testing.assert_array_equal(np.isnan(A_g[:, q]), mask)
    A_r = PR.acq_arrays(ref.mu, ref.var, ref.f_best, ref.lam, mask)
    scales = (np.sqrt(ogp.amp), 1.0, ymax)
    for q in range(3):
        err = PR.normwise_err(A_g[keep, q], A_r[keep, q], scales[q])
        assert err <= tol, (q, err)
        assert PR.index_ok(int(r.idx[q]), int(ref.idx[q]), A_r, q, mask, tol, scales[q]), (q, r.idx, ref.idx)
        assert r.score[q] == A_g[r.idx[q], q]
    return r, A_g, ref


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_acquisition_values(bo, precision, cfg):
    s = W.config_c1(2) if cfg == "c1" else W.config_c2(1)
    S = bo.Session(s.N, s.d, s.n, precision)
    S.set_grid(s.levels, s.cand, s.invalid)
    S.fit(s.obs_idx, s.y)
    X = oracle.normalize_grid(s.levels, s.cand, s.N)
    mu_s = float(np.mean(s.y[:s.n_init]))
    _values_vs_oracle(bo, S, X, s.invalid, s.visited(), s.obs_idx, s.y, bo.AcqParams(mode=1, mu_s=mu_s),
                      oracle.Acq(mode=1, mu_s=mu_s), oracle.GP(), TOL, np.abs(s.y).max())
    S.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [300, 1000])
def test_above_256_observations(bo, n, precision):
    # 8,640 candidates of a 5-parameter grid, 20% restricted
    s = W.make_session(70 + n, (6, 6, 6, 5, 8), n, invalid_frac=0.2)
    rep = _parity(bo, s, precision)
    print(f"{precision} n={n}: " + ", ".join(f"{k} {rep[k]:.2e}" for k in ("mu", "var", "ei", "pi", "lcb")))


def _dup_space(seed, n_obs=12, n_other=150, d=3):
    """Candidates given as coordinates: n_obs observed points (visited), an
    unvisited exact duplicate of each, and n_other further random points."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = rng.uniform(0, 1, size=(n_obs, d))
    Q = rng.uniform(0, 1, size=(n_other, d))
    X = np.concatenate([P, P, Q])
    N = X.shape[0]
    inv = np.zeros(N, np.uint8)
    vis = np.zeros(N, np.uint8)
    vis[:n_obs] = 1
    obs = np.arange(n_obs)
    y = 1.0 + rng.uniform(0, 1, size=n_obs)
    return X, inv, vis, obs, y


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sigma_zero_limits(bo, precision):
    """Zero noise: at a candidate that duplicates an observed point the latent
    variance is zero, clamped, and EI, PI and LCB take their sigma -> 0 limits
    (EI = max(tau - mu, 0), PI in {0, 1/2, 1}, LCB = mu) on both sides."""
    X, inv, vis, obs, y = _dup_space(3)
    n = obs.shape[0]
    gp = bo.GpParams(noise=0.0)
    ogp = oracle.GP(noise=0.0)
    S = bo.Session(X.shape[0], X.shape[1], n, precision, gp=gp)
    S.set_candidates(X, inv)
    S.fit(obs, y)
    ga, oa = bo.AcqParams(mode=0, lambda_const=0.01), oracle.Acq(mode=0, lambda_const=0.01)
    r, A_g, ref = _values_vs_oracle(bo, S, X, inv, vis, obs, y, ga, oa, ogp, TOL, np.abs(y).max())
    mu, var, _ = S.posterior(vis)
    mu, var = mu.cpu().numpy(), var.cpu().numpy()
    dup = np.arange(n, 2 * n)
    assert np.all(var[dup] <= 1e-12), var[dup]
    zero = dup[var[dup] == 0.0]
    assert zero.size > 0, var[dup]  # the clamp fired: the sigma = 0 branch ran on the GPU
    tau = r.f_best - r.lam
    for c in zero:
        assert A_g[c, 0] == max(tau - mu[c], 0.0)
        assert A_g[c, 1] == (1.0 if tau > mu[c] else (0.5 if tau == mu[c] else 0.0))
        assert A_g[c, 2] == mu[c]
    # mean interpolates the observation at its duplicate
    np.testing.assert_allclose(mu[dup], y, rtol=0, atol=1e-6 * np.abs(y).max())
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lam", [3.0, 1.0e3])
def test_far_tail(bo, precision, lam):
    """A large exploration offset puts every candidate deep in the lower tail
    of EI and PI: z < -2 everywhere, and with lambda = 1000 every EI and PI
    underflows to zero, so the arg-max is the lowest predicted index on both
    sides (ties to the lowest index)."""
    s = W.config_c1(4)
    S = bo.Session(s.N, s.d, s.n, precision)
    S.set_grid(s.levels, s.cand, s.invalid)
    S.fit(s.obs_idx, s.y)
    X = oracle.normalize_grid(s.levels, s.cand, s.N)
    ga, oa = bo.AcqParams(mode=0, lambda_const=lam), oracle.Acq(mode=0, lambda_const=lam)
    r, A_g, ref = _values_vs_oracle(bo, S, X, s.invalid, s.visited(), s.obs_idx, s.y, ga, oa, oracle.GP(), TOL,
                                    np.abs(s.y).max())
    keep = ~(s.invalid.astype(bool) | s.visited().astype(bool))
    if lam > 100:
        assert np.all(A_g[keep, 0] == 0.0) and np.all(A_g[keep, 1] == 0.0)
        first = int(np.flatnonzero(keep)[0])
        assert r.idx[0] == ref.idx[0] == first and r.idx[1] == ref.idx[1] == first
    else:
        assert np.all(A_g[keep, 1] < 0.03)
    S.close()


def _history(seed, levels=(7, 6, 6, 5), n_valid=24, n_fail=5):
    """A session's evaluations in order: (idx, y, valid) with failures mixed in."""
    s = W.make_session(seed, levels, n_valid + n_fail, invalid_frac=0.15)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    fail = set(rng.choice(np.arange(2, s.n), size=n_fail, replace=False).tolist())
    ev = [(int(s.obs_idx[i]), float(s.y[i]), i not in fail) for i in range(s.n)]
    return s, ev


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_observe_matches_fit(bo, precision):
    """bo_observe one evaluation at a time (bordered appends, failures only
    marked) and the session's own record as the mask, against a fresh
    bo_gp_fit on the valid history with an explicit mask after every step,
    and the last step against the oracle."""
    s, ev = _history(11)
    S = bo.Session(s.N, s.d, s.n, precision)
    S.set_grid(s.levels, s.cand, s.invalid)
    R = bo.Session(s.N, s.d, s.n, precision)
    R.set_grid(s.levels, s.cand, s.invalid)
    vis = np.zeros(s.N, np.uint8)
    obs, ys = [], []
    mu_s = float(np.mean([y for _, y, v in ev[:6] if v]))
    acq = bo.AcqParams(mode=1, mu_s=mu_s)
    X = oracle.normalize_grid(s.levels, s.cand, s.N)
    ymax = float(np.abs(s.y).max())
    for k, (i, y, valid) in enumerate(ev):
        S.observe(i, y, valid)
        vis[i] = 1
        if valid:
            obs.append(i)
            ys.append(y)
        if len(obs) < 2:
            continue
        a = S.acquire(None, acq)
        R.fit(np.array(obs), np.array(ys))
        b = R.acquire(vis, acq)
        assert a.n_obs == b.n_obs == len(obs)
        assert a.n_unmasked == b.n_unmasked
        assert a.jitter == b.jitter and a.f_best == b.f_best
        assert abs(a.lam - b.lam) <= 1e-9 * abs(b.lam)
        assert abs(a.var_mean - b.var_mean) <= 1e-9 * b.var_mean
        for q in range(3):
            sc = 1.0 if q < 2 else ymax
            assert abs(a.score[q] - b.score[q]) <= 1e-8 * max(abs(b.score[q]), sc), (k, q)
            if a.idx[q] != b.idx[q]:  # a tie within rounding of the two factorizations
                assert abs(a.score[q] - b.score[q]) <= 1e-8 * max(abs(b.score[q]), sc)
    ref = oracle.step(X, s.invalid, vis, np.array(obs), np.array(ys), oracle.GP(), oracle.Acq(mode=1, mu_s=mu_s),
                      want_posterior=True)
    r = S.acquire(None, acq)
    mu, var, _ = S.posterior(None)
    mask = (s.invalid | vis).astype(bool)
    rep = PR.check_step(r, ref, mu.cpu().numpy(), var.cpu().numpy(), ref.mu, ref.var, mask, np.array(ys), 1.0, TOL)
    for key in ("mu", "var", "ei", "pi", "lcb", "lambda", "var_mean"):
        assert rep[key] <= TOL, (key, rep)
    S.close()
    R.close()


def test_observe_errors(bo):
    s = W.config_c1(0)
    S = bo.Session(s.N, s.d, 3, "fp64")
    with pytest.raises(bo.BOError) as e:
        S.observe(0, 1.0)
    assert e.value.status == bo.BO_E_STATE  # no candidate set
    S.set_grid(s.levels, s.cand, s.invalid)
    for args in [(-1, 1.0, True), (s.N, 1.0, True), (0, float("nan"), True)]:
        with pytest.raises(bo.BOError) as e:
            S.observe(*args)
        assert e.value.status == bo.BO_E_INVALID_ARG
    # a failed evaluation of a restricted point is only a mark; a valid one is a device-side error
    bad = int(np.flatnonzero(s.invalid)[0])
    S.observe(bad, 0.0, valid=False)
    for i in s.obs_idx[:3]:
        S.observe(int(i), 1.0 + 0.1 * int(i % 7))
    with pytest.raises(bo.BOError) as e:
        S.observe(int(s.obs_idx[3]), 1.0)  # n_max = 3 reached
    assert e.value.status == bo.BO_E_INVALID_ARG
    r = S.acquire(None, bo.AcqParams(mode=0))
    assert r.n_obs == 3 and r.n_unmasked == int((s.invalid == 0).sum()) - 3
    T = bo.Session(s.N, s.d, 3, "fp64")
    T.set_grid(s.levels, s.cand, s.invalid)
    T.observe(bad, 1.0)
    assert T.acquire(None, bo.AcqParams(mode=0), check=False).status == bo.BO_E_INVALID_ARG
    S.close()
    T.close()
