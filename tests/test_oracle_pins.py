"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks one part of the oracle against an independent reference: the
general Bessel form of the Matern covariance, LAPACK's Cholesky, dense
multiprecision Gaussian conditioning, closed forms for one and two
observations, sampling and quadrature of the acquisition definitions, and
invariants (interpolation, monotone information, symmetries, tie rules).
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, special

import oracle
from paper_2111_14991_amd import workloads as W
from tests import bruteforce as BF


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# --- P1: Matern closed forms equal the general Bessel definition -------------

@pytest.mark.parametrize("nu2", [3, 5])
@pytest.mark.parametrize("l", [0.5, 1.0, 2.0])
def test_matern_matches_bessel_form(orc, nu2, l):
    r = np.concatenate([np.linspace(1e-6, 4.0, 200), [0.1 / 3, 1.0 / 3, math.sqrt(2.0)]])
    got = oracle.matern(nu2, r, l)
    with mp.workdps(30):
        ref = np.array([float(BF.matern_bessel_mp(mp.mpf(nu2) / 2, mp.mpf(float(x)), mp.mpf(l))) for x in r])
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("nu2", [3, 5])
def test_matern_limit_and_monotone(orc, nu2):
    assert oracle.matern(nu2, 0.0, 1.0) == 1.0
    r = np.linspace(0.0, 10.0, 2001)
    k = oracle.matern(nu2, r, 1.3)
    assert np.all(np.diff(k) < 0.0)
    assert np.all(k > 0.0) and k[0] == 1.0


# --- a1: linear normalization of the discrete space ------------------------------

def test_normalize_grid_matches_unravel(orc):
    levels = (8, 1, 6, 4, 3)
    X = oracle.normalize_grid(levels)
    assert X.shape == (8 * 6 * 4 * 3, 5)
    idx = np.stack(np.unravel_index(np.arange(X.shape[0]), levels), axis=1)
    den = np.array([max(k - 1, 1) for k in levels], dtype=np.float64)
    # unravel_index is C order (last axis fastest); every level lands on i/(k-1) exactly
    for j, k in enumerate(levels):
        for i in range(k):
            sel = idx[:, j] == i
            want = 0.0 if k == 1 else i / (k - 1)
            assert np.all(X[sel, j] == want)
    assert X.min() == 0.0 and X.max() == 1.0
    # subset enumeration equals the rows of the full grid
    cand = _rng(3).choice(X.shape[0], 50, replace=False)
    np.testing.assert_array_equal(oracle.normalize_grid(levels, cand), X[cand])
    assert np.all(np.abs(X - idx / den) <= 1e-16)


def test_normalize_grid_rejects_out_of_range(orc):
    with pytest.raises(oracle.OracleError):
        oracle.normalize_grid((3, 3), np.array([0, 9], dtype=np.int64))


# --- P2: Cholesky and the fit -----------------------------------------------------

def _rand_obs(seed, n, d):
    r = _rng(seed)
    Xo = r.integers(0, 5, size=(4 * n, d)) / 4.0
    Xo = np.unique(Xo, axis=0)[:n]
    r.shuffle(Xo)
    y = 1.0 + r.uniform(0.0, 2.0, size=Xo.shape[0])
    return Xo, y


@pytest.mark.parametrize("seed", range(3))
def test_fit_cholesky_vs_lapack_and_bessel(orc, seed):
    Xo, y = _rand_obs(seed, 40, 4)
    gp = oracle.GP(nu2=5, lengthscale=1.0, amp=1.7, noise=1e-6)
    f = oracle.fit(Xo, y, gp)
    D = np.sqrt(((Xo[:, None, :] - Xo[None, :, :]) ** 2).sum(-1))
    K = gp.amp * BF.matern_bessel(2.5, D, gp.lengthscale) + gp.noise * np.eye(Xo.shape[0])
    assert f.jitter == gp.noise
    n = Xo.shape[0]
    resid = np.linalg.norm(f.L @ f.L.T - K) / np.linalg.norm(K)
    assert resid <= 10 * n * 2.0**-52 + 1e-14
    np.testing.assert_allclose(f.L, np.linalg.cholesky(K), rtol=1e-10, atol=1e-12)
    assert np.all(np.triu(f.L, 1) == 0.0)
    # alpha solves K alpha = y - mean(y) (LU solve, a different algorithm)
    np.testing.assert_allclose(f.alpha, np.linalg.solve(K, y - y.mean()), rtol=1e-8, atol=1e-10)
    assert f.mean_y == pytest.approx(y.mean(), rel=1e-15)
    assert f.f_best == y.min()


# --- P3: posterior vs dense multiprecision conditioning ----------------------

@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("nu2", [3, 5])
def test_posterior_vs_dense_conditioning(orc, seed, nu2):
    s = W.tiny_session(seed, levels=(4, 3, 5), n_obs=6)
    X = oracle.normalize_grid(s.levels)
    gp = oracle.GP(nu2=nu2, lengthscale=0.8, amp=1.3, noise=1e-4)
    f = oracle.fit(X[s.obs_idx], s.y, gp)
    P = X[::3]
    mu, var = oracle.predict(f, P)
    mref, vref = BF.dense_conditioning(P, X[s.obs_idx], s.y, mp.mpf(nu2) / 2, gp.lengthscale, gp.amp, gp.noise)
    scale_mu = np.abs(s.y).max()
    assert np.max(np.abs(mu - mref)) <= 1e-11 * scale_mu
    assert np.max(np.abs(var - np.maximum(vref, 0.0))) <= 1e-11 * gp.amp


# --- P4: interpolation ----------------------------------------------------------------

def test_interpolates_observations_without_noise(orc):
    s = W.tiny_session(11, levels=(5, 5, 4), n_obs=10)
    X = oracle.normalize_grid(s.levels)
    gp = oracle.GP(noise=1e-12, lengthscale=0.5)
    f = oracle.fit(X[s.obs_idx], s.y, gp)
    mu, var = oracle.predict(f, X[s.obs_idx])
    assert np.max(np.abs(mu - s.y)) <= 1e-8 * np.abs(s.y).max()
    assert np.max(var) <= 1e-8


# --- P5 / P6: one and two observations --------------------------------------------

def test_single_observation_closed_form(orc):
    Xo = np.array([[0.25, 0.5, 1.0]])
    y = np.array([1.7])
    gp = oracle.GP(noise=1e-3)
    f = oracle.fit(Xo, y, gp)
    assert f.alpha[0] == 0.0
    P = _rng(0).uniform(size=(50, 3))
    mu, var = oracle.predict(f, P)
    assert np.all(mu == 1.7)
    r = np.linalg.norm(P - Xo, axis=1)
    k = BF.matern_bessel(2.5, r, 1.0)
    np.testing.assert_allclose(var, 1.0 - k * k / (1.0 + 1e-3), rtol=0, atol=1e-14)


def test_two_observations_closed_form(orc):
    Xo = np.array([[0.0, 0.0], [0.5, 1.0]])
    y = np.array([1.0, 2.0])
    amp, noise, l = 2.0, 1e-3, 0.7
    f = oracle.fit(Xo, y, oracle.GP(nu2=3, lengthscale=l, amp=amp, noise=noise))
    c = amp * BF.matern_bessel(1.5, np.linalg.norm(Xo[0] - Xo[1]), l)
    a = amp + noise
    det = a * a - c * c
    inv = np.array([[a, -c], [-c, a]]) / det
    P = _rng(1).uniform(size=(40, 2))
    mu, var = oracle.predict(f, P)
    K = amp * BF.matern_bessel(1.5, np.linalg.norm(P[:, None, :] - Xo[None], axis=2), l)
    r = y - 1.5
    np.testing.assert_allclose(mu, 1.5 + K @ (inv @ r), rtol=1e-13)
    np.testing.assert_allclose(var, amp - np.einsum("ij,jk,ik->i", K, inv, K), rtol=0, atol=1e-13)


# --- P7 / P8: monotone information and symmetries ---------------------------------

def test_variance_never_grows_with_more_data(orc):
    s = W.tiny_session(5, levels=(6, 5, 4), n_obs=12)
    X = oracle.normalize_grid(s.levels)
    prev = None
    for n in range(1, 13):
        f = oracle.fit(X[s.obs_idx[:n]], s.y[:n])
        _, var = oracle.predict(f, X)
        if prev is not None:
            assert np.all(var <= prev + 1e-12)
        prev = var


def test_permutation_and_translation_invariance(orc):
    s = W.tiny_session(8, levels=(6, 5, 4), n_obs=9)
    X = oracle.normalize_grid(s.levels)
    f = oracle.fit(X[s.obs_idx], s.y)
    mu, var = oracle.predict(f, X)
    perm = _rng(2).permutation(s.n)
    f2 = oracle.fit(X[s.obs_idx[perm]], s.y[perm])
    mu2, var2 = oracle.predict(f2, X)
    shift = np.array([0.3, -0.7, 0.125])
    f3 = oracle.fit(X[s.obs_idx] + shift, s.y)
    mu3, var3 = oracle.predict(f3, X + shift)
    for m, v in ((mu2, var2), (mu3, var3)):
        assert np.max(np.abs(m - mu)) <= 1e-12 * np.abs(s.y).max()
        assert np.max(np.abs(v - var)) <= 1e-12


# --- P9 / P10: acquisition functions -------------------------------------------

@pytest.mark.parametrize("mu,sigma,tau", [(1.0, 0.3, 0.9), (2.0, 0.05, 1.5), (0.5, 1.2, 0.6)])
def test_ei_poi_monte_carlo_and_quadrature(orc, mu, sigma, tau):
    lam = 0.05
    a = oracle.acquisitions(mu, sigma * sigma, tau + lam, lam)
    ei_mc, ei_se, pi_mc, pi_se = BF.ei_poi_monte_carlo(mu, sigma, tau, 10_000_000, 17)
    assert abs(a[0] - ei_mc) <= 5 * ei_se + 1e-12
    assert abs(a[1] - pi_mc) <= 5 * pi_se + 1e-12
    dens = lambda g: math.exp(-0.5 * ((g - mu) / sigma) ** 2) / (sigma * math.sqrt(2 * math.pi))
    ei_q, _ = integrate.quad(lambda g: (tau - g) * dens(g), mu - 40 * sigma, tau, epsabs=1e-14, epsrel=1e-12)
    assert a[0] == pytest.approx(ei_q, rel=1e-10, abs=1e-14)
    assert a[2] == pytest.approx(mu - lam * sigma, rel=1e-15)


def test_acquisition_invariants(orc):
    r = _rng(4)
    for _ in range(300):
        mu = r.uniform(0.5, 3.0)
        s1, s2 = np.sort(r.uniform(0.0, 1.0, 2))
        fb, lam = r.uniform(0.5, 3.0), r.uniform(0.0, 0.5)
        a1 = oracle.acquisitions(mu, s1 * s1, fb, lam)
        a2 = oracle.acquisitions(mu, s2 * s2, fb, lam)
        tau = fb - lam
        assert a1[0] >= max(tau - mu, 0.0) - 1e-15
        assert a2[0] >= a1[0] - 1e-15          # EI grows with sigma at fixed mu
        assert 0.0 <= a1[1] <= 1.0
        assert a1[2] <= mu
    # sigma = 0 limits
    assert list(oracle.acquisitions(1.0, 0.0, 1.5, 0.25)) == [0.25, 1.0, 1.0]
    assert list(oracle.acquisitions(2.0, 0.0, 1.5, 0.25)) == [0.0, 0.0, 2.0]
    assert list(oracle.acquisitions(1.25, 0.0, 1.5, 0.25)) == [0.0, 0.5, 1.25]


def test_phi_tail_vs_mpmath(orc):
    for z in np.linspace(-37.0, 8.0, 451):
        pi = oracle.acquisitions(-z, 1.0, 0.0, 0.0)[1]
        with mp.workdps(40):
            ref = float(mp.ncdf(mp.mpf(float(z))))
        assert abs(pi - ref) <= 4e-16 * (1.0 + z * z) * ref


# --- P11: exploration factor ---------------------------------------------------------

def test_contextual_lambda_first_step_and_constant(orc):
    s = W.config_c1(1)
    X = oracle.normalize_grid(s.levels)
    mu_s = float(np.mean(s.y))
    r = oracle.step(X, s.invalid, s.visited(), s.obs_idx, s.y, acq=oracle.Acq(mode=1, mu_s=mu_s, var_s_mean=0.0))
    assert r.lam == pytest.approx(r.f_best / mu_s, rel=1e-14)
    r2 = oracle.step(X, s.invalid, s.visited(), s.obs_idx, s.y, acq=oracle.Acq(mode=0, lambda_const=0.01))
    assert r2.lam == 0.01
    assert r2.var_mean == r.var_mean
    r3 = oracle.step(X, s.invalid, s.visited(), s.obs_idx, s.y,
                     acq=oracle.Acq(mode=1, mu_s=mu_s, var_s_mean=2.0 * r.var_mean))
    assert r3.lam == pytest.approx(0.5 * r.f_best / mu_s, rel=1e-14)


# --- P12: arg-optimum, masks and ties ------------------------------------------------

def test_argmax_masks_and_brute_force(orc):
    s = W.config_c1(2)
    X = oracle.normalize_grid(s.levels)
    acq = oracle.Acq(mode=0, lambda_const=0.01)
    r = oracle.step(X, s.invalid, s.visited(), s.obs_idx, s.y, acq=acq, want_posterior=True)
    mask = (s.invalid | s.visited()).astype(bool)
    assert np.all(np.isnan(r.mu[mask])) and not np.any(np.isnan(r.mu[~mask]))
    assert r.n_unmasked == int((~mask).sum())
    A = np.array([oracle.acquisitions(m, v, r.f_best, r.lam) if ok else [np.nan] * 3
                  for m, v, ok in zip(r.mu, r.var, ~mask)])
    assert r.idx[0] == np.argmax(np.where(mask, -np.inf, A[:, 0]))
    assert r.idx[1] == np.argmax(np.where(mask, -np.inf, A[:, 1]))
    assert r.idx[2] == np.argmin(np.where(mask, np.inf, A[:, 2]))
    assert not np.any(mask[r.idx])
    assert r.var_mean == pytest.approx(np.mean(r.var[~mask]), rel=1e-13)


def test_ties_pick_lowest_index(orc):
    # identical candidate rows give identical scores: the lowest index wins
    Xo = np.array([[0.0, 0.0], [1.0, 1.0]])
    X = np.array([[0.0, 0.0], [0.5, 0.5], [0.2, 0.7], [0.5, 0.5], [1.0, 1.0], [0.2, 0.7]])
    inv = np.zeros(6, np.uint8)
    vis = np.array([1, 0, 0, 0, 1, 0], np.uint8)
    r = oracle.step(X, inv, vis, np.array([0, 4]), np.array([1.0, 1.0]), acq=oracle.Acq(mode=0), want_posterior=True)
    assert r.mu[1] == r.mu[3] and r.var[1] == r.var[3]
    for q in range(3):
        assert r.idx[q] in (1, 2)
    # with the point (0.5, 0.5) masked, its twin at index 3 is chosen instead
    vis2 = vis.copy()
    vis2[1] = 1
    r2 = oracle.step(X, inv, vis2, np.array([0, 4]), np.array([1.0, 1.0]), acq=oracle.Acq(mode=0))
    assert set(r2.idx.tolist()) <= {2, 3}
    assert r.idx[0] == (1 if r.score[0] == r2.score[0] and r2.idx[0] == 3 else r.idx[0])


def test_all_masked_reports_no_candidate(orc):
    X = oracle.normalize_grid((2, 2))
    r = oracle.step(X, np.array([0, 0, 1, 1], np.uint8), np.array([1, 1, 0, 0], np.uint8),
                    np.array([0, 1]), np.array([1.0, 2.0]), acq=oracle.Acq(mode=0), check=False)
    assert r.status == oracle.E_NO_CANDIDATE
    assert list(r.idx) == [-1, -1, -1]


# --- P13: jitter escalation and error codes ------------------------------------------

def test_jitter_escalation_on_duplicate_observations(orc):
    Xo = np.array([[0.1, 0.2], [0.6, 0.9], [0.1, 0.2]])
    y = np.array([1.0, 1.5, 1.1])
    f = oracle.fit(Xo, y, oracle.GP(noise=0.0, jitter_tries=7))
    assert f.jitter == 1e-10 * 10.0          # first escalation step passes
    K = BF.matern_bessel(2.5, np.linalg.norm(Xo[:, None] - Xo[None], axis=2), 1.0) + f.jitter * np.eye(3)
    np.testing.assert_allclose(f.L @ f.L.T, K, rtol=0, atol=1e-15)
    with pytest.raises(oracle.OracleError) as e:
        oracle.fit(Xo, y, oracle.GP(noise=0.0, jitter_tries=1))
    assert e.value.code == oracle.E_NOT_PD


def test_error_codes(orc):
    X = oracle.normalize_grid((3, 3))
    inv = np.zeros(9, np.uint8)
    inv[8] = 1
    vis = np.zeros(9, np.uint8)
    vis[[0, 4]] = 1
    ok_idx, ok_y = np.array([0, 4]), np.array([1.0, 2.0])
    assert oracle.step(X, inv, vis, ok_idx[:0], ok_y[:0], check=False).status == oracle.E_STATE
    assert oracle.step(X, inv, vis, ok_idx, np.array([1.0, np.nan]), check=False).status == oracle.E_INVALID_ARG
    assert oracle.step(X, inv, vis, np.array([0, 8]), ok_y, check=False).status == oracle.E_INVALID_ARG
    assert oracle.step(X, inv, vis, ok_idx, np.array([-1.0, 2.0]), acq=oracle.Acq(mode=1, mu_s=1.0),
                       check=False).status == oracle.E_INVALID_ARG
    assert oracle.step(X, inv, vis, ok_idx, ok_y, acq=oracle.Acq(mode=1, mu_s=0.0),
                       check=False).status == oracle.E_INVALID_ARG
    assert oracle.step(X, inv, vis, ok_idx, ok_y, gp=oracle.GP(nu2=4), check=False).status == oracle.E_INVALID_ARG
    assert oracle.step(X, inv, vis, ok_idx, ok_y, acq=oracle.Acq(mode=0)).status == oracle.OK
