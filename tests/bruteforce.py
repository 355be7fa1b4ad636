"""Independent references used to pin the oracle (tests only).

Nothing here shares arithmetic with the oracle or the GPU library: the Matern
covariance comes from its general modified-Bessel definition (Section III-B),
the posterior from dense joint-Gaussian conditioning in multiprecision, and the
acquisitions from sampling or numerical integration of their definitions.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np
from scipy import special


def matern_bessel(nu: float, r, l: float) -> np.ndarray:
    """2^(1-nu)/Gamma(nu) (sqrt(2 nu) r / l)^nu K_nu(sqrt(2 nu) r / l), with the
    r -> 0 limit 1, evaluated with scipy's Bessel function."""
    r = np.asarray(r, dtype=np.float64)
    t = np.sqrt(2.0 * nu) * r / l
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        v = (2.0 ** (1.0 - nu) / special.gamma(nu)) * t ** nu * special.kv(nu, t)
    return np.where(t == 0.0, 1.0, v)


def matern_bessel_mp(nu, r, l):
    """Same definition in mpmath at the current working precision."""
    r = mp.mpf(r)
    if r == 0:
        return mp.mpf(1)
    t = mp.sqrt(2 * mp.mpf(nu)) * r / mp.mpf(l)
    return mp.power(2, 1 - mp.mpf(nu)) / mp.gamma(nu) * mp.power(t, nu) * mp.besselk(nu, t)


def dense_conditioning(X, Xo, y, nu, l, amp, noise, dps=50):
    """Posterior mean and latent variance at the rows of X by conditioning the
    joint Gaussian [f(Xo) + noise; f(X)] on y, with the constant prior mean
    m = mean(y), in mpmath at `dps` digits:
        mu  = m + S_xn S_nn^-1 (y - m)
        var = amp - S_xn S_nn^-1 S_nx
    """
    with mp.workdps(dps):
        n = Xo.shape[0]
        def dist(a, b):
            return mp.sqrt(mp.fsum((mp.mpf(float(p)) - mp.mpf(float(q))) ** 2 for p, q in zip(a, b)))
        Snn = mp.matrix(n, n)
        for i in range(n):
            for j in range(n):
                Snn[i, j] = amp * matern_bessel_mp(nu, dist(Xo[i], Xo[j]), l) + (noise if i == j else 0)
        m = mp.fsum(mp.mpf(float(v)) for v in y) / n
        r = mp.matrix([mp.mpf(float(v)) - m for v in y])
        w = mp.lu_solve(Snn, r)
        mus, vars_ = [], []
        for x in X:
            k = mp.matrix([amp * matern_bessel_mp(nu, dist(x, Xo[i]), l) for i in range(n)])
            mus.append(float(m + mp.fsum(k[i] * w[i] for i in range(n))))
            u = mp.lu_solve(Snn, k)
            vars_.append(float(amp - mp.fsum(k[i] * u[i] for i in range(n))))
        return np.array(mus), np.array(vars_)


def ei_poi_monte_carlo(mu, sigma, tau, samples, seed):
    """Sample means of max(tau - g, 0) and of [g < tau] for g ~ N(mu, sigma^2),
    with their standard errors."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = mu + sigma * rng.standard_normal(samples)
    imp = np.maximum(tau - g, 0.0)
    hit = (g < tau).astype(np.float64)
    return (imp.mean(), imp.std(ddof=1) / np.sqrt(samples),
            hit.mean(), hit.std(ddof=1) / np.sqrt(samples))
