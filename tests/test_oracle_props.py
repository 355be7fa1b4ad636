"""Property tests of the oracle: random tiny spaces against dense
multiprecision conditioning, and independence from the OpenMP thread count."""
import os
import subprocess
import sys

import mpmath as mp
import numpy as np
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle
from paper_2111_14991_amd import workloads as W
from tests import bruteforce as BF

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@settings(max_examples=12, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(seed=st.integers(0, 2**31 - 1), d=st.integers(1, 4), n=st.integers(1, 8),
       nu2=st.sampled_from([3, 5]), l=st.floats(0.3, 2.5), noise=st.sampled_from([1e-6, 1e-3, 0.1]))
def test_random_tiny_spaces_match_dense_conditioning(orc, seed, d, n, nu2, l, noise):
    rng = np.random.Generator(np.random.PCG64(seed))
    levels = tuple(int(k) for k in rng.integers(2, 5, size=d))
    X = oracle.normalize_grid(levels)
    if X.shape[0] < n + 1:
        return
    obs = rng.choice(X.shape[0], size=n, replace=False)
    y = rng.uniform(0.5, 3.0, size=n)
    gp = oracle.GP(nu2=nu2, lengthscale=l, noise=noise)
    f = oracle.fit(X[obs], y, gp)
    P = X[: min(24, X.shape[0])]
    mu, var = oracle.predict(f, P)
    mref, vref = BF.dense_conditioning(P, X[obs], y, mp.mpf(nu2) / 2, l, 1.0, noise, dps=40)
    assert np.max(np.abs(mu - mref)) <= 1e-10 * np.abs(y).max()
    assert np.max(np.abs(var - np.maximum(vref, 0.0))) <= 1e-10


_SNIPPET = r"""
import sys, numpy as np
sys.path.insert(0, {root!r})
import oracle
from paper_2111_14991_amd import workloads as W
s = W.config_c1(4)
X = oracle.normalize_grid(s.levels)
r = oracle.step(X, s.invalid, s.visited(), s.obs_idx, s.y, acq=oracle.Acq(mode=1, mu_s=1.2), want_posterior=True)
print(oracle.threads(), r.idx.tolist(), r.var_mean.hex(), r.lam.hex(), np.nansum(r.var).hex(), np.nansum(r.mu).hex())
"""


def test_results_independent_of_thread_count(orc):
    outs = []
    for t in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        p = subprocess.run([sys.executable, "-c", _SNIPPET.format(root=ROOT)], env=env, capture_output=True,
                           text=True, check=True)
        outs.append(p.stdout.split(None, 1))
    assert [o[0] for o in outs] == ["1", "3", "8"]
    assert outs[0][1] == outs[1][1] == outs[2][1]
