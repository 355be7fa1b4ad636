"""Rank-1 (bordered) append of one observation (bo_gp_append) against a full
refit on the same observations (bo_gp_fit) and against the FP64 oracle:
L^-1, alpha, the accepted jitter, and the whole step's results, across the
64-observation boundaries of the padded layout, with a forced jitter, a
duplicate observation (the new pivot fails, so the append refits) and an
observation of a pruned candidate."""
import numpy as np
import pytest

import oracle
from paper_2111_14991_amd import workloads as W
from tests import parity as PR

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


def _session(bo, s, precision, n_max=256, gp=None):
    S = bo.Session(s.N, s.d, n_max, precision, gp=gp)
    S.set_grid(s.levels, s.cand, s.invalid)
    return S


def _vis(s, n, obs=None):
    obs = s.obs_idx if obs is None else obs
    v = np.zeros(s.N, np.uint8)
    v[obs[:n]] = 1
    return v


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_append_matches_refit(bo, precision):
    s = W.make_session(21, (7, 6, 6, 5), 140, invalid_frac=0.2)
    A = _session(bo, s, precision)
    R = _session(bo, s, precision)
    acq = bo.AcqParams(mode=0, lambda_const=0.01)
    n0 = 58
    A.fit(s.obs_idx[:n0], s.y[:n0])
    # through the 64 and 128 boundaries of the padded layout
    for n in list(range(n0 + 1, 72)) + list(range(125, 131)):
        if n == 125:
            A.fit(s.obs_idx[:124], s.y[:124])
        A.append(s.obs_idx[:n], s.y[:n])
        R.fit(s.obs_idx[:n], s.y[:n])
        rca, ia, alpha_a, Li_a = A.fit_read(True, True)
        rcr, ir, alpha_r, Li_r = R.fit_read(True, True)
        assert rca == rcr == 0
        assert ia.jitter == ir.jitter and ia.f_best == ir.f_best and ia.n == ir.n == n
        assert ia.mean_y == ir.mean_y
        np.testing.assert_allclose(Li_a, Li_r, rtol=1e-9, atol=1e-9 * np.abs(Li_r).max())
        np.testing.assert_allclose(alpha_a, alpha_r, rtol=1e-8, atol=1e-9 * np.abs(alpha_r).max())
        ra = A.acquire(_vis(s, n), acq)
        rr = R.acquire(_vis(s, n), acq)
        assert ra.n_unmasked == rr.n_unmasked
        assert ra.var_mean == pytest.approx(rr.var_mean, rel=1e-9)
        for q in range(3):
            assert ra.score[q] == pytest.approx(rr.score[q], rel=1e-8, abs=1e-12)
    # the appended state against the oracle
    n = 130
    X = oracle.normalize_grid(s.levels, s.cand, s.N)
    v = _vis(s, n)
    ref = oracle.step(X, s.invalid, v, s.obs_idx[:n], s.y[:n], oracle.GP(), oracle.Acq(mode=0, lambda_const=0.01),
                      want_posterior=True)
    mu, var, vm = A.posterior(v)
    r = A.acquire(v, acq)
    mask = (s.invalid | v).astype(bool)
    rep = PR.check_step(r, ref, mu.cpu().numpy(), var.cpu().numpy(), ref.mu, ref.var, mask, s.y[:n], 1.0, TOL)
    for k in ("mu", "var", "ei", "pi", "lcb", "var_mean", "score0", "score1", "score2", "mean_y"):
        assert rep[k] <= TOL, (k, rep)
    assert rep["jitter_equal"]
    A.close()
    R.close()


def test_append_keeps_escalated_jitter(bo):
    # zero noise and a near-singular K_nn: the fit escalates the jitter; the
    # appended factor keeps it, as a refit on n + 1 points does
    s = W.make_session(5, (10, 10, 10), 40, invalid_frac=0.0)
    obs = s.obs_idx.copy()
    obs[10] = obs[0]  # duplicate point: K_nn singular without jitter
    gp = bo.GpParams(noise=0.0)
    A = _session(bo, s, "fp64", gp=gp)
    R = _session(bo, s, "fp64", gp=gp)
    A.fit(obs[:30], s.y[:30])
    for n in range(31, 41):
        A.append(obs[:n], s.y[:n])
        R.fit(obs[:n], s.y[:n])
        _, ia, alpha_a, _ = A.fit_read(True, False)
        _, ir, alpha_r, _ = R.fit_read(True, False)
        assert ia.status == ir.status == 0
        assert ia.jitter == ir.jitter > 0.0
        np.testing.assert_allclose(alpha_a, alpha_r, rtol=1e-6, atol=1e-6 * np.abs(alpha_r).max())
    X = oracle.normalize_grid(s.levels)
    f = oracle.fit(X[obs[:40]], s.y[:40], oracle.GP(noise=0.0))
    assert ia.jitter == f.jitter
    A.close()
    R.close()


def test_append_duplicate_falls_back_to_refit(bo):
    # appending an already observed point with zero noise makes the new pivot
    # vanish: the append must refit with the jitter schedule, like bo_gp_fit
    s = W.make_session(8, (9, 9, 9), 30, invalid_frac=0.0)
    gp = bo.GpParams(noise=0.0)
    A = _session(bo, s, "fp32", gp=gp)
    R = _session(bo, s, "fp32", gp=gp)
    A.fit(s.obs_idx[:29], s.y[:29])
    obs = s.obs_idx.copy()
    obs[29] = obs[3]
    A.append(obs[:30], s.y[:30])
    R.fit(obs[:30], s.y[:30])
    _, ia, alpha_a, Li_a = A.fit_read(True, True)
    _, ir, alpha_r, Li_r = R.fit_read(True, True)
    assert ia.status == ir.status == 0 and ia.jitter == ir.jitter > 0.0
    np.testing.assert_array_equal(Li_a, Li_r)
    np.testing.assert_array_equal(alpha_a, alpha_r)
    A.close()
    R.close()


def test_append_errors_and_state(bo):
    s = W.make_session(9, (8, 8, 8), 20, invalid_frac=0.3)
    A = _session(bo, s, "fp64")
    # without a fit of n - 1 points the append is a plain fit
    A.append(s.obs_idx[:12], s.y[:12])
    rc, info, _, _ = A.fit_read(False, False)
    assert rc == 0 and info.n == 12
    # an observation of a restriction-pruned candidate is refused on the device
    bad = s.obs_idx[:13].copy()
    bad[12] = int(np.flatnonzero(s.invalid)[0])
    A.append(bad, s.y[:13])
    rc, info, _, _ = A.fit_read(False, False)
    assert rc == bo.BO_E_INVALID_ARG
    r = A.acquire(_vis(s, 12), bo.AcqParams(mode=0), check=False)
    assert r.status == bo.BO_E_INVALID_ARG and list(r.idx) == [-1, -1, -1]
    # recovers with a full fit
    A.fit(s.obs_idx[:13], s.y[:13])
    assert A.acquire(_vis(s, 13), bo.AcqParams(mode=0)).status == 0
    with pytest.raises(bo.BOError) as e:
        A.append(s.obs_idx[:0], s.y[:0])
    assert e.value.status == bo.BO_E_STATE
    A.close()
