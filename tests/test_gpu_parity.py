"""GPU parity: the HIP library through its C ABI against the FP64 oracle on the
same seeded inputs, element by element (posterior mean and variance of every
candidate, the three acquisitions, lambda, the mean variance) plus the chosen
indices, masks and error codes."""
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


def _session(bo, s, precision, n_max=None, gp=None):
    S = bo.Session(s.N, s.d, n_max or s.n, precision, gp=gp)
    nv = S.set_grid(s.levels, s.cand, s.invalid)
    assert nv == int((s.invalid == 0).sum())
    return S


def _gpu_step(S, s, obs, y, visited, acq):
    S.fit(obs, y)
    r = S.acquire(visited, acq)
    mu, var, vm = S.posterior(visited)
    return r, mu.cpu().numpy(), var.cpu().numpy(), vm


def _oracle_step(s, obs, y, visited, acq, gp=oracle.GP()):
    X = oracle.normalize_grid(s.levels, s.cand, s.N)
    return X, oracle.step(X, s.invalid, visited, obs, y, gp, acq, want_posterior=True)


def _acq_pair(bo, mu_s, var_s=0.0, mode=1):
    return (bo.AcqParams(mode=mode, mu_s=mu_s, var_s_mean=var_s),
            oracle.Acq(mode=mode, mu_s=mu_s, var_s_mean=var_s))


def _parity(bo, s, precision, acq_mode=1, tol=TOL, gp=None):
    gpp = gp or bo.GpParams()
    ogp = oracle.GP(gpp.nu2, gpp.lengthscale, gpp.amp, gpp.noise, gpp.jitter_tries)
    S = _session(bo, s, precision, gp=gpp)
    vis = s.visited()
    mu_s = float(np.mean(s.y[:s.n_init]))
    # contextual constants: each side computes its own from the initial sample
    var_s_g = var_s_o = 0.0
    if acq_mode == 1 and s.n > s.n_init:
        vis0 = np.zeros(s.N, np.uint8)
        vis0[s.obs_idx[:s.n_init]] = 1
        S.fit(s.obs_idx[:s.n_init], s.y[:s.n_init])
        var_s_g = S.acquire(vis0, bo.AcqParams(mode=0)).var_mean
        X = oracle.normalize_grid(s.levels, s.cand, s.N)
        var_s_o = oracle.step(X, s.invalid, vis0, s.obs_idx[:s.n_init], s.y[:s.n_init], ogp,
                              oracle.Acq(mode=0)).var_mean
        assert abs(var_s_g - var_s_o) <= tol * var_s_o
    ga = bo.AcqParams(mode=acq_mode, mu_s=mu_s, var_s_mean=var_s_g)
    oa = oracle.Acq(mode=acq_mode, mu_s=mu_s, var_s_mean=var_s_o)
    r, mu, var, vm = _gpu_step(S, s, s.obs_idx, s.y, vis, ga)
    _, ref = _oracle_step(s, s.obs_idx, s.y, vis, oa, ogp)
    mask = (s.invalid | vis).astype(bool)
    rep = PR.check_step(r, ref, mu, var, ref.mu, ref.var, mask, s.y, gpp.amp, tol)
    assert vm == pytest.approx(r.var_mean, rel=1e-12)
    for k in ("mu", "var", "ei", "pi", "lcb", "lambda", "var_mean", "score0", "score1", "score2", "mean_y"):
        assert rep[k] <= tol, (k, rep)
    assert rep["f_best"] == 0.0
    assert rep["jitter_equal"]
    S.close()
    return rep


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1_parity(bo, seed, precision):
    rep = _parity(bo, W.config_c1(seed), precision)
    if precision == "fp64":
        assert rep["mu"] < 1e-11 and rep["var"] < 1e-11, rep


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tiny_spaces(bo, seed, precision):
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    d = int(rng.integers(1, 7))
    levels = tuple(int(k) for k in rng.integers(1, 6, size=d))
    if W.grid_size(levels) < 12:
        levels = levels + (12,)
    n = int(rng.integers(1, 11))
    s = W.make_session(seed, levels, n, invalid_frac=float(rng.uniform(0, 0.4)))
    gp = bo.GpParams(nu2=int(rng.choice([3, 5])), lengthscale=float(rng.uniform(0.4, 2.0)),
                     amp=float(rng.uniform(0.5, 2.0)), noise=float(rng.choice([1e-6, 1e-3])))
    _parity(bo, s, precision, acq_mode=int(seed % 2), gp=gp)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c2_parity(bo, precision):
    _parity(bo, W.config_c2(0), precision)


def test_large_fit_parity(bo):
    # n > 256 takes the multi-workgroup fit
    s = W.make_session(3, (9, 8, 7, 6, 5), 300, invalid_frac=0.2)
    _parity(bo, s, "fp64")


def test_fit_matches_oracle(bo):
    s = W.config_c1(1)
    S = _session(bo, s, "fp64")
    S.fit(s.obs_idx, s.y)
    rc, info, alpha, Linv = S.fit_read(True, True)
    assert rc == 0 and info.status == 0
    X = oracle.normalize_grid(s.levels)
    f = oracle.fit(X[s.obs_idx], s.y)
    np.testing.assert_allclose(alpha, f.alpha, rtol=1e-10, atol=1e-10 * np.abs(f.alpha).max())
    np.testing.assert_allclose(Linv, np.linalg.inv(f.L), rtol=1e-10, atol=1e-12)
    assert info.jitter == f.jitter and info.f_best == f.f_best
    assert info.mean_y == pytest.approx(f.mean_y, rel=1e-15)


@pytest.mark.parametrize("n", [200, 520, 1000])
def test_large_fit_matches_oracle(bo, n):
    # the multi-workgroup fit (one launch per blocked step) against the
    # oracle's Cholesky: alpha and L^-1 normwise, scaled by the condition
    # of K that the errors of both sides grow with
    s = W.make_session(40 + n, (4,) * 8, n, invalid_frac=0.2)
    S = _session(bo, s, "fp64")
    S.fit(s.obs_idx, s.y)
    rc, info, alpha, Linv = S.fit_read(True, True)
    assert rc == 0 and info.status == 0
    X = oracle.normalize_grid(s.levels)
    f = oracle.fit(X[s.obs_idx], s.y)
    Li = np.linalg.inv(f.L)
    cond = np.linalg.cond(f.L @ f.L.T)
    tol = 1e-15 * cond * n
    assert np.max(np.abs(alpha - f.alpha)) <= tol * np.max(np.abs(f.alpha)), (np.max(np.abs(alpha - f.alpha)), tol)
    assert np.max(np.abs(Linv - Li)) <= tol * np.max(np.abs(Li))
    assert info.jitter == f.jitter and info.f_best == f.f_best
    S.close()


@pytest.mark.parametrize("n", [3, 300])
def test_jitter_escalation_and_not_pd(bo, n):
    # duplicate observations with zero noise make K_nn singular
    s = W.make_session(5, (10, 10, 10), n, invalid_frac=0.0)
    obs = s.obs_idx.copy()
    obs[-1] = obs[0]
    y = s.y.copy()
    X = oracle.normalize_grid(s.levels)
    f = oracle.fit(X[obs], y, oracle.GP(noise=0.0))
    S = _session(bo, s, "fp64", n_max=n, gp=bo.GpParams(noise=0.0))
    S.fit(obs, y)
    rc, info, _, _ = S.fit_read(False, False)
    assert rc == 0 and info.status == 0
    assert info.jitter == f.jitter and info.jitter > 0.0
    r = S.acquire(s.visited(), bo.AcqParams(mode=0))
    assert r.status == 0 and r.jitter == f.jitter
    S.close()
    S = _session(bo, s, "fp64", n_max=n, gp=bo.GpParams(noise=0.0, jitter_tries=1))
    S.fit(obs, y)
    r = S.acquire(s.visited(), bo.AcqParams(mode=0), check=False)
    assert r.status == bo.BO_E_NOT_PD
    assert list(r.idx) == [-1, -1, -1]


@pytest.mark.parametrize("n", [300, 1000])
def test_async_jitter_escalation_on_device(bo, n):
    # Section III-B fit with a singular K_nn (a duplicated observation, zero
    # noise) stepped only through bo_acquire_async: the jitter schedule is
    # escalated on the device, so the result carries the oracle's accepted
    # jitter and equals the synchronous step's
    import torch
    s = W.make_session(6, (12, 12, 12), n, invalid_frac=0.0)
    obs = s.obs_idx.copy()
    obs[-1] = obs[0]
    y = s.y.copy()
    X = oracle.normalize_grid(s.levels)
    f = oracle.fit(X[obs], y, oracle.GP(noise=0.0))
    assert f.jitter > 0.0
    S = _session(bo, s, "fp64", n_max=n, gp=bo.GpParams(noise=0.0))
    acq = bo.AcqParams(mode=0)
    vis = torch.as_tensor(s.visited()).cuda()
    out = torch.zeros(bo.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    S.fit(obs, y)
    S.acquire_async(out, vis, acq)
    torch.cuda.synchronize()
    ra = bo.result_from_bytes(out.cpu().numpy().tobytes())
    assert ra.status == 0 and ra.jitter == f.jitter
    S.fit(obs, y)
    r = S.acquire(vis, acq)
    np.testing.assert_array_equal(ra.idx, r.idx)
    np.testing.assert_array_equal(ra.score, r.score)
    assert ra.jitter == r.jitter and ra.var_mean == r.var_mean
    S.close()


def test_error_codes(bo):
    s = W.config_c1(0)
    S = _session(bo, s, "fp64")
    with pytest.raises(bo.BOError) as e:
        S.acquire(s.visited(), bo.AcqParams(mode=0))
    assert e.value.status == bo.BO_E_STATE
    # observation of a restriction-pruned candidate
    bad = s.obs_idx.copy()
    bad[3] = int(np.flatnonzero(s.invalid)[0])
    S.fit(bad, s.y)
    assert S.acquire(s.visited(), bo.AcqParams(mode=0), check=False).status == bo.BO_E_INVALID_ARG
    yb = s.y.copy()
    yb[2] = np.nan
    S.fit(s.obs_idx, yb)
    assert S.acquire(s.visited(), bo.AcqParams(mode=0), check=False).status == bo.BO_E_INVALID_ARG
    S.fit(s.obs_idx, -s.y)
    r = S.acquire(s.visited(), bo.AcqParams(mode=1, mu_s=1.0), check=False)
    assert r.status == bo.BO_E_INVALID_ARG
    S.fit(s.obs_idx, s.y)
    with pytest.raises(bo.BOError) as e:
        S.acquire(s.visited(), bo.AcqParams(mode=1, mu_s=0.0))
    assert e.value.status == bo.BO_E_INVALID_ARG
    # everything excluded
    allvis = np.ones(s.N, np.uint8)
    r = S.acquire(allvis, bo.AcqParams(mode=0), check=False)
    assert r.status == bo.BO_E_NO_CANDIDATE and list(r.idx) == [-1, -1, -1]
    # and a normal step still works afterwards
    assert S.acquire(s.visited(), bo.AcqParams(mode=0)).status == 0
    with pytest.raises(bo.BOError) as e:
        S.fit(s.obs_idx[:0], s.y[:0])
    assert e.value.status == bo.BO_E_STATE
    S.close()


def test_ties_lowest_index_and_coordinates(bo):
    # duplicated candidate rows given as coordinates: identical scores, the
    # lowest index must win on both sides
    X = np.array([[0.0, 0.0], [0.5, 0.5], [0.2, 0.7], [0.5, 0.5], [1.0, 1.0], [0.2, 0.7]])
    inv = np.zeros(6, np.uint8)
    vis = np.array([1, 0, 0, 0, 1, 0], np.uint8)
    obs = np.array([0, 4])
    y = np.array([1.0, 1.0])
    S = bo.Session(6, 2, 2, "fp64")
    S.set_candidates(X, inv)
    S.fit(obs, y)
    r = S.acquire(vis, bo.AcqParams(mode=0))
    ref = oracle.step(X, inv, vis, obs, y, acq=oracle.Acq(mode=0))
    np.testing.assert_array_equal(r.idx, ref.idx)


def test_async_matches_sync(bo):
    import torch
    s = W.config_c1(3)
    S = _session(bo, s, "fp32")
    S.fit(s.obs_idx, s.y)
    acq = bo.AcqParams(mode=1, mu_s=float(np.mean(s.y)))
    r = S.acquire(s.visited(), acq)
    out = torch.zeros(bo.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    vis = torch.as_tensor(s.visited()).cuda()
    S.acquire_async(out, vis, acq)
    torch.cuda.synchronize()
    ra = bo.result_from_bytes(out.cpu().numpy().tobytes())
    np.testing.assert_array_equal(ra.idx, r.idx)
    assert ra.lam == r.lam and ra.var_mean == r.var_mean
