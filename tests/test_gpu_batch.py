"""Batched form (bo_batch_*): many sessions of uneven candidate counts,
dimensions and observation counts in one captured graph of kernels.

Each session's result must be, bit for bit, the one the single-session path
gives on the same inputs (the same kernels per candidate, and the mean
variance summed over the same 64-candidate slots in the same order), and, for
the smaller sessions, the FP64 oracle's within the 1e-6 rules.  The graph is
replayed with changed plans (more observations, other unit sizes and grids)
and after autotuning."""
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


def _population(seed, k, n_lo=10, n_hi=220):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [W._population_member(rng, seed, n_lo, n_hi) for _ in range(k)]


def _open(bo, pop, precisions, n_max=256):
    out = []
    for s, p in zip(pop, precisions):
        S = bo.Session(s.N, s.d, n_max, p)
        S.set_grid(s.levels, s.cand, s.invalid)
        out.append(S)
    return out


def _acq(bo, s, mode):
    if mode == 0:
        return bo.AcqParams(mode=0, lambda_const=0.01)
    return bo.AcqParams(mode=1, mu_s=float(np.mean(s.y[:s.n_init])), var_s_mean=0.0)


def _single(bo, s, precision, n, acq):
    S = bo.Session(s.N, s.d, 256, precision)
    S.set_grid(s.levels, s.cand, s.invalid)
    vis = np.zeros(s.N, np.uint8)
    vis[s.obs_idx[:n]] = 1
    S.fit(s.obs_idx[:n], s.y[:n])
    r = S.acquire(vis, acq, check=False)
    S.close()
    return r


def _bits(x):
    return np.float64(x).view(np.uint64)


def _same(rb, rs):
    """Batched and single-session results are the same bit for bit: status,
    counts, indices, scores and every scalar of the step."""
    assert rb.status == rs.status, (rb.status, rs.status)
    assert rb.n_unmasked == rs.n_unmasked and rb.n_obs == rs.n_obs
    for f in ("jitter", "f_best", "mean_y", "var_mean", "lam"):
        assert _bits(getattr(rb, f)) == _bits(getattr(rs, f)), (f, getattr(rb, f), getattr(rs, f))
    for q in range(3):
        assert rb.idx[q] == rs.idx[q], (q, rb.idx[q], rs.idx[q])
        assert _bits(rb.score[q]) == _bits(rs.score[q]), (q, rb.score[q], rs.score[q])


def _step_inputs(pop, ns):
    obs = [s.obs_idx[:n] for s, n in zip(pop, ns)]
    ys = [s.y[:n] for s, n in zip(pop, ns)]
    vis = []
    for s, n in zip(pop, ns):
        v = np.zeros(s.N, np.uint8)
        v[s.obs_idx[:n]] = 1
        vis.append(v)
    return obs, ys, vis


def test_batch_matches_single_sessions(bo):
    pop = _population(3, 14)
    precs = ["fp32"] * 10 + ["fp64"] * 4
    modes = [1, 0] * 7
    S = _open(bo, pop, precs)
    B = bo.Batch(S)
    acqs = [_acq(bo, s, m) for s, m in zip(pop, modes)]
    # step 1: the first half of each session's observations; step 2: all of
    # them (the graph captured in step 1 replays a changed plan)
    for frac in (0.5, 1.0):
        ns = [max(1, int(round(frac * s.n))) for s in pop]
        obs, ys, vis = _step_inputs(pop, ns)
        res, _ = B.step(obs, ys, vis, acqs)
        for i, (s, r) in enumerate(zip(pop, res)):
            _same(r, _single(bo, s, precs[i], ns[i], acqs[i]))
    B.close()
    for x in S:
        x.close()


def test_batch_tile_shapes_and_tuner(bo):
    pop = _population(5, 10, n_lo=10, n_hi=120)
    precs = ["fp32"] * 7 + ["fp64"] * 3
    S = _open(bo, pop, precs)
    B = bo.Batch(S)
    acqs = [_acq(bo, s, 1) for s in pop]
    obs, ys, vis = _step_inputs(pop, [s.n for s in pop])
    base, _ = B.step(obs, ys, vis, acqs)
    for po in (1, 0):
        for chunk in (2048, 32768):
            for order in (0, 1):
                B.set_config(post_order=po, acq_chunk=chunk, fit_order=order)
                res, _ = B.step(obs, ys, vis, acqs)
                for a, b_ in zip(res, base):
                    _same(a, b_)
    cfg = B.tune(obs, ys, vis, acqs, reps=2)
    assert cfg["post_order"] in (0, 1) and cfg["acq_chunk"] % 2048 == 0 and cfg["fit_order"] in (0, 1)
    assert B.config() == cfg
    res, _ = B.step(obs, ys, vis, acqs)
    for a, b_ in zip(res, base):
        _same(a, b_)
    B.close()
    for x in S:
        x.close()


def test_batch_oracle_parity(bo):
    pop = sorted(_population(11, 12), key=lambda s: s.N)[:4]
    precs = ["fp32", "fp64", "fp32", "fp64"]
    S = _open(bo, pop, precs)
    B = bo.Batch(S)
    acqs = [_acq(bo, s, 0) for s in pop]
    obs, ys, vis = _step_inputs(pop, [s.n for s in pop])
    res, _ = B.step(obs, ys, vis, acqs)
    for s, r, v in zip(pop, res, vis):
        X = oracle.normalize_grid(s.levels, s.cand, s.N)
        ref = oracle.step(X, s.invalid, v, s.obs_idx, s.y, oracle.GP(), oracle.Acq(mode=0, lambda_const=0.01),
                          want_posterior=True)
        assert r.status == ref.status == 0
        assert r.n_unmasked == ref.n_unmasked
        assert r.var_mean == pytest.approx(ref.var_mean, rel=TOL)
        mask = (s.invalid | v).astype(bool)
        A = PR.acq_arrays(ref.mu, ref.var, ref.f_best, ref.lam, mask)
        scales = (1.0, 1.0, float(np.max(np.abs(s.y))))
        for q in range(3):
            assert PR.index_ok(int(r.idx[q]), int(ref.idx[q]), A, q, mask, TOL, scales[q]), (q, r, ref)
            g = int(r.idx[q])
            assert abs(r.score[q] - A[g, q]) <= TOL * max(abs(A[g, q]), scales[q])
    B.close()
    for x in S:
        x.close()


def test_batch_errors(bo):
    pop = _population(7, 3, n_lo=10, n_hi=40)
    S = _open(bo, pop, ["fp32", "fp64", "fp32"])
    B = bo.Batch(S)
    acqs = [_acq(bo, s, 0) for s in pop]
    obs, ys, vis = _step_inputs(pop, [s.n for s in pop])
    # an observation of a restriction-pruned candidate fails only its session
    bad = obs[1].copy()
    pruned = np.flatnonzero(pop[1].invalid)
    if pruned.size:
        bad[0] = pruned[0]
        res, _ = B.step([obs[0], bad, obs[2]], ys, vis, acqs)
        assert res[1].status == bo.BO_E_INVALID_ARG and res[1].idx[0] == -1
        assert res[0].status == 0 and res[2].status == 0
        _same(res[0], _single(bo, pop[0], "fp32", pop[0].n, acqs[0]))
    # a fit above the batched limit is refused before anything runs
    with pytest.raises(bo.BOError) as e:
        B.step([np.arange(257)] + obs[1:], [np.ones(257)] + ys[1:], vis, acqs)
    assert e.value.status == bo.BO_E_INVALID_ARG
    # the batch still works afterwards
    res, _ = B.step(obs, ys, vis, acqs)
    assert all(r.status == 0 for r in res)
    B.close()
    # BF16X3 sessions are not batched
    T = bo.Session(pop[0].N, pop[0].d, 64, "bf16x3")
    with pytest.raises(bo.BOError):
        bo.Batch([S[0], T])
    T.close()
    for x in S:
        x.close()
