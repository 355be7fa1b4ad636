"""Host logic of the tuning loop (CPU): the loop module driven through a
stand-in session whose step is the oracle's must reproduce the oracle loop's
run exactly (evaluations, choosers, active functions), for every strategy.
This checks the loop's bookkeeping independently of the GPU; the GPU loop's
parity is in test_gpu_loop.py."""
from dataclasses import dataclass
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from oracle import loop as OL
from paper_2111_14991_amd import bo_loop as BL
from paper_2111_14991_amd import workloads as W


@dataclass
class _Acq:
    mode: int = 0
    lambda_const: float = 0.01
    mu_s: float = 0.0
    var_s_mean: float = 0.0


class _OracleSession:
    def __init__(self, levels, invalid):
        self.X = oracle.normalize_grid(levels)
        self.invalid = invalid
        self.fits = self.appends = 0

    def fit(self, oi, yy):
        self.obs, self.y = np.array(oi), np.array(yy)
        self.fits += 1

    def append(self, oi, yy):
        assert oi.shape[0] == self.obs.shape[0] + 1 and np.array_equal(oi[:-1], self.obs)
        self.obs, self.y = np.array(oi), np.array(yy)
        self.appends += 1

    def acquire(self, visited, acq, check=True):
        a = oracle.Acq(mode=acq.mode, lambda_const=acq.lambda_const, mu_s=acq.mu_s, var_s_mean=acq.var_s_mean)
        return oracle.step(self.X, self.invalid, visited, self.obs, self.y, acq=a, check=False)


BO = SimpleNamespace(AcqParams=_Acq, BO_OK=oracle.OK, BO_E_NO_CANDIDATE=oracle.E_NO_CANDIDATE)


@pytest.mark.parametrize("strategy,kw", [("ei", {}), ("poi", {}), ("lcb", {}),
                                         ("multi", dict(skip_threshold=1)),
                                         ("advanced_multi", dict(skip_threshold=2, improvement=0.01)),
                                         ("advanced_multi", dict(lambda_mode=0))])
def test_loop_matches_oracle_loop(strategy, kw):
    sim = W.make_simulation(9, (6, 5, 4, 4), invalid_frac=0.2, hidden_frac=0.08)
    dr = W.loop_draws(21, 20, sim.d)
    ev = lambda i: float(sim.table[i])
    S = _OracleSession(sim.levels, sim.invalid)
    tb = BL.TuningRun(BO, S, sim.levels, sim.invalid, ev, dr, BL.LoopParams(strategy=strategy, budget=110, **kw)).run()
    to = OL.run(sim.levels, sim.invalid, ev, dr, OL.LoopParams(strategy=strategy, budget=110, **kw))
    assert tb.evaluated == to.evaluated
    assert tb.chooser == to.chooser
    assert tb.active == to.active
    assert np.array_equal(tb.best_after(), np.asarray(OL.incumbents(to.values)))
    assert BL.mean_abs_error(tb.best_after(), np.nanmin(sim.table)) == \
        pytest.approx(OL.mae(OL.incumbents(to.values), np.nanmin(sim.table)), rel=1e-15)
    # one new observation per step: rank-1 appends after the first fit
    if strategy in ("ei", "poi", "lcb"):
        assert S.fits == 1 and S.appends > 50


def test_maximin_design_matches_oracle():
    # the last space's squared-distance scale exceeds 64-bit integers
    for seed, levels in enumerate([(6, 6, 6, 6), (12, 7, 5, 3, 3, 3, 3, 3), (2, 9), (4, 3, 5),
                                   (24, 30, 32, 38, 42, 44, 48)]):
        dr = W.loop_draws(seed, 20, len(levels))
        assert BL.maximin_lhs(levels, dr.perm, dr.off).tolist() == OL.maximin_design(levels, dr.perm, dr.off)


def test_mdf_matches_oracle():
    t = np.random.default_rng(3).uniform(0.01, 1.0, size=(5, 3))
    m, sd = BL.mean_deviation_factor(t)
    ref = OL.mdf(t.tolist())
    assert np.allclose(m, [a for a, _ in ref], rtol=1e-14) and np.allclose(sd, [b for _, b in ref], rtol=1e-12)


def test_step_failure_raises():
    # a failing step (here: every fit rejected) ends the run with an error, not silently
    class _Failing(_OracleSession):
        def acquire(self, visited, acq, check=True):
            return SimpleNamespace(status=oracle.E_NOT_PD, idx=np.full(3, -1), var_mean=0.0)

    sim = W.make_simulation(4, (5, 4, 3))
    S = _Failing(sim.levels, sim.invalid)
    with pytest.raises(RuntimeError):
        BL.TuningRun(BO, S, sim.levels, sim.invalid, lambda i: float(sim.table[i]), W.loop_draws(1, 20, sim.d),
                     BL.LoopParams(strategy="ei", budget=40)).run()


def test_unknown_strategy():
    sim = W.make_simulation(1, (3, 3))
    with pytest.raises(ValueError):
        BL.TuningRun(BO, None, sim.levels, sim.invalid, lambda i: 1.0, W.loop_draws(0, 4, 2),
                     BL.LoopParams(strategy="hedge"))
