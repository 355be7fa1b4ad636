"""Tuning-loop parity: the loop over the GPU step against the oracle loop on
the same simulated tuning problem and the same random draws.  The evaluation
sequences, choosers and active-function histories must be identical; where
the two runs part, the GPU loop's choice must be within the step tolerance of
the oracle's best at the state the oracle saw (the chosen-index rule of the
single step), and the comparison ends there."""
import numpy as np
import pytest

import oracle
from oracle import loop as OL
from paper_2111_14991_amd import workloads as W
from tests import parity as PR

pytestmark = pytest.mark.gpu

CASES = [("ei", {}), ("poi", {}), ("lcb", {}), ("multi", dict(skip_threshold=2)),
         ("advanced_multi", dict(skip_threshold=2, improvement=0.02))]


@pytest.fixture(scope="module")
def bo():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2111_14991_amd as bo
    bo.lib()
    return bo


def _compare(bo, sim, draws, strategy, kw, precision, budget, tol, lambda_mode=1):
    from paper_2111_14991_amd import bo_loop as BL
    ev = lambda i: float(sim.table[i])
    tg = BL.run(bo, sim.levels, sim.invalid, ev, draws,
                BL.LoopParams(strategy=strategy, budget=budget, lambda_mode=lambda_mode, **kw), precision)
    to = OL.run(sim.levels, sim.invalid, ev, draws,
                OL.LoopParams(strategy=strategy, budget=budget, lambda_mode=lambda_mode, **kw))
    n = min(len(tg.evaluated), len(to.evaluated))
    part = next((e for e in range(n) if tg.evaluated[e] != to.evaluated[e]), None)
    if part is None:
        assert tg.evaluated == to.evaluated
        assert tg.chooser == to.chooser
        assert np.array_equal(np.asarray(tg.values), np.asarray(to.values), equal_nan=True)
        assert tg.active == to.active
        return None
    # the initial samples take no step: they must agree exactly
    q = to.chooser[part]
    assert q >= 0 and tg.chooser[part] == q, (part, q, tg.chooser[part])
    obs, y, vis, acq = to.states[sum(1 for c in to.chooser[:part] if c >= 0)]
    X = oracle.normalize_grid(sim.levels)
    ref = oracle.step(X, sim.invalid, vis, obs, y, acq=acq, want_posterior=True)
    mask = (sim.invalid | vis).astype(bool)
    A = PR.acq_arrays(ref.mu, ref.var, ref.f_best, ref.lam, mask)
    scale = (1.0, 1.0, float(np.max(np.abs(y))))[q]
    assert PR.index_ok(tg.evaluated[part], to.evaluated[part], A, q, mask, tol, scale), (part, q)
    return part


@pytest.mark.parametrize("strategy,kw", CASES)
def test_loop_trajectory_fp64(bo, strategy, kw):
    sim = W.make_simulation(3, (6, 6, 6, 6), invalid_frac=0.2, hidden_frac=0.06)
    part = _compare(bo, sim, W.loop_draws(11, 20, sim.d), strategy, kw, "fp64", 100, 1e-6)
    print(f"{strategy}: parted at {part}")


@pytest.mark.parametrize("strategy,kw", [CASES[0], CASES[4]])
def test_loop_trajectory_fp32(bo, strategy, kw):
    sim = W.make_simulation(4, (8, 8, 6, 4), invalid_frac=0.1, hidden_frac=0.05)
    part = _compare(bo, sim, W.loop_draws(12, 20, sim.d), strategy, kw, "fp32", 80, 1e-6)
    print(f"{strategy}: parted at {part}")


def test_loop_constant_lambda(bo):
    sim = W.make_simulation(5, (5, 5, 5, 5), invalid_frac=0.15, hidden_frac=0.05)
    _compare(bo, sim, W.loop_draws(13, 20, sim.d), "multi", dict(skip_threshold=1), "fp64", 70, 1e-6,
             lambda_mode=0)


def test_loop_exhausts_space(bo):
    # a budget beyond the space: every restriction-valid configuration once
    from paper_2111_14991_amd import bo_loop as BL
    sim = W.make_simulation(2, (4, 3, 5), invalid_frac=0.2, hidden_frac=0.1)
    tr = BL.run(bo, sim.levels, sim.invalid, lambda i: float(sim.table[i]), W.loop_draws(3, 20, sim.d),
                BL.LoopParams(strategy="ei", budget=60), "fp64")
    assert sorted(tr.evaluated) == np.flatnonzero(sim.invalid == 0).tolist()
    assert tr.best_after()[-1] == np.nanmin(sim.table)
