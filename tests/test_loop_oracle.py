"""Pins of the oracle tuning loop (CPU): the initial design against an
independent distance routine and the Latin hypercube property, the
discounted observation score against its closed form, the strategy updates
on scripted scores, the error metric on a constructed trace, and run
invariants on small simulations."""
import math

import numpy as np
import pytest
from scipy.spatial.distance import pdist

from oracle import loop as OL
from paper_2111_14991_amd import workloads as W


@pytest.mark.parametrize("levels", [(6, 6, 6, 6), (8, 8, 6, 4), (12, 7, 5, 3, 3), (2, 9)])
def test_lhs_strata_and_maximin(levels):
    S = 20
    dr = W.loop_draws(5, S, len(levels), designs=12)
    k = np.asarray(levels)
    crits = []
    for m in range(dr.perm.shape[0]):
        pts = np.array(OL.lhs_design(levels, dr.perm[m], dr.off[m]))
        # Latin hypercube: each of the S strata of [0, 1) once per parameter,
        # so each level of parameter j gets S/k_j samples up to the two strata
        # split by its boundaries
        for j, kj in enumerate(levels):
            cnt = np.bincount(pts[:, j], minlength=kj)
            assert cnt.sum() == S
            assert cnt.min() >= math.floor(S / kj) - 1 and cnt.max() <= math.ceil(S / kj) + 1
        x = pts / np.maximum(k - 1, 1)
        crits.append(pdist(x).min())
    chosen = OL.maximin_design(levels, dr.perm, dr.off)
    best = int(np.argmax(np.array(crits) >= max(crits) - 1e-12))
    want = [OL.grid_index(levels, lv) for lv in OL.lhs_design(levels, dr.perm[best], dr.off[best])]
    assert chosen == want
    # grid indices decode back to the design's levels (row-major, last fastest)
    assert [OL.grid_point(levels, c) for c in chosen] == OL.lhs_design(levels, dr.perm[best], dr.off[best])
    assert np.array_equal(np.ravel_multi_index(np.array(OL.lhs_design(levels, dr.perm[best], dr.off[best])).T,
                                               levels), chosen)


@pytest.mark.parametrize("g", [0.65, 0.75, 0.9])
def test_discounted_score(g):
    # constant observations: a geometric series
    for t in (1, 2, 7, 30):
        assert OL.discounted_score([2.5] * t, g) == pytest.approx(2.5 * (1 - g ** t) / (1 - g), rel=1e-14)
    # the newest observation has weight 1, each older one g times the next
    o = [3.0, 1.0, 4.0, 1.0, 5.0]
    prev = 0.0
    for t in range(1, len(o) + 1):
        cur = OL.discounted_score(o[:t], g)
        assert cur == pytest.approx(g * prev + o[t - 1], rel=1e-14)
        prev = cur


def test_advanced_update_promotes_and_drops():
    act = [0, 1, 2]
    win, miss = dict.fromkeys(act, 0), dict.fromkeys(act, 0)
    # function 2 scores 15% above the mean twice (the others 8% below): dropped at T = 2
    sc = {0: 1.2, 1: 1.2, 2: 1.5}
    assert OL.advanced_update(act, sc, win, miss, 0.1, 2) == act
    assert miss == {0: 0, 1: 0, 2: 1}
    act = OL.advanced_update(act, sc, win, miss, 0.1, 2)
    assert act == [0, 1] and win == {0: 0, 1: 0, 2: 0} and miss[0] == 0 and miss[1] == 0
    # function 0 scores 25% below the mean of the two twice: the only one left
    sc = {0: 1.0, 1: 1.7}
    assert OL.advanced_update(act, sc, win, miss, 0.1, 2) == [0, 1]
    assert OL.advanced_update(act, sc, win, miss, 0.1, 2) == [0]
    # within the improvement band nothing changes
    act, win, miss = [0, 1, 2], dict.fromkeys([0, 1, 2], 0), dict.fromkeys([0, 1, 2], 0)
    for _ in range(10):
        assert OL.advanced_update(act, {0: 1.0, 1: 1.05, 2: 0.97}, win, miss, 0.1, 2) == act


def test_multi_resolve_keeps_lowest_score():
    hist = {0: [1.0, 1.2], 1: [0.9, 1.0], 2: [2.0, 2.0]}
    dup = {0: 3, 1: 3, 2: 0}
    assert OL.multi_resolve([0, 1, 2], [[0, 1]], dup, hist, 0.65) == [1, 2]
    assert dup[1] == 0
    # ties go to the earlier function
    hist = {0: [1.0], 1: [1.0], 2: [1.0]}
    assert OL.multi_resolve([0, 1, 2], [[1, 2]], {0: 0, 1: 9, 2: 9}, hist, 0.9) == [0, 1]


def test_mae_definition():
    best = [1.0 + 1.0 / e for e in range(1, 221)]
    want = sum(1.0 / (20 * i) for i in range(2, 12)) / 10
    assert OL.mae(best, 1.0) == pytest.approx(want, rel=1e-14)
    # a run that stopped early keeps its last incumbent
    assert OL.mae([3.0] * 50, 1.0) == pytest.approx(2.0)
    assert OL.incumbents([5.0, float("nan"), 4.0, 6.0]) == [5.0, 5.0, 4.0, 4.0]


def test_mdf_definition():
    # two problems on different scales: only the ratios within a problem count
    t = [[1.0, 100.0], [3.0, 300.0]]
    assert OL.mdf(t) == [(0.5, 0.0), (1.5, 0.0)]
    t = [[1.0, 2.0], [1.0, 6.0]]
    (m0, s0), (m1, s1) = OL.mdf(t)
    assert m0 == pytest.approx((1.0 + 0.5) / 2) and s0 == pytest.approx(0.25)
    assert m1 == pytest.approx((1.0 + 1.5) / 2) and s1 == pytest.approx(0.25)
    # the factors of one problem average to one
    rng = np.random.default_rng(0)
    t = rng.uniform(0.1, 2.0, size=(5, 3)).tolist()
    assert sum(m for m, _ in OL.mdf(t)) / 5 == pytest.approx(1.0)


def test_table2_problem_sizes():
    ps = W.table2_problems(0)
    assert [p.N for p in ps] == [82944, 18432, 8184]
    valid = [int((p.invalid == 0).sum()) for p in ps]
    assert abs(valid[0] - 17956) < 0.1 * 17956 and abs(valid[1] - 9400) < 0.01 * 9400 and valid[2] == 8184
    assert ps[0].hidden.sum() == 0
    assert abs(ps[1].hidden.sum() / valid[1] - 0.385) < 0.03 and abs(ps[2].hidden.sum() / 8184 - 0.039) < 0.01


@pytest.mark.parametrize("strategy", ["ei", "poi", "lcb", "multi", "advanced_multi"])
def test_run_invariants(strategy):
    sim = W.make_simulation(7, (6, 5, 4, 3), invalid_frac=0.2, hidden_frac=0.08)
    dr = W.loop_draws(17, 20, sim.d)
    p = OL.LoopParams(strategy=strategy, budget=90, skip_threshold=2, improvement=0.02)
    tr = OL.run(sim.levels, sim.invalid, lambda i: sim.table[i], dr, p)
    ev = np.array(tr.evaluated)
    assert len(ev) == 90 and len(set(ev.tolist())) == 90        # budget spent, nothing twice
    assert not sim.invalid[ev].any()                           # restricted ones pruned
    vals = np.array(tr.values)
    assert np.array_equal(np.isnan(vals), sim.hidden[ev] == 1)  # failures are discovered
    ch = np.array(tr.chooser)
    n_init = int(np.argmax(ch >= 0))
    assert (ch[:n_init] == -1).all() and (ch[n_init:] >= 0).all()
    assert int((~np.isnan(vals[:n_init])).sum()) == 20          # 20 valid initial samples
    inc = OL.incumbents(tr.values)
    assert all(inc[i + 1] <= inc[i] for i in range(len(inc) - 1))
    if strategy in ("ei", "poi", "lcb"):
        assert set(ch[n_init:].tolist()) == {("ei", "poi", "lcb").index(strategy)}
    for a in tr.active:
        assert len(a) >= 1 and a == sorted(a, key=[0, 1, 2].index)


def test_run_exhausts_tiny_space():
    sim = W.make_simulation(2, (4, 3, 5), invalid_frac=0.2, hidden_frac=0.1)
    dr = W.loop_draws(3, 20, sim.d)
    tr = OL.run(sim.levels, sim.invalid, lambda i: sim.table[i], dr, OL.LoopParams(strategy="ei", budget=500))
    # every restriction-valid configuration evaluated once, then no candidate is left
    assert sorted(tr.evaluated) == np.flatnonzero(sim.invalid == 0).tolist()
    assert OL.incumbents(tr.values)[-1] == np.nanmin(sim.table)
