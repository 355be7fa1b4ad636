"""Pins of the oracle tuning loop's 'multi' and 'advanced multi' rounds
(Section III-H, Table I) with scripted inputs.

The surrogate step is replaced by a script of suggestions and the objective
by a table, so each trajectory below -- which configurations are evaluated,
by which function, the duplicate counts, the skip of a function, the
promotion of a function and the dropping of another -- is derived by hand
from the strategy's rules, independently of the GP.  The stub also checks
what each step sees: 'multi' steps once per round; 'advanced multi' steps once
per active function with the round's observations (no refit within a round)
and the round's earlier choices masked; failed configurations are masked and
never enter the fit (Section III-D.2).
"""
import math
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from oracle import loop as OL

EI, PI, LCB = 0, 1, 2


class Script:
    """Stand-in for the oracle step: returns the scripted (EI, PI, LCB) choices
    in turn and records the observations and mask each call saw."""

    def __init__(self, picks):
        self.picks = list(picks)
        self.calls = []

    def __call__(self, X, invalid, visited, obs, y, gp, acq, want_posterior=False, check=True):
        self.calls.append((np.flatnonzero(visited).tolist(), [int(i) for i in obs], [float(v) for v in y]))
        idx = self.picks.pop(0)
        return SimpleNamespace(status=oracle.OK, idx=np.array(idx, dtype=np.int64), var_mean=0.25)


def _run(monkeypatch, picks, table, **params):
    script = Script(picks)
    monkeypatch.setattr(OL, "step", script)
    monkeypatch.setattr(OL, "maximin_design", lambda levels, perm, off: [0, 1])
    draws = SimpleNamespace(perm=None, off=None, repl=np.array([0.5]))
    invalid = np.zeros(64, np.uint8)
    p = OL.LoopParams(init_samples=2, **params)
    tr = OL.run((8, 8), invalid, lambda c: table[c], draws, p)
    return tr, script


def _table(**vals):
    t = {0: 5.0, 1: 4.0}
    t.update({int(k[1:]): v for k, v in vals.items()})
    return t


def test_multi_duplicates_skip_and_keep_lowest_score(monkeypatch):
    # skip threshold 1, discount 1/2.  Round 1: EI and PI both suggest 10
    # (evaluated once, one duplicate each), LCB 11.  Round 2: EI and PI both
    # suggest 12: their counts reach 2 > 1, their discounted scores tie
    # (3*1/2 + 2.5 = 4.0 each) and the earlier function, EI, is kept.
    # Round 3: EI and LCB both suggest 14 (a duplicate each); round 4 both 15:
    # counts 2 > 1, scores EI 3/8 + 2.5/4 + 1/2 + 0.8 = 2.3 against LCB
    # 2/8 + 1.5/4 + 1/2 + 0.8 = 1.925, so LCB alone remains; round 5 it takes 20.
    table = _table(c10=3.0, c11=2.0, c12=2.5, c13=1.5, c14=1.0, c15=0.8, c20=0.7)
    picks = [(10, 10, 11), (12, 12, 13), (14, 63, 14), (15, 62, 15), (61, 60, 20)]
    tr, sc = _run(monkeypatch, picks, table, strategy="multi", budget=9, skip_threshold=1, discount=0.5)
    assert tr.evaluated == [0, 1, 10, 11, 12, 13, 14, 15, 20]
    assert tr.chooser == [-1, -1, EI, LCB, EI, LCB, EI, EI, LCB]
    assert tr.active == [[EI, PI, LCB], [EI, LCB], [EI, LCB], [LCB], [LCB]]
    assert len(sc.calls) == 5 and not sc.picks
    # one step per round, over everything evaluated before the round
    assert sc.calls[2][1] == [0, 1, 10, 11, 12, 13]


def test_multi_failure_scores_as_median_and_tie_keeps_earlier(monkeypatch):
    # As above but 13 fails: it is masked, never fitted, and LCB's score for
    # it is the median of the valid observations then (5, 4, 3, 2, 2.5 -> 3).
    # At round 4 the scores tie exactly (EI 3/8 + 2.5/4 + 1/2 + 0.8 against
    # LCB 2/8 + 3/4 + 1/2 + 0.8, both 1.0 + 0.5 + 0.8) and EI, the earlier,
    # is kept; round 5 is EI's.
    table = _table(c10=3.0, c11=2.0, c12=2.5, c13=math.nan, c14=1.0, c15=0.8, c20=0.7)
    picks = [(10, 10, 11), (12, 12, 13), (14, 63, 14), (15, 62, 15), (20, 60, 59)]
    tr, sc = _run(monkeypatch, picks, table, strategy="multi", budget=9, skip_threshold=1, discount=0.5)
    assert tr.evaluated == [0, 1, 10, 11, 12, 13, 14, 15, 20]
    assert tr.chooser == [-1, -1, EI, LCB, EI, LCB, EI, EI, EI]
    assert tr.active == [[EI, PI, LCB], [EI, LCB], [EI, LCB], [EI], [EI]]
    assert math.isnan(tr.values[5])
    vis, obs, y = sc.calls[2]
    assert 13 in vis and 13 not in obs and len(obs) == len(y) == 5


def test_multi_budget_ends_inside_a_round(monkeypatch):
    # budget 5: round 2 evaluates 12 (EI; PI's 12 is the same configuration),
    # then LCB's new suggestion 13 finds no budget left: the round stops, the
    # duplicate still counts, no skip is resolved.
    table = _table(c10=3.0, c11=2.0, c12=2.5, c13=1.5)
    picks = [(10, 10, 11), (12, 12, 13)]
    tr, sc = _run(monkeypatch, picks, table, strategy="multi", budget=5, skip_threshold=5, discount=0.5)
    assert tr.evaluated == [0, 1, 10, 11, 12]
    assert tr.chooser == [-1, -1, EI, LCB, EI]
    assert tr.active == [[EI, PI, LCB], [EI, PI, LCB]]


def test_advanced_multi_drop_then_promote(monkeypatch):
    # threshold 2, improvement factor 0.1, discount 1/2.
    # Round 1 (EI 3.2, PI 4.0, LCB 3.2): mean 3.467; PI > 1.1 mean (miss 1);
    # nobody below 0.9 mean = 3.12.  Round 2 (same values): discounted 4.8,
    # 6.0, 4.8, mean 5.2: PI misses again (6 > 5.72) and is dropped; EI and
    # LCB restart their counts.  Round 3 (EI 2.0, LCB 3.2): 4.4 and 5.6, mean
    # 5.0: EI wins (4.4 < 4.5), LCB misses (5.6 > 5.5).  Round 4 (EI 2.0, LCB
    # 3.2): 4.2 and 6.0, mean 5.1: EI's second win (4.2 < 4.59) promotes it
    # to the only function before LCB's second miss is looked at.
    table = _table(c10=3.2, c11=4.0, c12=3.2, c13=3.2, c14=4.0, c15=3.2, c16=2.0, c17=3.2, c18=2.0,
                   c19=3.2, c20=1.0)
    picks = [(10, 50, 51), (52, 11, 53), (54, 55, 12), (13, 56, 57), (58, 14, 59), (60, 61, 15),
             (16, 62, 63), (48, 47, 17), (18, 46, 45), (44, 43, 19), (20, 42, 41)]
    tr, sc = _run(monkeypatch, picks, table, strategy="advanced_multi", budget=13, skip_threshold=2,
                  improvement=0.1, discount=0.5)
    assert tr.evaluated == [0, 1, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20]
    assert tr.chooser == [-1, -1, EI, PI, LCB, EI, PI, LCB, EI, LCB, EI, LCB, EI]
    assert tr.active == [[EI, PI, LCB], [EI, LCB], [EI, LCB], [EI], [EI]]
    assert len(sc.calls) == 11 and not sc.picks
    # within round 1 every function steps on the round's observations, the
    # earlier choices of the round masked
    assert [c[1] for c in sc.calls[:3]] == [[0, 1]] * 3
    assert sc.calls[1][0] == [0, 1, 10] and sc.calls[2][0] == [0, 1, 10, 11]
    assert sc.calls[3][1] == [0, 1, 10, 11, 12]


@pytest.mark.parametrize("g", [0.65, 0.75])
def test_discounted_score_hand_values(g):
    assert OL.discounted_score([2.0, 1.0], g) == pytest.approx(2.0 * g + 1.0, rel=1e-15)
    assert OL.discounted_score([1.0, 0.0, 3.0], g) == pytest.approx(g * g + 3.0, rel=1e-15)


def test_advanced_multi_promotion_comes_before_a_drop(monkeypatch):
    # threshold 2, factor 0.1, discount 1/2.  EI 2.0, PI 3.0, LCB 4.0 in both
    # rounds: round 1 mean 3.0, EI wins (2 < 2.7), LCB misses (4 > 3.3);
    # round 2 discounted 3.0, 4.5, 6.0, mean 4.5: EI's second win and LCB's
    # second miss come in the same round; the win is looked at first, so EI
    # becomes the only function (dropping LCB would leave EI and PI).
    table = _table(c10=2.0, c11=3.0, c12=4.0, c13=2.0, c14=3.0, c15=4.0, c16=1.0)
    picks = [(10, 50, 51), (52, 11, 53), (54, 55, 12), (13, 56, 57), (58, 14, 59), (60, 61, 15),
             (16, 62, 63)]
    tr, sc = _run(monkeypatch, picks, table, strategy="advanced_multi", budget=9, skip_threshold=2,
                  improvement=0.1, discount=0.5)
    assert tr.evaluated == [0, 1, 10, 11, 12, 13, 14, 15, 16]
    assert tr.chooser == [-1, -1, EI, PI, LCB, EI, PI, LCB, EI]
    assert tr.active == [[EI, PI, LCB], [EI], [EI]]
