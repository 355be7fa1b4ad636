"""Oracle tuning loop in simulation mode (test infrastructure only).

The outer loop around the surrogate step, written plainly over the FP64
oracle step: the initial sample (Section III-E), the search over the
non-evaluated configurations with failures discovered at evaluation (Section
III-D), the contextual-variance exploration factor (Section III-F), the
single, 'multi' and 'advanced multi' acquisition strategies (Section III-H)
and the run metrics of Section IV-A.  The random numbers a run consumes come
in as inputs (LoopDraws).  Readings where the text leaves room:

- Latin hypercube: S samples; sample s of design m puts parameter j at level
  floor((perm[m, j, s] + off[m, j, s]) / S * k_j) (clamped to k_j - 1), so
  each of the S strata of [0, 1) holds one sample per parameter.  Maximin:
  of the designs, the one whose smallest pairwise distance between samples
  (normalized coordinates, duplicates at distance 0) is largest, compared
  exactly (squared and scaled to integers); ties to the first design.
- Initial sample: the design's samples in order; one that is restricted, a
  repeat, or fails when evaluated is replaced by random configurations
  (uniform over the restriction-valid, not yet evaluated ones, in index
  order, from the replacement stream) until a valid one is found.  Restricted
  configurations are never evaluated (pruned); failures are.
- Budget: every evaluation counts, failed ones included.  The initial phase
  ends with `init_samples` valid observations.  A step with nothing left to
  choose ends the run.
- Failed configurations are masked from then on and never enter the fit.
- Observation score of an acquisition function: dos_t = sum_i o_i g^(t-i)
  over the observations of the configurations it chose, a failed one scored
  as the median of the valid observations at that time.
- 'multi': one step per round, its three argmax results shared; the active
  functions in order take their suggestion; a suggestion another function
  made earlier in the round is not evaluated again, and every function of
  such a group counts a duplicate.  After the round, a group with a member
  whose duplicate count exceeds the skip threshold keeps only its member of
  lowest score (ties to the earlier function); the counts of the kept one
  restart.
- 'advanced multi': each active function in turn takes the step's choice
  over the configurations not yet evaluated (the round's earlier choices
  are evaluated, hence removed from the predictions; no refit within a
  round).  After a round with more than one active function: with m the
  mean score, a score above m (1 + f) counts a miss, below m (1 - f) a win;
  the first function with `skip_threshold` wins becomes the only one;
  otherwise the first with `skip_threshold` misses is dropped and the
  counts of the others restart.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import Acq, GP, E_NO_CANDIDATE, OK, OracleError, normalize_grid, step

AF_NAMES = ("ei", "poi", "lcb")


@dataclass
class LoopParams:
    strategy: str = "advanced_multi"   # "ei", "poi", "lcb", "multi", "advanced_multi"
    init_samples: int = 20
    budget: int = 220
    lambda_mode: int = 1               # 1 contextual variance, 0 constant
    lambda_const: float = 0.01
    skip_threshold: int = 5
    discount: Optional[float] = None   # default 0.65 (multi), 0.75 (advanced multi)
    improvement: float = 0.1
    order: Sequence[str] = AF_NAMES
    gp: GP = field(default_factory=GP)


@dataclass
class Trace:
    evaluated: List[int] = field(default_factory=list)
    values: List[float] = field(default_factory=list)   # NaN where the configuration failed
    chooser: List[int] = field(default_factory=list)    # acquisition index, -1 initial sample
    active: List[List[int]] = field(default_factory=list)  # active functions after each round
    # per evaluation chosen by a step: (observations, values, visited mask, Acq) the step saw
    states: List[tuple] = field(default_factory=list)


def grid_point(levels: Sequence[int], idx: int) -> List[int]:
    lv = []
    for k in reversed(levels):
        lv.append(idx % k)
        idx //= k
    return lv[::-1]


def grid_index(levels: Sequence[int], lv: Sequence[int]) -> int:
    idx = 0
    for k, v in zip(levels, lv):
        idx = idx * k + v
    return idx


def lhs_design(levels: Sequence[int], perm: np.ndarray, off: np.ndarray) -> List[List[int]]:
    S = perm.shape[1]
    pts = []
    for s in range(S):
        lv = []
        for j, k in enumerate(levels):
            u = (perm[j, s] + off[j, s]) / S
            lv.append(min(int(math.floor(u * k)), k - 1))
        pts.append(lv)
    return pts


def min_pair_distance2(levels: Sequence[int], pts: List[List[int]]) -> int:
    """Smallest squared distance between two samples in normalized
    coordinates, times the least common multiple L of the (k_j - 1)^2 (an
    exact integer)."""
    L = 1
    for k in levels:
        L = math.lcm(L, max(k - 1, 1) ** 2)
    best = None
    for a in range(len(pts)):
        for b in range(a + 1, len(pts)):
            s = 0
            for j, k in enumerate(levels):
                s += (pts[a][j] - pts[b][j]) ** 2 * (L // max(k - 1, 1) ** 2)
            best = s if best is None else min(best, s)
    return best


def maximin_design(levels: Sequence[int], perm: np.ndarray, off: np.ndarray) -> List[int]:
    """Candidate indices of the chosen design's samples, in sample order."""
    best_m, best_v = 0, -1
    for m in range(perm.shape[0]):
        v = min_pair_distance2(levels, lhs_design(levels, perm[m], off[m]))
        if v > best_v:
            best_m, best_v = m, v
    return [grid_index(levels, lv) for lv in lhs_design(levels, perm[best_m], off[best_m])]


def discounted_score(obs: Sequence[float], g: float) -> float:
    t = len(obs)
    return sum(obs[i] * g ** (t - 1 - i) for i in range(t))


def multi_resolve(act: List[int], groups: List[List[int]], dup: dict, hist: dict, g: float) -> List[int]:
    """End of a 'multi' round: each group of functions that suggested one
    configuration, with a member whose duplicate count exceeds the threshold
    (the caller passes only those groups), keeps its member of lowest
    discounted score, ties to the earlier function; the kept one's count
    restarts."""
    for grp in groups:
        keep = grp[0]
        for a in grp[1:]:
            if discounted_score(hist[a], g) < discounted_score(hist[keep], g):
                keep = a
        act = [a for a in act if a == keep or a not in grp]
        dup[keep] = 0
    return act


def advanced_update(act: List[int], sc: dict, win: dict, miss: dict, f: float, T: int) -> List[int]:
    """End of an 'advanced multi' round with scores sc of the active
    functions: count misses (above the mean by more than f) and wins (below
    it by more than f); T wins promote a function to the only one, else T
    misses drop one and restart the others' counts."""
    m = sum(sc[a] for a in act) / len(act)
    for a in act:
        if sc[a] > m * (1.0 + f):
            miss[a] += 1
        if sc[a] < m * (1.0 - f):
            win[a] += 1
    for a in act:
        if win[a] >= T:
            return [a]
    for a in act:
        if miss[a] >= T:
            rest = [b for b in act if b != a]
            for b in rest:
                win[b] = miss[b] = 0
            return rest
    return act


def mae(best_after: Sequence[float], f_opt: float) -> float:
    """(1/10) sum_{i=2..11} |f(x+ after 20 i evaluations) - f(x')|; a run that
    ended early keeps its last incumbent."""
    tot = 0.0
    for i in range(2, 12):
        e = min(20 * i, len(best_after))
        tot += abs(best_after[e - 1] - f_opt)
    return tot / 10.0


def mdf(mean_mae):
    """Mean deviation factor (Section IV-A) from mean_mae[s][k], the mean MAE
    of strategy s on problem k over its runs: each problem's values divided
    by their mean over the strategies, then the mean and the standard
    deviation over the problems.  Returns [(mdf, std)] per strategy."""
    S, K = len(mean_mae), len(mean_mae[0])
    out = []
    for s in range(S):
        f = []
        for k in range(K):
            col = sum(mean_mae[t][k] for t in range(S)) / S
            f.append(mean_mae[s][k] / col)
        m = sum(f) / K
        out.append((m, math.sqrt(sum((v - m) ** 2 for v in f) / K)))
    return out


def incumbents(values: Sequence[float]) -> List[float]:
    out, b = [], math.inf
    for v in values:
        if not math.isnan(v) and v < b:
            b = v
        out.append(b)
    return out


class _Run:
    def __init__(self, levels, invalid, evaluate, draws, p: LoopParams):
        self.levels = tuple(int(k) for k in levels)
        self.invalid = np.asarray(invalid, dtype=np.uint8)
        self.N = self.invalid.shape[0]
        self.evaluate = evaluate
        self.draws = draws
        self.p = p
        self.X = normalize_grid(self.levels)
        self.visited = np.zeros(self.N, dtype=np.uint8)
        self.obs: List[int] = []
        self.y: List[float] = []
        self.tr = Trace()
        self.rp = 0  # position in the replacement stream

    def left(self) -> int:
        return self.p.budget - len(self.tr.evaluated)

    def do_eval(self, c: int, who: int) -> float:
        v = float(self.evaluate(c))
        self.visited[c] = 1
        self.tr.evaluated.append(c)
        self.tr.values.append(v)
        self.tr.chooser.append(who)
        if not math.isnan(v):
            self.obs.append(c)
            self.y.append(v)
        return v

    def random_pick(self) -> Optional[int]:
        pool = [i for i in range(self.N) if self.invalid[i] == 0 and self.visited[i] == 0]
        if not pool:
            return None
        u = self.draws.repl[self.rp % self.draws.repl.shape[0]]
        self.rp += 1
        return pool[min(int(math.floor(u * len(pool))), len(pool) - 1)]

    def initial(self):
        design = maximin_design(self.levels, self.draws.perm, self.draws.off)
        for c in design:
            if len(self.y) >= self.p.init_samples or self.left() <= 0:
                return
            if self.invalid[c] == 0 and self.visited[c] == 0:
                if not math.isnan(self.do_eval(c, -1)):
                    continue
            while self.left() > 0:
                r = self.random_pick()
                if r is None:
                    return
                if not math.isnan(self.do_eval(r, -1)):
                    break

    def take(self, c: int, who: int, obs, y, acq: Acq, vis=None) -> float:
        self.tr.states.append((obs, y, self.visited.copy() if vis is None else vis, acq))
        return self.do_eval(c, who)

    def stepped(self, r) -> bool:
        """True to go on; False when nothing is left to choose; raises on
        any other failure of the step."""
        if r.status == E_NO_CANDIDATE:
            return False
        if r.status != OK:
            raise OracleError(r.status, "loop step")
        return True

    def acq(self, var_s: float) -> Acq:
        if self.p.lambda_mode == 0:
            return Acq(mode=0, lambda_const=self.p.lambda_const)
        return Acq(mode=1, mu_s=self.mu_s, var_s_mean=var_s)

    def score_value(self, v: float) -> float:
        return float(np.median(self.y)) if math.isnan(v) else v

    def run(self) -> Trace:
        self.initial()
        if not self.y:
            return self.tr
        self.mu_s = sum(self.y) / len(self.y)
        var_s = 0.0
        strat = self.p.strategy
        names = list(self.p.order)
        act = [AF_NAMES.index(a) for a in names]
        hist = {a: [] for a in act}
        dup = {a: 0 for a in act}
        win = {a: 0 for a in act}
        miss = {a: 0 for a in act}
        g = self.p.discount if self.p.discount is not None else (0.65 if strat == "multi" else 0.75)
        while self.left() > 0:
            obs = np.array(self.obs, dtype=np.int64)
            y = np.array(self.y)
            if strat in AF_NAMES:
                ac = self.acq(var_s)
                r = step(self.X, self.invalid, self.visited, obs, y, self.p.gp, ac, check=False)
                if not self.stepped(r):
                    break
                if var_s == 0.0:
                    var_s = r.var_mean
                a = AF_NAMES.index(strat)
                self.take(int(r.idx[a]), a, obs, y, ac)
            elif strat == "multi":
                ac = self.acq(var_s)
                r = step(self.X, self.invalid, self.visited, obs, y, self.p.gp, ac, check=False)
                if not self.stepped(r):
                    break
                if var_s == 0.0:
                    var_s = r.var_mean
                vis0 = self.visited.copy()
                seen = {}   # candidate -> value, this round
                groups = {}  # candidate -> functions that suggested it
                stop = False
                for a in act:
                    c = int(r.idx[a])
                    groups.setdefault(c, []).append(a)
                    if c not in seen:
                        if self.left() <= 0:
                            stop = True
                            break
                        seen[c] = self.take(c, a, obs, y, ac, vis0)
                    hist[a].append(self.score_value(seen[c]))
                for c, grp in groups.items():
                    if len(grp) > 1:
                        for a in grp:
                            dup[a] += 1
                if not stop:
                    over = [grp for grp in groups.values()
                            if len(grp) > 1 and max(dup[a] for a in grp) > self.p.skip_threshold]
                    act = multi_resolve(act, over, dup, hist, g)
                self.tr.active.append(list(act))
                if stop:
                    break
            elif strat == "advanced_multi":
                ended = False
                for a in act:
                    if self.left() <= 0:
                        ended = True
                        break
                    ac = self.acq(var_s)
                    r = step(self.X, self.invalid, self.visited, obs, y, self.p.gp, ac, check=False)
                    if not self.stepped(r):
                        ended = True
                        break
                    if var_s == 0.0:
                        var_s = r.var_mean
                    v = self.take(int(r.idx[a]), a, obs, y, ac)
                    hist[a].append(self.score_value(v))
                if ended:
                    self.tr.active.append(list(act))
                    break
                if len(act) > 1:
                    sc = {a: discounted_score(hist[a], g) for a in act}
                    act = advanced_update(act, sc, win, miss, self.p.improvement, self.p.skip_threshold)
                self.tr.active.append(list(act))
            else:
                raise ValueError(strat)
        return self.tr


def run(levels: Sequence[int], invalid: np.ndarray, evaluate: Callable[[int], float], draws,
        params: LoopParams = LoopParams()) -> Trace:
    """One tuning run over the full grid of `levels` (row-major, last parameter
    fastest); `evaluate(i)` returns the time of configuration i, NaN if it
    fails."""
    return _Run(levels, invalid, evaluate, draws, params).run()
