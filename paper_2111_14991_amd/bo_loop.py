"""Bayesian-optimization tuning loop in simulation mode.

Host orchestration around the GPU step (`Session.fit`/`append` +
`Session.acquire`): every surrogate fit, posterior, exploration factor,
acquisition and masked argmax runs in the library's kernels; this module only
decides which configuration to evaluate next and keeps the run's books.

- Initial sample (Section III-E): Latin hypercube designs, the maximin one
  kept (largest smallest distance between its samples in normalized
  coordinates, compared exactly; first design on ties); samples that are restricted, repeated
  or fail when evaluated are replaced by random restriction-valid
  configurations not yet evaluated, until `init_samples` valid observations
  are in.  Sample s of a design puts parameter j at level
  floor((perm + off) / S * k_j), clamped to k_j - 1.
- Search (Sections III-D, III-G): only configurations neither restricted nor
  evaluated are candidates; a configuration that fails when evaluated is
  masked from then on and never enters the fit.  Every evaluation, failed or
  not, counts against the budget.
- Exploration factor (Section III-F): contextual variance with mu_s the mean
  of the initial sample and the mean variance of the first step after it as
  the normalizer, or the constant 0.01.
- Strategies (Section III-H): a single acquisition function; 'multi' (one
  prediction per round shared by the active functions in order; a
  suggestion made earlier in the round is not evaluated again and every
  function suggesting it counts a duplicate; a group whose duplicate count
  exceeds the skip threshold keeps only its member of lowest discounted
  observation score); 'advanced multi' (each active function in turn takes
  its choice over the configurations not yet evaluated, the round's earlier
  choices thereby removed from the predictions; after each round a score
  above the mean by more than the improvement factor counts a miss, below it
  a win; `skip_threshold` wins make a function the only one, else
  `skip_threshold` misses drop it and restart the others' counts).  The
  discounted observation score is sum_i o_i g^(t-i) over a function's own
  observations, a failed configuration counted as the median of the valid
  observations at that time.
- Metrics (Section IV-A): the incumbent after every evaluation, the mean
  absolute error against the optimum over evaluations 40, 60, ..., 220, and
  the mean deviation factor of strategies over several problems (each
  problem's mean errors divided by their mean over the strategies, averaged
  over the problems).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

ACQS = ("ei", "poi", "lcb")
STRATEGIES = ACQS + ("multi", "advanced_multi")


@dataclass
class LoopParams:
    strategy: str = "advanced_multi"
    init_samples: int = 20
    budget: int = 220
    lambda_mode: int = 1            # 1: contextual variance; 0: constant
    lambda_const: float = 0.01
    skip_threshold: int = 5
    discount: Optional[float] = None  # None: 0.65 for multi, 0.75 for advanced multi (Table I)
    improvement: float = 0.1        # required improvement factor (Table I)
    order: Sequence[str] = ACQS


@dataclass
class RunTrace:
    evaluated: List[int] = field(default_factory=list)
    values: List[float] = field(default_factory=list)    # NaN: the configuration failed
    chooser: List[int] = field(default_factory=list)     # acquisition index; -1 initial sample
    active: List[List[int]] = field(default_factory=list)
    steps: int = 0                                       # GPU steps taken

    def best_after(self) -> np.ndarray:
        v = np.asarray(self.values, dtype=np.float64)
        return np.fmin.accumulate(np.where(np.isnan(v), np.inf, v)) if v.size else v


def mean_abs_error(best_after: np.ndarray, f_opt: float) -> float:
    marks = np.minimum(20 * np.arange(2, 12), best_after.shape[0]) - 1
    return float(np.mean(np.abs(best_after[marks] - f_opt)))


def mean_deviation_factor(mean_mae: np.ndarray):
    """MDF of Section IV-A: mean_mae[s, k] (strategy s, problem k) divided by
    the problem's mean over the strategies, then mean and standard deviation
    over the problems, per strategy."""
    m = np.asarray(mean_mae, dtype=np.float64)
    f = m / m.mean(axis=0, keepdims=True)
    return f.mean(axis=1), f.std(axis=1)


def maximin_lhs(levels: Sequence[int], perm: np.ndarray, off: np.ndarray) -> np.ndarray:
    """Candidate indices (row-major grid) of the maximin design's samples.
    Squared distances are compared exactly: scaled by the least common
    multiple of the (k_j - 1)^2 they are integers."""
    k = np.asarray(levels, dtype=np.int64)
    S = perm.shape[2]
    u = (perm + off) / S                                           # (designs, d, S)
    lv = np.minimum(np.floor(u * k[None, :, None]).astype(np.int64), (k - 1)[None, :, None])
    den = [max(int(v) - 1, 1) ** 2 for v in k]
    L = 1
    for v in den:
        L = math.lcm(L, v)
    diff = lv[:, :, :, None] - lv[:, :, None, :]                   # (designs, d, S, S)
    if L * max(den) * len(den) < 2 ** 62:
        wt = np.array([L // v for v in den], dtype=np.int64)
        d2 = np.einsum("mjab,j->mab", diff * diff, wt)
    else:  # beyond int64: exact Python integers
        wt = np.array([L // v for v in den], dtype=object)
        d2 = np.einsum("mjab,j->mab", (diff * diff).astype(object), wt)
    iu = np.triu_indices(S, 1)
    crit = d2[:, iu[0], iu[1]].min(axis=1)
    best = int(np.argmax(crit))
    return np.ravel_multi_index(tuple(lv[best]), tuple(int(v) for v in k))


def _dos(obs: Sequence[float], g: float) -> float:
    t, s = len(obs), 0.0
    for i, o in enumerate(obs):
        s += o * g ** (t - 1 - i)
    return s


class TuningRun:
    """One run over the full grid of `levels` (row-major, last parameter
    fastest); `evaluate(i)` returns configuration i's time, NaN if it fails."""

    def __init__(self, bo, session, levels: Sequence[int], invalid: np.ndarray,
                 evaluate: Callable[[int], float], draws, params: LoopParams):
        if params.strategy not in STRATEGIES:
            raise ValueError(f"unknown strategy {params.strategy!r}")
        self.bo, self.S, self.p = bo, session, params
        self.levels = tuple(int(k) for k in levels)
        self.invalid = np.asarray(invalid, dtype=np.uint8)
        self.evaluate, self.draws = evaluate, draws
        self.visited = np.zeros(self.invalid.shape[0], dtype=np.uint8)
        self.obs: List[int] = []
        self.y: List[float] = []
        self.fitted = -1      # observations in the current fit
        self.repl_pos = 0
        self.tr = RunTrace()

    # -- books -------------------------------------------------------------
    def remaining(self) -> int:
        return self.p.budget - len(self.tr.evaluated)

    def _evaluate(self, c: int, who: int) -> float:
        v = float(self.evaluate(c))
        self.visited[c] = 1
        self.tr.evaluated.append(c)
        self.tr.values.append(v)
        self.tr.chooser.append(who)
        if v == v:
            self.obs.append(c)
            self.y.append(v)
        return v

    def _score(self, v: float) -> float:
        return v if v == v else float(np.median(np.asarray(self.y)))

    # -- initial sample ----------------------------------------------------
    def _replacement(self) -> Optional[int]:
        pool = np.flatnonzero((self.invalid == 0) & (self.visited == 0))
        if pool.size == 0:
            return None
        u = self.draws.repl[self.repl_pos % self.draws.repl.shape[0]]
        self.repl_pos += 1
        return int(pool[min(int(math.floor(u * pool.size)), pool.size - 1)])

    def initial_sample(self):
        for c in maximin_lhs(self.levels, self.draws.perm, self.draws.off):
            c = int(c)
            if len(self.y) >= self.p.init_samples or self.remaining() <= 0:
                return
            if not self.invalid[c] and not self.visited[c] and not math.isnan(self._evaluate(c, -1)):
                continue
            while self.remaining() > 0:
                r = self._replacement()
                if r is None:
                    return
                if not math.isnan(self._evaluate(r, -1)):
                    break

    # -- steps -------------------------------------------------------------
    def _refit(self):
        n = len(self.obs)
        if n == self.fitted:
            return
        oi = np.asarray(self.obs, dtype=np.int64)
        yy = np.asarray(self.y, dtype=np.float64)
        if n == self.fitted + 1 and self.fitted > 0:
            self.S.append(oi, yy)
        else:
            self.S.fit(oi, yy)
        self.fitted = n

    def _acq(self):
        bo = self.bo
        if self.p.lambda_mode == 0:
            return bo.AcqParams(mode=0, lambda_const=self.p.lambda_const)
        return bo.AcqParams(mode=1, mu_s=self.mu_s, var_s_mean=self.var_s)

    def _step(self):
        """One GPU step; None when no configuration is left to choose (the
        run ends), an exception for any other failure."""
        r = self.S.acquire(self.visited, self._acq(), check=False)
        self.tr.steps += 1
        if r.status == self.bo.BO_E_NO_CANDIDATE:
            return None
        if r.status != self.bo.BO_OK:
            raise RuntimeError(f"tuning step failed with status {r.status}")
        if self.var_s == 0.0:
            self.var_s = r.var_mean
        return r

    def run(self) -> RunTrace:
        self.initial_sample()
        if not self.y:
            return self.tr
        self.mu_s = float(np.mean(np.asarray(self.y)))
        self.var_s = 0.0
        strat, p = self.p.strategy, self.p
        active = [ACQS.index(a) for a in p.order]
        g = p.discount if p.discount is not None else (0.65 if strat == "multi" else 0.75)
        hist = {a: [] for a in active}
        dup = dict.fromkeys(active, 0)
        wins = dict.fromkeys(active, 0)
        misses = dict.fromkeys(active, 0)
        while self.remaining() > 0:
            self._refit()
            if strat in ACQS:
                r = self._step()
                if r is None:
                    break
                a = ACQS.index(strat)
                self._evaluate(int(r.idx[a]), a)
                continue
            if strat == "multi":
                r = self._step()
                if r is None:
                    break
                taken, suggested, cut = {}, {}, False
                for a in active:
                    c = int(r.idx[a])
                    suggested.setdefault(c, []).append(a)
                    if c not in taken:
                        if self.remaining() <= 0:
                            cut = True
                            break
                        taken[c] = self._evaluate(c, a)
                    hist[a].append(self._score(taken[c]))
                for grp in suggested.values():
                    if len(grp) > 1:
                        for a in grp:
                            dup[a] += 1
                if not cut:
                    for grp in suggested.values():
                        if len(grp) < 2 or max(dup[a] for a in grp) <= p.skip_threshold:
                            continue
                        keep = grp[0]
                        for a in grp[1:]:
                            if _dos(hist[a], g) < _dos(hist[keep], g):
                                keep = a
                        active = [a for a in active if a == keep or a not in grp]
                        dup[keep] = 0
                self.tr.active.append(list(active))
                if cut:
                    break
                continue
            # advanced multi
            done = False
            for a in active:
                if self.remaining() <= 0:
                    done = True
                    break
                r = self._step()
                if r is None:
                    done = True
                    break
                hist[a].append(self._score(self._evaluate(int(r.idx[a]), a)))
            if not done and len(active) > 1:
                sc = {a: _dos(hist[a], g) for a in active}
                m = sum(sc[a] for a in active) / len(active)
                for a in active:
                    misses[a] += sc[a] > m * (1.0 + p.improvement)
                    wins[a] += sc[a] < m * (1.0 - p.improvement)
                top = next((a for a in active if wins[a] >= p.skip_threshold), None)
                if top is not None:
                    active = [top]
                else:
                    out = next((a for a in active if misses[a] >= p.skip_threshold), None)
                    if out is not None:
                        active = [a for a in active if a != out]
                        for a in active:
                            wins[a] = misses[a] = 0
            self.tr.active.append(list(active))
            if done:
                break
        return self.tr


def run(bo, levels: Sequence[int], invalid: np.ndarray, evaluate: Callable[[int], float], draws,
        params: LoopParams = LoopParams(), precision="fp64", gp=None, session=None) -> RunTrace:
    """One tuning run; opens a session for the grid unless one is given (a
    given session must hold this grid and at least `params.budget`
    observations)."""
    own = session is None
    if own:
        d = len(levels)
        session = bo.Session(int(np.prod(levels)), d, params.budget, precision, gp=gp)
        session.set_grid(levels, None, invalid)
    try:
        return TuningRun(bo, session, levels, invalid, evaluate, draws, params).run()
    finally:
        if own:
            session.close()
