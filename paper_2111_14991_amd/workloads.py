"""Seeded synthetic inputs for the BO surrogate step.

This module only *draws* inputs: discrete search spaces (value-list lengths per
parameter and, optionally, a subset of the grid), restriction masks, a synthetic
objective standing in for measured kernel run times, and observation lists.  It
holds none of the method's arithmetic (no normalization of the candidate
matrix, no covariance, no posterior, no acquisition).  Both the FP64 oracle and
the HIP path consume its outputs.

Stand-ins for the paper's measured search spaces (Section IV-A, Tables II and
III: 4,654 to 17,956 configurations, 5 to 15 parameters, 0 to 50.8% invalid),
which are not available: every space here is a Cartesian grid of integer levels,
pruned by seeded restrictions, with a positive objective in milliseconds.

Objective (all workloads):
    f(p) = 1 + sum_{b<6} a_b exp(-1/2 sum_j ((u_j - c_bj) / s_bj)^2)
             + 0.05 sin(2 pi sum_j w_j u_j + phi0)
where u_j = i_j / (k_j - 1) is the position of level i_j of parameter j on the
unit interval (0 for a one-level parameter) -- the objective's own coordinate
system.  a_b ~ U[0.5, 2], c_bj ~ U[0, 1], s_bj ~ U[0.1, 0.5], w_j ~ U[4, 8],
phi0 ~ U[0, 2 pi).  An observation is y = f(p) exp(0.02 eps), eps ~ N(0, 1).

Random draws use numpy.random.Generator(PCG64(seed)) in a fixed order:
landscape, restrictions, observations, observation noise.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Landscape", "Session", "grid_size", "decode_levels", "make_landscape",
    "product_restriction", "quantile_restrictions", "make_session",
    "config_c1", "config_c2", "config_c3", "config_c4", "config_c5_population",
    "tiny_session", "Simulation", "make_simulation", "LoopDraws", "loop_draws", "table2_problems",
]


def grid_size(levels: Sequence[int]) -> int:
    n = 1
    for k in levels:
        n *= int(k)
    return n


def decode_levels(levels: Sequence[int], grid_idx: np.ndarray) -> np.ndarray:
    """Level index of every parameter for each grid index (row-major, last
    parameter fastest).  Returns an int16 array of shape (len(grid_idx), d)."""
    g = np.asarray(grid_idx, dtype=np.int64).copy()
    d = len(levels)
    out = np.empty((g.shape[0], d), dtype=np.int16)
    for j in range(d - 1, -1, -1):
        k = int(levels[j])
        out[:, j] = g % k
        g //= k
    return out


def _unit_positions(levels: Sequence[int], lv: np.ndarray) -> np.ndarray:
    k = np.asarray(levels, dtype=np.float64)
    den = np.where(k > 1, k - 1, 1.0)
    return lv.astype(np.float64) / den


@dataclass
class Landscape:
    """Synthetic run-time landscape over a discrete grid (milliseconds, > 0)."""
    levels: tuple
    a: np.ndarray
    c: np.ndarray
    s: np.ndarray
    w: np.ndarray
    phi0: float

    def value(self, grid_idx: np.ndarray) -> np.ndarray:
        u = _unit_positions(self.levels, decode_levels(self.levels, grid_idx))
        acc = np.ones(u.shape[0])
        for b in range(self.a.shape[0]):
            q = ((u - self.c[b]) / self.s[b]) ** 2
            acc += self.a[b] * np.exp(-0.5 * q.sum(axis=1))
        acc += 0.05 * np.sin(2.0 * np.pi * (u @ self.w) + self.phi0)
        return acc


def make_landscape(rng: np.random.Generator, levels: Sequence[int], bumps: int = 6) -> Landscape:
    d = len(levels)
    a = rng.uniform(0.5, 2.0, size=bumps)
    c = rng.uniform(0.0, 1.0, size=(bumps, d))
    s = rng.uniform(0.1, 0.5, size=(bumps, d))
    w = rng.uniform(4.0, 8.0, size=d)
    phi0 = float(rng.uniform(0.0, 2.0 * np.pi))
    return Landscape(tuple(int(k) for k in levels), a, c, s, w, phi0)


def product_restriction(levels: Sequence[int], grid_idx: np.ndarray, p: int, q: int, limit: int) -> np.ndarray:
    """Invalid where level(p) * level(q) > limit (0-based level indices)."""
    lv = decode_levels(levels, grid_idx).astype(np.int64)
    return (lv[:, p] * lv[:, q] > limit).astype(np.uint8)


def quantile_restrictions(rng: np.random.Generator, levels: Sequence[int], grid_idx: np.ndarray,
                          target: float, tol: float = 0.005) -> np.ndarray:
    """Three seeded restrictions: two linear (w . u over a random parameter
    subset exceeds a threshold) and one product (u_a * u_b exceeds a threshold).
    Each threshold is the (1 - q) quantile of its score over the candidates;
    one common q is set by bisection so that the union of the three removes
    `target` of the candidates (within `tol` where the grid allows)."""
    d = len(levels)
    n = grid_idx.shape[0]
    u = _unit_positions(levels, decode_levels(levels, grid_idx))
    scores = []
    for _ in range(2):
        m = int(rng.integers(2, min(d, 4) + 1)) if d >= 2 else 1
        dims = rng.choice(d, size=m, replace=False)
        wts = rng.uniform(0.5, 1.5, size=m)
        scores.append(u[:, dims] @ wts)
    if d >= 2:
        pa, pb = rng.choice(d, size=2, replace=False)
    else:
        pa = pb = 0
    scores.append(u[:, pa] * u[:, pb])
    if target <= 0.0 or n == 0:
        return np.zeros(n, dtype=np.uint8)
    sorted_scores = [np.sort(sc) for sc in scores]

    def union(qv: float) -> np.ndarray:
        inv = np.zeros(n, dtype=bool)
        for sc, srt in zip(scores, sorted_scores):
            pos = min(n - 1, max(0, int(np.floor((1.0 - qv) * (n - 1)))))
            inv |= sc > srt[pos]
        return inv

    lo, hi = 0.0, 1.0
    best = union(target)
    best_err = abs(best.mean() - target)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        inv = union(mid)
        frac = inv.mean()
        err = abs(frac - target)
        if err < best_err:
            best, best_err = inv, err
        if err <= tol:
            break
        if frac < target:
            lo = mid
        else:
            hi = mid
    return best.astype(np.uint8)


@dataclass
class Session:
    """One tuning session's inputs.

    `levels` are the value-list lengths of the parameters.  `cand` holds the grid
    index of every candidate in the caller's enumeration (None: the full grid in
    row-major order, last parameter fastest).  `invalid` and indices in `obs_idx`
    refer to that enumeration.  `obs_idx`/`y` are the valid observations in
    observation order; the first `n_init` of them form the initial sample."""
    levels: tuple
    cand: Optional[np.ndarray]
    invalid: np.ndarray
    obs_idx: np.ndarray
    y: np.ndarray
    landscape: Landscape
    n_init: int = 20
    seed: int = 0
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.invalid.shape[0])

    @property
    def d(self) -> int:
        return len(self.levels)

    @property
    def n(self) -> int:
        return int(self.obs_idx.shape[0])

    def grid_index(self, idx: np.ndarray) -> np.ndarray:
        idx = np.asarray(idx, dtype=np.int64)
        return idx if self.cand is None else self.cand[idx]

    def visited(self) -> np.ndarray:
        v = np.zeros(self.N, dtype=np.uint8)
        v[self.obs_idx] = 1
        return v

    def observe(self, rng: np.random.Generator, idx: np.ndarray) -> np.ndarray:
        f = self.landscape.value(self.grid_index(idx))
        return f * np.exp(0.02 * rng.standard_normal(f.shape[0]))


def make_session(seed: int, levels: Sequence[int], n_obs: int, *, invalid_rule: str = "quantile",
                 invalid_frac: float = 0.25, cand_count: Optional[int] = None,
                 rng: Optional[np.random.Generator] = None, name: str = "") -> Session:
    """Draw one session: landscape, restrictions, then `n_obs` valid observations
    uniformly without replacement, then their noise."""
    rng = np.random.Generator(np.random.PCG64(seed)) if rng is None else rng
    levels = tuple(int(k) for k in levels)
    total = grid_size(levels)
    land = make_landscape(rng, levels)
    cand = None
    if cand_count is not None and cand_count < total:
        cand = np.sort(rng.permutation(total)[:cand_count]).astype(np.int64)
    gidx = np.arange(total, dtype=np.int64) if cand is None else cand
    if invalid_rule == "c1":
        invalid = product_restriction(levels, gidx, 0, 1, 30)
    elif invalid_rule == "none":
        invalid = np.zeros(gidx.shape[0], dtype=np.uint8)
    else:
        invalid = quantile_restrictions(rng, levels, gidx, invalid_frac)
    valid = np.flatnonzero(invalid == 0)
    n_obs = min(int(n_obs), valid.shape[0])
    obs_idx = rng.choice(valid, size=n_obs, replace=False).astype(np.int64)
    sess = Session(levels, cand, invalid, obs_idx, np.zeros(0), land, min(20, n_obs), seed, name)
    sess.y = sess.observe(rng, obs_idx)
    sess.extra["rng"] = rng
    return sess


def config_c1(seed: int = 0) -> Session:
    """Plain FP64 step: levels (8, 8, 6, 4), 1,536 points; invalid where
    level0 * level1 > 30 (144 points); 20 valid observations."""
    return make_session(seed, (8, 8, 6, 4), 20, invalid_rule="c1", name="c1")


def config_c2(seed: int = 0) -> Session:
    """Single session, FP32: levels (12, 7, 5, 3, 3, 3, 3, 3), 102,060 points,
    25% invalid from three restrictions; 220 valid observations."""
    return make_session(seed, (12, 7, 5, 3, 3, 3, 3, 3), 220, invalid_frac=0.25, name="c2")


def config_c3(seed: int = 0) -> Session:
    """Precision form: 4^10 = 1,048,576 points, 30% invalid; 1,000 observations."""
    return make_session(seed, (4,) * 10, 1000, invalid_frac=0.30, name="c3")


def _population_member(rng: np.random.Generator, seed: int, n_lo: int, n_hi: int) -> Session:
    n_s = int(round(float(np.exp(rng.uniform(np.log(1e3), np.log(2e5))))))
    d_s = int(rng.integers(3, 11))
    k = int(np.ceil(n_s ** (1.0 / d_s) - 1e-12))
    levels = (k,) * d_s
    while grid_size(levels) < n_s:
        k += 1
        levels = (k,) * d_s
    frac = float(rng.uniform(0.0, 0.4))
    n_obs = int(rng.integers(n_lo, n_hi + 1))
    sub_seed = int(rng.integers(0, 2**63 - 1))
    return make_session(sub_seed, levels, n_obs, invalid_frac=frac, cand_count=n_s, name=f"s{seed}")


def config_c4(seed: int = 0, sessions: int = 256) -> List[Session]:
    """Batched form: `sessions` independent sessions; candidate counts
    log-uniform in [1e3, 2e5], 3 to 10 parameters with ceil(N^(1/d)) levels each
    (the candidates are the first N of a seeded permutation of that grid),
    invalid fraction U[0, 0.4], 10 to 220 valid observations."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [_population_member(rng, seed, 10, 220) for _ in range(sessions)]


def config_c5_population(seed: int = 0, sessions: int = 1024) -> List[Session]:
    """Serving form: live sessions drawn as in the batched form, each starting
    with 10 to 200 observations (they retire at 220)."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    return [_population_member(rng, seed, 10, 200) for _ in range(sessions)]


def c5_fresh_session(seed: int, k: int) -> Session:
    """The k-th replacement session of the serving form (drawn as the
    population's members, from its own seeded generator): a live session
    retires at 220 observations and a fresh one takes its place."""
    rng = np.random.Generator(np.random.PCG64([seed + 7919, k + 1]))
    return _population_member(rng, seed, 10, 200)


def tiny_session(seed: int, levels: Sequence[int] = (4, 3, 5), n_obs: int = 5,
                 invalid_frac: float = 0.2) -> Session:
    """A few-dozen-point space for brute-force checks."""
    return make_session(seed, levels, n_obs, invalid_frac=invalid_frac, name="tiny")


# ---------------------------------------------------------------------------
# Tuning runs in simulation mode (the outer loop around the step)


@dataclass
class Simulation:
    """A cached tuning problem: the run time of every configuration drawn once
    (a measurement cache replayed by the loop), restrictions known before
    tuning (`invalid`, pruned from the search), and configurations that only
    fail when run (`hidden`, unknown to the optimizer until evaluated).
    `table` is NaN where a configuration is invalid or fails."""
    levels: tuple
    invalid: np.ndarray
    hidden: np.ndarray
    table: np.ndarray
    seed: int = 0

    @property
    def N(self) -> int:
        return int(self.invalid.shape[0])

    @property
    def d(self) -> int:
        return len(self.levels)


def make_simulation(seed: int, levels: Sequence[int], invalid_frac: float = 0.2,
                    hidden_frac: float = 0.05) -> Simulation:
    """Landscape, restrictions, failing configurations (each restriction-valid
    configuration with probability `hidden_frac`), then one noisy measurement
    per configuration, drawn in that order from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    levels = tuple(int(k) for k in levels)
    total = grid_size(levels)
    land = make_landscape(rng, levels)
    g = np.arange(total, dtype=np.int64)
    invalid = quantile_restrictions(rng, levels, g, invalid_frac)
    hidden = ((rng.random(total) < hidden_frac) & (invalid == 0)).astype(np.uint8)
    f = land.value(g) * np.exp(0.02 * rng.standard_normal(total))
    table = np.where((invalid == 0) & (hidden == 0), f, np.nan)
    return Simulation(levels, invalid, hidden, table, seed)


@dataclass
class LoopDraws:
    """The random numbers one tuning run consumes.  `perm[m, j]` is a
    permutation of the `samples` strata of parameter j in Latin hypercube
    design m and `off[m, j]` the positions within the strata (uniform on
    [0, 1)); `repl` is a stream of uniforms for the random replacements of
    invalid initial samples."""
    perm: np.ndarray
    off: np.ndarray
    repl: np.ndarray


def loop_draws(seed: int, samples: int, d: int, designs: int = 32, repl: int = 4096) -> LoopDraws:
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = np.empty((designs, d, samples), dtype=np.int64)
    for m in range(designs):
        for j in range(d):
            perm[m, j] = rng.permutation(samples)
    off = rng.random((designs, d, samples))
    return LoopDraws(perm, off, rng.random(repl))


def table2_problems(seed: int = 0) -> List[Simulation]:
    """Three simulated problems sized like the paper's test kernels (Table II):
    a 82,944-point 9-parameter grid restricted to about 17,956 configurations
    with none failing; an 18,432-point 7-parameter grid restricted to about
    9,400 of which 38.5% fail when run; an 8,184-point 6-parameter grid,
    unrestricted, 3.9% failing.  Synthetic landscapes stand in for the
    measured run times, which are not available."""
    return [
        make_simulation(seed * 3 + 1, (4, 4, 4, 4, 4, 3, 3, 3, 3), invalid_frac=1 - 17956 / 82944, hidden_frac=0.0),
        make_simulation(seed * 3 + 2, (8, 8, 6, 4, 3, 2, 2), invalid_frac=1 - 9400 / 18432, hidden_frac=0.385),
        make_simulation(seed * 3 + 3, (31, 11, 3, 2, 2, 2), invalid_frac=0.0, hidden_frac=0.039),
    ]
