#!/usr/bin/env python3
"""Benchmark of the Gaussian-process surrogate BO step on one MI355X.

One step = refit on the session's observations (FP64 Cholesky, jitter,
alpha, L^-1) + posterior over every valid candidate + EI/PI/LCB with the
contextual-variance exploration factor + masked arg-optimum, result on the
host.  Inputs are seeded synthetic landscapes resident in HBM before timing.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c1]

Prints one JSON line: throughput in candidate posterior+acquisition evals/s
(unmasked candidates per step / step time), step latency percentiles, phase
times, the roofline of the posterior kernel and of the whole step, one whole
FP64 CPU oracle step on the same inputs timed on this host, and the error of
every GPU result against that oracle step.
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}  # dense TFLOP/s, MI355X
HBM_GBS = 8000.0

MULTI = {
    "c4": "256 independent sessions (candidates log-uniform in [1e3, 2e5], 3-10 parameters, invalid U[0, 0.4], "
          "10-220 observations), FP32 posterior (FP64 products, FP32 results), FP64 fit, one captured graph "
          "per step (fits, posterior slots, exploration factors, acquisition chunks, selections), "
          "autotuned work order and chunk size",
    "c5": "1024 live sessions (sizes as in c4, 10-200 initial observations), Poisson arrivals of step requests, "
          "rank-1 append per request, 64 GB HBM admission budget, continuous batching",
    "loop": "tuning runs in simulation mode on the 102,060-point 8-parameter grid (25% restricted, 5% failing "
            "when run): maximin LHS initial sample of 20, 200 further evaluations, contextual variance, "
            "advanced multi acquisition (Table I settings)",
}

WORKLOADS = {
    "c3": dict(fn="config_c3", precision="bf16x3", dtype="bf16", peak="bf16",
               desc="1,048,576-point 4^10 grid, 30% invalid, n=1000 observations, BF16X3 posterior"),
    # the FP32 mode at n <= 256 stores FP32 results from FP64 products
    "c2": dict(fn="config_c2", precision="fp32", dtype="fp64", peak="fp64",
               desc="102,060-point 8-parameter grid, 25% invalid, n=220 observations, FP32 posterior "
                    "(FP64 products, FP32 results)"),
    "c1": dict(fn="config_c1", precision="fp64", dtype="fp64", peak="fp64",
               desc="1,536-point 8x8x6x4 grid, 144 invalid, n=20 observations, FP64 posterior"),
}
POSTERIOR_KERNEL = {"bf16x3": "k_post_bf16x3", "fp32": "k_post16r", "fp64": "k_post16r"}
KERNEL_SOURCE = {"bf16x3": "paper_2111_14991_amd/csrc/k_bf16x3.hip", "fp32": "paper_2111_14991_amd/csrc/k_posterior.hip",
                 "fp64": "paper_2111_14991_amd/csrc/k_posterior.hip"}


def source_hash(rel: str) -> str:
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profile(precision: str, workload: str):
    """HBM bytes per launch of the posterior kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{POSTERIOR_KERNEL[precision]}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256_16") != source_hash(KERNEL_SOURCE[precision]):
        return None
    return rec.get("bytes_per_launch")


def _quantiles(err):
    q = np.quantile(err, [0.5, 0.99, 1.0]) if err.size else np.zeros(3)
    return {"median": float(q[0]), "p99": float(q[1]), "max": float(q[2])}


def oracle_step_and_errors(s, S, bo, vis, acq_g, ms_step):
    """One whole FP64 oracle step on the benchmark's inputs, timed on this
    host's cores (the CPU baseline), and the error of every GPU result against
    it: normwise errors (scale floors max|y| for mu and LCB, amp = 1 for the
    variance, 1 for EI and PI) of the mean, variance and the kernel's own EI,
    PI, LCB over all predicted candidates, the scalars, and the chosen
    indices (exact, or within tolerance of the oracle's optimum)."""
    import oracle
    X = oracle.normalize_grid(s.levels, s.cand, s.N)
    n0 = s.n_init
    vis0 = np.zeros(s.N, np.uint8)
    vis0[s.obs_idx[:n0]] = 1
    var_s = oracle.step(X, s.invalid, vis0, s.obs_idx[:n0], s.y[:n0], oracle.GP(), oracle.Acq(mode=0)).var_mean
    oa = oracle.Acq(mode=1, mu_s=float(np.mean(s.y[:n0])), var_s_mean=var_s)
    t0 = time.perf_counter()
    ref = oracle.step(X, s.invalid, vis, s.obs_idx, s.y, oracle.GP(), oa, want_posterior=True)
    t_cpu = time.perf_counter() - t0
    cpu = {"value": ref.n_unmasked / t_cpu, "unit": "candidate-evals/s", "cores": oracle.threads(),
           "kind": "oracle",
           "sample": f"one whole FP64 oracle step on the benchmark's inputs: fit on {s.n} observations, posterior "
                     f"and EI/PI/LCB of all {ref.n_unmasked} predicted candidates, arg-optima ({t_cpu:.2f} s)",
           "step_s": t_cpu, "gpu_speedup": t_cpu / (ms_step * 1e-3)}
    S.fit(s.obs_idx, s.y)
    r, vals = S.acquire_values(vis, acq_g)
    mu, var, _ = S.posterior(vis)
    mu, var = mu.cpu().numpy(), var.cpu().numpy()
    A_g = np.stack([v.cpu().numpy() for v in vals], axis=1)
    mask = (s.invalid | vis).astype(bool)
    keep = ~mask
    A_r = oracle.acquisition_arrays(np.nan_to_num(ref.mu), np.nan_to_num(ref.var), mask, ref.f_best, ref.lam)
    ymax = float(np.abs(s.y).max())
    scales = {"mu": ymax, "var": 1.0, "ei": 1.0, "pi": 1.0, "lcb": ymax}
    got = {"mu": mu, "var": var, "ei": A_g[:, 0], "pi": A_g[:, 1], "lcb": A_g[:, 2]}
    want = {"mu": ref.mu, "var": ref.var, "ei": A_r[:, 0], "pi": A_r[:, 1], "lcb": A_r[:, 2]}
    err = {}
    for k in got:
        g, w = got[k][keep], want[k][keep]
        err[k] = _quantiles(np.abs(g - w) / np.maximum(np.abs(w), scales[k]))
    err["var_mean_rel"] = abs(r.var_mean - ref.var_mean) / ref.var_mean
    err["lambda_rel"] = abs(r.lam - ref.lam) / ref.lam
    agree = []
    for q, name in enumerate(("ei", "pi", "lcb")):
        g, o = int(r.idx[q]), int(ref.idx[q])
        a = A_r[:, q] if q < 2 else -A_r[:, q]
        gap = float(a[o] - a[g]) / max(abs(a[o]), scales[name]) if g >= 0 else float("inf")
        agree.append({"gpu": g, "oracle": o, "equal": g == o, "ref_gap": gap})
    err["indices"] = agree
    err["masks_equal"] = bool(all(np.array_equal(np.isnan(v), mask) for v in got.values()))
    return cpu, err


def _post_flops(N_valid, n, d):
    """Algorithmic flops of one posterior over N_valid candidates (see the
    single-session roofline)."""
    return float(N_valid) * (n * n + (3 * d + 12) * n + 2 * n)


def _cpu_sessions(sessions, budget_s=12.0):
    """FP64 oracle on this host over whole sessions of the population, in order,
    until the budget is spent; returns (evals/s, cores, description)."""
    import oracle
    done_c, t_tot, k = 0, 0.0, 0
    for s in sessions:
        Xo = oracle.normalize_grid(s.levels, s.grid_index(s.obs_idx))
        mask = (s.invalid | s.visited()).astype(bool)
        pool = np.flatnonzero(~mask)
        P = oracle.normalize_grid(s.levels, s.grid_index(pool))
        t0 = time.perf_counter()
        f = oracle.fit(Xo, s.y)
        oracle.predict(f, P)
        t_tot += time.perf_counter() - t0
        done_c += pool.size
        k += 1
        if t_tot > budget_s:
            break
    return done_c / t_tot, oracle.threads(), f"FP64 oracle fit + posterior of the first {k} sessions " \
        f"({done_c} candidates, {t_tot:.2f} s)"


def bench_batched(args, torch, bo, W) -> int:
    pop = W.config_c4(0)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prec = args.precision or "fp32"
    S = []
    for s in pop:
        x = bo.Session(s.N, s.d, 256, prec, device=dev)
        x.set_grid(s.levels, s.cand, s.invalid)
        S.append(x)
    B = bo.Batch(S)
    obs = [torch.as_tensor(s.obs_idx).to(dev) for s in pop]
    ys = [torch.as_tensor(s.y).to(dev) for s in pop]
    vis = [torch.as_tensor(s.visited()).to(dev) for s in pop]
    acqs = [bo.AcqParams(mode=1, mu_s=float(np.mean(s.y[:s.n_init])), var_s_mean=0.0) for s in pop]
    t0 = time.perf_counter()
    cfg = B.tune(obs, ys, vis, acqs, reps=2)
    t_tune = time.perf_counter() - t0
    B.set_timing(True)
    for _ in range(args.warmup):
        res, _ = B.step(obs, ys, vis, acqs)
    torch.cuda.synchronize()
    lat, gms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        res, ms = B.step(obs, ys, vis, acqs)
        lat.append(time.perf_counter() - ts)
        gms.append(ms)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert all(r.status == 0 for r in res), [r.status for r in res if r.status]
    unmasked = sum(int(r.n_unmasked) for r in res)
    ms_per_step = (t1 - t0) / args.steps * 1e3
    # the plain path: the same sessions stepped one after another
    for x, o, y_, v, a in zip(S, obs, ys, vis, acqs):
        x.fit(o, y_)
        x.acquire(v, a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for x, o, y_, v, a in zip(S, obs, ys, vis, acqs):
        x.fit(o, y_)
        x.acquire(v, a)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3
    g = float(np.mean(gms))
    flops = sum(_post_flops(int((s.invalid == 0).sum()), s.n, s.d) for s in pop)
    achieved = flops / (g * 1e-3) / 1e12
    line = {
        "metric": "candidate posterior+acquisition evals/s; BO step p50/p99 latency",
        "value": unmasked / (ms_per_step * 1e-3), "unit": "candidate-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp64", "data": "synthetic",
        "config": {"workload": "c4: " + MULTI["c4"].replace("FP32 posterior (FP64 products, FP32 results)",
                                                           prec.upper() + " posterior"),
                   "sessions": len(pop), "unmasked": unmasked,
                   "candidates": int(sum(s.N for s in pop)), "tuned": cfg, "tune_s": t_tune},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "graph_ms": g,
        "plain_path": {"ms_per_round": plain_ms, "value": unmasked / (plain_ms * 1e-3),
                       "speedup_batched": plain_ms / ms_per_step},
        # the whole graph's time (HIP events around the replay), fits included
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK["fp64"], "traffic": None, "kernel": "graph", "kernel_ms": g},
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        v, cores, desc = _cpu_sessions(pop)
        line["cpu_baseline"] = {"value": v, "unit": "candidate-evals/s", "cores": cores, "kind": "oracle",
                                "sample": desc}
    print(json.dumps(line), flush=True)
    B.close()
    for x in S:
        x.close()
    return 0


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _objective_table(s):
    """Noise-free objective of every candidate of a session (the simulated
    evaluations of the serving run read it; Session.observe's noise is applied
    per evaluation)."""
    return s.landscape.value(s.grid_index(np.arange(s.N)))


class _Draws:
    """A stream of pre-drawn variates (one generator call per block), so that
    the load generator's own cost per request stays small."""

    def __init__(self, draw, block=1 << 16):
        self.draw, self.block = draw, block
        self.buf, self.k = draw(block).tolist(), 0

    def __call__(self):
        if self.k == len(self.buf):
            self.buf, self.k = self.draw(self.block).tolist(), 0
        self.k += 1
        return self.buf[self.k - 1]


class _ServedPool:
    """The serving form's live sessions on one server: each has at most one
    request in flight (BO is sequential), evaluates the EI choice of its last
    result next (closed loop), and retires at 220 observations, when a fresh
    seeded session (drawn before the timed runs, `spares`) takes its place."""

    RETIRE = 220

    def __init__(self, srv, bo, W, prec, rng, spares, population, seed=0):
        self.srv, self.bo, self.W, self.prec, self.rng, self.seed = srv, bo, W, prec, rng, seed
        self.spares = spares
        self.fresh = 0
        self.noise = _Draws(lambda k: rng.standard_normal(k))
        self.slots = [self._open(s, f) for s, f in population]
        self.idle = list(range(len(self.slots)))
        self.live = {}
        self.retired = 0

    def wait_setup(self, limit_s=120.0):
        """Waits until the server has set up every admitted session."""
        t0 = time.perf_counter()
        while self.srv.stats()["sessions_setting_up"] and time.perf_counter() - t0 < limit_s:
            time.sleep(0.01)
        return time.perf_counter() - t0

    def _open(self, s, f):
        sid = self.srv.open(s.levels, s.obs_idx, s.y, N=s.N, cand=s.cand, invalid=s.invalid, n_max=256,
                            precision=self.prec)
        vis = s.visited().astype(bool)
        pool = np.flatnonzero((s.invalid == 0) & ~vis)
        acq = self.bo.AcqParams(mode=1, mu_s=float(np.mean(s.y[:s.n_init])), var_s_mean=0.0)
        return {"s": s, "f": f, "sid": sid, "vis": vis, "n": s.n, "next": int(self.rng.choice(pool)),
                "acq": acq.c()}

    def _replacement(self):
        k = self.fresh
        self.fresh += 1
        if k < len(self.spares):
            return self.spares[k]
        s = self.W.c5_fresh_session(self.seed, k)
        return s, _objective_table(s)

    def take_idle(self, u):
        """Removes and returns the idle session at uniform position u in [0, 1)."""
        idle = self.idle
        k = int(u * len(idle))
        idle[k], idle[-1] = idle[-1], idle[k]
        return idle.pop()

    def submit(self, i, t_arrive):
        c = self.slots[i]
        idx = c["next"]
        # the run-time measurement: the objective with its lognormal noise
        y = c["f"].item(idx) * math.exp(0.02 * self.noise())
        c["vis"][idx] = True
        c["n"] += 1
        self.live[self.srv.submit(c["sid"], idx, y, True, c["acq"])] = (i, t_arrive)

    def collect(self, timeout_us=0):
        """Finished requests (from the server's completion queue, waiting up to
        timeout_us for the first): [(latency from submission ms, latency from
        arrival ms, n_unmasked)]."""
        out = []
        got = self.srv.wait_any(1024, int(timeout_us), raw=True)
        now = time.perf_counter()
        for t, r, ms in got:
            i, t_arrive = self.live.pop(t)
            assert r.status == 0, r.status
            c = self.slots[i]
            c["next"] = r.idx[0]
            out.append((ms, (now - t_arrive) * 1e3, r.n_unmasked))
            if c["n"] >= self.RETIRE:
                self.srv.close_session(c["sid"])
                self.slots[i] = self._open(*self._replacement())
                self.retired += 1
            self.idle.append(i)
        return out


def _served_run(pool, rate, warm, count, rng, limit_s=120.0):
    """Runs until `warm` + `count` requests have finished (or `limit_s`
    seconds); rate None: closed loop (every idle session submits at once: the
    saturated rate), else Poisson arrivals at `rate` requests/s, each to a
    uniformly random idle session (an arrival with no idle session waits for
    one).  Statistics over the finished requests after the first `warm`; the
    mean number of requests inside the server (rate x mean latency) shows
    whether the server or this load generator set the pace."""
    done, lat, e2e, unm = 0, [], [], 0
    t_meas = None
    total = warm + count
    uni = _Draws(lambda k: rng.random(k))
    gap = _Draws(lambda k: rng.exponential(1.0 / rate, k)) if rate else None
    t0 = time.perf_counter()
    t_next = t0
    pending = collections.deque()  # arrival times waiting for an idle session
    t_note = t0
    while done < total and time.perf_counter() - t0 < limit_s:
        if time.perf_counter() - t_note > 20.0:
            t_note = time.perf_counter()
            _progress(f"{done} of {total} requests done")
        now = time.perf_counter()
        if rate is None:
            while pool.idle:
                pool.submit(pool.take_idle(uni()), now)
        else:
            while now >= t_next:
                pending.append(t_next)
                t_next += gap()
            while pending and pool.idle:
                pool.submit(pool.take_idle(uni()), pending.popleft())
        # wait for a completion until the next arrival is due, at most 200 us
        wait_us = 200 if rate is None else max(0.0, min(t_next - time.perf_counter(), 2e-4)) * 1e6
        for ms, ms_e2e, u in pool.collect(wait_us):
            done += 1
            if done == warm:
                t_meas = time.perf_counter()
            elif done > warm:
                lat.append(ms)
                e2e.append(ms_e2e)
                unm += u
    t_run = time.perf_counter() - (t_meas or t0)
    # requests still in flight finish outside this point's statistics; under
    # a budget that holds only some sessions, requests of waiting sessions
    # cannot finish once no request retires a resident one: those are left
    # to the server's close
    t_drain = time.perf_counter() + 10.0
    while pool.live and time.perf_counter() < t_drain:
        pool.collect(1000)
    q = lambda v, p: float(np.percentile(v, p)) if v else None
    rps = len(lat) / t_run
    return {"requests": len(lat), "requests_per_s": rps, "value": unm / t_run,
            "complete": done >= total, "left_in_flight": len(pool.live),
            "latency_ms": {"p50": q(lat, 50), "p99": q(lat, 99), "mean": float(np.mean(lat)) if lat else None},
            "arrival_to_result_ms": {"p50": q(e2e, 50), "p99": q(e2e, 99)},
            "in_server_mean": rps * float(np.mean(lat)) * 1e-3 if lat else None}


def bench_serving(args, torch, bo, W) -> int:
    """Serving form: 1,024 live sessions; the saturated request rate from a
    closed-loop run, then Poisson arrivals at 0.5, 0.6, 0.8, 0.95 and 1.1 times it
    (1,000 warm-up and --requests measured requests each) with a 64 GB
    admission budget, and one run at 0.8 times it with a 512 MB budget that
    forces admission; the plain per-session path (one step at a time, one
    stream, same precision) beside it.  Every run starts from the same 1,024
    sessions on a fresh server (every request adds an observation, so a
    population left from an earlier run would cost more per request than the
    one the saturated rate was measured on)."""
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prec = args.precision or "fp32"
    rng = np.random.Generator(np.random.PCG64(17))
    warm, count = 1000, int(args.requests)
    t0 = time.perf_counter()
    pop = W.config_c5_population(0, 1024)
    population = [(s, _objective_table(s)) for s in pop]
    spares = [(s, _objective_table(s)) for s in (W.c5_fresh_session(0, k) for k in range(320))]
    _progress(f"{len(population)} sessions and {len(spares)} replacements drawn in {time.perf_counter() - t0:.1f} s")

    def fresh(budget):
        srv = bo.Server(hbm_budget=budget, max_batch=args.max_batch, streams=args.streams)
        t0 = time.perf_counter()
        pool = _ServedPool(srv, bo, W, prec, np.random.Generator(np.random.PCG64(18)), spares, population)
        pool.wait_setup()
        return srv, pool, time.perf_counter() - t0

    def finish(srv, pool, res):
        st = srv.stats()
        srv.close()
        res["mean_batch"] = st["mean_batch"]
        res["server_us"] = {"wait_to_launch": st["mean_wait_us"], "launch_call": st["mean_launch_us"],
                            "graph_on_device": st["mean_gpu_us"]}
        res["sessions_retired_and_replaced"] = pool.retired
        return res

    srv, pool, t_open = fresh(64 << 30)
    sat = finish(srv, pool, _served_run(pool, None, warm, count, rng))
    lam = sat["requests_per_s"]
    _progress(f"saturated: {lam:.0f} requests/s, p50 {sat['latency_ms']['p50']} ms")
    sweep = {}
    for f in (0.5, 0.6, 0.8, 0.95, 1.1):
        srv, pool, _ = fresh(64 << 30)
        sweep[str(f)] = finish(srv, pool, dict(_served_run(pool, f * lam, warm, count, rng), rate_rps=f * lam))
        _progress(f"{f} x saturated: {sweep[str(f)]['requests']} requests, p50 {sweep[str(f)]['latency_ms']['p50']} "
                  f"ms, p99 {sweep[str(f)]['latency_ms']['p99']} ms")
    # forced admission: the same sessions under a 512 MB budget
    srv2, pool2, _ = fresh(512 << 20)
    st2_open = srv2.stats()
    forced = finish(srv2, pool2, dict(_served_run(pool2, 0.8 * lam, warm, count, rng), rate_rps=0.8 * lam,
                                      sessions_resident_at_open=st2_open["sessions_resident"],
                                      sessions_waiting_at_open=st2_open["sessions_waiting"]))
    _progress(f"forced admission: {forced['requests']} requests, complete {forced['complete']}")
    # the plain per-session path on the first 64 sessions, one request at a time
    acqs = [bo.AcqParams(mode=1, mu_s=float(np.mean(s.y[:s.n_init])), var_s_mean=0.0) for s in pop[:64]]
    P = []
    for s in pop[:64]:
        x = bo.Session(s.N, s.d, 256, prec, device=dev)
        x.set_grid(s.levels, s.cand, s.invalid)
        o = list(s.obs_idx)
        yv = list(s.y)
        x.fit(np.array(o), np.array(yv))
        P.append([x, o, yv, s.visited()])
    plat, punm = [], 0
    t0 = time.perf_counter()
    for k in range(256):
        i = k % 64
        x, o, yv, v = P[i]
        s = pop[i]
        cand_pool = np.flatnonzero((s.invalid == 0) & (v == 0))
        idx = int(cand_pool[k % cand_pool.size])
        ts = time.perf_counter()
        o.append(idx)
        yv.append(float(s.observe(rng, np.array([idx]))[0]))
        v[idx] = 1
        x.append(np.array(o), np.array(yv))
        r = x.acquire(v, acqs[i])
        plat.append((time.perf_counter() - ts) * 1e3)
        punm += r.n_unmasked
    t_plain = time.perf_counter() - t0
    for x in P:
        x[0].close()
    head = sweep["0.8"]
    line = {
        "metric": "candidate posterior+acquisition evals/s; BO step p50/p99 latency",
        "value": head["value"], "unit": "candidate-evals/s",
        "n_gpus": 1, "steps": head["requests"], "warmup": warm,
        "ms_per_step": 1e3 / head["requests_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp64", "data": "synthetic",
        "config": {"workload": "c5: " + MULTI["c5"] + f" over {args.streams} launch streams of at most "
                   f"{args.max_batch} requests, {prec.upper()} posterior"
                   + (" (FP64 products, FP32 results)" if prec == "fp32" else ""), "sessions": len(pool.slots),
                   "headline_rate": "0.8 x saturated", "open_s": t_open},
        "latency_ms": head["latency_ms"],
        "saturated": sat,
        "sweep": sweep,
        "forced_admission_512MB": forced,
        "plain_path": {"requests": len(plat), "value": punm / t_plain, "requests_per_s": len(plat) / t_plain,
                       "latency_ms": {"p50": float(np.percentile(plat, 50)), "p99": float(np.percentile(plat, 99))}},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_loop(args, torch, bo, W) -> int:
    """Whole tuning runs: `--steps` runs after `--warmup` runs, each a fresh
    draw of the initial design on one simulated problem.  value = BO
    iterations (evaluations chosen by a step) per second."""
    from paper_2111_14991_amd import bo_loop as BL
    precision = args.precision or "fp32"
    sim = W.make_simulation(0, (12, 7, 5, 3, 3, 3, 3, 3), invalid_frac=0.25, hidden_frac=0.05)
    f_opt = float(np.nanmin(sim.table))
    ev = lambda i: float(sim.table[i])
    params = BL.LoopParams()
    S = bo.Session(sim.N, sim.d, params.budget, precision, device="cuda:0")
    S.set_grid(sim.levels, None, sim.invalid)

    def one(r):
        return BL.TuningRun(bo, S, sim.levels, sim.invalid, ev, W.loop_draws(1000 + r, 20, sim.d), params).run()

    for r in range(args.warmup):
        one(r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    traces = [one(args.warmup + r) for r in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = sum(sum(1 for c in t.chooser if c >= 0) for t in traces)
    steps = sum(t.steps for t in traces)
    maes = [BL.mean_abs_error(t.best_after(), f_opt) for t in traces]
    cpu = None
    if not args.no_cpu:
        # one whole oracle run (about 15 s on 8 cores) on the first timed run's problem and draws
        from oracle import loop as OL
        t1 = time.perf_counter()
        tr = OL.run(sim.levels, sim.invalid, ev, W.loop_draws(1000 + args.warmup, 20, sim.d), OL.LoopParams())
        t_cpu = time.perf_counter() - t1
        n_it = sum(1 for c in tr.chooser if c >= 0)
        import oracle
        cpu = {"value": n_it / t_cpu, "unit": "BO iterations/s", "cores": oracle.threads(), "kind": "oracle",
               "sample": f"one oracle tuning run of {len(tr.evaluated)} evaluations ({n_it} chosen by a step) "
                         "on the problem and draws of the first timed run"}
    # strategies compared on the three Table II-sized problems (Section IV-A's MAE and MDF)
    strategies = BL.STRATEGIES
    probs = W.table2_problems(0)
    runs = 5
    mm = np.zeros((len(strategies), len(probs)))
    for k, pr in enumerate(probs):
        Sk = bo.Session(pr.N, pr.d, params.budget, precision, device="cuda:0")
        Sk.set_grid(pr.levels, None, pr.invalid)
        opt = float(np.nanmin(pr.table))
        evk = lambda i, t=pr.table: float(t[i])
        for si, st in enumerate(strategies):
            e = [BL.mean_abs_error(BL.TuningRun(bo, Sk, pr.levels, pr.invalid, evk, W.loop_draws(2000 + r, 20, pr.d),
                                                BL.LoopParams(strategy=st)).run().best_after(), opt)
                 for r in range(runs)]
            mm[si, k] = np.mean(e)
        Sk.close()
    mdf, mdf_sd = BL.mean_deviation_factor(mm)
    line = {
        "metric": "BO iterations/s in simulation-mode tuning runs",
        "value": iters / dt, "unit": "BO iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / max(iters, 1) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "fp64", "fp32": "fp32"}.get(precision, precision), "data": "synthetic",
        "config": {"workload": "loop: " + MULTI["loop"], "configurations": sim.N, "runs": args.steps,
                   "precision": precision, "strategy": params.strategy},
        "ms_per_run": dt / args.steps * 1e3, "gpu_steps": steps,
        "mae": {"mean": float(np.mean(maes)), "std": float(np.std(maes)), "f_opt": f_opt},
        "strategy_comparison": {
            "problems": [f"{p.N} configurations, {int((p.invalid == 0).sum())} unrestricted, "
                         f"{int(p.hidden.sum())} failing" for p in probs],
            "runs": runs, "mean_mae": {st: mm[i].tolist() for i, st in enumerate(strategies)},
            "mdf": {st: [float(mdf[i]), float(mdf_sd[i])] for i, st in enumerate(strategies)}},
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    S.close()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS) + sorted(MULTI))
    ap.add_argument("--requests", type=int, default=10000,
                    help="c5: measured requests per arrival rate (after 1,000 warm-up requests)")
    ap.add_argument("--streams", type=int, default=4, help="c5: the server's launch contexts")
    ap.add_argument("--max-batch", type=int, default=128, help="c5: most requests in one launch")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16x3"], default=None,
                    help="c1-c3: posterior arithmetic other than the workload's own")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB three times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the BO step runs on a single MI355X); --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        return 2

    import torch
    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 3}), flush=True)
        return 0
    import paper_2111_14991_amd as bo
    from paper_2111_14991_amd import workloads as W

    if args.workload == "c4":
        return bench_batched(args, torch, bo, W)
    if args.workload == "c5":
        return bench_serving(args, torch, bo, W)
    if args.workload == "loop":
        return bench_loop(args, torch, bo, W)
    wl = dict(WORKLOADS[args.workload])
    if args.precision and args.precision != wl["precision"]:
        # the FP64 and FP32 modes both take FP64 products
        wl.update(precision=args.precision, dtype="bf16" if args.precision == "bf16x3" else "fp64",
                  peak="bf16" if args.precision == "bf16x3" else "fp64",
                  desc=wl["desc"].rsplit(",", 1)[0] + f", {args.precision.upper()} posterior")
    s = getattr(W, wl["fn"])(0)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    S = bo.Session(s.N, s.d, s.n, wl["precision"], device=dev)
    n_valid = S.set_grid(s.levels, s.cand, s.invalid)
    obs = torch.as_tensor(s.obs_idx).to(dev)
    y = torch.as_tensor(s.y).to(dev)
    vis = torch.as_tensor(s.visited()).to(dev)
    n_unmasked = int(n_valid - s.n)

    # contextual-variance constants from the initial sample (Section III-F)
    n0 = s.n_init
    vis0 = torch.zeros_like(vis)
    vis0[obs[:n0]] = 1
    S.fit(obs[:n0].contiguous(), y[:n0].contiguous())
    var_s = S.acquire(vis0, bo.AcqParams(mode=0)).var_mean
    acq = bo.AcqParams(mode=1, mu_s=float(np.mean(s.y[:n0])), var_s_mean=var_s)

    S.set_timing(True)
    for _ in range(args.warmup):
        S.fit(obs, y)
        r = S.acquire(vis, acq)
    torch.cuda.synchronize()
    lat, phases = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        S.fit(obs, y)
        r = S.acquire(vis, acq)
        lat.append(time.perf_counter() - ts)
        phases.append(S.timing())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert r.status == 0 and r.n_unmasked == n_unmasked, (r.status, r.n_unmasked, n_unmasked)

    ms_per_step = (t1 - t0) / args.steps * 1e3
    ph = np.array(phases)
    post_ms = float(ph[:, 1].mean())
    n, d = s.n, s.d
    peak = PEAK[wl["peak"]]
    # algorithmic work of the posterior: the triangular solve, n^2 flops per
    # predicted candidate (distance, Matern and mean add (3d + 14) n)
    flops = float(n_unmasked) * n * n
    achieved = flops / (post_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic_from_profile(wl["precision"], args.workload),
                "kernel": POSTERIOR_KERNEL[wl["precision"]] + ("big" if wl["precision"] != "bf16x3" and n > 256 else ""),
                "kernel_ms": post_ms,
                "flops_per_launch": flops}
    fit_flops = 2.0 * n ** 3 / 3.0  # Cholesky n^3/3 + triangular inverse n^3/3, FP64
    if wl["precision"] == "bf16x3":
        # three bfloat16 products per multiply-add of the compensated contraction
        mfma = 3.0 * flops
        roofline["mfma_issued_tflops"] = mfma / (post_ms * 1e-3) / 1e12
        roofline["mfma_issued_frac"] = roofline["mfma_issued_tflops"] / peak
        roofline["graded_step_frac"] = (mfma / (PEAK["bf16"] * 1e12) + fit_flops / (PEAK["fp64"] * 1e12)) / \
            (ms_per_step * 1e-3)
    else:
        roofline["graded_step_frac"] = (flops / (peak * 1e12) + fit_flops / (PEAK["fp64"] * 1e12)) / \
            (ms_per_step * 1e-3)

    line = {
        "metric": "candidate posterior+acquisition evals/s; BO step p50/p99 latency",
        "value": n_unmasked / (ms_per_step * 1e-3),
        "unit": "candidate-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": wl["dtype"], "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "candidates": int(s.N), "valid": int(n_valid),
                   "unmasked": n_unmasked, "observations": int(n), "dims": int(d), "precision": wl["precision"]},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                       "mean": float(np.mean(lat) * 1e3)},
        "phases_ms": {"fit": float(ph[:, 0].mean()), "posterior": post_ms, "acquire": float(ph[:, 2].mean())},
        "roofline": roofline,
        "cpu_baseline": None,
        "chosen": [int(v) for v in r.idx],
    }
    if not args.no_cpu:
        line["cpu_baseline"], line["error_vs_oracle"] = oracle_step_and_errors(s, S, bo, s.visited(), acq,
                                                                                ms_per_step)
    print(json.dumps(line), flush=True)
    S.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
