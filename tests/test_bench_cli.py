"""The benchmark's command line on the CPU: more than one GPU is refused with a
message before anything touches a device, and the workload table names every
workload the line can report."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_workload_table():
    sys.path.insert(0, ROOT)
    import bench
    assert set(bench.WORKLOADS) == {"c1", "c2", "c3"}
    assert set(bench.MULTI) == {"c4", "c5", "loop"}
    assert bench.WORKLOADS["c3"]["precision"] == "bf16x3" and bench.WORKLOADS["c3"]["peak"] == "bf16"
    # the traffic summary belongs to the posterior kernel source it was taken on
    t = bench.traffic_from_profile("bf16x3", "c3")
    assert t is None or 4.0e7 < t < 1.0e8


class _InstantServer:
    """Stands in for the serving runtime: every request finishes at once, with
    a result that names the candidate after the one it was given (candidate
    counts of 400)."""

    def __init__(self, result_type):
        self.t = 0
        self.sid = 0
        self.queue = []
        self.closed = []
        self.arr = (result_type * 1024)()
        self.idx_of = {}

    def open(self, *a, **k):
        self.sid += 1
        return self.sid

    def submit(self, sid, idx, y, valid, acq):
        assert valid and y > 0.0
        self.t += 1
        self.queue.append(self.t)
        self.idx_of[self.t] = idx
        return self.t

    def wait_any(self, m, timeout_us, raw=False):
        assert raw
        out = []
        for k, t in enumerate(self.queue[:m]):
            r = self.arr[k]
            r.status = 0
            r.n_unmasked = 10
            r.idx[0] = (self.idx_of.pop(t) + 1) % 400
            out.append((t, r, 0.1))
        del self.queue[:m]
        return out

    def close_session(self, sid):
        self.closed.append(sid)

    def stats(self):
        return {"sessions_setting_up": 0}


class _Member:
    def __init__(self, N, n):
        self.levels, self.N, self.cand, self.n, self.n_init = [N], N, None, n, n
        self.obs_idx = np.arange(n)
        self.y = np.ones(n)
        self.invalid = np.zeros(N, np.uint8)

    def visited(self):
        v = np.zeros(self.N, np.uint8)
        v[:self.n] = 1
        return v


def test_served_load_generator():
    # the serving benchmark's closed loop and Poisson arrivals over a server
    # that answers at once: every session has at most one request in flight,
    # evaluates the candidate its last result named, and retires at 220
    # observations for the next pre-drawn replacement
    sys.path.insert(0, ROOT)
    import bench
    import paper_2111_14991_amd as bo
    rng = np.random.Generator(np.random.PCG64(3))
    pop = [(_Member(400, 200 + i % 20), np.full(400, 2.0)) for i in range(32)]
    spares = [(_Member(400, 10), np.full(400, 2.0)) for _ in range(64)]
    srv = _InstantServer(bo.bo_acq_result)
    pool = bench._ServedPool(srv, bo, None, "fp32", rng, spares, pop)
    starts = {c["sid"]: c["next"] for c in pool.slots}
    r = bench._served_run(pool, None, 50, 500, rng)
    assert r["complete"] and r["requests"] >= 500 and r["left_in_flight"] == 0
    assert sorted(pool.idle) == list(range(32)) and not pool.live
    # sessions that reached 220 observations were closed and replaced
    assert pool.retired == len(srv.closed) > 0
    assert all(c["n"] < 220 for c in pool.slots)
    # a session's next candidate is the one its last result named
    for c in pool.slots:
        if c["sid"] in starts and c["n"] > c["s"].n:
            assert c["next"] == (starts[c["sid"]] + c["n"] - c["s"].n) % 400
    r = bench._served_run(pool, 20000.0, 50, 300, rng)
    assert r["complete"] and r["requests"] >= 300
    assert 0.5 * 20000.0 < r["requests_per_s"] < 2.0 * 20000.0
