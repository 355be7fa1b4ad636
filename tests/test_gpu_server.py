"""Serving form (bo_server_*): requests from several sessions submitted in
bursts are batched continuously over two launch contexts; every result must
be, bit for bit, the one the plain single-session path gives for the same history (fit on
the initial sample, rank-1 appends, failed evaluations as visited marks
only).  Memory admission: sessions beyond the HBM budget wait, with their
requests, until a resident session closes."""
import numpy as np
import pytest

from paper_2111_14991_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bo():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2111_14991_amd as bo
    bo.lib()
    return bo


def _sessions(seed, k, n_obs=40):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(k):
        d = int(rng.integers(3, 7))
        lv = tuple(int(v) for v in rng.integers(3, 9, size=d))
        total = int(np.prod(lv))
        cnt = int(min(total, rng.integers(800, 6000)))
        out.append(W.make_session(int(rng.integers(0, 2**31)), lv, n_obs, invalid_frac=float(rng.uniform(0, 0.3)),
                                  cand_count=cnt if cnt < total else None))
    return out


class Alone:
    """The plain single-session path over the same history."""

    def __init__(self, bo, s, precision, n0):
        self.bo, self.s = bo, s
        self.S = bo.Session(s.N, s.d, 64, precision)
        self.S.set_grid(s.levels, s.cand, s.invalid)
        self.obs = list(s.obs_idx[:n0])
        self.y = list(s.y[:n0])
        self.vis = np.zeros(s.N, np.uint8)
        self.vis[s.obs_idx[:n0]] = 1
        self.S.fit(np.array(self.obs), np.array(self.y))

    def step(self, idx, y, valid, acq):
        self.vis[idx] = 1
        if valid:
            self.obs.append(idx)
            self.y.append(y)
            self.S.append(np.array(self.obs), np.array(self.y))
        return self.S.acquire(self.vis, acq, check=False)


def _bits(x):
    return np.float64(x).view(np.uint64)


def _same(rm, ra):
    """Served and plain results are the same bit for bit (the same kernels per
    candidate, the same slot order of the mean variance)."""
    assert rm.status == ra.status, (rm.status, ra.status)
    assert rm.n_unmasked == ra.n_unmasked and rm.n_obs == ra.n_obs
    for f in ("jitter", "f_best", "mean_y", "var_mean", "lam"):
        assert _bits(getattr(rm, f)) == _bits(getattr(ra, f)), (f, getattr(rm, f), getattr(ra, f))
    for q in range(3):
        assert rm.idx[q] == ra.idx[q], (q, rm.idx[q], ra.idx[q])
        assert _bits(rm.score[q]) == _bits(ra.score[q]), (q, rm.score[q], ra.score[q])


def test_server_mix_equals_alone(bo):
    pop = _sessions(1, 8)
    precs = ["fp32", "fp64"] * 4
    n0 = 15
    srv = bo.Server(hbm_budget=8 << 30, max_batch=3, streams=2)
    sids, alone, acqs = [], [], []
    for s, p in zip(pop, precs):
        sids.append(srv.open(s.levels, s.obs_idx[:n0], s.y[:n0], N=s.N, cand=s.cand, invalid=s.invalid, n_max=64,
                             precision=p))
        alone.append(Alone(bo, s, p, n0))
        acqs.append(bo.AcqParams(mode=1, mu_s=float(np.mean(s.y[:n0])), var_s_mean=0.0))
    rng = np.random.Generator(np.random.PCG64(3))
    nxt = [n0] * len(pop)
    for rnd in range(5):
        reqs = []
        for i, s in enumerate(pop):
            if rnd == 2 and i % 3 == 0:
                # a failed evaluation: a not yet visited valid candidate, marked only
                cand = np.flatnonzero((s.invalid == 0) & (alone[i].vis == 0))
                idx, y, valid = int(rng.choice(cand)), 0.0, False
            else:
                idx, y, valid = int(s.obs_idx[nxt[i]]), float(s.y[nxt[i]]), True
                nxt[i] += 1
            reqs.append((i, idx, y, valid))
        # one burst: more requests than a launch holds, so launches queue and overlap
        tickets = [srv.submit(sids[i], idx, y, valid, acqs[i]) for i, idx, y, valid in reqs]
        if rnd % 2 == 0:
            got = [srv.wait(t) for t in tickets]
        else:
            # through the completion queue, a few at a time
            done = {}
            while len(done) < len(tickets):
                for t, r, ms in srv.wait_any(3, 100000):
                    assert t in tickets and t not in done
                    done[t] = (r, ms)
            got = [done[t] for t in tickets]
            assert srv.wait_any(4, 0) == []
        for (i, idx, y, valid), (rm, ms) in zip(reqs, got):
            assert ms > 0.0
            _same(rm, alone[i].step(idx, y, valid, acqs[i]))
    st = srv.stats()
    assert st["steps_done"] == 5 * len(pop) and st["pending"] == 0
    assert st["sessions_resident"] == len(pop) and st["sessions_waiting"] == 0
    assert st["launches"] >= 5 * len(pop) / 3
    srv.close()
    for a in alone:
        a.S.close()


def test_server_memory_admission(bo):
    # four sessions of one problem size; the budget holds two of them
    pop = [W.make_session(40 + i, (6, 5, 5, 4), 40, invalid_frac=0.2) for i in range(4)]
    b = bo.server_session_bytes(pop[0].N, pop[0].d, 64, "fp32")
    srv = bo.Server(hbm_budget=int(2.5 * b), max_batch=8, streams=2)
    n0 = 12
    sids = [srv.open(s.levels, s.obs_idx[:n0], s.y[:n0], N=s.N, cand=s.cand, invalid=s.invalid, n_max=64,
                     precision="fp32") for s in pop]
    st = srv.stats()
    assert st["sessions_resident"] == 2 and st["sessions_waiting"] == 2
    acq = bo.AcqParams(mode=0, lambda_const=0.01)
    tickets = [srv.submit(sid, int(s.obs_idx[n0]), float(s.y[n0]), True, acq) for sid, s in zip(sids, pop)]
    res = {0: srv.wait(tickets[0])[0], 1: srv.wait(tickets[1])[0]}
    # the waiting sessions' requests cannot run before memory frees up
    assert not srv.poll(tickets[2]) and not srv.poll(tickets[3])
    srv.close_session(sids[0])
    res[2] = srv.wait(tickets[2])[0]
    srv.close_session(sids[1])
    res[3] = srv.wait(tickets[3])[0]
    for i, s in enumerate(pop):
        a = Alone(bo, s, "fp32", n0)
        _same(res[i], a.step(int(s.obs_idx[n0]), float(s.y[n0]), True, acq))
        a.S.close()
    st = srv.stats()
    assert st["sessions_resident"] == 2 and st["sessions_waiting"] == 0
    srv.close()


def test_server_errors(bo):
    s = _sessions(4, 1)[0]
    b = bo.server_session_bytes(s.N, s.d, 64, "fp32")
    srv = bo.Server(hbm_budget=b // 2, max_batch=4, streams=1)
    with pytest.raises(bo.BOError) as e:
        srv.open(s.levels, s.obs_idx[:10], s.y[:10], N=s.N, cand=s.cand, invalid=s.invalid, n_max=64)
    assert e.value.status == bo.BO_E_BUDGET
    srv.close()
    srv = bo.Server(hbm_budget=4 * b, max_batch=4, streams=1)
    sid = srv.open(s.levels, s.obs_idx[:10], s.y[:10], N=s.N, cand=s.cand, invalid=s.invalid, n_max=64)
    acq = bo.AcqParams(mode=0)
    with pytest.raises(bo.BOError) as e:
        srv.submit(sid, s.N, 1.0, True, acq)
    assert e.value.status == bo.BO_E_INVALID_ARG
    with pytest.raises(bo.BOError):
        srv.submit(sid + 1, 0, 1.0, True, acq)
    # an evaluation of a restriction-pruned candidate fails that step only
    pruned = np.flatnonzero(s.invalid)
    if pruned.size:
        r, _ = srv.wait(srv.submit(sid, int(pruned[0]), 1.0, True, acq))
        assert r.status == bo.BO_E_INVALID_ARG
    r, _ = srv.wait(srv.submit(sid, int(s.obs_idx[10]), float(s.y[10]), True, acq))
    assert r.status == 0 and r.n_obs == 11
    srv.close()


def test_server_close_while_setting_up(bo):
    # sessions are set up by the server's setup thread; one closed right after
    # it was opened (typically before its setup ends) refuses requests and
    # returns its memory, and the others are not affected
    pop = [W.make_session(60 + i, (6, 5, 5, 4), 40, invalid_frac=0.2) for i in range(3)]
    srv = bo.Server(hbm_budget=8 << 30, max_batch=4, streams=2)
    n0 = 12
    sids = [srv.open(s.levels, s.obs_idx[:n0], s.y[:n0], N=s.N, cand=s.cand, invalid=s.invalid, n_max=64,
                     precision="fp64") for s in pop]
    srv.close_session(sids[0])
    acq = bo.AcqParams(mode=0, lambda_const=0.01)
    with pytest.raises(bo.BOError):
        srv.submit(sids[0], int(pop[0].obs_idx[n0]), float(pop[0].y[n0]), True, acq)
    for i in (1, 2):
        s = pop[i]
        r, _ = srv.wait(srv.submit(sids[i], int(s.obs_idx[n0]), float(s.y[n0]), True, acq))
        a = Alone(bo, s, "fp64", n0)
        _same(r, a.step(int(s.obs_idx[n0]), float(s.y[n0]), True, acq))
        a.S.close()
    b = bo.server_session_bytes(pop[0].N, pop[0].d, 64, "fp64")
    import time
    t_end = time.time() + 10.0
    while time.time() < t_end:
        st = srv.stats()
        if st["sessions_resident"] == 2 and st["bytes_in_use"] == 2 * b:
            break
        time.sleep(0.01)
    assert st["sessions_resident"] == 2 and st["bytes_in_use"] == 2 * b, st
    srv.close()
