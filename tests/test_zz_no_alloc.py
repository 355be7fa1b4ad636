"""bo_step_noalloc (one whole step over the library's static device array, no
session, no workspace, no allocation) against the session entry points it
stands for: bo_session_create + bo_set_candidates + bo_gp_fit + bo_acquire on
the same arguments.  Both run the same kernels in the same order, so every
field of the result must be identical.  Two calls in a row, the second on a
smaller problem (the array keeps the first call's contents), then a problem
too large for the array (refused on the host, nothing enqueued)."""
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


def _coords(s):
    gidx = np.arange(s.N, dtype=np.int64) if s.cand is None else s.cand
    lv = W.decode_levels(s.levels, gidx)
    k = np.asarray(s.levels, dtype=np.float64)
    return lv.astype(np.float64) / np.where(k > 1, k - 1, 1.0)


def _both(bo, s, precision, visited):
    import torch
    X = torch.as_tensor(_coords(s), device="cuda")
    if precision != "fp64":
        X = X.to(torch.float32)
    mu_s = float(np.mean(s.y[:s.n_init]))
    acq = bo.AcqParams(mode=1, mu_s=mu_s)
    S = bo.Session(s.N, s.d, s.n, precision)
    S.set_candidates(X, s.invalid)
    S.fit(s.obs_idx, s.y)
    ref = S.acquire(visited, acq)
    S.close()
    print(f"noalloc case: {s.name or 'session'} N={s.N} d={s.d} n={s.n} {precision}", flush=True)
    got = bo.bo_step_noalloc(X, s.obs_idx, s.y, precision, invalid=s.invalid, visited=visited, acq=acq)
    return got, ref


def _same(got, ref):
    assert got.status == ref.status == 0
    assert list(got.idx) == list(ref.idx)
    np.testing.assert_array_equal(got.score, ref.score)
    for f in ("lam", "var_mean", "jitter", "f_best", "mean_y", "n_unmasked", "n_obs"):
        assert getattr(got, f) == getattr(ref, f), f


def test_noalloc_equals_session_two_calls(bo):
    big = W.config_c2(3)            # 102,060 candidates, n = 220 (multi-workgroup fit)
    got, ref = _both(bo, big, "fp32", big.visited())
    _same(got, ref)
    small = W.config_c1(4)          # 1,536 candidates, n = 20, on the same array
    got2, ref2 = _both(bo, small, "fp64", small.visited())
    _same(got2, ref2)
    # visited = NULL: nothing evaluated yet, against the session's own (empty) record
    got3, ref3 = _both(bo, small, "fp64", None)
    _same(got3, ref3)


def test_noalloc_refuses_beyond_the_array(bo):
    import torch
    X = torch.zeros((1 << 20, 10), dtype=torch.float32, device="cuda")
    with pytest.raises(bo.BOError) as e:
        bo.bo_step_noalloc(X, np.arange(1000), np.ones(1000), "bf16x3")
    assert e.value.status == bo.BO_E_WORKSPACE
    assert "static scratch" in bo.last_error()
