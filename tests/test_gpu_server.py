"""Build server: each result in a concurrent mix equals the same request built alone
(bit-exact), small budgets queue instead of failing, and admitted builds overlap (GPU only)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    import torch

    import paper_1312_0526_amd as mx

    assert torch.cuda.is_available()
    mx.lib()
    return mx


def _dev(a):
    import torch

    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).cuda()


def _requests():
    """Sizes on both sides of the batching lane's limit (2^17 keys by default)."""
    reqs = []
    for i, n in enumerate([1000, 5000, 200_000, 3_000_000, 777, 60_000, 100, 131_072, 131_073]):
        reqs.append(("u64", _dev(workloads.u64_keys(n, gen_seed=100 + i)), None, 10 + i))
    for i, n in enumerate([2000, 150_000, 1_000_000, 30, 9000]):
        d, o = workloads.str_keys(n, gen_seed=200 + i)
        reqs.append(("str", _dev(d), _dev(o), 20 + i))
    return reqs


def _alone(mx, r):
    kind, a, b, seed = r
    if kind == "u64":
        return mx.mphf_build_u64(a, seed=seed)
    return mx.mphf_build_str(a, b, seed=seed)


def _submit(srv, r):
    kind, a, b, seed = r
    return srv.submit_u64(a, seed=seed) if kind == "u64" else srv.submit_str(a, b, seed=seed)


def test_mix_equals_alone(mx):
    import torch

    reqs = _requests()
    alone = [_alone(mx, r) for r in reqs]
    srv = mx.Server(hbm_budget=8 << 30, slots=4)
    base = srv.stats()["in_use"]  # the batching lane's reserved workspace
    assert base > 0
    tickets = [_submit(srv, r) for r in reqs]
    res = [srv.wait(t) for t in tickets]
    torch.cuda.synchronize()
    for r, a in zip(res, alone):
        assert r["status"] == 0
        assert r["tries"] == a["tries"] and r["seed_used"] == a["seed_used"] and r["P"] == a["P"]
        assert torch.equal(r["codes"], a["codes"]) and torch.equal(r["rank"], a["rank"])
    # overlap: some admitted build started before another one finished
    spans = sorted((r["t_start"], r["t_done"]) for r in res)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["in_use"] == base and st["peak_in_use"] > base
    srv.close()
    # spot-check results against the oracle
    o = oracle.Oracle()
    keys = workloads.u64_keys(5000, gen_seed=101)
    rc, ref = o.mphf_build_u64(keys, seed=11)
    assert np.array_equal(res[1]["codes"].cpu().numpy().view(np.uint64), ref["words"])
    d, of = workloads.str_keys(9000, gen_seed=204)
    rc, ref = o.mphf_build_str(d, of, seed=24)
    assert np.array_equal(res[-1]["codes"].cpu().numpy().view(np.uint64), ref["words"])


def test_tiny_budget_queues_but_never_fails(mx):
    import torch

    reqs = _requests()[:4]
    ws = [(mx.mphf_workspace_bytes(r[1].numel()) + 255) // 256 * 256 for r in reqs]
    budget = max(ws) + 4096
    srv = mx.Server(hbm_budget=budget, slots=4)
    assert srv.stats()["in_use"] == 0  # no room for a batching lane at this budget
    tickets = [_submit(srv, r) for r in reqs]
    res = [srv.wait(t) for t in tickets]
    assert all(r["status"] == 0 for r in res)
    # the workspaces of the builds running at any instant fit in the budget
    for r in res:
        t = r["t_start"]
        live = sum(w for q, w in zip(res, ws) if q["t_start"] <= t < q["t_done"])
        assert live <= budget
    assert srv.stats()["peak_in_use"] <= budget
    alone = [_alone(mx, r) for r in reqs]
    for r, a in zip(res, alone):
        assert torch.equal(r["codes"], a["codes"])
    srv.close()


def test_over_budget_request_fails_fast(mx):
    small = _dev(workloads.u64_keys(1000))
    big = _dev(workloads.u64_keys(1_000_000))
    srv = mx.Server(hbm_budget=mx.mphf_workspace_bytes(1000) + 4096, slots=2)
    tb = srv.submit_u64(big)
    ts = srv.submit_u64(small)
    assert srv.wait(tb)["status"] == mx.ENOMEM
    assert srv.wait(ts)["status"] == 0
    srv.close()


def _n_with_workspace_in(mx, lo, hi):
    """Some n whose build workspace lies in (lo, hi] bytes (bisection on n)."""
    a, b = 1, 1 << 31
    while a < b:
        mid = (a + b) // 2
        if mx.mphf_workspace_bytes(mid) <= lo:
            a = mid + 1
        else:
            b = mid
    assert lo < mx.mphf_workspace_bytes(a) <= hi
    return a


def test_request_beyond_the_lane_reservation_fails_at_once(mx):
    """With the batching lane holding part of the pool, a plain request whose workspace fits the
    budget but not the rest of the pool can never start: it completes with ENOMEM at submission
    instead of blocking the queue (and the server's shutdown) for good."""
    budget = 2 << 30
    srv = mx.Server(hbm_budget=budget, slots=2)
    base = srv.stats()["in_use"]
    assert base > 0  # the lane's reservation
    n = _n_with_workspace_in(mx, budget - base, budget - 4096)
    big = _dev(workloads.u64_keys(n, gen_seed=5))
    tb = srv.submit_u64(big)
    assert srv.poll(tb)["status"] == mx.ENOMEM  # done at submission
    small = _dev(workloads.u64_keys(300_000, gen_seed=6))  # above the lane limit: a plain build
    ts = srv.submit_u64(small, seed=4)
    r = srv.wait(ts)
    assert r["status"] == 0
    a = mx.mphf_build_u64(small, seed=4)
    assert r["seed_used"] == a["seed_used"] and np.array_equal(r["codes"].cpu().numpy(), a["codes"].cpu().numpy())
    srv.close()


def test_small_requests_pass_a_blocked_head_a_bounded_number_of_times(mx):
    """A large request that does not fit beside a running one waits at the queue head; small
    requests behind it that fit are admitted first (continuous admission), but at most 8 of
    them before the head, and every request completes."""
    n_big, n_small, k = 120_000_000, 200_000, 12
    ws_big, ws_small = mx.mphf_workspace_bytes(n_big), mx.mphf_workspace_bytes(n_small)
    budget = (ws_big + 255) // 256 * 256 + 4 * ((ws_small + 255) // 256 * 256) + 4096
    srv = mx.Server(hbm_budget=budget, slots=4, batch_max_keys=0)
    big1 = _dev(workloads.u64_keys(n_big, gen_seed=8))
    big2 = _dev(workloads.u64_keys(n_big, gen_seed=9))
    smalls = [_dev(workloads.u64_keys(n_small, gen_seed=30 + i)) for i in range(k)]
    t1 = srv.submit_u64(big1, seed=1)
    t2 = srv.submit_u64(big2, seed=2)
    ts = [srv.submit_u64(x, seed=40 + i) for i, x in enumerate(smalls)]
    r1, r2 = srv.wait(t1), srv.wait(t2)
    rs = [srv.wait(t) for t in ts]
    assert r1["status"] == 0 and r2["status"] == 0 and all(r["status"] == 0 for r in rs)
    ahead = sum(r["t_start"] < r2["t_start"] for r in rs)
    assert 1 <= ahead <= 8, ahead
    # the two large builds never ran at once: the pool holds only one
    assert r2["t_start"] >= r1["t_done"]
    a = mx.mphf_build_u64(smalls[-1], seed=40 + k - 1)
    assert np.array_equal(rs[-1]["codes"].cpu().numpy(), a["codes"].cpu().numpy())
    srv.close()


def test_shutdown_with_queued_requests_waits_for_the_running_build_only(mx):
    """Destroying the server with requests still queued completes them with MPHX_ECANCELED
    instead of building them: it returns once the build already admitted is done."""
    import time

    import torch

    n, k = 60_000_000, 16
    ws = mx.mphf_workspace_bytes(n)
    keys = [_dev(workloads.u64_keys(n, gen_seed=70 + i)) for i in range(k)]
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        mx.mphf_build_u64(keys[0])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t_one = sorted(times)[1]
    srv = mx.Server(hbm_budget=(ws + 255) // 256 * 256 + 4096, slots=1, batch_max_keys=0)
    for i, x in enumerate(keys):
        srv.submit_u64(x, seed=i)
    assert srv.stats()["pending"] >= k // 2
    t0 = time.perf_counter()
    srv.close()
    t_close = time.perf_counter() - t0
    assert t_close < 3 * t_one, (t_close, t_one)  # building the queue would take about k t_one
