"""Serving loop: admission, continuous batching, lanes and latency accounting
(CPU, simulated executor)."""
import threading

import numpy as np
import pytest

import synthetic as syn
from paper_2312_13051_amd import serve as S


def req(L, n=4, kind=S.KIND_WILSON, lo=None):
    hl = syn.bhz_disordered(L, 1.0, [8, L, n]) if L > 1 else syn.bhz()
    kg = syn.kplane(n, n)
    m = hl.N // 2
    return S.Request(hoplist=hl, kappa=kg, lo=0 if lo is None else lo, hi=m, kind=kind)


def test_resident_bytes_counts_vectors_values_and_status():
    r = req(2, 4)
    N, m, nk = r.N, r.m, r.n_k
    assert S.resident_bytes(r) == nk * (N * m * 16 + (m + 2) * 8 + 4)
    ex = S.FakeExecutor(sleep=False, chunk_k=8)
    assert ex.footprint(r) == S.resident_bytes(r) + 8 * N * N * 16


def test_admission_respects_budget_and_all_complete():
    ex = S.FakeExecutor(sleep=False, chunk_k=16)
    reqs = [req(2, 4) for _ in range(5)]
    fp = ex.footprint(reqs[0])
    eng = S.Engine(ex, hbm_budget=int(2.5 * fp))
    for r in reqs:
        eng.submit(r)
    eng.run_until_idle()
    assert len(eng.completed) == 5 and all(r.done.is_set() for r in reqs)
    assert eng.peak_used <= eng.budget
    assert ex.live == 0 and eng.used == 0


def test_continuous_batching_mixes_compatible_requests():
    ex = S.FakeExecutor(sleep=False, chunk_k=10)
    eng = S.Engine(ex, hbm_budget=1 << 40)
    a = eng.submit(req(2, 4))          # 16 k-points
    eng.step()                         # a alone: 10 k-points
    b = eng.submit(req(2, 4))          # arrives while a is in flight
    eng.step()                         # a's last 6 + b's first 4
    eigs = [c for c in ex.calls if c[0] == "eig"]
    assert eigs[0][1] == [a.rid] and eigs[0][2] == 10
    assert eigs[1][1] == [a.rid, b.rid] and eigs[1][2] == 10
    eng.run_until_idle()
    assert a.done.is_set() and b.done.is_set()


def test_incompatible_requests_never_share_a_launch():
    ex = S.FakeExecutor(sleep=False, chunk_k=64)
    eng = S.Engine(ex, hbm_budget=1 << 40)
    for L in (2, 3, 2, 1, 3):
        eng.submit(req(L, 4))
    eng.run_until_idle()   # FakeExecutor asserts one (N, bands, precision) per launch
    assert len(eng.completed) == 5


def test_oversized_request_rejected():
    eng = S.Engine(S.FakeExecutor(sleep=False), hbm_budget=1000)
    with pytest.raises(ValueError):
        eng.submit(req(2, 4))


def test_poisson_stream_latencies():
    ex = S.FakeExecutor(flops_per_s=5e10, sleep=True, chunk_k=16)
    reqs = [req(L, 4) for L in (1, 2, 2, 1, 2, 1)]
    eng = S.Engine(ex, hbm_budget=1 << 40)
    t = S.drive(eng, reqs, S.poisson_arrivals(200.0, len(reqs), [5, 0]))
    st = S.latency_stats(reqs)
    assert st["n"] == 6 and 0 < st["p50_ms"] <= st["p99_ms"]
    assert all(r.t_done >= r.t_admit >= r.t_submit for r in reqs)
    assert t > 0


def test_two_lanes_overlap_different_sizes_never_one_key_twice():
    """Two lanes: launches of different sizes run at the same time, one size
    never on both lanes at once (the executor asserts it), and every request
    completes with its k-points processed in order, once."""
    ex = S.FakeExecutor(flops_per_s=2e9, sleep=True, n_lanes=2, chunk_k=4)
    reqs = [req(L, 4) for L in (3, 1, 3, 2, 1, 3, 2, 1)]
    eng = S.Engine(ex, hbm_budget=1 << 40)
    S.drive(eng, reqs, np.zeros(len(reqs)))
    assert all(r.done.is_set() and r.error is None for r in reqs)
    assert ex.overlaps > 0
    lanes = {c[3] for c in ex.calls if c[0] == "eig"}
    assert lanes == {0, 1}
    assert ex.live == 0 and eng.used == 0


def test_executor_error_is_reported_on_the_request():
    class Failing(S.FakeExecutor):
        def run_eig(self, parts, lane):
            raise RuntimeError("launch failed")

    ex = Failing(sleep=False)
    eng = S.Engine(ex, hbm_budget=1 << 40)
    r = eng.submit(req(2, 4))
    eng.run_until_idle()
    assert r.done.is_set() and isinstance(r.error, RuntimeError) and r.result is None
    assert ex.live == 0 and eng.used == 0


def test_cancel_waiting_request_never_runs():
    ex = S.FakeExecutor(sleep=False, chunk_k=8)
    a, b = req(2, 4), req(2, 4)
    eng = S.Engine(ex, hbm_budget=ex.footprint(a))      # room for one request at a time
    eng.submit(a)
    eng.submit(b)
    eng.step()                                          # a admitted, its first chunk runs; b waits
    assert eng.cancel(b) and b.done.is_set() and isinstance(b.error, S.RequestCancelled)
    eng.run_until_idle()
    assert a.error is None and a.result["n_k"] == a.n_k
    assert all(b.rid not in (c[1] if c[0] == "eig" else [c[1]]) for c in ex.calls)
    assert eng.used == 0 and ex.live == 0 and not eng.cancel(b)


def test_cancel_admitted_request_stops_its_launches_and_frees_memory():
    ex = S.FakeExecutor(sleep=False, chunk_k=4)
    a, c = req(2, 4), req(3, 4)                          # 16 k-points each, different keys
    eng = S.Engine(ex, hbm_budget=1 << 40)
    eng.submit(a)
    eng.submit(c)
    eng.step()                                          # a's first 4 k-points
    assert eng.cancel(a)
    eng.run_until_idle()
    assert isinstance(a.error, S.RequestCancelled) and a.result is None and a.done.is_set()
    assert [k for k in ex.calls if k[0] == "eig" and a.rid in k[1]] == [("eig", [a.rid], 4, 0)]
    assert ("loop", a.rid, 0) not in ex.calls           # no loop stage for a
    assert c.error is None and c.result["n_k"] == c.n_k  # the other request is unaffected
    assert eng.used == 0 and ex.live == 0


def test_timeouts_stop_waiting_and_admitted_requests():
    now = [0.0]
    ex = S.FakeExecutor(sleep=False, chunk_k=4)
    a, b = req(2, 4), req(2, 4)
    a.timeout, b.timeout = 5.0, 1.0
    eng = S.Engine(ex, hbm_budget=ex.footprint(a), clock=lambda: now[0])
    eng.submit(a)
    eng.submit(b)
    eng.step()                                          # a: first chunk; b waits for memory
    now[0] = 2.0                                        # b is past its timeout, a is not
    eng.step()
    assert isinstance(b.error, S.RequestTimeout) and b.done.is_set() and b.t_admit is None
    now[0] = 10.0                                       # now a is too, mid-way through its k-points
    eng.run_until_idle()
    assert isinstance(a.error, S.RequestTimeout) and a.result is None
    assert eng.used == 0 and ex.live == 0


def test_request_log_has_one_line_per_request(tmp_path):
    import json
    log = tmp_path / "requests.jsonl"
    ex = S.FakeExecutor(sleep=False, chunk_k=8)
    a, b, c = req(2, 4), req(2, 4), req(1, 4)
    eng = S.Engine(ex, hbm_budget=ex.footprint(a), log_path=str(log))
    for r in (a, b, c):
        eng.submit(r)
    eng.step()
    eng.cancel(b)
    eng.run_until_idle()
    recs = {r["rid"]: r for r in map(json.loads, log.read_text().splitlines())}
    assert set(recs) == {a.rid, b.rid, c.rid}
    assert recs[a.rid]["outcome"] == "ok" and recs[c.rid]["outcome"] == "ok"
    assert recs[b.rid]["outcome"] == "cancelled" and recs[b.rid]["queue_s"] is None
    ra = recs[a.rid]
    assert (ra["N"], ra["m"], ra["k_points"], ra["kind"]) == (a.N, a.m, a.n_k, "wilson")
    assert ra["latency_s"] >= ra["queue_s"] >= 0.0


def test_srpt_policy_serves_the_smallest_remaining_work_first():
    ex = S.FakeExecutor(sleep=False, chunk_k=8)
    big, small = req(3, 4), req(1, 4)              # same k-points, N = 36 against N = 4
    with pytest.raises(ValueError):
        S.Engine(ex, hbm_budget=1 << 40, policy="lifo")
    eng = S.Engine(ex, hbm_budget=1 << 40, policy="srpt")
    eng.submit(big)
    eng.submit(small)
    eng.run_until_idle()
    eigs = [c[1] for c in ex.calls if c[0] == "eig"]
    assert eigs[0] == [small.rid] and eigs[1] == [small.rid]   # the small request's two chunks go first
    assert small.t_done <= big.t_done and all(r.error is None for r in (big, small))
    ex2 = S.FakeExecutor(sleep=False, chunk_k=8)
    eng2 = S.Engine(ex2, hbm_budget=1 << 40)       # fifo: the older request first
    b2, s2 = eng2.submit(req(3, 4)), eng2.submit(req(1, 4))
    eng2.run_until_idle()
    assert [c[1] for c in ex2.calls if c[0] == "eig"][0] == [b2.rid]
