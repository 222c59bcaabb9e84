"""Serving loop: admission, continuous batching and latency accounting (CPU, fake executor)."""
import numpy as np
import pytest

import synthetic as syn
from paper_2312_13051_amd import serve as S


def req(L, n=4, kind=S.KIND_WILSON, lo=None):
    hl = syn.bhz_disordered(L, 1.0, [8, L, n]) if L > 1 else syn.bhz()
    kg = syn.kplane(n, n)
    m = hl.N // 2
    return S.Request(hoplist=hl, kappa=kg, lo=0 if lo is None else lo, hi=m, kind=kind)


def test_footprint_counts_resident_vectors_and_h_chunk():
    r = req(2, 4)
    N, m, nk = r.N, r.m, r.n_k
    fp = S.footprint_bytes(r, chunk_k=8)
    assert fp == nk * (N * m * 16 + (m + 2) * 8 + 4) + 8 * N * N * 16


def test_admission_respects_budget_and_all_complete():
    ex = S.FakeExecutor(sleep=False)
    reqs = [req(2, 4) for _ in range(5)]
    fp = S.footprint_bytes(reqs[0], 16)
    eng = S.Engine(ex, hbm_budget=int(2.5 * fp), chunk_k=16)
    for r in reqs:
        eng.submit(r)
    eng.run_until_idle()
    assert len(eng.completed) == 5 and all(r.done.is_set() for r in reqs)
    assert eng.peak_used <= eng.budget
    assert ex.live == 0 and eng.used == 0


def test_continuous_batching_mixes_compatible_requests():
    ex = S.FakeExecutor(sleep=False)
    eng = S.Engine(ex, hbm_budget=1 << 40, chunk_k=10)
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
    ex = S.FakeExecutor(sleep=False)
    eng = S.Engine(ex, hbm_budget=1 << 40, chunk_k=64)
    for L in (2, 3, 2, 1, 3):
        eng.submit(req(L, 4))
    eng.run_until_idle()   # FakeExecutor asserts one (N, bands, precision) per launch
    assert len(eng.completed) == 5


def test_oversized_request_rejected():
    eng = S.Engine(S.FakeExecutor(sleep=False), hbm_budget=1000)
    with pytest.raises(ValueError):
        eng.submit(req(2, 4))


def test_poisson_stream_latencies():
    ex = S.FakeExecutor(flops_per_s=5e10, sleep=True)
    reqs = [req(L, 4) for L in (1, 2, 2, 1, 2, 1)]
    eng = S.Engine(ex, hbm_budget=1 << 40, chunk_k=16)
    t = S.drive(eng, reqs, S.poisson_arrivals(200.0, len(reqs), [5, 0]))
    st = S.latency_stats(reqs)
    assert st["n"] == 6 and 0 < st["p50_ms"] <= st["p99_ms"]
    assert all(r.t_done >= r.t_admit >= r.t_submit for r in reqs)
    assert t > 0
