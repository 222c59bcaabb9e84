"""Served streams on the GPU: every request's result is the same alone and in
the mix (continuous batching, two lanes), and equals the oracle."""
import numpy as np
import pytest

import synthetic as syn
from oracle import berry as orc
from tests import gpu_util as gu
from tests.phase_metrics import phase_set_error

torch = gu.torch
pytestmark = pytest.mark.gpu


def make_requests(S):
    kg = syn.kplane(8, 6)
    reqs = []
    for r in range(3):
        hl = syn.bhz_disordered(3, 4.0 * (r + 1) / 4, [5, 1, r])
        reqs.append(S.Request(hoplist=hl, kappa=kg, lo=0, hi=hl.N // 2, kind=S.KIND_SPIN,
                              spin_diag=syn.bhz_spin_diag(hl)))
    wl = syn.wannier_like(16, [5, 2, 0])
    reqs.append(S.Request(hoplist=wl, kappa=kg, lo=0, hi=8, kind=S.KIND_WILSON))
    reqs.append(S.Request(hoplist=syn.bbh(0.5, 1.0), kappa=syn.kplane(12, 12), lo=0, hi=2, kind=S.KIND_NESTED))
    hl = syn.bhz_disordered(3, 2.0, [5, 1, 9])
    reqs.append(S.Request(hoplist=hl, kappa=kg, lo=0, hi=hl.N // 2, kind=S.KIND_WILSON))
    reqs.append(S.Request(hoplist=syn.qwz(1.5), kappa=syn.kplane(10, 8), lo=0, hi=1, kind=S.KIND_FLUX))
    hl = syn.bhz_disordered(3, 1.0, [5, 1, 7])
    reqs.append(S.Request(hoplist=hl, kappa=kg, lo=0, hi=hl.N // 2, kind=S.KIND_SPIN_FLUX,
                          spin_diag=syn.bhz_spin_diag(hl)))
    return reqs


def circ(a, b):
    return float(np.max(np.abs(np.mod(np.asarray(a) - np.asarray(b) + np.pi, 2 * np.pi) - np.pi)))


def alone(S, reqs, budget=8 << 30):
    out = []
    ex = S.GpuExecutor(n_lanes=1, chunk_cap=64)
    for r in reqs:
        e1 = S.Engine(ex, hbm_budget=budget)
        e1.submit(r)
        e1.run_until_idle()
        assert r.error is None
        out.append(r.result)
    return out


def test_served_mix_equals_alone():
    gu.need_gpu()
    from paper_2312_13051_amd import serve as S
    ex = S.GpuExecutor(n_lanes=2, chunk_cap=64)
    mix = make_requests(S)
    eng = S.Engine(ex, hbm_budget=8 << 30)
    # the first half arrives together (so compatible requests must share
    # launches); the rest follow as a Poisson stream while those run
    arr = np.concatenate([np.zeros(3), S.poisson_arrivals(500.0, len(mix) - 3, [5, 0])])
    S.drive(eng, mix, arr)
    assert all(r.error is None for r in mix)
    launches_with_two = [s for s in eng.step_log if len(s["requests"]) > 1]
    assert launches_with_two, "continuous batching never mixed two requests"
    ref_alone = alone(S, make_requests(S))
    for a, b, r in zip(ref_alone, [x.result for x in mix], mix):
        if r.kind == S.KIND_SPIN:
            md = b["m_dn"][0]
            assert a["m_dn"] == b["m_dn"]
            assert phase_set_error(a["theta_dn"][0, :, :md], b["theta_dn"][0, :, :md]) < 1e-10
            assert phase_set_error(a["theta_up"][0, :, :r.m - md], b["theta_up"][0, :, :r.m - md]) < 1e-10
            assert int(a["C_dn"][0]) == int(b["C_dn"][0])
        elif r.kind == S.KIND_NESTED:
            assert abs(float(a["p_mean"][0]) - float(b["p_mean"][0])) < 1e-10
            assert abs(float(b["p_mean"][0]) - 0.5) < 1e-10
        elif r.kind == S.KIND_FLUX:
            ref = orc.plaquette_flux(r.hoplist, r.kappa, r.lo, r.hi)
            assert circ(a["flux"][0], b["flux"][0]) < 1e-10 and circ(b["flux"][0], ref["flux"]) < 1e-10
            assert int(b["chern"][0]) == ref["chern"] == 1
        elif r.kind == S.KIND_SPIN_FLUX:
            ref = orc.spin_resolved_flux(r.hoplist, r.spin_diag, r.kappa, r.lo, r.hi)
            assert a["m_dn"] == b["m_dn"] == [ref["m_dn"]]
            for key in ("flux_dn", "flux_up"):
                assert circ(a[key][0], b[key][0]) < 1e-10 and circ(b[key][0], ref[key]) < 1e-10
            assert float(b["C_s"][0]) == ref["C_s"]
        else:
            assert phase_set_error(a["theta"][0], b["theta"][0]) < 1e-10
            ref = orc.wilson_surface(r.hoplist, r.kappa, r.lo, r.hi)
            assert phase_set_error(b["theta"][0], ref["theta"]) < 1e-10
    st = S.latency_stats(mix)
    assert st["n"] == len(mix) and st["p99_ms"] >= st["p50_ms"] > 0


def test_served_stream_at_full_request_sizes():
    """One request of each type of the served workload (BHZ supercells L = 8,
    12, 16, 24 with disorder, and the 96-orbital model; 32 x 32 k-grids, all
    occupied bands, mixed path) arriving together on two lanes: launches of
    different sizes run at the same time on the two lanes; each result equals
    the same request run alone (1e-10 rad) and, for the three smallest types,
    one transverse line equals the FP64 oracle's within 1e-6 rad (mixed path
    for the supercells, refined mixed path for the 96-orbital model)."""
    gu.need_gpu()
    from paper_2312_13051_amd import _lib as L
    from paper_2312_13051_amd import serve as S
    kg = syn.kplane(32, 32)

    def reqs():
        out = []
        for q, kind in enumerate(syn.SERVED_TYPES):
            hl = syn.served_model(kind, q)
            out.append(S.Request(hoplist=hl, kappa=kg, lo=0, hi=hl.N // 2, kind=S.KIND_WILSON,
                                 precision=S.served_precision(kind), tag=kind))
        return out

    mix = reqs()
    eng = S.Engine(S.GpuExecutor(n_lanes=2), hbm_budget=150 << 30)
    S.drive(eng, mix, np.zeros(len(mix)))
    assert all(r.error is None for r in mix)
    by_lane = {}
    for s in eng.step_log:
        by_lane.setdefault(s["lane"], []).append((s["t0"], s["t"]))
    assert set(by_lane) == {0, 1}
    assert any(a0 < b1 and b0 < a1 for a0, a1 in by_lane[0] for b0, b1 in by_lane[1]), "the lanes never overlapped"
    ref_alone = alone(S, reqs(), budget=150 << 30)
    for a, b, r in zip(ref_alone, [x.result for x in mix], mix):
        # the random 96-orbital model has no resolved winding on a 32-point
        # transverse grid: every other status bit must be clear
        assert int(np.bitwise_or.reduce(np.asarray(b["status"]).ravel())) & ~orc.WINDING_UNRESOLVED == 0
        assert not b["eig_status"]
        assert phase_set_error(a["theta"][0], b["theta"][0]) < 1e-10, r.tag
        if r.tag in ("w96", "bhz8", "bhz12"):
            ev, U, st = orc.eigh_grid(r.hoplist, kg[0], 0, r.m)
            W, _ = orc.wilson_matrix(U)
            assert phase_set_error(b["theta"][0, 0], orc.eigphases(W)) < 1e-6, r.tag


def test_cancelled_request_frees_its_buffers_and_leaves_others_unchanged(tmp_path):
    """Cancelling an admitted request on the GPU executor: no further launches
    for it, its eigenvector grid and its key's Hamiltonian buffer are
    released, and the other request's result is bitwise the one it has alone."""
    gu.need_gpu()
    import json
    from paper_2312_13051_amd import serve as S
    kg = syn.kplane(8, 6)

    def pair():
        h1 = syn.bhz_disordered(3, 2.0, [5, 1, 9])
        h2 = syn.bhz_disordered(4, 2.0, [5, 1, 4])
        return (S.Request(hoplist=h1, kappa=kg, lo=0, hi=h1.N // 2, kind=S.KIND_WILSON),
                S.Request(hoplist=h2, kappa=kg, lo=0, hi=h2.N // 2, kind=S.KIND_WILSON))

    ex = S.GpuExecutor(n_lanes=1, chunk_cap=16)
    log = tmp_path / "req.jsonl"
    eng = S.Engine(ex, hbm_budget=8 << 30, log_path=str(log))
    keep, gone = pair()
    eng.submit(gone)
    eng.submit(keep)
    eng.step()                        # gone's first chunk (16 of its 48 k-points)
    assert gone.key in ex._H
    assert eng.cancel(gone)
    eng.run_until_idle()
    torch.cuda.synchronize()
    assert isinstance(gone.error, S.RequestCancelled) and gone.result is None
    assert [s["k_points"] for s in eng.step_log if gone.rid in s["requests"]] == [16]
    assert gone.key not in ex._H and gone.key not in ex._key_users
    assert keep.error is None and eng.used == 0
    (ref,) = alone(S, [pair()[0]])
    assert np.array_equal(ref["theta"], keep.result["theta"])
    outcomes = {r["rid"]: r["outcome"] for r in map(json.loads, log.read_text().splitlines())}
    assert outcomes == {keep.rid: "ok", gone.rid: "cancelled"}
