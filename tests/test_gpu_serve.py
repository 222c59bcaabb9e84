"""Served mix on the GPU: every request's result is the same alone and in the mix."""
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


def test_served_mix_equals_alone():
    gu.need_gpu()
    from paper_2312_13051_amd import serve as S
    c = gu.ctx()
    ex = S.GpuExecutor(c, chunk_k=64)
    mix = make_requests(S)
    eng = S.Engine(ex, hbm_budget=8 << 30, chunk_k=64)
    # the first half arrives together (so compatible requests must share
    # launches); the rest follow as a Poisson stream while those run
    arr = np.concatenate([np.zeros(3), S.poisson_arrivals(500.0, len(mix) - 3, [5, 0])])
    S.drive(eng, mix, arr)
    launches_with_two = [s for s in eng.step_log if len(s["requests"]) > 1]
    assert launches_with_two, "continuous batching never mixed two requests"
    # the same requests, each alone, compared in submission order
    alone = []
    for r in make_requests(S):
        e1 = S.Engine(S.GpuExecutor(c, chunk_k=64), hbm_budget=8 << 30, chunk_k=64)
        e1.submit(r)
        e1.run_until_idle()
        alone.append(r.result)
    for a, b, r in zip(alone, [x.result for x in mix], mix):
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
