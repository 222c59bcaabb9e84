"""The hot path captured into a HIP graph: build_hk -> eigh_batched ->
wilson_loop (and the plaquette flux) recorded once on a stream and replayed;
every replay reproduces the uncaptured results bit for bit. Inside capture
the library takes no host read-back (its iterations run on a fixed schedule
with per-matrix predicates) and may not grow its workspace."""
import numpy as np
import pytest

import synthetic as syn
from tests import gpu_util as gu

torch = gu.torch
pytestmark = pytest.mark.gpu


def _setup(prec, L_cell=3):
    from paper_2312_13051_amd import _lib as L
    c = gu.ctx()
    hls = [syn.bhz_disordered(L_cell, 1.0 + r, [13, r]) for r in range(2)]
    plan = c.hk_plan(hls)
    kg = syn.kplane(8, 6)
    n_k = kg.shape[0] * kg.shape[1]
    N = hls[0].N
    m = N // 2
    mixed = prec == L.BE_MIXED_FP32
    kap = torch.from_numpy(np.ascontiguousarray(kg.reshape(-1, 3))).cuda()
    H = torch.empty((2 * n_k, N, N), dtype=torch.complex64 if mixed else torch.complex128, device="cuda")
    bufs = {
        "U": torch.empty((2 * n_k, m, N), dtype=torch.complex128, device="cuda"),
        "ev": torch.empty((2 * n_k, m + 2), dtype=torch.float64, device="cuda"),
        "est": torch.empty(2 * n_k, dtype=torch.int32, device="cuda"),
        "theta": torch.empty((2, 6, m), dtype=torch.float64, device="cuda"),
        "phi": torch.empty((2, 6), dtype=torch.float64, device="cuda"),
        "wind": torch.empty(2, dtype=torch.int32, device="cuda"),
        "st": torch.empty(2, dtype=torch.int32, device="cuda"),
        "flux": torch.empty((2, 6, 8), dtype=torch.float64, device="cuda"),
        "chern": torch.empty(2, dtype=torch.int32, device="cuda"),
        "tot": torch.empty(2, dtype=torch.float64, device="cuda"),
        "fst": torch.empty(2, dtype=torch.int32, device="cuda"),
    }
    dt = L.BE_C64 if mixed else L.BE_C128

    def run():
        c.build_hk(plan, 0, 2, kap, H, N * N, N, dt)
        c.eigh_batched(H, dt, N, N, N * N, 2 * n_k, 0, m, prec, bufs["ev"], bufs["U"], N, bufs["U"].stride(0),
                       bufs["est"])
        c.wilson_loop(bufs["U"], N, m, N, bufs["U"].stride(0), 2, 8, 6, L.BE_OVL_POLAR, bufs["theta"], bufs["phi"],
                      bufs["wind"], bufs["st"])
        c.plaquette_flux(bufs["U"], N, m, N, bufs["U"].stride(0), 2, 8, 6, bufs["flux"], bufs["chern"], bufs["tot"],
                         bufs["fst"])
    return c, run, bufs


@pytest.mark.parametrize("prec,L_cell", [(0, 3), (1, 3), (2, 3), (0, 8), (1, 8)])
def test_captured_hot_path_replays_bitwise(prec, L_cell):
    """L_cell = 8: Wilson matrices of order 128, whose eigenphases take the
    Hermitian route (an eigensolver call and the checked QR fallback inside
    the graph); prec 2: the refined eigensolver."""
    gu.need_gpu()
    c, run, bufs = _setup(prec, L_cell)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        run()           # sizes the workspace outside capture
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in bufs.items()}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        run()
    torch.cuda.synchronize()
    for rep in range(3):
        for v in bufs.values():
            v.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in bufs.items():
            # bit for bit (NaN where the layout defines it, e.g. the eigenvalue below band 0)
            a, b = v.view(torch.float64) if v.is_complex() else v, ref[k].view(torch.float64) if v.is_complex() else ref[k]
            if a.is_floating_point():
                assert torch.equal(torch.isnan(a), torch.isnan(b)), (rep, k)
                a, b = torch.nan_to_num(a, nan=0.0), torch.nan_to_num(b, nan=0.0)
            assert torch.equal(a, b), (rep, k)
        # eager work between the replays
        x = torch.randn(1000, device="cuda")
        assert float(x.abs().sum()) > 0


def test_captured_spin_resolved_wilson_replays_bitwise():
    """Spin-resolved loop (mixed path) under capture: the sector sizes of an
    uncaptured call are passed in; replays equal the uncaptured results."""
    gu.need_gpu()
    from paper_2312_13051_amd import _lib as L
    c = gu.ctx()
    hls = [syn.bhz_disordered(3, 1.0, [14, r]) for r in range(2)]
    plan = c.hk_plan(hls)
    kg = syn.kplane(8, 6)
    n_k = 48
    N, m = hls[0].N, hls[0].N // 2
    kap = torch.from_numpy(np.ascontiguousarray(kg.reshape(-1, 3))).cuda()
    sd = torch.from_numpy(np.stack([syn.bhz_spin_diag(h) for h in hls])).cuda()
    H = torch.empty((2 * n_k, N, N), dtype=torch.complex64, device="cuda")
    U = torch.empty((2 * n_k, m, N), dtype=torch.complex128, device="cuda")
    ev = torch.empty((2 * n_k, m + 2), dtype=torch.float64, device="cuda")
    est = torch.empty(2 * n_k, dtype=torch.int32, device="cuda")
    outs = {"pso": torch.empty((2, 6, 8, m), dtype=torch.float64, device="cuda"),
            "tdn": torch.empty((2, 6, m), dtype=torch.float64, device="cuda"),
            "tup": torch.empty((2, 6, m), dtype=torch.float64, device="cuda"),
            "cdn": torch.empty(2, dtype=torch.int32, device="cuda"),
            "cup": torch.empty(2, dtype=torch.int32, device="cuda"),
            "cs": torch.empty(2, dtype=torch.float64, device="cuda"),
            "st": torch.empty(2, dtype=torch.int32, device="cuda")}

    def run(m_dn_in=None):
        c.build_hk(plan, 0, 2, kap, H, N * N, N, L.BE_C64)
        c.eigh_batched(H, L.BE_C64, N, N, N * N, 2 * n_k, 0, m, L.BE_MIXED_FP32, ev, U, N, U.stride(0), est)
        return c.spin_resolved_wilson(U, N, m, N, U.stride(0), 2, 8, 6, L.BE_OVL_POLAR, sd, outs["pso"], outs["tdn"],
                                      outs["tup"], outs["cdn"], outs["cup"], outs["cs"], outs["st"],
                                      L.BE_MIXED_FP32, m_dn_in=m_dn_in)

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        mdn = run()
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in outs.items()}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        assert run(m_dn_in=mdn) == mdn
    for rep in range(2):
        for v in outs.values():
            v.fill_(-3)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in outs.items():
            if k in ("tdn", "tup"):   # entries past each sector size are NaN fill
                assert torch.equal(torch.nan_to_num(v, nan=7.0), torch.nan_to_num(ref[k], nan=7.0)), (rep, k)
            else:
                assert torch.equal(v, ref[k]), (rep, k)
