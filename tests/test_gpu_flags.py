"""GPU status flags against the oracle's on the cases that make each of the
oracle's flag branches fire (the same inputs as its CPU pins).

OVERLAP_SINGULAR: link grids with prescribed singular values (the smallest
below or above 1e-8, or all of them moderately below one at a high order,
where |det| < 1e-8 although no singular value is small), through both the
plaquette flux (one-wave LU up to order 128, workgroup LU above) and the
Wilson loop. WANNIER_GAP, PSO_GAP and NAN_INF: the cases of the oracle pins.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import berry as orc
from tests import gpu_util as gu

torch = gu.torch
pytestmark = pytest.mark.gpu


def upload_grid(g):
    """U-grid (n_perp, n_par, N, m) -> device (n_mat, m, N), ld = N."""
    n_perp, n_par, N, m = g.shape
    return gu.from_np(g.reshape(n_perp * n_par, N, m), N), N, m


def gpu_flux_status(c, g):
    U, N, m = upload_grid(g)
    n_perp, n_par = g.shape[:2]
    f = torch.empty((n_perp, n_par), dtype=torch.float64, device="cuda")
    ch = torch.empty(1, dtype=torch.int32, device="cuda")
    tot = torch.empty(1, dtype=torch.float64, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    c.plaquette_flux(U, N, m, N, U.stride(0), 1, n_par, n_perp, f, ch, tot, st)
    torch.cuda.synchronize()
    return int(st[0]), f.cpu().numpy()


def gpu_wilson_status(c, g):
    U, N, m = upload_grid(g)
    n_perp, n_par = g.shape[:2]
    th = torch.empty((n_perp, m), dtype=torch.float64, device="cuda")
    ph = torch.empty(n_perp, dtype=torch.float64, device="cuda")
    w = torch.empty(1, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    c.wilson_loop(U, N, m, N, U.stride(0), 1, n_par, n_perp, 0, th, ph, w, st)
    torch.cuda.synchronize()
    return int(st[0])


@pytest.mark.parametrize("m,cos", [(100, 0.8), (300, 0.95), (640, 0.97)])
def test_high_order_links_are_regular(m, cos):
    """Every singular value of order one, |det| = cos^m < 1e-8: not singular
    (flux, both LU kernels; Wilson loop), as in the oracle; the flux is zero."""
    gu.need_gpu()
    c = gu.ctx()
    g = syn.link_grid(np.full(m, cos))
    ref = orc.plaquette_flux_from_grid(g)
    assert not ref["status"] & orc.OVERLAP_SINGULAR
    st, f = gpu_flux_status(c, g)
    assert not st & orc.OVERLAP_SINGULAR
    assert np.max(np.abs(f)) < 1e-10
    if m <= 300:
        assert not gpu_wilson_status(c, g) & orc.OVERLAP_SINGULAR


@pytest.mark.parametrize("m", [1, 100, 200])
@pytest.mark.parametrize("small,flagged", [(1e-9, True), (1e-7, False)])
def test_one_small_singular_value(m, small, flagged):
    """One singular value of 1e-9 among ones is singular (sigma_min < 1e-8);
    1e-7 is not: flux (one-wave LU at m <= 128, workgroup LU at 200) and
    Wilson loop agree with the oracle."""
    gu.need_gpu()
    c = gu.ctx()
    cs = np.ones(m)
    cs[m // 2] = small
    g = syn.link_grid(cs)
    ref = orc.plaquette_flux_from_grid(g)
    assert bool(ref["status"] & orc.OVERLAP_SINGULAR) == flagged
    st, _ = gpu_flux_status(c, g)
    assert bool(st & orc.OVERLAP_SINGULAR) == flagged
    assert bool(orc.wilson_loop_grid(g)[3] & orc.OVERLAP_SINGULAR) == flagged
    assert bool(gpu_wilson_status(c, g) & orc.OVERLAP_SINGULAR) == flagged


def test_random_high_order_links_match_oracle():
    """Random orthonormal bases (N = 700, m = 600): |det| of every link is far
    below 1e-8, the smallest singular value is not; no flag on either side."""
    gu.need_gpu()
    c = gu.ctx()
    rng = np.random.default_rng([22, 700])
    g = np.linalg.qr(rng.standard_normal((2, 2, 700, 600)) + 1j * rng.standard_normal((2, 2, 700, 600)))[0]
    ref = orc.plaquette_flux_from_grid(g)
    st, f = gpu_flux_status(c, g)
    assert (st & orc.OVERLAP_SINGULAR) == (ref["status"] & orc.OVERLAP_SINGULAR)
    d = np.abs(np.mod(f - ref["flux"] + np.pi, 2 * np.pi) - np.pi)
    assert d.max() < 1e-9


def test_wannier_gap_when_sector_size_varies():
    """Chern insulator, one band: the number of phases in (0, 1/2) changes
    between transverse lines; the nested loop carries WANNIER_GAP on both
    sides."""
    gu.need_gpu()
    from paper_2312_13051_amd import pipeline as P
    c = gu.ctx()
    kg = syn.kplane(12, 16, k0=(0.0, 0.013, 0.0))
    ref = orc.nested_wilson(syn.qwz(1.5), kg, 0, 1)
    assert ref["status"] & orc.WANNIER_GAP
    out = P.wnwl(c, [syn.qwz(1.5)], kg, 0, 1)
    assert int(out["status"][0]) & orc.WANNIER_GAP
    # a fixed sector (BBH): no flag on either side
    kb = syn.kplane(10, 10)
    assert not orc.nested_wilson(syn.bbh(0.5, 1.0), kb, 0, 2)["status"] & orc.WANNIER_GAP
    assert not int(P.wnwl(c, [syn.bbh(0.5, 1.0)], kb, 0, 2)["status"][0]) & orc.WANNIER_GAP


def test_pso_gap_flags_match_oracle():
    """P S P with a zero eigenvalue, and with a spin-down count that changes
    across the zone: PSO_GAP on both sides; BHZ: neither."""
    gu.need_gpu()
    from paper_2312_13051_amd import pipeline as P
    from synthetic.models import _from_blocks
    c = gu.ctx()
    cases = [(syn.atomic([-1.0, 2.0]), np.array([0.0, 1.0]), syn.kplane(4, 3), 1),
             (_from_blocks(2, 1, {(0,): np.zeros((2, 2)), (1,): np.diag([0.5, -0.5])}), np.array([1.0, -1.0]),
              syn.kplane(8, 2, k0=(1.0 / 16, 0.0, 0.0)), 1),
             (syn.bhz(), np.array([1.0, -1.0, -1.0, 1.0]), syn.kplane(8, 6), 2)]
    for hl, sd, kg, m in cases:
        ref = orc.spin_resolved_wilson(hl, sd, kg, 0, m)
        out = P.wspinsurf(c, [hl], sd[None], kg, 0, m)
        assert (int(out["status"][0]) & orc.PSO_GAP) == (ref["status"] & orc.PSO_GAP)


def test_nan_inf_flag_matches_oracle():
    """A non-finite Hamiltonian entry: the eigensolver reports NAN_INF for
    that matrix only, as the oracle's eigh_bands does."""
    gu.need_gpu()
    c = gu.ctx()
    rng = np.random.default_rng(31)
    A = rng.standard_normal((3, 12, 12)) + 1j * rng.standard_normal((3, 12, 12))
    Hs = A + np.conj(np.swapaxes(A, 1, 2))
    Hs[1, 3, 5] = Hs[1, 5, 3] = np.nan
    dH = gu.from_np(Hs, 12)
    U = gu.colmajor(3, 12, 6, 12, fill=0)
    ev = torch.empty((3, 8), dtype=torch.float64, device="cuda")
    st = torch.empty(3, dtype=torch.int32, device="cuda")
    c.eigh_batched(dH, 0, 12, 12, dH.stride(0), 3, 0, 6, 0, ev, U, 12, U.stride(0), st)
    torch.cuda.synchronize()
    for q in range(3):
        ref = orc.eigh_bands(Hs[q], 0, 6)[2]
        assert (int(st[q]) & orc.NAN_INF) == (ref & orc.NAN_INF), q
