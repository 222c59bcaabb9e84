"""GPU parity of the Berry flux per plaquette (coupling-matrix method of the
disordered quadrupolar-insulator example, Sec. IV) against the oracle.

Flux maps must agree with the FP64 oracle to 1e-10 rad per plaquette
(circular distance), Chern numbers exactly. The flux of one plaquette is a
function of its four corners only: the oracle's map of the 2 x 2 grid of
those corners holds it at entry (0, 0), which is how full-size maps are
sampled.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import berry as orc
from tests import gpu_util as gu

torch = gu.torch
pytestmark = pytest.mark.gpu
TOL = 1e-10
TOL_MIXED = 1e-6   # spin sectors from the FP32-reduction eigensolver


def pipe():
    from paper_2312_13051_amd import pipeline
    return pipeline


def circ(a, b):
    return np.abs(np.mod(np.asarray(a) - np.asarray(b) + np.pi, 2 * np.pi) - np.pi)


def corners(kg, i, j):
    n_perp, n_par = kg.shape[:2]
    return kg[[i, (i + 1) % n_perp]][:, [j, (j + 1) % n_par]]


@pytest.mark.parametrize("m,C", [(-1.0, 1), (1.5, -1), (2.5, 0)])
def test_qwz_flux_map_and_chern(m, C):
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    kg = syn.kplane(24, 20, e_par=(0, 1, 0), e_perp=(1, 0, 0))
    hl = syn.qwz(m)
    out = P.wflux(c, [hl], kg, 0, 1)
    ref = orc.plaquette_flux(hl, kg, 0, 1)
    assert int(out["status"][0]) == ref["status"] == 0
    assert int(out["chern"][0]) == ref["chern"] == C
    assert circ(out["flux"][0].cpu().numpy(), ref["flux"]).max() < TOL
    assert abs(float(out["total"][0]) - ref["total"]) < 1e-9
    # the sum over the zone is 2 pi times the Wilson-loop winding on the same grid
    assert int(P.wsurf(c, [hl], kg, 0, 1)["winding"][0]) == C


@pytest.mark.parametrize("name", ["bhz_clean", "bhz_L3_W2", "bhz_L4_vac", "wannier24"])
def test_flux_parity_models(name):
    """Several bands per link (m up to 32), ragged grids."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = {"bhz_clean": lambda: syn.bhz(),
          "bhz_L3_W2": lambda: syn.bhz_disordered(3, 2.0, [3, 1, 5]),
          "bhz_L4_vac": lambda: syn.bhz_vacancies(4, 0.1, [4, 1, 2]),
          "wannier24": lambda: syn.wannier_like(24, [5, 2, 9])}[name]()
    kg = syn.kplane(9, 7)
    m = hl.N // 2
    out = P.wflux(c, [hl], kg, 0, m)
    ref = orc.plaquette_flux(hl, kg, 0, m)
    st = int(out["status"][0])
    assert (st & ~4) == (ref["status"] & ~4)
    assert circ(out["flux"][0].cpu().numpy(), ref["flux"]).max() < TOL
    if st == 0 and ref["status"] == 0:
        assert int(out["chern"][0]) == ref["chern"]


def test_flux_batch_of_systems():
    """Four disordered systems in one call, each against the oracle."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hls = [syn.bhz_disordered(2, 1.0 + r, [7, r]) for r in range(4)]
    kg = syn.kplane(6, 8)
    m = hls[0].N // 2
    out = P.wflux(c, hls, kg, 0, m)
    for s, hl in enumerate(hls):
        ref = orc.plaquette_flux(hl, kg, 0, m)
        assert circ(out["flux"][s].cpu().numpy(), ref["flux"]).max() < TOL
        assert (int(out["status"][s]) & ~4) == (ref["status"] & ~4)


def test_flux_empty_band_set_and_no_systems():
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    kg = syn.kplane(5, 4)
    out = P.wflux(c, [syn.bhz()], kg, 1, 1)
    assert float(out["flux"].abs().max()) == 0.0
    assert int(out["chern"][0]) == 0 and int(out["status"][0]) == 0
    # no systems: nothing is written (pointers must still be valid)
    f = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    i = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    U = torch.zeros((1, 1, 4), dtype=torch.complex128, device="cuda")
    c.plaquette_flux(U, 4, 1, 4, 4, 0, 5, 4, f, i, f, i)
    torch.cuda.synchronize()
    assert float(f[0]) == 7.0 and int(i[0]) == 7


def test_flux_bad_arguments():
    gu.need_gpu()
    from paper_2312_13051_amd import _lib as L
    c = gu.ctx()
    U = torch.zeros((4, 2, 4), dtype=torch.complex128, device="cuda")
    f = torch.empty(8, dtype=torch.float64, device="cuda")
    i = torch.empty(8, dtype=torch.int32, device="cuda")
    with pytest.raises(L.BerryError):
        c.plaquette_flux(U, 4, 5, 4, 8, 1, 2, 2, f, i, f, i)      # m > N
    with pytest.raises(L.BerryError):
        c.plaquette_flux(U, 4, 2, 3, 8, 1, 2, 2, f, i, f, i)      # ldu < N
    with pytest.raises(L.BerryError):
        c.plaquette_flux(U, 4, 2, 4, 8, 1, 0, 2, f, i, f, i)      # n_par = 0


def test_flux_singular_link_flagged():
    """Two uncoupled orbitals whose occupied state switches between grid
    points: det of the link across the switch is exactly zero."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    from synthetic.models import _from_blocks
    hl = _from_blocks(2, 1, {(0,): np.zeros((2, 2)), (1,): np.diag([0.5, -0.5])})
    kg = syn.kplane(8, 3, k0=(1.0 / 16, 0.0, 0.0))
    out = P.wflux(c, [hl], kg, 0, 1)
    ref = orc.plaquette_flux(hl, kg, 0, 1)
    assert ref["status"] & orc.OVERLAP_SINGULAR
    assert int(out["status"][0]) & orc.OVERLAP_SINGULAR
    assert np.isfinite(out["flux"][0].cpu().numpy()).all()


@pytest.mark.parametrize("precision,tol", [(0, TOL), (1, TOL_MIXED)])
def test_spin_flux_bhz(precision, tol):
    """Spin sectors of BHZ (Sec. IV): C_dn = -1, C_up = +1, C_s = +1, flux maps
    of both sectors against the oracle."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    sd = np.array([1.0, -1, -1, 1])
    kg = syn.kplane(16, 16)
    out = P.wspinflux(c, [syn.bhz()], sd[None, :], kg, 0, 2, precision=precision)
    ref = orc.spin_resolved_flux(syn.bhz(), sd, kg, 0, 2)
    assert int(out["status"][0]) == ref["status"] == 0
    assert out["m_dn"] == [ref["m_dn"]]
    assert (int(out["C_dn"][0]), int(out["C_up"][0]), float(out["C_s"][0])) == (-1, 1, 1.0)
    assert circ(out["flux_dn"][0].cpu().numpy(), ref["flux_dn"]).max() < tol
    assert circ(out["flux_up"][0].cpu().numpy(), ref["flux_up"]).max() < tol


def test_spin_flux_disordered_supercell():
    """Spinful BHZ 3x3 supercell with weak disorder: sector flux maps and the
    spin Chern number against the oracle."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = syn.bhz_disordered(3, 1.0, [11, 4])
    sd = syn.bhz_spin_diag(hl)
    kg = syn.kplane(7, 6)
    m = hl.N // 2
    out = P.wspinflux(c, [hl], sd[None, :], kg, 0, m)
    ref = orc.spin_resolved_flux(hl, sd, kg, 0, m)
    assert (int(out["status"][0]) & ~4) == (ref["status"] & ~4)
    if not ref["status"] & orc.PSO_GAP:
        assert out["m_dn"] == [ref["m_dn"]]
        assert circ(out["flux_dn"][0].cpu().numpy(), ref["flux_dn"]).max() < TOL
        assert circ(out["flux_up"][0].cpu().numpy(), ref["flux_up"]).max() < TOL
        if ref["status"] == 0:
            assert float(out["C_s"][0]) == ref["C_s"]


@pytest.mark.parametrize("precision,tol", [(0, TOL), (1, TOL_MIXED)])
def test_spin_flux_full_size_supercells(precision, tol):
    """The coupling-matrix workload at full size and in the benchmark's launch
    configuration: eight disordered spinful BHZ 10x10 supercells (N = 400,
    m = 200) on a 24 x 24 plaquette grid in one eigensolver call. Sampled
    plaquettes of both sectors against the oracle (2 x 2 corner grids); every
    system's spin Chern number equals the spin-resolved Wilson-loop winding on
    the same grid whenever both are resolved."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hls = [syn.bhz_disordered(10, 1.0, [6, r]) for r in range(8)]
    kg = syn.kplane(24, 24)
    m = hls[0].N // 2
    sd = np.stack([syn.bhz_spin_diag(h) for h in hls])
    out = P.wspinflux(c, hls, sd, kg, 0, m, precision=precision, chunk=8 * 576)
    st = out["status"].cpu().numpy()
    w = P.spin(c, out["eig"], sd, precision=precision)
    wst = w["status"].cpu().numpy()
    for s in range(8):
        if st[s] == 0 and wst[s] == 0:
            assert int(out["C_dn"][s]) == int(w["C_dn"][s])
            assert int(out["C_up"][s]) == int(w["C_up"][s])
    assert (st == 0).sum() >= 6
    for s, (i, j) in ((0, (0, 0)), (3, (7, 19)), (6, (23, 11))):
        ref = orc.spin_resolved_flux(hls[s], sd[s], corners(kg, i, j), 0, m)
        assert not ref["status"] & orc.PSO_GAP
        assert out["m_dn"][s] == ref["m_dn"]
        assert circ(float(out["flux_dn"][s, i, j]), ref["flux_dn"][0, 0]) < tol
        assert circ(float(out["flux_up"][s, i, j]), ref["flux_up"][0, 0]) < tol


@pytest.mark.parametrize("N,m", [(20, 17), (300, 256), (300, 257), (700, 600)])
def test_flux_random_bases_panel_widths(N, m):
    """Random orthonormal bases on a 3 x 4 grid: link determinants of every
    panel width (16 up to m = 256, 8 up to 512, 4 beyond) with ragged last
    panels, against the oracle's determinants."""
    gu.need_gpu()
    c = gu.ctx()
    rng = np.random.default_rng([21, N, m])
    n_perp, n_par = 3, 4
    Ug = np.linalg.qr(rng.standard_normal((n_perp, n_par, N, m)) + 1j * rng.standard_normal((n_perp, n_par, N, m)))[0]
    U = torch.from_numpy(np.ascontiguousarray(np.swapaxes(Ug, -1, -2).reshape(-1, m, N))).cuda()
    f = torch.empty((n_perp, n_par), dtype=torch.float64, device="cuda")
    ch = torch.empty(1, dtype=torch.int32, device="cuda")
    tot = torch.empty(1, dtype=torch.float64, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    c.plaquette_flux(U, N, m, N, m * N, 1, n_par, n_perp, f, ch, tot, st)
    ref = orc.plaquette_flux_from_grid(Ug)
    assert circ(f.cpu().numpy(), ref["flux"]).max() < 1e-9
    assert (int(st[0]) & orc.OVERLAP_SINGULAR) == (ref["status"] & orc.OVERLAP_SINGULAR)


def test_flux_multi_pass_matches_single_systems():
    """Three BHZ 10x10 supercells (m = 200 occupied bands, 24 x 24 grid): their
    links take 369 MB per system and direction, so one call runs them in two
    passes; every system's flux map equals the one computed alone."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hls = [syn.bhz_disordered(10, 1.0 + r, [8, r]) for r in range(3)]
    kg = syn.kplane(24, 24)
    m = hls[0].N // 2
    g = P.eig_grid(c, c.hk_plan(hls), 0, 3, kg, 0, m, precision=1)
    both = P.flux(c, g)
    for s in range(3):
        one = P.flux(c, P.EigGrid(g.U[s * 576:(s + 1) * 576], g.evals, g.status, g.N, g.m, g.ldu, 1, 24, 24))
        assert float((both["flux"][s] - one["flux"][0]).abs().max()) == 0.0
        assert int(both["chern"][s]) == int(one["chern"][0]) and int(both["status"][s]) == int(one["status"][0])


def test_spin_sectors_bad_arguments():
    gu.need_gpu()
    from paper_2312_13051_amd import _lib as L
    c = gu.ctx()
    U = torch.zeros((4, 2, 4), dtype=torch.complex128, device="cuda")
    V = torch.zeros((4, 2, 4), dtype=torch.complex128, device="cuda")
    sd = torch.ones((1, 4), dtype=torch.float64, device="cuda")
    mu = torch.empty((4, 2), dtype=torch.float64, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    with pytest.raises(L.BerryError):
        c.spin_sectors(U, 4, 2, 4, 8, 1, 4, sd, mu, V, 3, 8, st)          # ldv < N
    with pytest.raises(L.BerryError):
        c.spin_sectors(U, 4, 2, 4, 8, 1, 4, sd, mu, V, 4, 8, st, precision=7)
    assert c.spin_sectors(U, 4, 2, 4, 8, 0, 4, sd, mu, V, 4, 8, st) == []
