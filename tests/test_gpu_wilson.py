"""GPU parity of the Wilson-loop, nested and spin-resolved calls against the oracle.

Phases must agree with the FP64 oracle to 1e-10 rad (best cyclic match of the
sorted sets, circular distance); topological integers exactly.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import berry as orc
from tests import gpu_util as gu
from tests.phase_metrics import phase_set_error

torch = gu.torch
pytestmark = pytest.mark.gpu
TOL = 1e-10


def pipe():
    from paper_2312_13051_amd import pipeline
    return pipeline


def test_qwz_config1_winding_and_phases():
    """QWZ m=-1, 64x64, loop along ky per kx: winding +1 (the oracle's sign pin)."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    kg = syn.kplane(64, 64, e_par=(0, 1, 0), e_perp=(1, 0, 0))
    hl = syn.qwz(-1.0)
    out = P.wsurf(c, [hl], kg, 0, 1)
    ref = orc.wilson_surface(hl, kg, 0, 1)
    assert int(out["status"][0]) == 0 and ref["status"] == 0
    assert int(out["winding"][0]) == ref["winding"] == 1
    assert phase_set_error(out["theta"][0].cpu().numpy(), ref["theta"]) < TOL
    d = np.abs(np.mod(out["phi"][0].cpu().numpy() - ref["phi"] + np.pi, 2 * np.pi) - np.pi)
    assert d.max() < TOL


def test_qwz_paper_value_and_raw_mode():
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    kg = syn.kplane(48, 40)
    hl = syn.qwz(1.5)
    out = P.wsurf(c, [hl], kg, 0, 1, mode=1)
    ref = orc.wilson_surface(hl, kg, 0, 1, mode="raw")
    assert int(out["winding"][0]) == ref["winding"] == 1
    assert phase_set_error(out["theta"][0].cpu().numpy(), ref["theta"]) < TOL


@pytest.mark.parametrize("name", ["bhz_clean", "bhz_L3_W2", "bhz_L4_vac", "wannier24"])
def test_wilson_parity_models(name):
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = {"bhz_clean": lambda: syn.bhz(),
          "bhz_L3_W2": lambda: syn.bhz_disordered(3, 2.0, [3, 1, 5]),
          "bhz_L4_vac": lambda: syn.bhz_vacancies(4, 0.1, [4, 1, 2]),
          "wannier24": lambda: syn.wannier_like(24, [5, 2, 9])}[name]()
    kg = syn.kplane(12, 7)
    m = hl.N // 2
    out = P.wsurf(c, [hl], kg, 0, m)
    ref = orc.wilson_surface(hl, kg, 0, m)
    st = int(out["status"][0])
    assert (st & ~4) == (ref["status"] & ~4)   # winding resolution may differ on coarse grids
    assert phase_set_error(out["theta"][0].cpu().numpy(), ref["theta"]) < TOL
    if st == 0 and ref["status"] == 0:
        assert int(out["winding"][0]) == ref["winding"]


def test_batch_composition_alone_vs_mixed():
    """A system's phases are the same alone and inside a batch of several."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hls = [syn.bhz_disordered(3, 1.5, [7, r]) for r in range(4)]
    kg = syn.kplane(10, 6)
    m = hls[0].N // 2
    mix = P.wsurf(c, hls, kg, 0, m)["theta"].cpu().numpy()
    for r in (0, 3):
        alone = P.wsurf(c, [hls[r]], kg, 0, m)["theta"].cpu().numpy()
        assert phase_set_error(alone[0], mix[r]) < 1e-12


def test_bbh_nested_half_and_parity():
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    kg = syn.kplane(30, 30)
    hl = syn.bbh(0.5, 1.0)
    out = P.wnwl(c, [hl], kg, 0, 2)
    ref = orc.nested_wilson(hl, kg, 0, 2)
    assert out["s"] == [1] and ref["s"] == 1
    assert int(out["status"][0]) == 0
    p = out["p"][0].cpu().numpy()
    assert np.max(np.abs(np.abs(p) - 0.5)) < 1e-12
    assert abs(float(out["p_mean"][0]) - 0.5) < 1e-12
    assert phase_set_error(out["theta"][0, :, :1].cpu().numpy(), ref["theta"]) < TOL


def test_bbh_config2_full_size_closed_form():
    """BBH gamma=0.5, lambda=1 on the 100x100 grid: p(kx) = 1/2 at every kx."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    kg = syn.kplane(100, 100)
    out = P.wnwl(c, [syn.bbh(0.5, 1.0), syn.bbh(1.5, 1.0)], kg, 0, 2)
    assert out["s"] == [1, 1]
    p = out["p"].cpu().numpy()
    assert np.max(np.abs(np.abs(p[0]) - 0.5)) < 1e-12
    assert np.max(np.abs(p[1])) < 1e-12
    pm = out["p_mean"].cpu().numpy()
    assert abs(pm[0] - 0.5) < 1e-12 and min(pm[1], 1 - pm[1]) < 1e-12


def test_nested_two_sectors():
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = syn.concat_hops([syn.product_state_2d(0.7, 0.5), syn.product_state_2d(0.3, 0.0)])
    kg = syn.kplane(16, 12)
    a = P.wnwl(c, [hl], kg, 0, 2, window=(0.0, 0.5))
    b = P.wnwl(c, [hl], kg, 0, 2, window=(-0.5, 0.0))
    assert a["s"] == [1] and b["s"] == [1]
    assert abs(float(a["p_mean"][0]) - 0.5) < 1e-12
    pb = float(b["p_mean"][0])
    assert min(pb, 1 - pb) < 1e-12


def test_bhz_spin_chern():
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    kg = syn.kplane(32, 32)
    hl = syn.bhz()
    sd = np.array([[1.0, -1, -1, 1]])
    out = P.wspinsurf(c, [hl], sd, kg, 0, 2)
    ref = orc.spin_resolved_wilson(hl, sd[0], kg, 0, 2)
    assert int(out["status"][0]) == 0
    assert out["m_dn"] == [1]
    assert int(out["C_dn"][0]) == ref["C_dn"] == -1
    assert int(out["C_up"][0]) == ref["C_up"] == 1
    assert float(out["C_s"][0]) == ref["C_s"] == 1.0
    mu = out["mu"][0].cpu().numpy()
    assert np.max(np.abs(np.abs(mu) - 1)) < 1e-12
    assert phase_set_error(out["theta_dn"][0, :, :1].cpu().numpy(), ref["theta_dn"]) < TOL
    assert phase_set_error(out["theta_up"][0, :, :1].cpu().numpy(), ref["theta_up"]) < TOL


@pytest.mark.parametrize("L,W", [(3, 2.0), (4, 3.0)])
def test_spin_parity_disordered_supercells(L, W):
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hls = [syn.bhz_disordered(L, W, [3, 1, r]) for r in range(2)]
    kg = syn.kplane(8, 6)
    m = hls[0].N // 2
    sd = np.stack([syn.bhz_spin_diag(h) for h in hls])
    out = P.wspinsurf(c, hls, sd, kg, 0, m)
    for r, hl in enumerate(hls):
        ref = orc.spin_resolved_wilson(hl, sd[r], kg, 0, m)
        md = out["m_dn"][r]
        assert md == ref["m_minus"]
        assert (int(out["status"][r]) & ~4) == (ref["status"] & ~4)
        assert phase_set_error(out["theta_dn"][r, :, :md].cpu().numpy(), ref["theta_dn"]) < TOL
        assert phase_set_error(out["theta_up"][r, :, :m - md].cpu().numpy(), ref["theta_up"]) < TOL
        mu = np.sort(out["mu"][r].cpu().numpy(), axis=-1)
        assert np.max(np.abs(mu - ref["mu"])) < 1e-10
        if int(out["status"][r]) == 0 and ref["status"] == 0:
            assert int(out["C_dn"][r]) == ref["C_dn"] and int(out["C_up"][r]) == ref["C_up"]


def test_choti_spin_nonconserved():
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    kg = syn.kplane(24, 24)
    hl = syn.choti(1.0)
    sd = np.array([[1.0, -1, -1, 1]])
    out = P.wspinsurf(c, [hl], sd, kg, 0, 2)
    ref = orc.spin_resolved_wilson(hl, sd[0], kg, 0, 2)
    assert int(out["status"][0]) == ref["status"] == 0
    assert abs(float(out["C_s"][0])) == 1.0 and float(out["C_s"][0]) == ref["C_s"]
    assert phase_set_error(out["theta_dn"][0, :, :1].cpu().numpy(), ref["theta_dn"]) < TOL


@pytest.mark.parametrize("name", ["bhz_L3_W2", "bhz_L4_vac", "bhz_L10_W3"])
def test_mixed_precision_phases_within_gate(name):
    """Mixed path (FP32 reduction and back-transformation, FP64 elsewhere):
    Wilson phases within the 1e-6 rad gate of the FP64 oracle, integers exact."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = {"bhz_L3_W2": lambda: syn.bhz_disordered(3, 2.0, [3, 1, 5]),
          "bhz_L4_vac": lambda: syn.bhz_vacancies(4, 0.1, [4, 1, 2]),
          "bhz_L10_W3": lambda: syn.bhz_disordered(10, 3.0, [3, 3, 0])}[name]()
    kg = syn.kplane(8, 3) if hl.N > 100 else syn.kplane(12, 7)
    m = hl.N // 2
    out = P.wsurf(c, [hl], kg, 0, m, precision=1)
    ref = orc.wilson_surface(hl, kg, 0, m)
    assert phase_set_error(out["theta"][0].cpu().numpy(), ref["theta"]) < 1e-6
    sd = syn.bhz_spin_diag(hl)
    plan = c.hk_plan([hl])
    g = P.eig_grid(c, plan, 0, 1, kg, 0, m, precision=1)
    sref = orc.spin_resolved_wilson(hl, sd, kg, 0, m)
    for inner in (0, 1):  # eigensolver of the projected spin operator: FP64, mixed
        sp = P.spin(c, g, sd[None], precision=inner)
        md = sp["m_dn"][0]
        assert md == sref["m_minus"]
        assert phase_set_error(sp["theta_dn"][0, :, :md].cpu().numpy(), sref["theta_dn"]) < 1e-6
        assert phase_set_error(sp["theta_up"][0, :, :m - md].cpu().numpy(), sref["theta_up"]) < 1e-6


@pytest.mark.parametrize("N,m,n_par", [(202, 101, 3), (260, 130, 4), (700, 420, 3)])
def test_wilson_large_order_random_bases(N, m, n_par):
    """Wilson loops whose matrices are too large for LDS (the workgroup
    eigenphase kernel): random orthonormal bases on an n_par x 2 grid, phases
    and windings against the oracle."""
    gu.need_gpu()
    c = gu.ctx()
    rng = np.random.default_rng([31, N, m])
    g = np.linalg.qr(rng.standard_normal((2, n_par, N, m)) + 1j * rng.standard_normal((2, n_par, N, m)))[0]
    U = gu.from_np(g.reshape(2 * n_par, N, m), N)
    th = torch.empty((2, m), dtype=torch.float64, device="cuda")
    ph = torch.empty(2, dtype=torch.float64, device="cuda")
    w = torch.empty(1, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    c.wilson_loop(U, N, m, N, U.stride(0), 1, n_par, 2, 0, th, ph, w, st)
    torch.cuda.synchronize()
    ref_th, ref_phi, ref_C, ref_st = orc.wilson_loop_grid(g)
    for i in range(2):
        assert phase_set_error(th[i].cpu().numpy(), ref_th[i]) < 1e-10
    assert (int(st[0]) & orc.OVERLAP_SINGULAR) == (ref_st & orc.OVERLAP_SINGULAR)


def test_wilson_large_order_raw_mode():
    """Raw overlaps (eq. 2 without polar factors) make W non-unitary, which
    the Hermitian route for large orders cannot represent: such matrices go to
    the QR kernel (order 128); phases against the oracle's."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = syn.bhz_disordered(8, 2.0, [3, 8, 1])
    kg = syn.kplane(16, 2)
    m = hl.N // 2
    out = P.wsurf(c, [hl], kg, 0, m, mode=1)
    for i in range(2):
        ev, U, st = orc.eigh_grid(hl, kg[i], 0, m)
        W, _ = orc.wilson_matrix(U, "raw")
        assert phase_set_error(out["theta"][0, i].cpu().numpy(), orc.eigphases(W)) < 1e-9


def test_nested_large_sector_eigenvectors():
    """Nested Wilson loop of a clean BBH 6x6 supercell (m = 72: the Wilson
    matrices' eigenvectors come from the Hermitian route), against the
    oracle."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = syn.supercell(syn.bbh(0.5, 1.0), 6)
    kg = syn.kplane(10, 8)
    m = hl.N // 2
    # the supercell's Wannier centres crowd at 0; the window takes the six
    # bands between 0.07 and 0.25 (far from its edges on every line)
    out = P.wnwl(c, [hl], kg, 0, m, window=(0.03, 0.3))
    ref = orc.nested_wilson(hl, kg, 0, m, window=(0.03, 0.3))
    assert ref["status"] == 0 and int(out["status"][0]) == 0
    assert out["s"] == [ref["s"]]
    assert phase_set_error(out["theta"][0, :, :ref["s"]].cpu().numpy(), ref["theta"]) < TOL


def test_wilson_clustered_phases_served_supercell():
    """A served BHZ L = 12 supercell (m = 288): most of its Wilson phases
    crowd within ~1e-9 of 0, which the eigenphase path must resolve (the
    eigenvalues of the Hermitian matrix fix the phases, the vectors only their
    signs); two lines against the oracle, FP64 path."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = syn.served_model("bhz12", 3)
    kg = syn.kplane(32, 2)
    m = hl.N // 2
    out = P.wsurf(c, [hl], kg, 0, m)
    assert int(out["status"][0]) & ~orc.WINDING_UNRESOLVED == 0
    for i in range(2):
        ev, U, st = orc.eigh_grid(hl, kg[i], 0, m)
        W, _ = orc.wilson_matrix(U)
        ref = orc.eigphases(W)
        assert np.sum(np.abs(ref) < 1e-6) > m // 3  # the crowded cluster is there
        assert phase_set_error(out["theta"][0, i].cpu().numpy(), ref) < 1e-10
