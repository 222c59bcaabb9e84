"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each checks a closed form from
the paper's model equations, a value the paper prints, an exact invariant, a
special case with a known answer, or an independent brute-force computation.
"""
import json
import os

import numpy as np
import pytest

import synthetic as syn
from oracle import berry as orc
from tests.phase_metrics import phase_set_error

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")
S0 = np.eye(2)
S1 = np.array([[0, 1], [1, 0]], dtype=complex)
S2 = np.array([[0, -1j], [1j, 0]])
S3 = np.diag([1.0, -1.0]).astype(complex)


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


# ---------------------------------------------------------------- Bloch H
def _rand_k(rng, n, dim=3):
    return rng.uniform(-1, 1, size=(n, dim))


def test_bloch_h_matches_eq4_eq7_closed_forms():
    rng = np.random.default_rng(1)
    for kap in _rand_k(rng, 20):
        kx, ky, kz = 2 * np.pi * kap
        # eq. 4 with a general mass
        for m in (1.5, -1.0):
            Hc = np.sin(kx) * S1 + np.sin(ky) * S2 + (np.cos(kx) + np.cos(ky) + m) * S3
            assert np.max(np.abs(orc.bloch_hamiltonian(syn.qwz(m), kap) - Hc)) < 1e-15
        # eq. 7
        Hb = (np.sin(kx) * np.kron(S1, S1) + np.sin(ky) * np.kron(S1, S2)
              + (np.cos(kx) + np.cos(ky) + 1.5) * np.kron(S3, S0))
        assert np.max(np.abs(orc.bloch_hamiltonian(syn.bhz(), kap) - Hb)) < 1e-15
        # eq. 9
        Hh = (np.sin(kx) * np.kron(S1, S1) + np.sin(ky) * np.kron(S1, S2) + np.sin(kz) * np.kron(S1, S3)
              + (np.cos(kx) + np.cos(ky) + np.cos(kz) - 1.5) * np.kron(S3, S0)
              + 1.0 * (np.cos(kx) - np.cos(ky)) * np.kron(S2, S0))
        assert np.max(np.abs(orc.bloch_hamiltonian(syn.choti(1.0), kap) - Hh)) < 1e-15


def test_bloch_h_bbh_closed_form():
    g, l = 0.5, 1.0
    G1, G2, G3, G4 = syn.models.bbh_gammas()
    # Gamma matrices anticommute pairwise and square to one (Clifford algebra)
    Gs = [G1, G2, G3, G4]
    for a in range(4):
        for b in range(4):
            ac = Gs[a] @ Gs[b] + Gs[b] @ Gs[a]
            assert np.allclose(ac, 2 * np.eye(4) * (a == b))
    rng = np.random.default_rng(2)
    for kap in _rand_k(rng, 10, 2):
        kx, ky = 2 * np.pi * kap
        Hc = ((g + l * np.cos(kx)) * G4 + l * np.sin(kx) * G3
              + (g + l * np.cos(ky)) * G2 + l * np.sin(ky) * G1)
        assert np.max(np.abs(orc.bloch_hamiltonian(syn.bbh(g, l), kap) - Hc)) < 1e-15


def test_bloch_h_hermitian_bruteforce_all_models():
    rng = np.random.default_rng(3)
    models = [syn.qwz(-1), syn.bhz(), syn.bbh(), syn.bhz_disordered(3, 2.0, [9, 9]),
              syn.bhz_vacancies(4, 0.1, [9, 1]), syn.wannier_like(8, [9, 2])]
    for hl in models:
        for kap in _rand_k(rng, 3):
            H = orc.bloch_hamiltonian(hl, kap)
            assert np.max(np.abs(H - H.conj().T)) <= 1e-14 * np.sum(np.abs(hl.t))


def test_supercell_band_folding():
    """Eigenvalues of the clean L x L supercell are the unit-cell bands at folded k."""
    L = 3
    cell = syn.bhz()
    sc = syn.supercell(cell, L)
    rng = np.random.default_rng(4)
    for kap in _rand_k(rng, 4, 2):
        ev_sc = np.linalg.eigvalsh(orc.bloch_hamiltonian(sc, kap))
        ev_cell = []
        for a in range(L):
            for b in range(L):
                ev_cell.append(np.linalg.eigvalsh(orc.bloch_hamiltonian(cell, (kap + np.array([a, b])) / L)))
        ev_cell = np.sort(np.concatenate(ev_cell))
        assert np.max(np.abs(ev_sc - ev_cell)) < 1e-13


def test_vacancy_and_disorder_counts():
    hl = syn.bhz_vacancies(10, 0.02, [4, 1, 0])
    assert hl.N == 4 * (100 - 2)
    hl = syn.bhz_disordered(10, 3.0, [3, 3, 0])
    assert hl.N == 400
    wl = syn.wannier_like(6, [5, 2, 0])
    assert wl.meta["n_R"] == 29


# ---------------------------------------------------------------- eigensolver
def test_jacobi_matches_lapack_small():
    rng = np.random.default_rng(5)
    mats = []
    for n in (1, 2, 3, 5, 8, 16):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        mats.append(A + A.conj().T)
    mats.append(orc.bloch_hamiltonian(syn.supercell(syn.bhz(), 2), [0.13, 0.31]))
    for H in mats:
        wj, Vj = orc.jacobi_eigh(H)
        w, V = np.linalg.eigh(H)
        assert np.max(np.abs(wj - w)) < 1e-13 * max(1, np.max(np.abs(w)))
        assert np.max(np.abs(H @ Vj - Vj * wj)) < 1e-12 * max(1, np.max(np.abs(w)))


def test_qwz_eigenvalues_closed_form_and_residual():
    rng = np.random.default_rng(6)
    for kap in _rand_k(rng, 10, 2):
        kx, ky = 2 * np.pi * kap
        d = np.array([np.sin(kx), np.sin(ky), 1.5 + np.cos(kx) + np.cos(ky)])
        H = orc.bloch_hamiltonian(syn.qwz(1.5), kap)
        w, U, st = orc.eigh_bands(H, 0, 1)
        assert abs(w[0] + np.linalg.norm(d)) < 1e-14 and abs(w[1] - np.linalg.norm(d)) < 1e-14
        assert np.max(np.abs(H @ U - U * w[0])) < 1e-14
        assert abs(np.trace(U @ U.conj().T).real - 1) < 1e-14


def test_gap_closed_flag():
    H = orc.bloch_hamiltonian(syn.atomic([0.0, 0.0, 1.0]), [0, 0])
    _, _, st = orc.eigh_bands(H, 0, 1)
    assert st & orc.GAP_CLOSED


# ---------------------------------------------------------------- Wilson loop
def test_chern_number_of_eq4_matches_paper():
    g = golden()["qwz_m1p5_chern"]
    kg = syn.kplane(48, 48, e_par=(1, 0, 0), e_perp=(0, 1, 0))
    out = orc.wilson_surface(syn.qwz(1.5), kg, 0, 1)
    assert out["status"] == 0
    assert out["winding"] == g["value"]


@pytest.mark.parametrize("m,axis,expect", [
    (2.5, "x", 0),      # |m| > 2: trivial
    (-1.0, "x", -1),    # H(k + (pi, pi); m) = -H(k; -m): C(-m) = -C(m)
    (-1.0, "y", +1),    # exchanging loop and transverse axes flips the orientation
    (1.5, "y", -1),
])
def test_qwz_windings_from_symmetry(m, axis, expect):
    ex, ey = (1, 0, 0), (0, 1, 0)
    e_par, e_perp = (ex, ey) if axis == "x" else (ey, ex)
    kg = syn.kplane(40, 40, e_par=e_par, e_perp=e_perp)
    out = orc.wilson_surface(syn.qwz(m), kg, 0, 1)
    assert out["status"] == 0 and out["winding"] == expect


def test_ssh_berry_phase_is_pi_or_zero():
    for (v, w, expect) in [(0.3, 1.0, np.pi), (1.0, 0.3, 0.0)]:
        kg = syn.kplane(64, 1, e_par=(1, 0, 0), e_perp=(0, 0, 0))
        out = orc.wilson_surface(syn.ssh(v, w), kg, 0, 1)
        assert phase_set_error(out["theta"], np.full((1, 1), expect)) < 1e-12


def test_bond_shift_raw_modulus_closed_form():
    """Lower state (1, e^{ik})/sqrt2: raw product = prod (1 + e^{-i dk})/2 = -cos^n(pi/n)."""
    n = 16
    kg = syn.kplane(n, 1, e_par=(1, 0, 0), e_perp=(0, 0, 0))
    _, U, _ = orc.eigh_grid(syn.bond_shift_1d(), kg, 0, 1)
    Wr, _ = orc.wilson_matrix(U[0], "raw")
    assert abs(Wr[0, 0] - (-np.cos(np.pi / n) ** n)) < 1e-14
    Wp, _ = orc.wilson_matrix(U[0], "polar")
    assert abs(Wp[0, 0] - (-1.0)) < 1e-14


def test_atomic_limit_trivial():
    kg = syn.kplane(8, 8)
    out = orc.wilson_surface(syn.atomic([-1.0, -0.5, 2.0]), kg, 0, 2)
    assert np.max(np.abs(out["theta"])) < 1e-14 and out["winding"] == 0


def test_unitarity_trace_and_gauge_invariance():
    hl = syn.bhz_disordered(2, 1.0, [1, 2, 3])
    kg = syn.kplane(10, 6)
    ev, U, st = orc.eigh_grid(hl, kg, 0, hl.N // 2)
    m = hl.N // 2
    for i in range(kg.shape[0]):
        W, _ = orc.wilson_matrix(U[i])
        assert np.max(np.abs(W.conj().T @ W - np.eye(m))) < 1e-12
    P = U[0, 0] @ U[0, 0].conj().T
    assert abs(np.trace(P).real - m) < 1e-12
    th0, _, C0, _ = orc.wilson_loop_grid(U)
    rng = np.random.default_rng(7)
    Ug = U.copy()
    for i in range(U.shape[0]):
        for j in range(U.shape[1]):
            G, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
            Ug[i, j] = U[i, j] @ G
    th1, _, C1, _ = orc.wilson_loop_grid(Ug)
    assert phase_set_error(th0, th1) < 1e-12 and C0 == C1


def test_raw_vs_polar_det_identity():
    hl = syn.bhz_disordered(2, 2.0, [2, 2, 2])
    kg = syn.kplane(8, 4)
    _, U, _ = orc.eigh_grid(hl, kg, 0, hl.N // 2)
    tp, php, _, _ = orc.wilson_loop_grid(U, "polar")
    tr, phr, _, _ = orc.wilson_loop_grid(U, "raw")
    d = np.mod(php - phr + np.pi, 2 * np.pi) - np.pi
    assert np.max(np.abs(d)) < 1e-13
    # m = 1: the polar factor of a 1x1 overlap is its phase, so theta agrees exactly
    _, U1, _ = orc.eigh_grid(syn.qwz(1.5), syn.kplane(12, 5), 0, 1)
    assert phase_set_error(orc.wilson_loop_grid(U1, "raw")[0], orc.wilson_loop_grid(U1, "polar")[0]) < 1e-13


def test_eigphases_two_by_two_closed_form():
    rng = np.random.default_rng(8)
    for _ in range(20):
        Q, _ = np.linalg.qr(rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)))
        tr, det = np.trace(Q), np.linalg.det(Q)
        disc = np.sqrt(tr * tr - 4 * det)
        lam = np.array([(tr + disc) / 2, (tr - disc) / 2])
        expect = np.sort(np.angle(lam))
        assert phase_set_error(orc.eigphases(Q)[None], expect[None]) < 1e-13


def test_uniform_grid_shift_preserves_winding():
    kg = syn.kplane(40, 40, k0=(0.013, 0.021, 0))
    assert orc.wilson_surface(syn.qwz(1.5), kg, 0, 1)["winding"] == 1


def test_bhz_wcc_spectrum_gapless():
    assert golden()["bhz_wcc_gapless"]["value"] is True
    kg = syn.kplane(40, 40)
    out = orc.wilson_surface(syn.bhz(), kg, 0, 2)
    x = np.sort(np.mod(out["theta"].ravel() / (2 * np.pi), 1.0))
    gaps = np.diff(np.concatenate([x, [x[0] + 1]]))
    assert gaps.max() < 0.1   # the centres sweep the whole unit interval


# ---------------------------------------------------------------- nested loop
def test_bbh_nested_polarization_half():
    kg = syn.kplane(40, 40)
    out = orc.nested_wilson(syn.bbh(0.5, 1.0), kg, 0, 2)
    assert out["status"] == 0 and out["s"] == 1
    assert np.max(np.abs(np.abs(out["p"]) - 0.5)) < 1e-12
    assert abs(out["p_mean"] - 0.5) < 1e-12
    # Wannier bands of the first loop come in +-nu pairs
    th = orc.wilson_surface(syn.bbh(0.5, 1.0), kg, 0, 2)["theta"]
    assert np.max(np.abs(th[:, 0] + th[:, 1])) < 1e-12


def test_bbh_trivial_control_zero():
    kg = syn.kplane(24, 24)
    out = orc.nested_wilson(syn.bbh(1.5, 1.0), kg, 0, 2)
    assert out["status"] == 0
    assert np.max(np.abs(out["p"])) < 1e-12 and min(out["p_mean"], 1 - out["p_mean"]) < 1e-12


def test_nested_sector_selection_two_sectors():
    """Direct sum of two rank-one product models with centres near +0.3 and -0.3.

    The (0, 1/2) sector is the first model, whose y Berry phase is pi (p = 1/2);
    the (-1/2, 0) sector is the second, with no y dependence (p = 0).
    """
    hl = syn.concat_hops([syn.product_state_2d(0.7, 0.5), syn.product_state_2d(0.3, 0.0)])
    kg = syn.kplane(16, 12)
    out = orc.nested_wilson(hl, kg, 0, 2, window=(0.0, 0.5))
    assert out["status"] == 0 and out["s"] == 1
    assert abs(out["p_mean"] - 0.5) < 1e-12
    out = orc.nested_wilson(hl, kg, 0, 2, window=(-0.5, 0.0))
    assert out["status"] == 0 and out["s"] == 1
    assert min(out["p_mean"], 1 - out["p_mean"]) < 1e-12


# ---------------------------------------------------------------- spin-resolved
def test_bhz_spin_chern():
    conv = golden()["spin_chern_sign_convention"]["value"]
    kg = syn.kplane(32, 32)
    out = orc.spin_resolved_wilson(syn.bhz(), np.array([1.0, -1, -1, 1]), kg, 0, 2)
    assert out["status"] == 0
    assert np.max(np.abs(np.abs(out["mu"]) - 1)) < 1e-13
    assert out["C_dn"] == conv["C_dn"] and out["C_s"] == conv["C_s"] and out["C_up"] == 1
    assert orc.wilson_surface(syn.bhz(), kg, 0, 2)["winding"] == 0


def test_spin_block_reduction_clean_and_disordered():
    """With [H, S_z] = 0 the S_z = -1 sector is a model of its own.

    The spin-down Wilson loop from the projected spin operator must equal the
    plain Wilson loop of the sub-Hamiltonian on the S_z = -1 orbitals.
    """
    def restrict(hl, keep_mask):
        keep = np.nonzero(keep_mask)[0]
        cmap = -np.ones(hl.N, dtype=np.int64)
        cmap[keep] = np.arange(keep.size)
        sel = keep_mask[hl.i] & keep_mask[hl.j]
        return syn.HopList(N=keep.size, dim=hl.dim, i=cmap[hl.i[sel]].astype(np.int32),
                           j=cmap[hl.j[sel]].astype(np.int32), R=hl.R[sel], t=hl.t[sel])

    for hl in (syn.bhz(), syn.bhz_disordered(2, 2.0, [6, 1, 0])):
        sd = syn.bhz_spin_diag(hl)
        kg = syn.kplane(16, 12)
        m = hl.N // 2
        out = orc.spin_resolved_wilson(hl, sd, kg, 0, m)
        dn = restrict(hl, sd < 0)
        up = restrict(hl, sd > 0)
        ref_dn = orc.wilson_surface(dn, kg, 0, dn.N // 2)
        ref_up = orc.wilson_surface(up, kg, 0, up.N // 2)
        assert out["status"] == 0
        assert phase_set_error(out["theta_dn"], ref_dn["theta"]) < 1e-12
        assert phase_set_error(out["theta_up"], ref_up["theta"]) < 1e-12
        assert out["C_dn"] == ref_dn["winding"] and out["C_up"] == ref_up["winding"]
    # clean BHZ down block is QWZ(kx, -ky): theta_dn(ky_i) = theta_QWZ(ky_{n-i})
    kg = syn.kplane(16, 12)
    out = orc.spin_resolved_wilson(syn.bhz(), np.array([1.0, -1, -1, 1]), kg, 0, 2)
    q = orc.wilson_surface(syn.qwz(1.5), kg, 0, 1)["theta"]
    n = kg.shape[0]
    flipped = q[[(n - i) % n for i in range(n)]]
    assert phase_set_error(out["theta_dn"], flipped) < 1e-12


def test_choti_spin_chern_matches_paper():
    g = golden()["choti_kz0_abs_spin_chern"]
    kg = syn.kplane(32, 32)
    hl = syn.choti(1.0)
    out = orc.spin_resolved_wilson(hl, np.array([1.0, -1, -1, 1]), kg, 0, 2)
    assert out["status"] == 0
    assert abs(out["C_s"]) == g["value"]
    assert np.max(np.abs(np.abs(out["mu"]) - 1)) > 1e-3   # spin not conserved here
    # the plain WCC spectrum is gapped at kz = 0 (Sec. III)
    th = orc.wilson_surface(hl, kg, 0, 2)["theta"]
    x = np.sort(np.mod(th.ravel() / (2 * np.pi), 1.0))
    gaps = np.diff(np.concatenate([x, [x[0] + 1]]))
    assert gaps.max() > 0.2


def test_singular_overlap_flagged():
    """Uncoupled orbitals with energies +-cos 2 pi k: the occupied state jumps
    from one orbital to the other between grid points, the overlap there is
    exactly zero and the loop is flagged instead of given a phase."""
    from synthetic.models import _from_blocks
    hl = _from_blocks(2, 1, {(0,): np.zeros((2, 2)), (1,): np.diag([0.5, -0.5])})
    kg = syn.kplane(8, 2, k0=(1.0 / 16, 0.0, 0.0))
    out = orc.wilson_surface(hl, kg, 0, 1)
    assert out["status"] & orc.OVERLAP_SINGULAR
    # a smooth path (no switch) is not flagged
    out = orc.wilson_surface(syn.qwz(1.5), syn.kplane(16, 4), 0, 1)
    assert not out["status"] & orc.OVERLAP_SINGULAR


# ---------------------------------------------------------------- Berry flux per plaquette
@pytest.mark.parametrize("m,C", [(-1.0, 1), (1.5, -1), (2.5, 0)])
def test_plaquette_flux_chern_equals_wilson_winding(m, C):
    """The plaquette sum is 2 pi times an integer to rounding, and it is the
    Chern number of the Wilson-loop winding (eq. 6) for QWZ in each phase."""
    kg = syn.kplane(24, 20, e_par=(0, 1, 0), e_perp=(1, 0, 0))
    f = orc.plaquette_flux(syn.qwz(m), kg, 0, 1)
    assert f["status"] == 0
    assert abs(f["total"] - round(f["total"])) < 1e-12
    assert f["chern"] == C
    assert orc.wilson_surface(syn.qwz(m), kg, 0, 1)["winding"] == C


def test_plaquette_flux_converges_to_two_band_curvature():
    """Closed form for a two-band model H = d(k).sigma: the Berry curvature of
    the lower band is (1/2) d.(d_x d x d_y d)/|d|^3 up to the orientation,
    so the flux per plaquette approaches it times the plaquette area."""
    n = 48
    M = -1.0
    kg = syn.kplane(n, n, e_par=(0, 1, 0), e_perp=(1, 0, 0))
    F = orc.plaquette_flux(syn.qwz(M), kg, 0, 1)["flux"]      # [i (kx), j (ky)]
    kx = 2 * np.pi * (np.arange(n) + 0.5) / n
    KX, KY = np.meshgrid(kx, kx, indexing="ij")
    d = np.stack([np.sin(KX), np.sin(KY), M + np.cos(KX) + np.cos(KY)])
    dx = np.stack([np.cos(KX), 0 * KX, -np.sin(KX)])
    dy = np.stack([0 * KY, np.cos(KY), -np.sin(KY)])
    omega = 0.5 * np.einsum("i...,i...->...", d, np.cross(dx, dy, axis=0)) / np.linalg.norm(d, axis=0) ** 3
    ref = omega * (2 * np.pi / n) ** 2
    sign = np.sign(np.sum(F * ref))
    assert sign != 0
    assert np.max(np.abs(F - sign * ref)) < 0.02 * np.max(np.abs(F))
    assert abs(sign * ref.sum() / (2 * np.pi) - round(F.sum() / (2 * np.pi))) < 0.02


def test_plaquette_flux_trivial_and_gauge_invariant():
    """An atomic insulator carries no flux; random unitary rotations of the
    occupied basis at every k leave every plaquette's flux unchanged."""
    kg = syn.kplane(6, 5)
    f = orc.plaquette_flux(syn.atomic([-1.0, -0.5, 2.0]), kg, 0, 2)
    assert np.max(np.abs(f["flux"])) < 1e-14 and f["chern"] == 0
    hl = syn.bhz_disordered(2, 1.0, [7, 7, 7])
    ev, U, st = orc.eigh_grid(hl, kg, 0, hl.N // 2)
    rng = np.random.default_rng(3)
    R = np.linalg.qr(rng.standard_normal(U.shape[:2] + (U.shape[-1],) * 2)
                     + 1j * rng.standard_normal(U.shape[:2] + (U.shape[-1],) * 2))[0]
    a = orc.plaquette_flux_from_grid(U)["flux"]
    b = orc.plaquette_flux_from_grid(U @ R)["flux"]
    assert np.max(np.abs(a - b)) < 1e-12


def test_spin_resolved_flux_bhz():
    """Spin sectors of BHZ (Sec. IV): C_dn = -1, C_up = +1, C_s = +1, the
    values the spin-resolved Wilson loop gives."""
    kg = syn.kplane(16, 16)
    out = orc.spin_resolved_flux(syn.bhz(), np.array([1.0, -1, -1, 1]), kg, 0, 2)
    assert out["status"] == 0
    assert (out["C_dn"], out["C_up"], out["C_s"]) == (-1, 1, 1.0)
    w = orc.spin_resolved_wilson(syn.bhz(), np.array([1.0, -1, -1, 1]), kg, 0, 2)
    assert (w["C_dn"], w["C_up"]) == (out["C_dn"], out["C_up"])


def test_plaquette_flux_singular_link_flagged():
    """The occupied state of two uncoupled orbitals with energies +-cos 2 pi k
    jumps from one orbital to the other: the link across the switch is the
    zero matrix and its plaquettes are flagged; a smooth grid is not."""
    from synthetic.models import _from_blocks
    hl = _from_blocks(2, 1, {(0,): np.zeros((2, 2)), (1,): np.diag([0.5, -0.5])})
    kg = syn.kplane(8, 3, k0=(1.0 / 16, 0.0, 0.0))
    f = orc.plaquette_flux(hl, kg, 0, 1)
    assert f["status"] & orc.OVERLAP_SINGULAR
    f = orc.plaquette_flux(syn.qwz(1.5), syn.kplane(12, 10), 0, 1)
    assert not f["status"] & orc.OVERLAP_SINGULAR


@pytest.mark.parametrize("m,c", [(100, 0.8), (640, 0.97)])
def test_flux_singular_flag_independent_of_order(m, c):
    """Links of order m whose singular values are all c: |det| = c^m is far
    below 1e-8 (2e-10 and 3e-9), yet every singular value is of order one,
    so no link is singular and the flux is defined (zero here: the link
    matrices are real and positive). The Wilson loop's criterion for the
    same overlaps (sigma_min < 1e-8) agrees."""
    assert c ** m < 1e-8
    g = syn.link_grid(np.full(m, c))
    f = orc.plaquette_flux_from_grid(g)
    assert not f["status"] & orc.OVERLAP_SINGULAR
    assert np.max(np.abs(f["flux"])) < 1e-12 and f["chern"] == 0
    assert not orc.wilson_loop_grid(g)[3] & orc.OVERLAP_SINGULAR


@pytest.mark.parametrize("m", [1, 100])
def test_flux_singular_flag_one_small_singular_value(m):
    """One singular value of 1e-9 among ones: the link is singular by the
    sigma_min < 1e-8 test (its |det| is 1e-9 too), and so is the Wilson-loop
    overlap; 1e-7 is not."""
    for s, flagged in ((1e-9, True), (1e-7, False)):
        cs = np.ones(m)
        cs[m // 2] = s
        g = syn.link_grid(cs)
        assert bool(orc.plaquette_flux_from_grid(g)["status"] & orc.OVERLAP_SINGULAR) == flagged
        assert bool(orc.wilson_loop_grid(g)[3] & orc.OVERLAP_SINGULAR) == flagged


def test_wannier_gap_flag_on_window_edge():
    """Atomic limit: the Wilson loop is the identity, so every phase is 0,
    exactly on the lower edge of the sector window (0, 1/2)."""
    out = orc.nested_wilson(syn.atomic([-1.0, -0.5, 2.0]), syn.kplane(6, 4), 0, 2)
    assert out["status"] & orc.WANNIER_GAP


def test_wannier_gap_flag_when_sector_size_varies():
    """Chern insulator (eq. 4, one band): the single Wilson phase winds once
    through (-pi, pi] across the transverse direction, so the number of
    phases inside (0, 1/2) changes from one line to the next although no
    phase on the grid sits within 1e-6 of a window edge (the transverse grid
    is shifted off the symmetric lines, where the phase is 0 or pi)."""
    kg = syn.kplane(12, 16, k0=(0.0, 0.013, 0.0))
    th = orc.wilson_surface(syn.qwz(1.5), kg, 0, 1)["theta"].ravel() / (2 * np.pi)
    assert np.min(np.abs(np.concatenate([th, th - 0.5]))) > 1e-6
    counts = {int(((x > 0) & (x < 0.5)).sum()) for x in th.reshape(-1, 1)}
    assert counts == {0, 1}
    out = orc.nested_wilson(syn.qwz(1.5), kg, 0, 1)
    assert out["status"] & orc.WANNIER_GAP
    # the BBH model's sector is fixed (one phase per line in (0, 1/2)): no flag
    assert not orc.nested_wilson(syn.bbh(0.5, 1.0), syn.kplane(10, 10), 0, 2)["status"] & orc.WANNIER_GAP


def test_pso_gap_flag_zero_eigenvalue():
    """A spin operator that vanishes on the occupied orbital: P S P has the
    eigenvalue 0 exactly."""
    out = orc.spin_resolved_wilson(syn.atomic([-1.0, 2.0]), np.array([0.0, 1.0]), syn.kplane(4, 3), 0, 1)
    assert out["status"] & orc.PSO_GAP
    assert np.max(np.abs(out["mu"])) == 0.0


def test_pso_gap_flag_when_sector_count_varies():
    """Two uncoupled orbitals with energies +-cos 2 pi k and spins +1, -1:
    the occupied orbital, hence the sign of P S P's single eigenvalue,
    switches across the zone, so the spin-down count varies while |mu| = 1
    everywhere."""
    from synthetic.models import _from_blocks
    hl = _from_blocks(2, 1, {(0,): np.zeros((2, 2)), (1,): np.diag([0.5, -0.5])})
    kg = syn.kplane(8, 2, k0=(1.0 / 16, 0.0, 0.0))
    out = orc.spin_resolved_wilson(hl, np.array([1.0, -1.0]), kg, 0, 1)
    assert out["status"] & orc.PSO_GAP
    ev, U, _ = orc.eigh_grid(hl, kg, 0, 1)
    mus = np.array([orc.spin_sectors(u, np.array([1.0, -1.0]))[0] for u in U.reshape(-1, 2, 1)])
    assert np.allclose(np.abs(mus), 1.0) and (mus < 0).any() and (mus > 0).any()
    # the same switch is a PSO gap for the flux of the spin sectors too
    assert orc.spin_resolved_flux(hl, np.array([1.0, -1.0]), kg, 0, 1)["status"] & orc.PSO_GAP


def test_nan_inf_flag():
    """A non-finite hopping amplitude makes H non-finite at every k: the
    eigenpairs carry NAN_INF instead of eigenvalues."""
    hl = syn.qwz(1.5)
    hl.t = hl.t.copy()
    hl.t[0] = np.nan
    ev, U, st = orc.eigh_grid(hl, syn.kplane(3, 2), 0, 1)
    assert st & orc.NAN_INF
    assert np.isnan(ev).all()
    assert not orc.eigh_grid(syn.qwz(1.5), syn.kplane(3, 2), 0, 1)[2] & orc.NAN_INF


def test_plaquette_flux_is_local():
    """A plaquette's flux depends on its four corners only: the map of the
    2 x 2 grid of those corners holds it at (0, 0) (how full-size maps are
    sampled in the parity tests)."""
    hl = syn.bhz_disordered(2, 1.0, [7, 1])
    kg = syn.kplane(5, 4)
    m = hl.N // 2
    full = orc.plaquette_flux(hl, kg, 0, m)["flux"]
    for i, j in ((0, 0), (3, 4), (2, 1)):
        sub = kg[[i, (i + 1) % 4]][:, [j, (j + 1) % 5]]
        assert abs(orc.plaquette_flux(hl, sub, 0, m)["flux"][0, 0] - full[i, j]) < 1e-12


# ---------------------------------------------------------------- spinful BBH with chiral disorder
def test_spinful_bbh_reading_chiral_and_gapped():
    """Eq. 10 with the quadrupolar mass read as s0 (x) t1: H anticommutes with
    S = s0 (x) t2 (also with the disorder w s0 (x) t3) and is gapped at half
    filling; the printed s0 (x) t0 commutes with S and closes the gap at
    half filling: at k = (pi, 0) and (0, pi) (sin kx = sin ky = 0, mass term
    +-1) it shifts the spectrum by -1 and +1, so the second band reaches 0 at
    one point and the third band comes down to 0 at the other."""
    S = np.kron(np.eye(2), np.array([[0, -1j], [1j, 0]]))
    rng = np.random.default_rng(8)
    hls = [syn.spinful_bbh(), syn.spinful_bbh_disordered(3, 2.0, [4, 4])]
    for hl in hls:
        Sb = np.kron(np.eye(hl.N // 4), S)
        for _ in range(4):
            H = orc.bloch_hamiltonian(hl, np.r_[rng.random(2), 0.0])
            assert np.abs(Sb @ H @ Sb.conj().T + H).max() < 1e-13
    w = np.linalg.eigvalsh(orc.bloch_hamiltonian(hls[0], np.array([0.5, 0.0, 0.0])))
    assert w[2] - w[1] > 1.0
    s3t3 = np.kron(np.diag([1.0, -1.0]), np.diag([1.0, -1.0]))
    # (pi, 0): mass cos pi + cos 0 + 1 = 1, printed term 0.5 (cos pi - cos 0) = -1; (0, pi): +1
    wa = np.linalg.eigvalsh(1.0 * s3t3 - 1.0 * np.eye(4))
    wb = np.linalg.eigvalsh(1.0 * s3t3 + 1.0 * np.eye(4))
    assert wb[1] >= wa[2] - 1e-15


def test_spinful_bbh_spin_chern_against_paper():
    """Fig. 5c-d: C_s = 1 at W = 1 and 0 at W = 9. Clean and weakly disordered
    supercells give C_s = +1 by the plaquette flux and by the spin-resolved
    Wilson loop (with a PSO spectrum away from +-1: spin is not conserved);
    at W = 9 no realization keeps |C_s| = 1 (each is 0, or its PSO gap has
    closed)."""
    g = golden()
    hl = syn.spinful_bbh()
    sd = syn.spinful_bbh_spin_diag(hl)
    kg = syn.kplane(12, 12)
    f = orc.spin_resolved_flux(hl, sd, kg, 0, 2)
    w = orc.spin_resolved_wilson(hl, sd, kg, 0, 2)
    assert f["status"] == 0 and w["status"] == 0
    assert f["C_s"] == w["C_s"] == g["spinful_bbh_W1_spin_chern"]["value"]
    assert np.abs(np.abs(w["mu"]) - 1).max() > 0.2
    for r in range(3):
        h = syn.spinful_bbh_disordered(5, 1.0, [2, r])
        o = orc.spin_resolved_flux(h, syn.spinful_bbh_spin_diag(h), syn.kplane(6, 6), 0, h.N // 2)
        assert o["status"] == 0 and o["C_s"] == g["spinful_bbh_W1_spin_chern"]["value"]
    for r in range(3):
        h = syn.spinful_bbh_disordered(5, 9.0, [2, r])
        o = orc.spin_resolved_flux(h, syn.spinful_bbh_spin_diag(h), syn.kplane(6, 6), 0, h.N // 2)
        assert (o["status"] & orc.PSO_GAP) or o["C_s"] == g["spinful_bbh_W9_spin_chern"]["value"]


def test_choti_nested_spectrum_gapless_against_kz():
    """Sec. III, Fig. 4b: the nested spectrum of the chiral HOTI (eq. 9,
    Delta0 = 1; loop along kx, nested along ky) is gapless against kz: the
    nested polarization p(kz) winds once around the circle as kz runs over
    the zone (a Chern-insulator-like flow), while each plane is resolved."""
    assert golden()["choti_nested_gapless_vs_kz"]["value"] is True
    hl = syn.choti(1.0)
    ps = []
    for kz in np.arange(20) / 20:
        out = orc.nested_wilson(hl, syn.kplane(16, 16, k0=(0.0, 0.0, kz)), 0, 2)
        assert out["status"] == 0 and out["s"] == 1
        ps.append(out["p_mean"])
    d = np.diff(np.r_[ps, ps[0]])
    d -= np.round(d)
    assert abs(abs(d.sum()) - 1.0) < 1e-9
    assert np.abs(d).max() < 0.3   # resolved: no step near half a turn
