"""Wannier90 ingestion and spin-axis rotation (host side, no GPU).

Files are written by ``synthetic.write_tb`` from seeded models and read back
by ``paper_2312_13051_amd.w90.read_tb``; Bloch Hamiltonians are compared with
the oracle's, and the spin-axis rotation is checked against the oracle's
projected spin spectrum of the dense operator n.sigma.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import berry as orc
from paper_2312_13051_amd import w90

S1 = np.array([[0, 1], [1, 0]], dtype=complex)
S2 = np.array([[0, -1j], [1j, 0]])
S3 = np.diag([1.0, -1.0]).astype(complex)


def pair_op(N, axis, order="interleaved"):
    n = np.asarray(axis, float) / np.linalg.norm(axis)
    s = n[0] * S1 + n[1] * S2 + n[2] * S3
    S = np.zeros((N, N), dtype=complex)
    for a, b in w90.spin_pairs(N, order):
        S[np.ix_([a, b], [a, b])] = s
    return S


def deg(R):
    return 1 + (abs(R[0]) + abs(R[1]) + abs(R[2]) >= 2) + 2 * (abs(R[0]) >= 3)


@pytest.mark.parametrize("which", ["rotated_bhz", "wannier24"])
def test_tb_round_trip(tmp_path, which):
    """write_tb then read_tb gives the same H(k) (degeneracies divided out)."""
    hl = syn.rotated_bhz((1, 0, 0)) if which == "rotated_bhz" else syn.wannier_like(24, [5, 2, 9])
    lat = np.array([[4.3, 0, 0], [-2.15, 3.72, 0], [0, 0, 20.0]])
    path = tmp_path / "m_tb.dat"
    syn.write_tb(hl, path, lat, degeneracy=deg)
    m = w90.read_tb(path, dim=2)
    assert m.N == hl.N and np.allclose(m.lattice, lat)
    rng = np.random.default_rng(3)
    for _ in range(4):
        k = np.r_[rng.random(2), 0.0]
        assert np.abs(orc.bloch_hamiltonian(m, k) - orc.bloch_hamiltonian(hl, k)).max() < 1e-13


def test_tb_cutoffs(tmp_path):
    """ECut keeps |t| >= ECut; HopCut keeps |R.A + c_j - c_i| <= HopCut."""
    hl = syn.wannier_like(12, [5, 2, 1])
    lat = np.diag([3.0, 3.0, 10.0])
    cen = np.random.default_rng(4).random((12, 3))
    syn.write_tb(hl, tmp_path / "w_tb.dat", lat)
    syn.write_centres(cen, tmp_path / "w_centres.xyz", atoms=[("Bi", (0.1, 0.2, 0.3))])
    full = w90.read_tb(tmp_path / "w_tb.dat", dim=2)
    assert np.allclose(w90.read_centres(tmp_path / "w_centres.xyz"), cen)
    ec = 0.05
    cut = w90.read_tb(tmp_path / "w_tb.dat", ecut=ec, dim=2)
    assert np.abs(cut.t).min() >= ec
    assert cut.nnz == int((np.abs(full.t) >= ec).sum())
    hc = 4.0
    hop = w90.read_tb(tmp_path / "w_tb.dat", hopcut=hc, centres=tmp_path / "w_centres.xyz", dim=2)
    d = np.linalg.norm(np.c_[hop.R, np.zeros(hop.nnz)] @ lat + cen[hop.j] - cen[hop.i], axis=1)
    assert d.max() <= hc
    dfull = np.linalg.norm(np.c_[full.R, np.zeros(full.nnz)] @ lat + cen[full.j] - cen[full.i], axis=1)
    assert hop.nnz == int((dfull <= hc).sum()) and hop.nnz < full.nnz
    # the cut model is still Hermitian: H(k) = H(k)^H
    H = orc.bloch_hamiltonian(hop, np.array([0.3, 0.7, 0.0]))
    assert np.abs(H - H.conj().T).max() < 1e-14


def test_tb_malformed(tmp_path):
    p = tmp_path / "bad_tb.dat"
    p.write_text("x\n1 0 0\n0 1 0\n0 0 1\n1\n1\n1\n\n1 0 0\n1 1 0.5 0.0\n")
    with pytest.raises(ValueError, match="partner"):
        w90.read_tb(p)
    hl = syn.choti(1.0)
    syn.write_tb(hl, tmp_path / "c_tb.dat")
    with pytest.raises(ValueError, match="layer"):
        w90.read_tb(tmp_path / "c_tb.dat", dim=2)
    assert w90.read_tb(tmp_path / "c_tb.dat").dim == 3


@pytest.mark.parametrize("order", ["interleaved", "blocked"])
def test_spin_axis_rotation_preserves_pso_spectrum(order):
    """The PSO spectrum of n.sigma in the original basis equals that of the
    diagonal operator in the rotated basis, for any axis."""
    hl = syn.wannier_like(8, [1, 2, 3])
    rng = np.random.default_rng(11)
    for _ in range(3):
        ax = rng.standard_normal(3)
        rot, diag = w90.rotate_spin_axis(hl, ax, order)
        for _ in range(2):
            k = np.r_[rng.random(2), 0.0]
            a = orc.pso_spectrum(hl, k, 0, 4, pair_op(8, ax, order))
            b = orc.pso_spectrum(rot, k, 0, 4, np.diag(diag))
            assert np.abs(a - b).max() < 1e-12


def test_rotated_bhz_conserves_spin_along_its_axis():
    """BHZ with the spin axis turned to x: the PSO of x.sigma is exactly +-1
    (spin conserved), that of z.sigma is not."""
    hl = syn.rotated_bhz((1, 0, 0))
    k = np.array([0.17, 0.41, 0.0])
    mx = orc.pso_spectrum(hl, k, 0, 2, pair_op(4, (1, 0, 0)))
    mz = orc.pso_spectrum(hl, k, 0, 2, pair_op(4, (0, 0, 1)))
    assert np.abs(np.abs(mx) - 1).max() < 1e-12
    assert np.abs(np.abs(mz) - 1).max() > 1e-3
    # BHZ itself (axis z) in the same interleaved basis
    hz = syn.rotated_bhz((0, 0, 1))
    assert np.abs(np.abs(orc.pso_spectrum(hz, k, 0, 2, pair_op(4, (0, 0, 1)))) - 1).max() < 1e-12


def test_axes_grid_covers_hemisphere():
    ax = w90.axes_grid(4, 6)
    assert np.allclose(np.linalg.norm(ax, axis=1), 1.0)
    assert (ax[:, 2] >= -1e-12).all()
    assert any(np.allclose(a, [1, 0, 0]) for a in ax) and any(np.allclose(a, [0, 1, 0]) for a in ax)
