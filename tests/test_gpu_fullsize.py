"""Parity at the full sizes of the workloads, on outputs the oracle can afford.

* Spin-resolved BHZ 10x10 supercells (N = 400, m = 200, 24 x 24 grid) in the
  launch configuration of the benchmark: eight systems (4608 matrices) per
  eigensolver call. Two transverse lines per chunk are recomputed by the FP64
  oracle; every line's spin Chern data are checked for consistency.
* The largest uneven-size supercell (L = 20 with 2 % vacancies, N = 1568, 16 x 16
  grid): one Wilson line against the oracle, eigenvalues at sampled k-points.
* The largest served request size (L = 24, N = 2304, one 32-point line):
  eigenvalues at sampled k-points against LAPACK, the invariant-subspace residual,
  the total Berry phase of the polar and raw overlap modes against each other
  (arg det W is the same in both, since the polar factor only rescales each
  det F by a positive number), and the phases of the mixed path against FP64.
Tolerances: 1e-10 rad for FP64 phases, 1e-6 rad for the mixed path.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import berry as orc
from tests import gpu_util as gu
from tests.phase_metrics import phase_set_error

torch = gu.torch
pytestmark = pytest.mark.gpu


def pipe():
    from paper_2312_13051_amd import pipeline
    return pipeline


def oracle_spin_line(hl, sd, kline, m):
    """theta_dn, theta_up of one Wilson line with the oracle (None if the sectors are uneven)."""
    ev, U, st = orc.eigh_grid(hl, kline, 0, m)
    vm, vp = [], []
    for j in range(kline.shape[0]):
        _, a, b = orc.spin_sectors(U[j], sd)
        vm.append(a)
        vp.append(b)
    out = []
    for V in (vm, vp):
        W, _ = orc.wilson_matrix(np.stack(V))
        out.append(orc.eigphases(W))
    return out


@pytest.mark.parametrize("w_idx,precision", [(0, 0), (3, 0), (3, 1), (3, 2)])
def test_bhz_supercell_bench_chunk(w_idx, precision):
    """Eight BHZ 10x10 systems at disorder W = w_idx in one eigensolver launch
    (FP64 and refined paths within 1e-10 rad of the oracle, mixed within 1e-6)."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hls = [syn.bhz_disordered(10, float(w_idx), [3, w_idx, r]) for r in range(8)]
    kg = syn.kplane(24, 24)
    m = hls[0].N // 2
    sd = np.stack([syn.bhz_spin_diag(h) for h in hls])
    out = P.wspinsurf(c, hls, sd, kg, 0, m, precision=precision, chunk=8 * 24 * 24)
    tol = 1e-6 if precision == 1 else 1e-10
    st = out["status"].cpu().numpy()
    eig_st = out["eig"].status.view(8, -1).cpu().numpy()
    assert (eig_st == 0).all()
    if w_idx == 0:
        # clean supercell: every realization is the same crystal, C_s = +1
        assert (st == 0).all()
        assert out["m_dn"] == [m // 2] * 8
        assert (out["C_s"].cpu().numpy() == 1.0).all()
    for r, i in ((0, 5), (5, 17)):
        md = out["m_dn"][r]
        a, b = oracle_spin_line(hls[r], sd[r], kg[i], m)
        assert a.size == md
        assert phase_set_error(out["theta_dn"][r, i, :md].cpu().numpy(), a) < tol
        assert phase_set_error(out["theta_up"][r, i, :m - md].cpu().numpy(), b) < tol


def test_largest_uneven_supercell_line():
    """BHZ 20x20 with 2 % vacancies (N = 1568), 16 x 16 grid, all occupied bands."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = syn.bhz_vacancies(20, 0.02, [4, 1, 0])
    assert hl.N == 1568
    kg = syn.kplane(16, 16)
    m = hl.N // 2
    out = P.wsurf(c, [hl], kg, 0, m)
    g = out["eig"]
    assert int(out["status"][0]) == 0
    i = 9
    ref = orc.wilson_surface(hl, kg[i:i + 1], 0, m)
    assert phase_set_error(out["theta"][0, i].cpu().numpy(), ref["theta"][0]) < 1e-10
    ev = g.evals.view(16, 16, m + 2).cpu().numpy()
    for (ii, jj) in ((0, 0), (11, 4)):
        w = np.linalg.eigvalsh(orc.bloch_hamiltonian(hl, kg[ii, jj]))
        assert np.max(np.abs(ev[ii, jj, 1:m + 1] - w[:m])) < 1e-12 * max(1.0, np.abs(w).max())
    mixed = P.wsurf(c, [hl], kg, 0, m, precision=1)
    assert phase_set_error(mixed["theta"][0, i].cpu().numpy(), ref["theta"][0]) < 1e-6


def test_largest_served_request_line():
    """BHZ 24x24 with disorder (N = 2304), one 32-point Wilson line: eigenpairs
    of one k-point against LAPACK, polar against raw overlaps, mixed against
    FP64, and the Wilson stage against the oracle's on the GPU eigenvectors."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = syn.bhz_disordered(24, 2.5, [5, 1, 0])
    assert hl.N == 2304
    kg = syn.kplane(32, 1, k0=(0.0, 0.3, 0.0))
    m = hl.N // 2
    out = P.wsurf(c, [hl], kg, 0, m)
    g = out["eig"]
    assert int(g.status.max()) == 0
    U = gu.to_np(g.U[7:8], hl.N)[0, :, :m]
    H = orc.bloch_hamiltonian(hl, kg[0, 7])
    w = np.linalg.eigvalsh(H)
    nrm = max(1.0, np.abs(w).max())
    ev = g.evals.cpu().numpy()
    assert np.max(np.abs(ev[7, 1:m + 1] - w[:m])) < 1e-12 * nrm
    assert np.max(np.abs(U.conj().T @ U - np.eye(m))) < 1e-10
    HU = H @ U
    assert np.max(np.abs(HU - U @ (U.conj().T @ HU))) < 1e-10 * nrm
    raw = P.wsurf(c, [hl], kg, 0, m, mode=1)
    d = float(out["phi"][0, 0]) - float(raw["phi"][0, 0])
    assert abs(np.mod(d + np.pi, 2 * np.pi) - np.pi) < 1e-8
    th = out["theta"][0, 0].cpu().numpy()
    mixed = P.wsurf(c, [hl], kg, 0, m, precision=1)
    assert phase_set_error(th, mixed["theta"][0, 0].cpu().numpy()) < 1e-6
    # the Wilson stage at order 1152 (overlaps, polar factors, product, eigenphases
    # through the Hermitian route) against the oracle's on the same eigenvectors
    Ul = gu.to_np(g.U, hl.N)[:, :, :m]
    W, _ = orc.wilson_matrix(Ul)
    assert phase_set_error(th, orc.eigphases(W)) < 1e-10
