"""GPU path on Wannier90-ingested models (Sec. V workflow: read the
tight-binding file with cutoffs, scan the projected spin spectrum over a
grid of 400 k-points for a gapped spin axis, then the spin-resolved loop),
against the oracle. Files are written from seeded models (the paper's
bismuthene and PdTe2 files are not available).
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import berry as orc
from paper_2312_13051_amd import w90
from tests import gpu_util as gu
from tests.phase_metrics import phase_set_error
from tests.test_w90 import deg, pair_op

torch = gu.torch
pytestmark = pytest.mark.gpu
TOL = 1e-10


def pipe():
    from paper_2312_13051_amd import pipeline
    return pipeline


@pytest.fixture(scope="module")
def rotated_model(tmp_path_factory):
    d = tmp_path_factory.mktemp("w90")
    hl = syn.rotated_bhz((1.0, 0.0, 0.0), L=2, W=1.0, seed=(3,))
    syn.write_tb(hl, d / "rb_tb.dat", np.diag([4.0, 4.0, 20.0]), degeneracy=deg)
    return w90.read_tb(d / "rb_tb.dat", ecut=1e-12, dim=2)


def test_spin_axis_scan_against_oracle(rotated_model):
    """PSO spectra of 19 candidate axes on a 20 x 20 grid in one batch; three
    axes checked at every k-point against the oracle's dense n.sigma; the
    scan picks the conserved axis x (spectrum +-1)."""
    gu.need_gpu()
    c = gu.ctx()
    m = rotated_model
    kg = syn.kplane(20, 20).reshape(-1, 3)
    axes = w90.axes_grid(4, 6)
    out = w90.scan_spin_axes(c, m, kg, 0, m.N // 2, axes)
    assert (out["status"] & ~8 == 0).all()
    assert abs(abs(out["axis"][0]) - 1.0) < 1e-12 and abs(out["gap"].max() - 1.0) < 1e-10
    for q in (0, 3, len(axes) - 1):
        S = pair_op(m.N, axes[q])
        ref = np.array([orc.pso_spectrum(m, k, 0, m.N // 2, S) for k in kg])
        assert np.abs(out["mu"][q] - ref).max() < TOL


def test_spin_chern_on_chosen_axis(rotated_model):
    """After rotating to the chosen axis, the spin-resolved Wilson loop and
    the spin-resolved plaquette flux give the oracle's C_s (|C_s| = 1)."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    m = rotated_model
    rot, diag = w90.rotate_spin_axis(m, (1.0, 0.0, 0.0))
    kg = syn.kplane(12, 10)
    nb = m.N // 2
    wl = P.wspinsurf(c, [rot], diag[None, :], kg, 0, nb)
    fl = P.wspinflux(c, [rot], diag[None, :], kg, 0, nb)
    ref = orc.spin_resolved_wilson(rot, diag, kg, 0, nb)
    assert int(wl["status"][0]) == ref["status"] == 0
    assert float(wl["C_s"][0]) == ref["C_s"] and abs(ref["C_s"]) == 1.0
    assert float(fl["C_s"][0]) == ref["C_s"]
    md = wl["m_dn"][0]
    assert phase_set_error(wl["theta_dn"][0, :, :md].cpu().numpy(), ref["theta_dn"]) < TOL


def test_many_band_file_wilson(tmp_path):
    """A 96-orbital model through a _tb.dat file with degeneracies and an
    energy cutoff: Wilson phases against the oracle on the parsed model."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = syn.wannier_like(96, [5, 2, 3])
    syn.write_tb(hl, tmp_path / "w96_tb.dat", np.diag([5.0, 5.0, 30.0]), degeneracy=deg)
    m = w90.read_tb(tmp_path / "w96_tb.dat", ecut=1e-3, dim=2)
    assert m.nnz < hl.nnz
    kg = syn.kplane(12, 6)
    out = P.wsurf(c, [m], kg, 0, 48)
    ref = orc.wilson_surface(m, kg, 0, 48)
    assert (int(out["status"][0]) & ~4) == (ref["status"] & ~4)
    assert phase_set_error(out["theta"][0].cpu().numpy(), ref["theta"]) < TOL
