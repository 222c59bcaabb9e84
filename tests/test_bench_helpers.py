"""Host logic of bench.py: algorithmic work counts, the traffic lookup of a
profile summary, and the one-GPU guard (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_hetrd_panel_bytes_is_one_triangle_of_the_trailing_matrix_per_column():
    N, n_mat = 37, 3
    brute = 0
    for j in range(N - 1):   # reflector column j: trailing matrix rows/cols j+1..N-1, r >= c
        brute += sum(1 for r in range(j + 1, N) for c in range(j + 1, N) if r >= c)
    assert bench.hetrd_panel_bytes(N, n_mat, 8) == 8 * brute * n_mat
    assert bench.hetrd_panel_bytes(N, n_mat, 16) == 2 * bench.hetrd_panel_bytes(N, n_mat, 8)


def test_det_phase_flops_counts_the_lu_updates():
    # unblocked LU of an ms x ms matrix: step k updates (ms-k-1)^2 entries,
    # one complex multiply-add (8 flops) each; two sectors, two directions
    m, md, n_k = 9, 4, 5
    per = 0
    for ms in (md, m - md):
        for k in range(ms):
            per += 8 * (ms - k - 1) ** 2
    assert bench.det_phase_flops([md], m, n_k) == 2 * n_k * per


def test_her2k_and_unmtr_flops():
    N, m, n_mat = 100, 40, 2
    nb = bench.NB
    her = sum(8.0 * (N - p * nb - nb) ** 2 * nb for p in range((N + nb - 1) // nb) if N - p * nb - nb > 0)
    assert bench.eigh_gemm_flops("her2k", N, m, n_mat) == n_mat * her
    with pytest.raises(KeyError):
        bench.eigh_gemm_flops("nope", N, m, n_mat)


def test_traffic_lookup_follows_digest_and_precision(tmp_path):
    src = os.path.join(ROOT, "paper_2312_13051_amd", "csrc", "eigh.hip")
    sha = bench.panel_source_digest(src)
    p = tmp_path / "prof.md"
    p.write_text(f"<!-- precision: mixed -->\n<!-- traffic_bytes_per_launch: 1.5e+10 -->\n"
                 f"<!-- kernel_source_sha256: {sha} -->\n")
    assert bench.traffic_from_profile(str(p), src, "mixed") == 1.5e10
    assert bench.traffic_from_profile(str(p), src, "fp64") is None
    p.write_text("<!-- precision: mixed -->\n<!-- traffic_bytes_per_launch: 1.5e+10 -->\n"
                 "<!-- kernel_source_sha256: 0000 -->\n")
    assert bench.traffic_from_profile(str(p), src, "mixed") is None
    assert bench.traffic_from_profile(str(tmp_path / "missing.md"), src, "mixed") is None


@pytest.mark.parametrize("name", ["hetrd_panel_bhz400_mixed.md", "hetrd_panel_served_bhz24_mixed.md"])
def test_committed_profile_matches_the_panel_source(name):
    src = os.path.join(ROOT, "paper_2312_13051_amd", "csrc", "eigh.hip")
    prof = os.path.join(ROOT, "profiles", name)
    assert bench.traffic_from_profile(prof, src, "mixed") is not None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_served_gemm_flops_and_phase_summary():
    import numpy as np
    from types import SimpleNamespace as NS
    REF = 2
    a = NS(N=64, m=32, n_k=12, kappa=np.zeros((3, 4, 3)), precision=1)
    b = NS(N=96, m=48, n_k=12, kappa=np.zeros((3, 4, 3)), precision=REF)   # refined: all bands in the eigensolver
    fl = bench.served_gemm_flops([a, b], REF)
    assert fl["her2k"] == bench.eigh_gemm_flops("her2k", 64, 32, 12) + bench.eigh_gemm_flops("her2k", 96, 96, 12)
    assert fl["unmtr"] == bench.eigh_gemm_flops("unmtr", 64, 32, 12) + bench.eigh_gemm_flops("unmtr", 96, 96, 12)
    assert fl["overlap"] == 8.0 * (64 * 32 * 32 + 96 * 48 * 48) * 12
    assert fl["chain"] == 8.0 * (32 ** 3 + 48 ** 3) * 3 * 3           # (n_par - 1) products per line, 3 lines
    # the summary: rates against the peak of each tag's type, time-weighted fraction
    s = bench.gemm_phase_summary({"her2k": 157.3e12, "overlap": 78.6e12 / 2, "absent": 1.0},
                                 {"her2k": 2000.0, "overlap": 1000.0}, ("her2k",), scale=2.0)
    assert s["per_tag"]["her2k"]["frac"] == 1.0 and s["per_tag"]["overlap"]["frac"] == 1.0
    assert "absent" not in s["per_tag"] and s["frac_of_mfma_peak"] == 1.0
