"""GPU edge cases, argument errors and physics status flags of the C ABI."""
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


def test_empty_batches_are_noops():
    gu.need_gpu()
    c = gu.ctx()
    z = torch.zeros(16, dtype=torch.complex128, device="cuda")
    d = torch.zeros(16, dtype=torch.float64, device="cuda")
    i = torch.zeros(16, dtype=torch.int32, device="cuda")
    c.eigh_batched(z, 0, 2, 2, 4, 0, 0, 1, 0, d, z, 2, 2, i)
    c.wilson_loop(z, 2, 1, 2, 2, 0, 4, 4, 0, d, d, i, i)
    plan = c.hk_plan([syn.qwz(1.0)])
    kap = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    c.build_hk(plan, 0, 0, kap, z, 4, 2, 0)   # no systems
    torch.cuda.synchronize()


def test_no_selected_bands_and_single_point_loops():
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    hl = syn.bhz()
    plan = c.hk_plan([hl])
    kg = syn.kplane(4, 3)
    g = P.eig_grid(c, plan, 0, 1, kg, 1, 1)       # m = 0
    ev = g.evals.cpu().numpy()
    ref = np.stack([np.linalg.eigvalsh(orc.bloch_hamiltonian(hl, k)) for k in kg.reshape(-1, 3)])
    assert np.max(np.abs(ev[:, 0] - ref[:, 0])) < 1e-12 and np.max(np.abs(ev[:, 1] - ref[:, 1])) < 1e-12
    # a loop of one point: the only overlap is U^H U = I, so every phase is 0
    kg1 = syn.kplane(1, 5)
    g1 = P.eig_grid(c, plan, 0, 1, kg1, 0, 2)
    out = P.wilson(c, g1)
    assert np.max(np.abs(out["theta"].cpu().numpy())) < 1e-12


def test_argument_errors():
    gu.need_gpu()
    from paper_2312_13051_amd import BerryError
    c = gu.ctx()
    # buffers large enough for every call below: the library's own argument
    # checks are what reject them (the binding's extent checks pass)
    z = torch.zeros(4096, dtype=torch.complex128, device="cuda")
    d = torch.zeros(4096, dtype=torch.float64, device="cuda")
    i = torch.zeros(4096, dtype=torch.int32, device="cuda")
    with pytest.raises(BerryError):
        c.eigh_batched(z, 0, 4, 4, 16, 1, 3, 2, 0, d, z, 4, 16, i)      # lo > hi
    with pytest.raises(BerryError):
        c.eigh_batched(z, 1, 4, 4, 16, 1, 0, 2, 0, d, z, 4, 16, i)      # FP64 needs c128
    with pytest.raises(BerryError):
        c.eigh_batched(z, 0, 4, 3, 16, 1, 0, 2, 0, d, z, 4, 16, i)      # ld < N
    with pytest.raises(BerryError, match="too large"):                  # order beyond the LDS-resident kernels
        c.eigh_batched(z, 0, 5000, 5000, 5000 * 5000, 0, 0, 2500, 0, d, z, 5000, 5000 * 2500, i)
    c.eigh_batched(z, 0, 4000, 4000, 4000 * 4000, 0, 0, 2000, 0, d, z, 4000, 4000 * 2000, i)  # within it: no-op
    with pytest.raises(BerryError):
        c.wilson_loop(z, 4, 2, 4, 8, 1, 4, 4, 7, d, d, i, i)            # bad mode
    with pytest.raises(BerryError):
        c.wilson_loop(z, 4, 5, 4, 20, 1, 4, 4, 0, d, d, i, i)           # m > N
    with pytest.raises(BerryError):
        c.wilson_loop(z, 4, 2, 4, 8, 1, 0, 4, 0, d, d, i, i)            # n_par = 0
    with pytest.raises(BerryError):
        c.tune_set("no_such_knob", 1)
    with pytest.raises(BerryError):
        c.tune_set("hetrd_panel_threads", 300)
    assert c.tune_get("hetrd_panel_threads") == 512
    with pytest.raises(BerryError):
        c.tune_get("no_such_knob")


def test_binding_rejects_short_or_foreign_buffers():
    """The binding checks every buffer's extent (from the documented layouts)
    and device before the call: a too-small or host tensor is an error on the
    host, and the device is never handed a pointer it would overrun."""
    gu.need_gpu()
    from paper_2312_13051_amd import BerryError
    c = gu.ctx()
    N, m, n = 8, 3, 4
    H = torch.zeros((n, N, N), dtype=torch.complex128, device="cuda")
    ev = torch.zeros((n, m + 2), dtype=torch.float64, device="cuda")
    U = torch.zeros((n, m, N), dtype=torch.complex128, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    for q in range(n):
        H[q] = torch.eye(N, dtype=torch.complex128) * torch.arange(N, dtype=torch.float64).to(torch.complex128)
    # (the extent counted is the allocation's from the tensor's first element:
    # views into a large enough allocation pass, so short buffers are fresh)
    U_short = torch.zeros((n - 1, m, N), dtype=torch.complex128, device="cuda")
    with pytest.raises(BerryError, match="U: the call accesses"):
        c.eigh_batched(H, 0, N, N, N * N, n, 0, m, 0, ev, U_short, N, m * N, st)
    with pytest.raises(BerryError, match="U: the call accesses"):
        c.eigh_batched(H, 0, N, N, N * N, n, 0, m, 0, ev, U[1:], N, m * N, st)   # starts one matrix in
    with pytest.raises(BerryError, match="evals: the call accesses"):
        c.eigh_batched(H, 0, N, N, N * N, n, 0, m, 0, torch.zeros((n, m), dtype=torch.float64, device="cuda"),
                       U, N, m * N, st)
    with pytest.raises(BerryError, match="H: the call accesses"):
        c.eigh_batched(H, 0, N, N + 1, N * N, n, 0, m, 0, ev, U, N, m * N, st)
    with pytest.raises(BerryError, match="must be a tensor on cuda"):
        c.eigh_batched(H, 0, N, N, N * N, n, 0, m, 0, ev, U, N, m * N, st.cpu())
    with pytest.raises(BerryError, match="theta: the call accesses"):
        c.wilson_loop(U, N, m, N, m * N, 1, 2, 2, 0, torch.zeros(5, dtype=torch.float64, device="cuda"),
                      ev.reshape(-1), st, st)
    # the same arguments with full buffers run
    c.eigh_batched(H, 0, N, N, N * N, n, 0, m, 0, ev, U, N, m * N, st)
    torch.cuda.synchronize()
    assert np.allclose(ev[:, 1:m + 1].cpu().numpy(), np.arange(m)[None, :])


def test_pso_gap_flag_with_zero_spin_operator():
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    out = P.wspinsurf(c, [syn.bhz()], np.zeros((1, 4)), syn.kplane(6, 4), 0, 2)
    assert int(out["status"][0]) & 8


def test_wannier_gap_flag_on_window_edge():
    """Atomic limit: every Wilson phase is exactly 0, on the edge of (0, 1/2)."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    out = P.wnwl(c, [syn.atomic([-1.0, -0.5, 2.0])], syn.kplane(6, 4), 0, 2)
    assert int(out["status"][0]) & 16


def test_gap_closed_and_nan_flags_in_wilson_chain():
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    # degenerate Fermi level: bands 0,1 at -1 and band 2 also at -1
    g = P.eig_grid(c, c.hk_plan([syn.atomic([-1.0, -1.0, -1.0, 2.0])]), 0, 1, syn.kplane(4, 2), 0, 2)
    assert np.all(g.status.cpu().numpy() & 1)


def test_uneven_sizes_one_call_per_size():
    """Uneven batches (vacancy supercells of several L): each size runs as its
    own call; results equal the oracle for every system."""
    gu.need_gpu()
    P = pipe()
    c = gu.ctx()
    kg = syn.kplane(6, 4)
    for L in (3, 4):
        hls = [syn.bhz_vacancies(L, 0.12, [4, 1, s]) for s in range(2)]
        Ns = {h.N for h in hls}
        for N in Ns:
            group = [h for h in hls if h.N == N]
            out = P.wsurf(c, group, kg, 0, N // 2)
            for r, h in enumerate(group):
                ref = orc.wilson_surface(h, kg, 0, N // 2)
                assert phase_set_error(out["theta"][r].cpu().numpy(), ref["theta"]) < 1e-10


def test_singular_overlap_flag_matches_oracle():
    """The occupied state switches orbital between two grid points (two
    uncoupled orbitals with energies cos 2 pi k and -cos 2 pi k), so the
    overlap across the switch vanishes: OVERLAP_SINGULAR on the GPU as in
    the oracle, whose criterion is a smallest singular value below 1e-8."""
    gu.need_gpu()
    from synthetic.models import _from_blocks
    P = pipe()
    c = gu.ctx()
    hl = _from_blocks(2, 1, {(0,): np.zeros((2, 2)), (1,): np.diag([0.5, -0.5])})
    kg = syn.kplane(8, 2, k0=(1.0 / 16, 0.0, 0.0))
    ref = orc.wilson_surface(hl, kg, 0, 1)
    assert ref["status"] & 2
    out = P.wsurf(c, [hl], kg, 0, 1)
    assert int(out["status"][0]) & 2
