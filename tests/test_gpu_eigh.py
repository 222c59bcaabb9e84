"""GPU parity of the batched Hermitian eigensolver against the oracle.

Eigenvalues are compared with LAPACK (through the oracle) to 1e-12 ||H||,
the occupied projector U U^H to 1e-10, and U must be orthonormal.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import berry as orc
from tests import gpu_util as gu

torch = gu.torch
pytestmark = pytest.mark.gpu


def run_eigh(c, Hs, lo, hi, ld_pad=0):
    """Hs: numpy (n, N, N). Returns evals (n, m+2), U (n, N, m), status."""
    n, N, _ = Hs.shape
    m = hi - lo
    ld = N + ld_pad
    dH = gu.from_np(Hs, ld)
    ldu = N + 1
    U = gu.colmajor(n, N, max(m, 1), ldu, fill=0)
    ev = torch.empty((n, m + 2), dtype=torch.float64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    c.eigh_batched(dH, 0, N, ld, dH.stride(0), n, lo, hi, 0, ev, U, ldu, U.stride(0), st)
    torch.cuda.synchronize()
    return ev.cpu().numpy(), gu.to_np(U, N)[:, :, :m], st.cpu().numpy()


def check(Hs, lo, hi, ev, U, st, expect_status=0):
    for q in range(Hs.shape[0]):
        H = Hs[q]
        w, V = np.linalg.eigh(H)
        nrm = max(1.0, np.max(np.abs(w)))
        m = hi - lo
        assert np.max(np.abs(ev[q, 1:m + 1] - w[lo:hi])) <= 1e-12 * nrm, q
        if lo > 0:
            assert abs(ev[q, 0] - w[lo - 1]) <= 1e-12 * nrm
        else:
            assert np.isnan(ev[q, 0])
        if hi < H.shape[0]:
            assert abs(ev[q, m + 1] - w[hi]) <= 1e-12 * nrm
        else:
            assert np.isnan(ev[q, m + 1])
        if m:
            Uq = U[q]
            # inverse iteration keeps vectors of clusters more than 1e-3 ||T|| apart
            # orthogonal to about eps ||T|| / gap, i.e. ~1e-12 with a small constant
            assert np.max(np.abs(Uq.conj().T @ Uq - np.eye(m))) < 2e-11
            P = Uq @ Uq.conj().T
            Pref = V[:, lo:hi] @ V[:, lo:hi].conj().T
            assert np.max(np.abs(P - Pref)) < 1e-10, (q, np.max(np.abs(P - Pref)))
            # U spans an invariant subspace: H U = U (U^H H U) (gauge invariant)
            A = Uq.conj().T @ H @ Uq
            assert np.max(np.abs(H @ Uq - Uq @ A)) < 1e-11 * nrm
            # per column: H u_c = lambda_c u_c up to the width of lambda_c's
            # cluster (eigenvalues of the reference spectrum whose consecutive
            # gaps are below 1e-9 ||H||: inside such a cluster any orthonormal
            # basis of its invariant subspace is correct), and U^H H U is
            # block diagonal over the clusters
            wl = w[lo:hi]
            cid = np.concatenate([[0], np.cumsum(np.diff(wl) > 1e-9 * nrm)])
            width = np.array([np.ptp(wl[cid == k]) for k in cid])
            res = np.linalg.norm(H @ Uq - Uq * ev[q, 1:m + 1], axis=0)
            assert np.all(res <= 1e-11 * nrm + width), (q, np.max(res - width))
            off = np.abs(A) * (cid[:, None] != cid[None, :])
            assert np.max(off, initial=0.0) < 1e-11 * nrm
        assert st[q] == expect_status, (q, st[q])


@pytest.mark.parametrize("N,lo,hi", [(1, 0, 1), (2, 0, 1), (3, 1, 2), (5, 0, 5), (31, 3, 17), (32, 0, 16),
                                     (33, 0, 16), (70, 10, 45), (100, 0, 50), (129, 64, 129)])
def test_eigh_random_hermitian(N, lo, hi):
    gu.need_gpu()
    rng = np.random.default_rng(N)
    A = rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))
    Hs = A + np.conj(np.swapaxes(A, 1, 2))
    c = gu.ctx()
    ev, U, st = run_eigh(c, Hs, lo, hi, ld_pad=2)
    check(Hs, lo, hi, ev, U, st)


@pytest.mark.parametrize("name", ["qwz", "bbh", "bhz_clean_L3", "bhz_L10_W2", "bhz_vac_L6", "wannier96"])
def test_eigh_model_hamiltonians(name):
    gu.need_gpu()
    hl = {"qwz": lambda: syn.qwz(-1.0), "bbh": lambda: syn.bbh(0.5, 1.0),
          "bhz_clean_L3": lambda: syn.supercell(syn.bhz(), 3),
          "bhz_L10_W2": lambda: syn.bhz_disordered(10, 2.0, [3, 2, 1]),
          "bhz_vac_L6": lambda: syn.bhz_vacancies(6, 0.05, [4, 1, 3]),
          "wannier96": lambda: syn.wannier_like(96, [5, 2, 1])}[name]()
    kap = syn.kplane(3, 2).reshape(-1, 3)
    Hs = np.stack([orc.bloch_hamiltonian(hl, k) for k in kap])
    c = gu.ctx()
    m = hl.N // 2
    ev, U, st = run_eigh(c, Hs, 0, m)
    check(Hs, 0, m, ev, U, st)


def test_eigh_degenerate_clusters_and_gap_flag():
    """Clean supercell at kappa = 0 has large degenerate clusters; the atomic
    model with a degenerate Fermi level must raise GAP_CLOSED."""
    gu.need_gpu()
    hl = syn.supercell(syn.bhz(), 4)
    Hs = np.stack([orc.bloch_hamiltonian(hl, [0.0, 0.0, 0.0]), orc.bloch_hamiltonian(hl, [0.5, 0.5, 0.0])])
    c = gu.ctx()
    ev, U, st = run_eigh(c, Hs, 0, hl.N // 2)
    check(Hs, 0, hl.N // 2, ev, U, st)
    Ha = np.stack([orc.bloch_hamiltonian(syn.atomic([0.0, 0.0, 1.0, 2.0]), [0, 0])])
    ev, U, st = run_eigh(c, Ha, 0, 1)
    assert st[0] & 1


def test_eigh_nan_input_flagged():
    gu.need_gpu()
    H = np.eye(6, dtype=complex)[None]
    H[0, 2, 3] = np.nan
    H[0, 3, 2] = np.nan
    c = gu.ctx()
    ev, U, st = run_eigh(c, H, 0, 3)
    assert st[0] & 64


def run_eigh_mixed(c, Hs, lo, hi):
    n, N, _ = Hs.shape
    m = hi - lo
    dH = gu.from_np(Hs, N, dtype=torch.complex64)
    U = gu.colmajor(n, N, max(m, 1), N, fill=0)
    ev = torch.empty((n, m + 2), dtype=torch.float64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    c.eigh_batched(dH, 1, N, N, dH.stride(0), n, lo, hi, 1, ev, U, N, U.stride(0), st)
    torch.cuda.synchronize()
    return ev.cpu().numpy(), gu.to_np(U, N)[:, :, :m], st.cpu().numpy()


@pytest.mark.parametrize("name", ["bhz_L10_W2", "bhz_vac_L6", "wannier96"])
def test_eigh_mixed_precision_bounds(name):
    """FP32 reduction + FP64 tridiagonal solve and re-orthonormalization:
    eigenvalues within 2e-5 ||H||, U orthonormal to FP64 level in Z and FP32
    level after the FP32 back-transformation, projector within 1e-4."""
    gu.need_gpu()
    hl = {"bhz_L10_W2": lambda: syn.bhz_disordered(10, 2.0, [3, 2, 1]),
          "bhz_vac_L6": lambda: syn.bhz_vacancies(6, 0.05, [4, 1, 3]),
          "wannier96": lambda: syn.wannier_like(96, [5, 2, 1])}[name]()
    kap = syn.kplane(2, 2).reshape(-1, 3)
    Hs = np.stack([orc.bloch_hamiltonian(hl, k) for k in kap])
    c = gu.ctx()
    m = hl.N // 2
    ev, U, st = run_eigh_mixed(c, Hs, 0, m)
    for q in range(Hs.shape[0]):
        w, V = np.linalg.eigh(Hs[q])
        nrm = max(1.0, np.max(np.abs(w)))
        assert np.max(np.abs(ev[q, 1:m + 1] - w[:m])) <= 2e-5 * nrm
        assert np.max(np.abs(U[q].conj().T @ U[q] - np.eye(m))) < 1e-5
        P = U[q] @ U[q].conj().T
        assert np.max(np.abs(P - V[:, :m] @ V[:, :m].conj().T)) < 1e-4
        assert st[q] == 0


@pytest.mark.parametrize("threads,loads", [(1024, 0), (512, 4), (512, 8), (256, 0)])
@pytest.mark.parametrize("N,lo,hi", [(257, 0, 128), (400, 7, 203), (463, 100, 300)])
def test_eigh_panel_variants(N, lo, hi, threads, loads):
    """The panel kernel with 256 to 1024 threads per matrix, and the FP32
    512-thread kernel in both loads-in-flight forms (the FP64 reduction has
    one form per thread count: the loads knob leaves it unchanged)."""
    gu.need_gpu()
    rng = np.random.default_rng([N, 7])
    A = rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))
    Hs = A + np.conj(np.swapaxes(A, 1, 2))
    c = gu.ctx()
    for knob in ("hetrd_panel_threads", "hetrd_panel_loads"):
        c.tune_clear(knob)  # no per-order table: one setting for every order
    c.tune_set("hetrd_panel_threads", threads)
    c.tune_set("hetrd_panel_loads", loads)
    assert c.tune_get("hetrd_panel_threads") == threads and c.tune_get("hetrd_panel_loads") == loads
    try:
        ev, U, st = run_eigh(c, Hs, lo, hi, ld_pad=1)
        check(Hs, lo, hi, ev, U, st)
        hl = syn.bhz_disordered(10, 2.0, [3, 2, 4])
        Hm = np.stack([orc.bloch_hamiltonian(hl, k) for k in syn.kplane(2, 1).reshape(-1, 3)])
        # mixed path on the BHZ supercell and on the random matrices (at
        # N = 257 the panel splits each 64-row tile into column groups)
        for H, m in ((Hm, 200), (Hs, hi)):
            ev, U, st = run_eigh_mixed(c, H, 0, m)
            for q in range(H.shape[0]):
                w = np.linalg.eigvalsh(H[q])
                assert np.max(np.abs(ev[q, 1:m + 1] - w[:m])) <= 2e-5 * max(1.0, np.abs(w).max())
                assert np.max(np.abs(U[q].conj().T @ U[q] - np.eye(m))) < 1e-5
                assert st[q] == 0
    finally:
        c.close()


def test_tune_loads_knob_checks_values():
    """hetrd_panel_loads takes 0, 4 or 8; tune_clear restores 0 (by order)."""
    gu.need_gpu()
    c = gu.ctx()
    try:
        with pytest.raises(Exception):
            c.tune_set("hetrd_panel_loads", 6)
        with pytest.raises(Exception):
            c.tune_set_orders("hetrd_panel_loads", 1, 100, 1, 16)
        c.tune_set("hetrd_panel_loads", 8)
        c.tune_clear("hetrd_panel_loads")
        assert c.tune_get("hetrd_panel_loads") == 0
    finally:
        c.close()


@pytest.mark.parametrize("N,n_minus", [(200, 100), (96, 40)])
def test_eigh_large_degenerate_clusters(N, n_minus):
    """Eigenvalues exactly -1 and +1 with large multiplicities (the projected
    spin operator of a spin-conserving model): clusters far larger than a
    wave's lane group go through the workgroup-wide orthonormalization."""
    gu.need_gpu()
    rng = np.random.default_rng([N, n_minus])
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    lam = np.r_[-np.ones(n_minus), np.ones(N - n_minus)]
    Hs = np.stack([(Q * lam) @ Q.conj().T for _ in range(2)])
    Hs = 0.5 * (Hs + np.conj(np.swapaxes(Hs, 1, 2)))
    c = gu.ctx()
    ev, U, st = run_eigh(c, Hs, 0, N)
    for q in range(2):
        assert np.max(np.abs(ev[q, 1:N + 1] - lam)) < 1e-12
        Uq = U[q]
        assert np.max(np.abs(Uq.conj().T @ Uq - np.eye(N))) < 1e-12
        Pm = Uq[:, :n_minus] @ Uq[:, :n_minus].conj().T
        Pref = Q[:, :n_minus] @ Q[:, :n_minus].conj().T
        assert np.max(np.abs(Pm - Pref)) < 1e-10
        assert st[q] == 0


def _tridiagonal_cases():
    """Tridiagonal Hermitian inputs, which the reduction passes through almost
    unchanged, so inverse iteration meets them directly: a zero diagonal under
    unit couplings (row interchanges at nearly every elimination step), exact
    splits into equal blocks (eigenvalues repeated across blocks), tiny
    diagonal entries next to large couplings, and complex couplings."""
    rng = np.random.default_rng(11)
    cases = []
    N = 61
    cases.append((np.diag(np.ones(N - 1), 1) + np.diag(np.ones(N - 1), -1), 0, 30))
    blk = np.diag(rng.standard_normal(10)) + np.diag(np.full(9, 0.7), 1) + np.diag(np.full(9, 0.7), -1)
    H = np.kron(np.eye(6), blk)
    cases.append((H, 0, 24))
    d = np.where(rng.random(N) < 0.5, 1e-9, 1.0) * rng.standard_normal(N)
    e = (5.0 + rng.random(N - 1)) * np.where(rng.random(N - 1) < 0.15, 0.0, 1.0)
    cases.append((np.diag(d) + np.diag(e, 1) + np.diag(e, -1), 5, 37))
    ec = rng.standard_normal(N - 1) * np.exp(1j * rng.uniform(0, 2 * np.pi, N - 1))
    Hc = np.diag(rng.standard_normal(N)).astype(complex) + np.diag(ec, -1)
    Hc = Hc + np.triu(Hc.conj().T, 1)
    cases.append((Hc, 10, 50))
    return cases


@pytest.mark.parametrize("case", range(4))
def test_eigh_tridiagonal_inputs(case):
    """Eigenpairs of tridiagonal inputs match LAPACK (inverse iteration's
    stored elimination diagonals rebuild every factor entry, with and without
    row interchanges and across exact splits)."""
    gu.need_gpu()
    H, lo, hi = _tridiagonal_cases()[case]
    w = np.linalg.eigvalsh(H)
    assert w[lo] - w[lo - 1] > 1e-6 if lo > 0 else True
    assert w[hi] - w[hi - 1] > 1e-6
    Hs = np.stack([H.astype(complex)] * 3)
    c = gu.ctx()
    ev, U, st = run_eigh(c, Hs, lo, hi)
    check(Hs, lo, hi, ev, U, st)


@pytest.mark.parametrize("precision", [0, 1])
def test_eigh_batch_invariant(precision):
    """A matrix's eigenvectors do not depend on the batch it is solved in: the
    same k-points solved in one call, and in two calls at other batch
    positions, give the same bits (spin-degenerate BHZ spectrum, where the
    basis inside each degenerate pair is decided by the inverse iteration's
    start vector)."""
    gu.need_gpu()
    hl = syn.bhz_disordered(3, 2.0, [5, 1, 3])
    kap = syn.kplane(8, 5).reshape(-1, 3)
    Hs = np.stack([orc.bloch_hamiltonian(hl, k) for k in kap])
    c = gu.ctx()
    m = hl.N // 2
    run = run_eigh_mixed if precision else (lambda c_, H_, lo_, hi_: run_eigh(c_, H_, lo_, hi_))
    ev, U, st = run(c, Hs, 0, m)
    ev1, U1, st1 = run(c, Hs[:17], 0, m)
    ev2, U2, st2 = run(c, Hs[17:], 0, m)
    assert np.array_equal(U, np.concatenate([U1, U2]))
    assert np.array_equal(ev[:, 1:m + 1], np.concatenate([ev1, ev2])[:, 1:m + 1])
    assert not st.any()


def run_eigh_refined(c, Hs, lo, hi):
    n, N, _ = Hs.shape
    m = hi - lo
    dH = gu.from_np(Hs, N + 3)
    H0 = dH.clone()
    U = gu.colmajor(n, N, max(m, 1), N + 1, fill=0)
    ev = torch.empty((n, m + 2), dtype=torch.float64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    c.eigh_batched(dH, 0, N, N + 3, dH.stride(0), n, lo, hi, 2, ev, U, N + 1, U.stride(0), st)
    torch.cuda.synchronize()
    assert torch.equal(dH, H0), "the refined path must leave H unchanged"
    return ev.cpu().numpy(), gu.to_np(U, N)[:, :, :m], st.cpu().numpy()


@pytest.mark.parametrize("name,lo,hi", [("bhz_L10_W2", 0, 200), ("bhz_vac_L6", 0, 70), ("wannier96", 0, 48),
                                        ("wannier96", 20, 48), ("bhz_L10_W2", 150, 400)])
def test_eigh_refined_precision(name, lo, hi):
    """Mixed path with the FP64 subspace correction: the window's projector
    within 1e-10 of LAPACK's and U orthonormal to 1e-13 (the FP32 path alone
    reaches 1e-4 and 1e-5), the invariant-subspace residual H U - U (U^H H U)
    within 1e-10 ||H||, Rayleigh-quotient eigenvalues within 1e-9 ||H|| on
    these models (second order in the FP32 columns' error; a nearly
    degenerate pair inside the window could keep the FP32 level), H left
    unchanged."""
    gu.need_gpu()
    hl = {"bhz_L10_W2": lambda: syn.bhz_disordered(10, 2.0, [3, 2, 1]),
          "bhz_vac_L6": lambda: syn.bhz_vacancies(6, 0.05, [4, 1, 3]),
          "wannier96": lambda: syn.wannier_like(96, [5, 2, 1])}[name]()
    kap = syn.kplane(2, 2).reshape(-1, 3)
    Hs = np.stack([orc.bloch_hamiltonian(hl, k) for k in kap])
    c = gu.ctx()
    m = hi - lo
    ev, U, st = run_eigh_refined(c, Hs, lo, hi)
    for q in range(Hs.shape[0]):
        w, V = np.linalg.eigh(Hs[q])
        nrm = max(1.0, np.max(np.abs(w)))
        assert np.max(np.abs(ev[q, 1:m + 1] - w[lo:hi])) <= 1e-9 * nrm, q
        if lo > 0:
            assert abs(ev[q, 0] - w[lo - 1]) <= 1e-4 * nrm
        else:
            assert np.isnan(ev[q, 0])
        if hi < hl.N:
            assert abs(ev[q, m + 1] - w[hi]) <= 1e-4 * nrm
        else:
            assert np.isnan(ev[q, m + 1])
        Uq = U[q]
        # Newton-Schulz from the FP32 level (~1e-6) until the error is below
        # 1e-8, then a last step: rounding is left (one step from 1e-6 left
        # ~1e-12, enough to split a spin operator's +-1 clusters)
        orth = np.max(np.abs(Uq.conj().T @ Uq - np.eye(m)))
        assert orth < 1e-13, (q, orth)
        P = Uq @ Uq.conj().T
        assert np.max(np.abs(P - V[:, lo:hi] @ V[:, lo:hi].conj().T)) < 1e-10, (q, np.max(np.abs(P - V[:, lo:hi] @ V[:, lo:hi].conj().T)))
        A = Uq.conj().T @ Hs[q] @ Uq
        assert np.max(np.abs(Hs[q] @ Uq - Uq @ A)) < 1e-10 * nrm
        assert st[q] == 0, (q, st[q])


def test_eigh_refined_gap_flag_and_batch_invariance():
    """The refined path flags a closed gap at the window's edge like the FP64
    path, and gives the same bits in any batch."""
    gu.need_gpu()
    c = gu.ctx()
    Ha = np.stack([orc.bloch_hamiltonian(syn.atomic([0.0, 0.0, 1.0, 2.0]), [0, 0])])
    ev, U, st = run_eigh_refined(c, Ha, 0, 1)
    assert st[0] & 1
    hl = syn.bhz_disordered(3, 2.0, [5, 1, 3])
    kap = syn.kplane(6, 5).reshape(-1, 3)
    Hs = np.stack([orc.bloch_hamiltonian(hl, k) for k in kap])
    m = hl.N // 2
    ev, U, st = run_eigh_refined(c, Hs, 0, m)
    ev1, U1, _ = run_eigh_refined(c, Hs[:11], 0, m)
    ev2, U2, _ = run_eigh_refined(c, Hs[11:], 0, m)
    assert np.array_equal(U, np.concatenate([U1, U2]))
    assert not st.any()


@pytest.mark.parametrize("spread", [0.0, 1e-14, 1e-12, 1e-10])
def test_eigh_fuzzy_clusters(spread):
    """Two 100-fold clusters at -1 and +1, each spread over `spread` (the
    projected spin operator of a spin-conserving model, formed from
    eigenvectors accurate to ~1e-12): the FP64 eigensolver returns an
    orthonormal basis whose lower half spans the -1 cluster to 1e-10, with
    no status bit (no orthonormalization left unconverged)."""
    gu.need_gpu()
    rng = np.random.default_rng([11, int(spread * 1e16)])
    n = 200
    Q = np.linalg.qr(rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n)))[0]
    w = np.concatenate([-1.0 + spread * rng.random(100), 1.0 + spread * rng.random(100)])
    Hs = np.stack([(Q[q] * w) @ Q[q].conj().T for q in range(2)])
    Hs = 0.5 * (Hs + np.conj(np.swapaxes(Hs, 1, 2)))
    c = gu.ctx()
    for lo, hi in ((0, 100), (0, 200)):
        ev, U, st = run_eigh(c, Hs, lo, hi)
        assert not st.any(), st
        for q in range(2):
            Uq = U[q]
            assert np.max(np.abs(Uq.conj().T @ Uq - np.eye(hi - lo))) < 2e-11
            P = Uq[:, :100] @ Uq[:, :100].conj().T
            Pref = Q[q][:, :100] @ Q[q][:, :100].conj().T
            assert np.max(np.abs(P - Pref)) < 1e-10


def test_eigh_per_order_tuning():
    """Per-order panel thread counts (as the autotuner stores them) select the
    kernel variant by order and precision; results stay correct."""
    gu.need_gpu()
    c = gu.ctx()
    try:
        c.load_tuning({"knobs": {"hetrd_panel_threads": [
            {"n_lo": 1, "n_hi": 100, "precision": -1, "value": 256},
            {"n_lo": 101, "n_hi": 1000, "precision": 0, "value": 1024},
            {"n_lo": 101, "n_hi": 1000, "precision": 1, "value": 256}]}})
        for N, lo, hi in ((70, 10, 45), (129, 64, 129)):
            rng = np.random.default_rng(N + 7)
            A = rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))
            Hs = A + np.conj(np.swapaxes(A, 1, 2))
            ev, U, st = run_eigh(c, Hs, lo, hi)
            check(Hs, lo, hi, ev, U, st)
        hl = syn.bhz_disordered(6, 2.0, [3, 2, 9])
        Hs = np.stack([orc.bloch_hamiltonian(hl, k) for k in syn.kplane(2, 1).reshape(-1, 3)])
        ev, U, st = run_eigh_mixed(c, Hs, 0, hl.N // 2)
        w, V = np.linalg.eigh(Hs[0])
        P = U[0] @ U[0].conj().T
        assert np.max(np.abs(P - V[:, :hl.N // 2] @ V[:, :hl.N // 2].conj().T)) < 1e-4
        # per-order loads in flight of the 512-thread FP32 kernel
        c.load_tuning({"knobs": {"hetrd_panel_threads": [{"n_lo": 1, "n_hi": 10000, "precision": -1, "value": 512}],
                                 "hetrd_panel_loads": [{"n_lo": 1, "n_hi": 200, "precision": 1, "value": 8},
                                                       {"n_lo": 201, "n_hi": 10000, "precision": 1, "value": 4}]}})
        ev2, U2, st2 = run_eigh_mixed(c, Hs, 0, hl.N // 2)
        P2 = U2[0] @ U2[0].conj().T
        assert np.max(np.abs(P2 - V[:, :hl.N // 2] @ V[:, :hl.N // 2].conj().T)) < 1e-4
        assert np.all(st2 == 0)
    finally:
        c.close()


@pytest.mark.parametrize("N,lo,hi", [(1, 0, 1), (5, 2, 2), (40, 0, 40), (70, 0, 1), (70, 69, 70)])
def test_eigh_refined_edges(N, lo, hi):
    """Refined path at its edges: one matrix element, an empty window, the
    whole spectrum (no complement), a single band at either end."""
    gu.need_gpu()
    rng = np.random.default_rng([N, lo, hi])
    A = rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))
    Hs = A + np.conj(np.swapaxes(A, 1, 2))
    c = gu.ctx()
    m = hi - lo
    ev, U, st = run_eigh_refined(c, Hs, lo, hi)
    for q in range(3):
        w, V = np.linalg.eigh(Hs[q])
        nrm = max(1.0, np.max(np.abs(w)))
        assert np.max(np.abs(ev[q, 1:m + 1] - w[lo:hi]), initial=0.0) <= 1e-9 * nrm
        if m:
            Uq = U[q]
            assert np.max(np.abs(Uq.conj().T @ Uq - np.eye(m))) < 5e-12
            P = Uq @ Uq.conj().T
            assert np.max(np.abs(P - V[:, lo:hi] @ V[:, lo:hi].conj().T)) < 1e-9
        assert (ev[q, 0] == ev[q, 0]) == (lo > 0) and (ev[q, m + 1] == ev[q, m + 1]) == (hi < N)


def test_bisection_cap_flags_nonconverged():
    """A bisection cap set from the host leaves eigenvalues short of their
    tolerance: every matrix is flagged NONCONVERGED (the kernels still end
    normally), and the default cap gives the uncapped results again."""
    gu.need_gpu()
    from paper_2312_13051_amd import BerryError
    N, lo, hi = 40, 5, 25
    rng = np.random.default_rng(11)
    A = rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))
    Hs = A + np.conj(np.swapaxes(A, 1, 2))
    c = gu.ctx()
    try:
        ev0, U0, st0 = run_eigh(c, Hs, lo, hi)
        assert np.all(st0 == 0)
        c.tune_set("tri_bisect_max_iter", 1)
        ev1, U1, st1 = run_eigh(c, Hs, lo, hi)
        assert np.all(st1 & 32), st1                       # BE_ST_NONCONVERGED
        assert np.all(np.isfinite(ev1[:, 1:hi - lo + 1]))
        assert np.max(np.abs(ev1[:, 1:hi - lo + 1] - ev0[:, 1:hi - lo + 1])) > 1e-6
        with pytest.raises(BerryError):
            c.tune_set_orders("tri_bisect_max_iter", 1, 100, -1, 4)
        with pytest.raises(BerryError):
            c.tune_set("tri_bisect_max_iter", 0)
        c.tune_clear("tri_bisect_max_iter")
        assert c.tune_get("tri_bisect_max_iter") == 128
        ev2, U2, st2 = run_eigh(c, Hs, lo, hi)
        assert np.all(st2 == 0) and np.array_equal(ev2, ev0) and np.array_equal(U2, U0)
    finally:
        c.close()


@pytest.mark.parametrize("name", ["random257", "bhz_L10_W2"])
def test_eigh_split_bf16_bounds(name):
    """BE_MIXED_BF16X (trailing updates and back-transformation as split-bf16
    products, ~2^-16 relative error per product): eigenvalues within 1e-5
    ||H||, U orthonormal to 1e-4, projector within 1e-4 (measured: 1.1e-6,
    1.3e-5 and 1.5e-5 on these inputs); it must not fall back to the FP32
    products (its eigenvalues differ from the FP32 mixed path's)."""
    gu.need_gpu()
    from paper_2312_13051_amd import _lib as L
    if name == "random257":
        rng = np.random.default_rng(3)
        A = rng.standard_normal((3, 257, 257)) + 1j * rng.standard_normal((3, 257, 257))
        Hs = A + np.conj(np.swapaxes(A, 1, 2))
    else:
        hl = syn.bhz_disordered(10, 2.0, [3, 2, 4])
        Hs = np.stack([orc.bloch_hamiltonian(hl, k) for k in syn.kplane(2, 2).reshape(-1, 3)])
    n, N, _ = Hs.shape
    m = N // 2
    c = gu.ctx()
    out = {}
    for prec in (L.BE_MIXED_FP32, L.BE_MIXED_BF16X):
        dH = gu.from_np(Hs, N, dtype=torch.complex64)
        U = gu.colmajor(n, N, m, N, fill=0)
        ev = torch.empty((n, m + 2), dtype=torch.float64, device="cuda")
        st = torch.empty(n, dtype=torch.int32, device="cuda")
        c.eigh_batched(dH, 1, N, N, dH.stride(0), n, 0, m, prec, ev, U, N, U.stride(0), st)
        torch.cuda.synchronize()
        out[prec] = (ev.cpu().numpy(), gu.to_np(U, N)[:, :, :m], st.cpu().numpy())
    ev, U, st = out[L.BE_MIXED_BF16X]
    assert np.all(st == 0)
    for q in range(n):
        w, V = np.linalg.eigh(Hs[q])
        nrm = np.abs(w).max()
        assert np.max(np.abs(ev[q, 1:m + 1] - w[:m])) <= 1e-5 * nrm
        assert np.max(np.abs(U[q].conj().T @ U[q] - np.eye(m))) < 1e-4
        assert np.max(np.abs(U[q] @ U[q].conj().T - V[:, :m] @ V[:, :m].conj().T)) < 1e-4
    assert not np.array_equal(ev, out[L.BE_MIXED_FP32][0])
    z = gu.from_np(Hs, N)                # c128 input is refused for this precision
    ev2 = torch.empty((n, m + 2), dtype=torch.float64, device="cuda")
    U2 = gu.colmajor(n, N, m, N, fill=0)
    st2 = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(L.BerryError):
        c.eigh_batched(z, L.BE_C128, N, N, z.stride(0), n, 0, m, L.BE_MIXED_BF16X, ev2, U2, N, U2.stride(0), st2)
