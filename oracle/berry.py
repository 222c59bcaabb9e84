"""FP64 CPU oracle for the Wilson-loop method (test infrastructure only).

This module is the correctness reference for the GPU library. It is test
infrastructure: only the test suite, the smoke entry point and the benchmark's
CPU-baseline leg may import it. The product path never calls it. It shares no
code with the HIP library; the two meet only through the seeded inputs of the
``synthetic`` package.

Everything is complex128/float64 NumPy with plain loops over k-points, links
and loops. LAPACK enters only through ``numpy.linalg`` (eigh, eigvals/eig,
svd, qr), one library primitive per step, in the order the paper gives.

Method (paper references are to sections and equations):

* Bloch Hamiltonian (Sec. II-A, closing remarks on periodic/twisted boundary
  conditions): H_ab(kappa) = sum over entries (a, b, R, t) of
  t * exp(2 pi i kappa . R), with kappa fractional in the reciprocal basis of
  the (super)cell. This lattice gauge gives H(kappa + G) = H(kappa) exactly,
  which is the periodicity the paper requires of the Bloch functions.
* Eigenpairs (Sec. I, "exact diagonalization ... at many points"): ascending
  eigenvalues; the selected bands [lo, hi) give U(kappa), N x m.
* Overlaps (eq. 2): F_j = U(kappa_{j+1})^H U(kappa_j), j = 0..n-1, with
  kappa_n identified with kappa_0 (the same U is reused at the closure).
* Re-unitarisation: F -> X Y^H from svd(F) = X S Y^H (polar factor). The raw
  product of eq. 2 is available as mode "raw".
* Wilson loop (eq. 2, path ordered, eq. 1 remark on non-Abelian connections):
  W = F_{n-1} ... F_1 F_0, eigenphases theta = arg eig(W) in (-pi, pi],
  sorted; the Wannier centres are x = theta / 2 pi (eq. 2, eq. 3).
* Chern winding (eq. 6) over a closed transverse loop:
  Phi_i = sum_n theta_{i,n} mod 2 pi, C = (1/2pi) sum_i wrap(Phi_{i+1}-Phi_i).
* Nested Wilson loop (Sec. III, eq. 8): the Wannier Hamiltonian of the first
  loop is diagonalised at every base point; the states of the chosen Wannier
  sector, w = U nu_S, are carried through a second Wilson loop along the other
  direction, giving nested phases and the nested polarisation.
* Spin-resolved Wilson loop (Sec. IV): the projected spin operator P s P is
  diagonalised inside the occupied space; its negative (positive) eigenstates
  give the spin-down (spin-up) Wilson loop and C_down (C_up);
  C_s = (C_up - C_down)/2, so that C_down = -1 means C_s = +1 (Sec. V).
* Berry flux per plaquette (Sec. IV, example of the disordered quadrupolar
  insulator: the coupling-matrix method on a grid of plaquettes, per spin
  sector): the phase of the product of the link
  variables det(U(k')^H U(k)) around each plaquette; the sum over the zone
  is 2 pi times the Chern number. A link whose smallest singular value is
  below 1e-8 is flagged, as an overlap of the Wilson loop is.
* Spectrum of the projected spin operator for any spin operator S (Sec. V,
  the scan over a grid of k-points for a spin axis with a gapped spectrum):
  the eigenvalues of U^H S U in the selected bands.

Where the paper is silent or garbled, the readings used here are listed in
the design notes of the repository (overlap index order, polar factor as the
canonical overlap, eigenphase branch, winding as a sum of wrapped steps,
nested sector window, unwrapping of the nested polarisation, spin-sector
sign convention).
"""
from __future__ import annotations

import numpy as np

# Status bits of a result (a physics condition, never an error).
GAP_CLOSED = 1
OVERLAP_SINGULAR = 2
WINDING_UNRESOLVED = 4
PSO_GAP = 8
WANNIER_GAP = 16
NONCONVERGED = 32
NAN_INF = 64

TWO_PI = 2.0 * np.pi


# ----------------------------------------------------------------------------
# Bloch Hamiltonian
# ----------------------------------------------------------------------------
def bloch_hamiltonian(hl, kappa) -> np.ndarray:
    """Dense H(kappa) = sum_e t_e exp(2 pi i kappa . R_e) placed at (i_e, j_e).

    Lattice-gauge Bloch sum (Sec. II-A, periodic boundary conditions along the
    integration path; supercells use kappa in units of the supercell
    reciprocal vectors, which is the 2pi -> 2pi/L rule).
    """
    kappa = np.asarray(kappa, dtype=np.float64).reshape(-1)
    H = np.zeros((hl.N, hl.N), dtype=np.complex128)
    if hl.nnz == 0:
        return H
    phase = np.exp(1j * TWO_PI * (hl.R.astype(np.float64) @ kappa[: hl.dim]))
    np.add.at(H, (hl.i, hl.j), hl.t * phase)
    return H


# ----------------------------------------------------------------------------
# Eigenpairs
# ----------------------------------------------------------------------------
def eigh_bands(H: np.ndarray, lo: int, hi: int):
    """Ascending eigenvalues and the eigenvectors of bands [lo, hi).

    Returns (evals (N,), U (N, hi-lo), status). GAP_CLOSED is set when a band
    edge of the selection is degenerate with its outside neighbour.
    """
    N = H.shape[0]
    status = 0
    if not np.all(np.isfinite(H)):
        return np.full(N, np.nan), np.full((N, hi - lo), np.nan + 0j), NAN_INF
    w, V = np.linalg.eigh(H)
    scale = max(1.0, float(np.max(np.abs(w))) if N else 1.0)
    gaps = []
    if lo > 0:
        gaps.append(w[lo] - w[lo - 1])
    if hi < N:
        gaps.append(w[hi] - w[hi - 1])
    if gaps and min(gaps) < 1e-9 * scale:
        status |= GAP_CLOSED
    return w, V[:, lo:hi], status


def eigh_grid(hl, kappa_grid: np.ndarray, lo: int, hi: int):
    """Eigenvalues and selected eigenvectors at every point of a k-grid.

    kappa_grid has shape (..., 3). Returns evals (..., N), U (..., N, m), status.
    """
    shp = kappa_grid.shape[:-1]
    flat = kappa_grid.reshape(-1, kappa_grid.shape[-1])
    ev = np.empty((flat.shape[0], hl.N))
    U = np.empty((flat.shape[0], hl.N, hi - lo), dtype=np.complex128)
    st = 0
    for q in range(flat.shape[0]):
        H = bloch_hamiltonian(hl, flat[q])
        ev[q], U[q], s = eigh_bands(H, lo, hi)
        st |= s
    return ev.reshape(shp + (hl.N,)), U.reshape(shp + (hl.N, hi - lo)), st


# ----------------------------------------------------------------------------
# Overlaps, polar factor, Wilson loop, eigenphases
# ----------------------------------------------------------------------------
def overlaps(U_line: np.ndarray) -> np.ndarray:
    """F_j = U_{j+1}^H U_j along a closed line (eq. 2); U_n is U_0."""
    n = U_line.shape[0]
    return np.stack([U_line[(j + 1) % n].conj().T @ U_line[j] for j in range(n)])


def polar_factor(F: np.ndarray):
    """Unitary polar factor X Y^H of F = X S Y^H, and the smallest singular value."""
    X, s, Yh = np.linalg.svd(F)
    return X @ Yh, float(s.min()) if s.size else 1.0


def wilson_matrix(U_line: np.ndarray, mode: str = "polar"):
    """Path-ordered product W = F_{n-1} ... F_0 of the overlaps of one closed line."""
    F = overlaps(U_line)
    m = U_line.shape[-1]
    W = np.eye(m, dtype=np.complex128)
    status = 0
    for j in range(F.shape[0]):
        Fj = F[j]
        if mode == "polar":
            Fj, smin = polar_factor(Fj)
            if smin < 1e-8:
                status |= OVERLAP_SINGULAR
        elif mode != "raw":
            raise ValueError(mode)
        W = Fj @ W
    return W, status


def eigphases(W: np.ndarray) -> np.ndarray:
    """theta = arg eig(W) in (-pi, pi], ascending (eq. 2: exp(i 2 pi x) = eig(W))."""
    th = np.angle(np.linalg.eigvals(W))
    th = np.where(th <= -np.pi, np.pi, th)
    return np.sort(th)


def winding(theta: np.ndarray):
    """Chern number as the winding of the summed hybrid centres (eq. 6).

    theta: (n_perp, m) eigenphases. Phi_i = sum_n theta_{i,n} mod 2pi; the
    winding adds the wrapped steps Phi_{i+1} - Phi_i around the closed
    transverse loop. Returns (C as int, phi (n_perp,), status).
    """
    phi = np.mod(theta.sum(axis=-1), TWO_PI)
    d = np.roll(phi, -1) - phi
    d = d - TWO_PI * np.round(d / TWO_PI)
    c = d.sum() / TWO_PI
    status = 0
    if np.max(np.abs(d)) > 0.8 * np.pi or abs(c - np.round(c)) > 1e-6:
        status |= WINDING_UNRESOLVED
    return int(np.round(c)), phi, status


def wilson_loop_grid(U_grid: np.ndarray, mode: str = "polar"):
    """Wilson loop of every transverse line of a U-grid (n_perp, n_par, N, m).

    Returns theta (n_perp, m), phi (n_perp,), winding, status.
    """
    n_perp = U_grid.shape[0]
    m = U_grid.shape[-1]
    theta = np.empty((n_perp, m))
    st = 0
    for i in range(n_perp):
        W, s = wilson_matrix(U_grid[i], mode)
        st |= s
        theta[i] = eigphases(W)
    C, phi, s = winding(theta)
    return theta, phi, C, st | s


def wilson_surface(hl, kappa_grid: np.ndarray, lo: int, hi: int, mode: str = "polar"):
    """Hybrid Wannier centres over a k-plane (eq. 3) and their winding (eq. 6).

    kappa_grid: (n_perp, n_par, 3) from a closed loop along the second axis.
    """
    ev, U, st = eigh_grid(hl, kappa_grid, lo, hi)
    theta, phi, C, s = wilson_loop_grid(U, mode)
    return {"theta": theta, "phi": phi, "winding": C, "status": st | s,
            "evals": ev, "U": U}


# ----------------------------------------------------------------------------
# Nested Wilson loop
# ----------------------------------------------------------------------------
def nested_from_grid(U_grid: np.ndarray, window=(0.0, 0.5), mode: str = "polar"):
    """Nested Wilson loop (Sec. III, eq. 8) from a U-grid (n_perp, n_par, N, m).

    For each transverse index i and base point j0 the Wilson loop along the
    parallel axis is formed by an explicit cyclic product starting at j0. Its
    eigenvectors with x = theta/2pi inside ``window`` form the Wannier sector;
    w = U(kappa_{i,j0}) nu_S is re-orthonormalised by QR. The nested loop then
    runs along the transverse axis at every j0.

    Returns dict with nested theta (n_par, s), p (n_par,) in (-1/2, 1/2],
    p_mean in [0, 1), s, status.
    """
    n_perp, n_par, N, m = U_grid.shape
    status = 0
    F = np.empty((n_perp, n_par, m, m), dtype=np.complex128)
    for i in range(n_perp):
        Fi = overlaps(U_grid[i])
        for j in range(n_par):
            if mode == "polar":
                F[i, j], smin = polar_factor(Fi[j])
                if smin < 1e-8:
                    status |= OVERLAP_SINGULAR
            else:
                F[i, j] = Fi[j]
    w_states = None
    s_count = None
    lo, hi = window
    for i in range(n_perp):
        for j0 in range(n_par):
            W = np.eye(m, dtype=np.complex128)
            for step in range(n_par):
                W = F[i, (j0 + step) % n_par] @ W
            lam, nu = np.linalg.eig(W)
            x = np.angle(lam) / TWO_PI
            x = np.where(x <= -0.5, 0.5, x)
            sel = (x > lo) & (x < hi)
            edge = np.min(np.abs(np.concatenate([x - lo, x - hi]))) if x.size else 1.0
            if edge < 1e-6:
                status |= WANNIER_GAP
            s = int(sel.sum())
            if s_count is None:
                s_count = s
                w_states = np.empty((n_perp, n_par, N, s), dtype=np.complex128)
            elif s != s_count:
                status |= WANNIER_GAP
                return {"theta": None, "p": None, "p_mean": np.nan, "s": s_count,
                        "status": status}
            w = U_grid[i, j0] @ nu[:, sel]
            q, _ = np.linalg.qr(w)
            w_states[i, j0] = q
    s = s_count
    theta_n = np.empty((n_par, s))
    p = np.empty(n_par)
    for j0 in range(n_par):
        line = w_states[:, j0]  # along the transverse axis, closed
        W, st = wilson_matrix(line, mode)
        status |= st
        theta_n[j0] = eigphases(W)
        pj = theta_n[j0].sum() / TWO_PI
        p[j0] = pj - np.round(pj) if abs(pj - np.round(pj)) != 0.5 else 0.5
    # unwrap along the base point, then average, then reduce mod 1
    pu = np.empty_like(p)
    pu[0] = p[0]
    for j0 in range(1, n_par):
        d = p[j0] - p[j0 - 1]
        d -= np.round(d)
        pu[j0] = pu[j0 - 1] + d
    p_mean = float(np.mod(pu.mean(), 1.0))
    return {"theta": theta_n, "p": p, "p_mean": p_mean, "s": s, "status": status}


def nested_wilson(hl, kappa_grid: np.ndarray, lo: int, hi: int, window=(0.0, 0.5),
                  mode: str = "polar"):
    """Nested Wilson loop of a model over a k-plane (Sec. III)."""
    ev, U, st = eigh_grid(hl, kappa_grid, lo, hi)
    out = nested_from_grid(U, window, mode)
    out["status"] |= st
    return out


# ----------------------------------------------------------------------------
# Spin-resolved Wilson loop
# ----------------------------------------------------------------------------
def spin_sectors(U: np.ndarray, spin_diag: np.ndarray):
    """Projected spin operator inside the occupied space (Sec. IV).

    A = U^H S U with S = diag(spin_diag); (mu, Q) = eigh(A). Returns mu
    (ascending), V_minus = U Q[:, mu<0], V_plus = U Q[:, mu>0].
    """
    A = U.conj().T @ (spin_diag[:, None] * U)
    mu, Q = np.linalg.eigh(A)
    return mu, U @ Q[:, mu < 0], U @ Q[:, mu > 0]


def spin_resolved_from_grid(U_grid: np.ndarray, spin_diag: np.ndarray, mode: str = "polar"):
    """Spin-resolved Wilson loops from a U-grid (n_perp, n_par, N, m)."""
    n_perp, n_par, N, m = U_grid.shape
    status = 0
    mu = np.empty((n_perp, n_par, m))
    n_minus = None
    Vm, Vp = None, None
    for i in range(n_perp):
        for j in range(n_par):
            mu[i, j], a, b = spin_sectors(U_grid[i, j], spin_diag)
            if np.min(np.abs(mu[i, j])) < 1e-6:
                status |= PSO_GAP
            if n_minus is None:
                n_minus = a.shape[1]
                Vm = np.empty((n_perp, n_par, N, a.shape[1]), dtype=np.complex128)
                Vp = np.empty((n_perp, n_par, N, b.shape[1]), dtype=np.complex128)
            if a.shape[1] != n_minus:
                status |= PSO_GAP
                return {"status": status, "mu": mu}
            Vm[i, j], Vp[i, j] = a, b
    out = {"mu": mu, "m_minus": n_minus, "m_plus": m - n_minus}
    th_m, phi_m, c_dn, s1 = wilson_loop_grid(Vm, mode) if n_minus else (np.zeros((n_perp, 0)), np.zeros(n_perp), 0, 0)
    th_p, phi_p, c_up, s2 = wilson_loop_grid(Vp, mode) if m - n_minus else (np.zeros((n_perp, 0)), np.zeros(n_perp), 0, 0)
    out.update({"theta_dn": th_m, "theta_up": th_p, "phi_dn": phi_m, "phi_up": phi_p,
                "C_dn": c_dn, "C_up": c_up, "C_s": 0.5 * (c_up - c_dn),
                "status": status | s1 | s2})
    return out


def spin_resolved_wilson(hl, spin_diag: np.ndarray, kappa_grid: np.ndarray, lo: int, hi: int,
                         mode: str = "polar"):
    """Spin-resolved Wilson loop of a model over a k-plane (Sec. IV)."""
    ev, U, st = eigh_grid(hl, kappa_grid, lo, hi)
    out = spin_resolved_from_grid(U, np.asarray(spin_diag, dtype=np.float64), mode)
    out["status"] |= st
    return out


# ----------------------------------------------------------------------------
# Berry flux through the plaquettes of the grid (coupling-matrix method)
# ----------------------------------------------------------------------------
def link_phases(U_grid: np.ndarray):
    """Phases of the link variables det(U(k')^H U(k)) between neighbouring
    grid points, along the loop direction (k' = k(i, j+1)) and across it
    (k' = k(i+1, j)), both closing periodically. Returns (phi_par, phi_perp,
    smallest singular value of any link). A link variable det/|det| is
    undetermined when the link matrix is singular; the test is the one the
    Wilson loop applies to its overlaps, sigma_min < 1e-8, which does not
    depend on the order of the link (|det|, the product of all singular
    values, shrinks geometrically with the order even when every singular
    value is close to one)."""
    n_perp, n_par = U_grid.shape[:2]
    phi_par = np.empty((n_perp, n_par))
    phi_perp = np.empty((n_perp, n_par))
    smin = np.inf
    for i in range(n_perp):
        for j in range(n_par):
            for phi, Un in ((phi_par, U_grid[i, (j + 1) % n_par]), (phi_perp, U_grid[(i + 1) % n_perp, j])):
                L = Un.conj().T @ U_grid[i, j]
                phi[i, j] = np.angle(np.linalg.det(L))
                if L.size:
                    smin = min(smin, float(np.linalg.svd(L, compute_uv=False).min()))
    return phi_par, phi_perp, smin


def plaquette_flux_from_grid(U_grid: np.ndarray):
    """Berry flux through every plaquette of a U-grid (n_perp, n_par, N, m).

    The disordered quadrupolar-insulator example (Sec. IV) cuts the zone into plaquettes
    and integrates the Berry flux through each along its closed boundary
    (the coupling-matrix method, generalised there to spin sectors). The
    flux through plaquette (i, j), with corners k(i, j), k(i, j+1),
    k(i+1, j+1), k(i+1, j), is the phase of the product of the four link
    variables around it, in (-pi, pi]:
        F(i, j) = wrap(phi_par(i+1, j) - phi_par(i, j) + phi_perp(i, j) - phi_perp(i, j+1)),
    oriented so that the sum over the zone is 2 pi times the winding of
    eq. 6. Every link enters two plaquettes with opposite signs, so the sum
    over the zone is an exact multiple of 2 pi (the Chern number).
    Returns flux (n_perp, n_par), chern (int), total (sum / 2 pi), status.
    """
    phi_par, phi_perp, smin = link_phases(U_grid)
    F = np.roll(phi_par, -1, axis=0) - phi_par + phi_perp - np.roll(phi_perp, -1, axis=1)
    F = F - TWO_PI * np.round(F / TWO_PI)
    F = np.where(F <= -np.pi, np.pi, F)
    total = F.sum() / TWO_PI
    status = 0
    if smin < 1e-8:
        status |= OVERLAP_SINGULAR
    if np.max(np.abs(F)) > 0.8 * np.pi or abs(total - np.round(total)) > 1e-6:
        status |= WINDING_UNRESOLVED
    return {"flux": F, "chern": int(np.round(total)), "total": total, "status": status}


def plaquette_flux(hl, kappa_grid: np.ndarray, lo: int, hi: int):
    """Berry flux map of the bands [lo, hi) of a model over a k-plane."""
    ev, U, st = eigh_grid(hl, kappa_grid, lo, hi)
    out = plaquette_flux_from_grid(U)
    out["status"] |= st
    return out


def spin_resolved_flux(hl, spin_diag: np.ndarray, kappa_grid: np.ndarray, lo: int, hi: int):
    """Berry flux maps of the two spin sectors of the occupied space (the
    spin-resolved coupling-matrix method of the disordered quadrupolar
    insulator example, Sec. IV); C_s = (C_up - C_dn)/2."""
    ev, U, st = eigh_grid(hl, kappa_grid, lo, hi)
    n_perp, n_par, N, m = U.shape
    spin_diag = np.asarray(spin_diag, dtype=np.float64)
    sectors = [[spin_sectors(U[i, j], spin_diag) for j in range(n_par)] for i in range(n_perp)]
    m_dn = {sec[1].shape[1] for row in sectors for sec in row}
    if len(m_dn) != 1 or any(np.min(np.abs(sec[0])) < 1e-6 for row in sectors for sec in row):
        return {"status": st | PSO_GAP}
    Vm = np.stack([np.stack([sec[1] for sec in row]) for row in sectors])
    Vp = np.stack([np.stack([sec[2] for sec in row]) for row in sectors])
    dn, up = plaquette_flux_from_grid(Vm), plaquette_flux_from_grid(Vp)
    return {"flux_dn": dn["flux"], "flux_up": up["flux"], "C_dn": dn["chern"], "C_up": up["chern"],
            "C_s": 0.5 * (up["chern"] - dn["chern"]), "m_dn": Vm.shape[-1],
            "status": st | dn["status"] | up["status"]}


def pso_spectrum(hl, kappa, lo: int, hi: int, S: np.ndarray):
    """Spectrum of the projected spin operator P S P in the bands [lo, hi) at
    one k-point, for any Hermitian spin operator S (N x N), e.g. n.sigma on
    every spinor pair (the spin_spectrum scan of Sec. V, used to choose the
    spin axis along which this spectrum is gapped)."""
    H = bloch_hamiltonian(hl, np.asarray(kappa, dtype=np.float64))
    w, U = eigh_bands(H, lo, hi)[:2]
    return np.linalg.eigvalsh(U.conj().T @ S @ U)


# ----------------------------------------------------------------------------
# Independent Hermitian eigensolver (cross-check of LAPACK on small N)
# ----------------------------------------------------------------------------
def jacobi_eigh(H: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Cyclic complex Jacobi method for a Hermitian matrix.

    Each (p, q) step first removes the phase of H_pq with a diagonal unitary,
    then applies the real symmetric Jacobi rotation that zeroes the pair.
    Returns ascending eigenvalues and eigenvectors (columns).
    """
    A = np.array(H, dtype=np.complex128)
    n = A.shape[0]
    V = np.eye(n, dtype=np.complex128)
    scale = max(np.linalg.norm(A), 1e-300)
    for _ in range(max_sweeps):
        off = np.linalg.norm(A - np.diag(np.diag(A)))
        if off <= tol * scale:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                c = A[p, q]
                r = abs(c)
                if r <= 1e-300:
                    continue
                a, b = A[p, p].real, A[q, q].real
                ph = c / r
                tau = (b - a) / (2.0 * r)
                t = (1.0 if tau >= 0 else -1.0) / (abs(tau) + np.sqrt(1.0 + tau * tau))
                cs = 1.0 / np.sqrt(1.0 + t * t)
                sn = t * cs
                # J = D G with D = diag(1, conj(ph)) on (p, q), G = [[cs, sn], [-sn, cs]]
                J = np.array([[cs, sn], [-np.conj(ph) * sn, np.conj(ph) * cs]], dtype=np.complex128)
                cols = A[:, [p, q]] @ J
                A[:, p], A[:, q] = cols[:, 0], cols[:, 1]
                rows = J.conj().T @ A[[p, q], :]
                A[p, :], A[q, :] = rows[0], rows[1]
                A[p, q] = 0.0
                A[q, p] = 0.0
                vc = V[:, [p, q]] @ J
                V[:, p], V[:, q] = vc[:, 0], vc[:, 1]
    w = np.real(np.diag(A))
    order = np.argsort(w)
    return w[order], V[:, order]
