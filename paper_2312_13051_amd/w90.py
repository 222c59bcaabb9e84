"""Wannier90 tight-binding ingestion and spin-axis selection (host side).

Sec. V builds the tight-binding model of a real material from the Wannier90
files ``<seed>_tb.dat`` (lattice, Wigner-Seitz vectors with their
degeneracies, Hamiltonian blocks H(R)) and ``<seed>_centres.xyz``, keeping
hoppings above an energy cutoff (ECut) and within a neighbour cutoff
(HopCut); it then scans the spectrum of the projected spin operator over a
grid of k-points (``spin_spectrum``) to find a spin axis along which that
spectrum is gapped, before the spin-resolved Wilson loop.

``read_tb`` returns a hopping list in the form the library's plan builder
takes (N, dim, i, j, R, t): entry e is the amplitude from orbital j in cell R
to orbital i in the home cell, H(R)_{ij} / ndegen(R). ``rotate_spin_axis``
changes the spinor basis of a hopping list so that a chosen axis n.sigma
becomes diagonal (+1, -1 on each spinor pair), which turns any spin axis into
the diagonal spin operator the spin-resolved calls take. No arithmetic of
the Wilson-loop method happens here.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np


@dataclass
class TBModel:
    """Hopping list of a Wannier90 model (duck-types the plan builder's input)."""
    N: int
    dim: int
    i: np.ndarray
    j: np.ndarray
    R: np.ndarray
    t: np.ndarray
    lattice: np.ndarray                      # rows: real-space lattice vectors (Angstrom)
    centres: Optional[np.ndarray] = None     # (N, 3) Wannier centres (Angstrom), if read
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.t.shape[0])


def _tokens(path):
    with open(path) as f:
        f.readline()                         # header (date / comment)
        rest = f.read().split()
    return rest


def read_centres(path) -> np.ndarray:
    """Wannier centres from ``<seed>_centres.xyz``: the rows whose symbol is X."""
    with open(path) as f:
        lines = f.read().splitlines()
    n = int(lines[0].split()[0])
    rows = [ln.split() for ln in lines[2:2 + n]]
    return np.array([[float(x) for x in r[1:4]] for r in rows if r and r[0] == "X"], dtype=np.float64)


def read_tb(path, ecut: float = 0.0, hopcut: float = np.inf, centres=None, dim: Optional[int] = None) -> TBModel:
    """Parse ``<seed>_tb.dat`` into a hopping list.

    ecut   keep hoppings with |t| >= ecut (energy units of the file, after
           the division by the Wigner-Seitz degeneracy);
    hopcut keep hoppings whose length |R.A + c_j - c_i| <= hopcut (Angstrom;
           c = Wannier centres if given, else 0);
    centres (N, 3) array or a path to ``<seed>_centres.xyz``;
    dim    2 for a layer (every kept R must have R3 = 0), default 3.
    The Hamiltonian blocks H(R) and H(-R) are conjugate transposes in the
    file up to its printed digits; each pair is averaged so that the list is
    Hermitian to rounding. The position-operator section is not used.
    """
    tok = _tokens(path)
    lat = np.array(tok[0:9], dtype=np.float64).reshape(3, 3)
    nw, nr = int(tok[9]), int(tok[10])
    p = 11
    deg = np.array(tok[p:p + nr], dtype=np.float64)
    p += nr
    if np.any(deg <= 0):
        raise ValueError(f"{path}: degeneracies must be positive")
    Rs = np.empty((nr, 3), dtype=np.int64)
    H = np.empty((nr, nw, nw), dtype=np.complex128)
    blk = nw * nw * 4
    for r in range(nr):
        Rs[r] = np.array(tok[p:p + 3], dtype=np.int64)
        p += 3
        a = np.array(tok[p:p + blk], dtype=np.float64).reshape(nw * nw, 4)
        p += blk
        m, n = a[:, 0].astype(np.int64) - 1, a[:, 1].astype(np.int64) - 1
        if m.min() < 0 or n.min() < 0 or m.max() >= nw or n.max() >= nw:
            raise ValueError(f"{path}: orbital index out of range in block {r}")
        H[r, m, n] = (a[:, 2] + 1j * a[:, 3]) / deg[r]
    # Hermitian pairs H(-R) = H(R)^H, averaged
    index = {tuple(R): r for r, R in enumerate(Rs)}
    for r, R in enumerate(Rs):
        q = index.get(tuple(-R))
        if q is None:
            raise ValueError(f"{path}: R = {tuple(R)} has no partner -R")
        if q >= r:
            avg = 0.5 * (H[r] + H[q].conj().T)
            H[r], H[q] = avg, avg.conj().T
    if centres is not None and not isinstance(centres, np.ndarray):
        centres = read_centres(centres)
    if centres is not None:
        centres = np.asarray(centres, dtype=np.float64)
        if centres.shape != (nw, 3):
            raise ValueError(f"centres: expected ({nw}, 3), got {centres.shape}")
    if dim is None:
        dim = 3
    ii, jj, RR, tt = [], [], [], []
    for r in range(nr):
        m, n = np.nonzero(np.abs(H[r]) >= max(ecut, 1e-300))
        if m.size == 0:
            continue
        d = np.tile(Rs[r] @ lat, (m.size, 1))
        if centres is not None:
            d += centres[n] - centres[m]
        keep = np.linalg.norm(d, axis=1) <= hopcut
        m, n = m[keep], n[keep]
        if m.size == 0:
            continue
        if dim < 3 and np.any(Rs[r, dim:] != 0):
            raise ValueError(f"{path}: R = {tuple(Rs[r])} leaves the {dim}D layer")
        ii.append(m)
        jj.append(n)
        RR.append(np.tile(Rs[r, :dim], (m.size, 1)))
        tt.append(H[r, m, n])
    if not ii:
        raise ValueError(f"{path}: no hopping survives the cutoffs")
    return TBModel(N=nw, dim=dim, i=np.concatenate(ii).astype(np.int32), j=np.concatenate(jj).astype(np.int32),
                   R=np.concatenate(RR).astype(np.int32).reshape(-1, dim), t=np.concatenate(tt),
                   lattice=lat, centres=centres,
                   meta={"source": str(path), "ecut": ecut, "hopcut": hopcut, "nrpts": nr})


def spin_pairs(N: int, order: str = "interleaved") -> np.ndarray:
    """Orbital pairs (up, down) of a spinor basis: (2p, 2p+1) for
    'interleaved', (p, p + N/2) for 'blocked'."""
    if N % 2:
        raise ValueError("a spinor basis has an even number of orbitals")
    p = np.arange(N // 2)
    if order == "interleaved":
        return np.stack([2 * p, 2 * p + 1], axis=1)
    if order == "blocked":
        return np.stack([p, p + N // 2], axis=1)
    raise ValueError(f"unknown spinor order {order!r}")


def axis_unitary(axis) -> np.ndarray:
    """2x2 unitary u with u^H (n.sigma) u = diag(1, -1), n = axis / |axis|."""
    n = np.asarray(axis, dtype=np.float64)
    n = n / np.linalg.norm(n)
    s = n[0] * np.array([[0, 1], [1, 0]]) + n[1] * np.array([[0, -1j], [1j, 0]]) + n[2] * np.diag([1.0, -1.0])
    w, v = np.linalg.eigh(s)
    return v[:, ::-1]                        # eigenvalue +1 first


def rotate_spin_axis(model, axis, order: str = "interleaved"):
    """Hopping list in the spinor basis where n.sigma is diagonal on every
    pair (up component +1, down component -1), and that diagonal.

    t'(R) = B^H t(R) B with B block diagonal (u on every spinor pair); the
    spectrum of the projected spin operator is unchanged by the change of
    basis, so a diagonal spin operator in the new basis is n.sigma in the old.
    """
    N = model.N
    pairs = spin_pairs(N, order)
    u = axis_unitary(axis)
    pos = np.empty(N, dtype=np.int64)        # position of each orbital within its pair
    mate = np.empty((N, 2), dtype=np.int64)  # the pair an orbital belongs to
    for a, b in pairs:
        pos[a], pos[b] = 0, 1
        mate[a], mate[b] = (a, b), (a, b)
    i, j, t = model.i.astype(np.int64), model.j.astype(np.int64), model.t
    # t'_{ab} = sum_{a' in pair(a), b' in pair(b)} conj(B_{a'a}) t_{a'b'} B_{b'b}
    ii, jj, RR, tt = [], [], [], []
    for pa in range(2):
        for pb in range(2):
            a = mate[i, pa]
            b = mate[j, pb]
            w = np.conj(u[pos[i], pa]) * t * u[pos[j], pb]
            ii.append(a)
            jj.append(b)
            RR.append(model.R)
            tt.append(w)
    i2, j2 = np.concatenate(ii), np.concatenate(jj)
    R2, t2 = np.concatenate(RR), np.concatenate(tt)
    key = np.concatenate([i2[:, None], j2[:, None], R2.astype(np.int64)], axis=1)
    uk, inv = np.unique(key, axis=0, return_inverse=True)
    tsum = np.zeros(uk.shape[0], dtype=np.complex128)
    np.add.at(tsum, inv.ravel(), t2)
    keep = np.abs(tsum) > 0.0
    uk, tsum = uk[keep], tsum[keep]
    diag = np.empty(N)
    diag[pairs[:, 0]], diag[pairs[:, 1]] = 1.0, -1.0
    out = TBModel(N=N, dim=model.dim, i=uk[:, 0].astype(np.int32), j=uk[:, 1].astype(np.int32),
                  R=uk[:, 2:].astype(np.int32).reshape(-1, model.dim), t=tsum,
                  lattice=getattr(model, "lattice", np.eye(3)), centres=getattr(model, "centres", None),
                  meta=dict(getattr(model, "meta", {}), spin_axis=list(np.asarray(axis, float)), spin_order=order))
    return out, diag


def axes_grid(n_theta: int = 7, n_phi: int = 12) -> np.ndarray:
    """Candidate spin axes on the upper hemisphere (n and -n give the same
    spectrum up to sign): the pole and n_phi azimuths at each polar angle."""
    axes = [np.array([0.0, 0.0, 1.0])]
    for th in np.linspace(0.0, np.pi / 2, n_theta)[1:]:
        for ph in np.arange(n_phi) * (np.pi / n_phi if th == np.pi / 2 else 2 * np.pi / n_phi):
            axes.append(np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)]))
    return np.array(axes)


def scan_spin_axes(ctx, model, kpoints: np.ndarray, lo: int, hi: int, axes: Sequence, order: str = "interleaved",
                   precision: int = 0):
    """Spectrum of the projected spin operator n.sigma for every candidate
    axis at every k-point (the paper's spin_spectrum over a grid), in one
    batch on the GPU: the rotated models are the systems of one call.
    Returns mu (n_axes, n_k, m), gap (n_axes,) = min |mu| over k and bands,
    and the axis with the largest gap."""
    from . import pipeline as P
    torch = P._torch()
    rot = [rotate_spin_axis(model, ax, order) for ax in axes]
    kp = np.asarray(kpoints, dtype=np.float64).reshape(1, -1, 3)
    plan = ctx.hk_plan([r[0] for r in rot])
    g = P.eig_grid(ctx, plan, 0, len(rot), kp, lo, hi, precision)
    m = max(g.m, 1)
    n_k = kp.shape[1]
    sd = torch.as_tensor(np.stack([r[1] for r in rot])).cuda()
    pso = torch.empty((len(rot), n_k, m), dtype=torch.float64, device="cuda")
    V = torch.empty((len(rot) * n_k, m, g.N), dtype=torch.complex128, device="cuda")
    st = torch.empty(len(rot), dtype=torch.int32, device="cuda")
    ctx.spin_sectors(g.U, g.N, g.m, g.ldu, g.U.stride(0), len(rot), n_k, sd, pso, V, g.N, V.stride(0), st,
                     precision)
    mu = pso[..., :g.m].cpu().numpy()
    gap = np.abs(mu).min(axis=(1, 2)) if g.m else np.zeros(len(rot))
    return {"mu": mu, "gap": gap, "axis": np.asarray(axes[int(np.argmax(gap))], dtype=np.float64),
            "status": st.cpu().numpy() | g.status.view(len(rot), n_k).cpu().numpy().max(axis=1)}
