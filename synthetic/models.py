"""Tight-binding models as hopping lists, plus k-point planes.

A hopping list entry ``(i, j, R, t)`` is the amplitude ``t`` from orbital ``j``
in the cell at integer lattice vector ``R`` to orbital ``i`` in the home cell.
Every list holds both Hermitian partners: ``(j, i, -R, conj(t))`` is present
whenever ``(i, j, R, t)`` is (for ``R = 0`` the on-site block itself is
Hermitian). Duplicate ``(i, j, R)`` keys may occur (e.g. a mass term and an
on-site disorder term on the same orbital); consumers must add them.

The models follow the paper:

* ``qwz``      -- the two-band Chern insulator of Sec. II (eq. 4), mass ``m``.
* ``bhz``      -- the four-band quantum spin-Hall model of eq. 7, spin (sigma)
                  as the outer Kronecker factor, orbital (tau) inner.
* ``bbh``      -- the Benalcazar-Bernevig-Hughes quadrupole model that the
                  nested Wilson-loop section (Sec. III) cites.
* ``supercell`` / ``bhz_disordered`` / ``bhz_vacancies`` -- the supercells of
                  Sec. II-C and Sec. IV-A with periodic boundary conditions at
                  the supercell period; vacancies and disorder only change the
                  hopping list.
* ``wannier_like`` -- a synthetic many-orbital stand-in for the Wannier90
                  models of Sec. V (the real Wannier data is not available).

Seeds are ``numpy.random.SeedSequence`` entropy lists so every realisation is
reproducible and independent of call order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

_S0 = np.eye(2, dtype=np.complex128)
_S1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_S2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_S3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)


@dataclass
class HopList:
    """Hopping list of one (super)cell.

    N    -- number of orbitals.
    dim  -- number of periodic directions (length of each R).
    i, j -- int32[nnz] orbital indices.
    R    -- int32[nnz, dim] lattice vectors in (super)cell units.
    t    -- complex128[nnz] amplitudes.
    """

    N: int
    dim: int
    i: np.ndarray
    j: np.ndarray
    R: np.ndarray
    t: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.t.shape[0])

    def validate(self) -> None:
        assert self.i.dtype == np.int32 and self.j.dtype == np.int32
        assert self.R.dtype == np.int32 and self.R.shape == (self.nnz, self.dim)
        assert self.t.dtype == np.complex128
        assert self.nnz == 0 or (self.i.min() >= 0 and self.i.max() < self.N)
        assert self.nnz == 0 or (self.j.min() >= 0 and self.j.max() < self.N)


def _from_blocks(N: int, dim: int, blocks: Dict[Tuple[int, ...], np.ndarray],
                 meta: Optional[dict] = None) -> HopList:
    """Hopping list from matrix blocks T(R).

    ``blocks`` holds T(0) (Hermitian) and one of each pair T(R), T(-R); the
    partner T(-R) = T(R)^H is added here.
    """
    ii, jj, RR, tt = [], [], [], []
    for R, T in blocks.items():
        R = tuple(int(r) for r in R)
        assert len(R) == dim
        T = np.asarray(T, dtype=np.complex128)
        assert T.shape == (N, N)
        zero = all(r == 0 for r in R)
        parts = [(R, T)] if zero else [(R, T), (tuple(-r for r in R), T.conj().T)]
        for Rv, Tm in parts:
            a, b = np.nonzero(Tm)
            ii.append(a)
            jj.append(b)
            RR.append(np.tile(np.array(Rv, dtype=np.int32), (a.size, 1)))
            tt.append(Tm[a, b])
    hl = HopList(
        N=N,
        dim=dim,
        i=np.concatenate(ii).astype(np.int32),
        j=np.concatenate(jj).astype(np.int32),
        R=np.concatenate(RR).astype(np.int32).reshape(-1, dim),
        t=np.concatenate(tt).astype(np.complex128),
        meta=dict(meta or {}),
    )
    hl.validate()
    return hl


def qwz(m: float = 1.5) -> HopList:
    """Two-band Chern insulator, H = sin kx s1 + sin ky s2 + (m + cos kx + cos ky) s3."""
    blocks = {
        (0, 0): m * _S3,
        (1, 0): 0.5 * _S3 + _S1 / 2j,
        (0, 1): 0.5 * _S3 + _S2 / 2j,
    }
    return _from_blocks(2, 2, blocks, {"model": "qwz", "m": m})


def bhz(mass: float = 1.5) -> HopList:
    """BHZ model of eq. 7: sin kx s1(x)t1 + sin ky s1(x)t2 + (cos kx + cos ky + mass) s3(x)t0.

    Orbital index = 2*spin + orbital (spin outer).
    """
    blocks = {
        (0, 0): mass * np.kron(_S3, _S0),
        (1, 0): 0.5 * np.kron(_S3, _S0) + np.kron(_S1, _S1) / 2j,
        (0, 1): 0.5 * np.kron(_S3, _S0) + np.kron(_S1, _S2) / 2j,
    }
    return _from_blocks(4, 2, blocks, {"model": "bhz", "mass": mass})


def bbh_gammas():
    """Gamma matrices of the BBH quadrupole model, Kronecker order tau (x) sigma."""
    g1 = -np.kron(_S2, _S1)
    g2 = -np.kron(_S2, _S2)
    g3 = -np.kron(_S2, _S3)
    g4 = np.kron(_S1, _S0)
    return g1, g2, g3, g4


def bbh(gamma: float = 0.5, lam: float = 1.0) -> HopList:
    """BBH quadrupole model:
    h = (g + l cos kx) G4 + l sin kx G3 + (g + l cos ky) G2 + l sin ky G1.
    """
    g1, g2, g3, g4 = bbh_gammas()
    blocks = {
        (0, 0): gamma * (g4 + g2),
        (1, 0): 0.5 * lam * g4 + lam * g3 / 2j,
        (0, 1): 0.5 * lam * g2 + lam * g1 / 2j,
    }
    return _from_blocks(4, 2, blocks, {"model": "bbh", "gamma": gamma, "lambda": lam})


def choti(delta0: float = 1.0) -> HopList:
    """Chiral higher-order TI of eq. 9 (3D):
    sin kx s1(x)t1 + sin ky s1(x)t2 + sin kz s1(x)t3
    + (cos kx + cos ky + cos kz - 1.5) s3(x)t0 + delta0 (cos kx - cos ky) s2(x)t0.
    """
    st0 = np.kron(_S3, _S0)
    s2t0 = np.kron(_S2, _S0)
    blocks = {
        (0, 0, 0): -1.5 * st0,
        (1, 0, 0): 0.5 * st0 + np.kron(_S1, _S1) / 2j + 0.5 * delta0 * s2t0,
        (0, 1, 0): 0.5 * st0 + np.kron(_S1, _S2) / 2j - 0.5 * delta0 * s2t0,
        (0, 0, 1): 0.5 * st0 + np.kron(_S1, _S3) / 2j,
    }
    return _from_blocks(4, 3, blocks, {"model": "choti", "delta0": delta0})


def ssh(v: float, w: float) -> HopList:
    """1D SSH chain, H(k) = (v + w cos k) s1 + w sin k s2."""
    blocks = {(0,): v * _S1, (1,): 0.5 * w * _S1 + w * _S2 / 2j}
    return _from_blocks(2, 1, blocks, {"model": "ssh", "v": v, "w": w})


def bond_shift_1d() -> HopList:
    """1D two-orbital chain whose lower state is (1, e^{ik})/sqrt(2) in the lattice gauge."""
    return ssh(0.0, -1.0)


def product_state_2d(bx2: float, dy2: float) -> HopList:
    """Four-orbital model H(k) = -|u(k)><u(k)| with a product lower state.

    u = (sqrt(1-bx2), sqrt(bx2) e^{i kx}) (x) (sqrt(1-dy2), sqrt(dy2) e^{i ky});
    the lower band (energy -1) is separated by a unit gap from three flat
    bands at 0. Its hybrid centre along x is set by bx2 and its Berry phase
    along y by dy2 (pi exactly for dy2 = 1/2).
    """
    a, b = np.sqrt(1.0 - bx2), np.sqrt(bx2)
    c, d = np.sqrt(1.0 - dy2), np.sqrt(dy2)
    tx = {0: np.diag([a * a, b * b]), 1: np.array([[0, 0], [a * b, 0]]), -1: np.array([[0, a * b], [0, 0]])}
    ty = {0: np.diag([c * c, d * d]), 1: np.array([[0, 0], [c * d, 0]]), -1: np.array([[0, c * d], [0, 0]])}
    blocks = {}
    for R in [(0, 0), (1, 0), (0, 1), (1, 1), (1, -1)]:
        blocks[R] = -np.kron(tx[R[0]], ty[R[1]]).astype(np.complex128)
    return _from_blocks(4, 2, blocks, {"model": "product_state_2d", "bx2": bx2, "dy2": dy2})


def atomic(energies: Sequence[float], dim: int = 2) -> HopList:
    """No hopping at all: H(k) = diag(energies) for every k."""
    e = np.asarray(energies, dtype=np.float64)
    return _from_blocks(e.size, dim, {(0,) * dim: np.diag(e).astype(np.complex128)},
                        {"model": "atomic"})


def supercell(cell: HopList, L: int, removed_sites: Optional[np.ndarray] = None,
              site_onsite: Optional[np.ndarray] = None,
              onsite_weights: Optional[np.ndarray] = None) -> HopList:
    """Fold a 2D unit-cell hopping list into an L x L supercell.

    Site (x, y) has index s = x*L + y. Orbital a of site s becomes supercell
    orbital ``n_orb*c(s) + a`` where c() compacts the surviving sites.
    Supercell lattice vectors are in units of the supercell (k -> 2pi/L).
    ``removed_sites`` drops every orbital of those sites (vacancies);
    ``site_onsite`` adds a per-site scalar on every orbital of the site,
    times ``onsite_weights[a]`` on orbital a (default 1: the identity).
    """
    assert cell.dim == 2
    n_orb = cell.N
    ns = L * L
    keep = np.ones(ns, dtype=bool)
    if removed_sites is not None and len(removed_sites):
        keep[np.asarray(removed_sites, dtype=np.int64)] = False
    compact = -np.ones(ns, dtype=np.int64)
    compact[keep] = np.arange(int(keep.sum()))
    xs, ys = np.divmod(np.arange(ns), L)
    ii, jj, RR, tt = [], [], [], []
    for e in range(cell.nnz):
        a, b = int(cell.i[e]), int(cell.j[e])
        Rx, Ry = int(cell.R[e, 0]), int(cell.R[e, 1])
        tx, ty = xs + Rx, ys + Ry
        Sx, Sy = np.floor_divide(tx, L), np.floor_divide(ty, L)
        tgt = np.mod(tx, L) * L + np.mod(ty, L)
        ok = keep & keep[tgt]
        src = np.arange(ns)[ok]
        ii.append(n_orb * compact[src] + a)
        jj.append(n_orb * compact[tgt[ok]] + b)
        RR.append(np.stack([Sx[ok], Sy[ok]], axis=1))
        tt.append(np.full(src.size, cell.t[e], dtype=np.complex128))
    if site_onsite is not None:
        eps = np.asarray(site_onsite, dtype=np.float64)
        assert eps.shape == (ns,)
        wts = np.ones(n_orb) if onsite_weights is None else np.asarray(onsite_weights, dtype=np.float64)
        assert wts.shape == (n_orb,)
        src = np.arange(ns)[keep]
        for a in range(n_orb):
            ii.append(n_orb * compact[src] + a)
            jj.append(n_orb * compact[src] + a)
            RR.append(np.zeros((src.size, 2), dtype=np.int64))
            tt.append((wts[a] * eps[src]).astype(np.complex128))
    N = n_orb * int(keep.sum())
    meta = dict(cell.meta)
    meta.update({"L": L, "n_removed": int(ns - keep.sum()), "n_orb_cell": n_orb})
    hl = HopList(
        N=N,
        dim=2,
        i=np.concatenate(ii).astype(np.int32),
        j=np.concatenate(jj).astype(np.int32),
        R=np.concatenate(RR).astype(np.int32).reshape(-1, 2),
        t=np.concatenate(tt),
        meta=meta,
    )
    hl.validate()
    return hl


def bhz_disordered(L: int, W: float, seed: Sequence[int], mass: float = 1.5) -> HopList:
    """BHZ on an L x L supercell with Anderson on-site disorder.

    One scalar eps_s ~ U[-W/2, W/2] per site, times the 4x4 identity (spin
    independent, so it commutes with the spin operator).
    """
    rng = np.random.default_rng(list(seed))
    eps = rng.uniform(-W / 2.0, W / 2.0, L * L)
    hl = supercell(bhz(mass), L, site_onsite=eps)
    hl.meta.update({"W": W, "seed": list(seed)})
    return hl


def bhz_vacancies(L: int, frac: float, seed: Sequence[int], W: float = 0.0,
                  disorder_seed: Optional[Sequence[int]] = None,
                  mass: float = 1.5) -> HopList:
    """BHZ L x L supercell with round(frac*L^2) sites removed (uniform, no replacement)."""
    rng = np.random.default_rng(list(seed))
    n_vac = int(round(frac * L * L))
    removed = np.sort(rng.choice(L * L, size=n_vac, replace=False)) if n_vac else np.zeros(0, np.int64)
    eps = None
    if W > 0.0:
        drng = np.random.default_rng(list(disorder_seed if disorder_seed is not None else list(seed) + [1]))
        eps = drng.uniform(-W / 2.0, W / 2.0, L * L)
    hl = supercell(bhz(mass), L, removed_sites=removed, site_onsite=eps)
    hl.meta.update({"removed": removed, "frac": frac, "seed": list(seed), "W": W})
    return hl


def bhz_spin_diag(hl: HopList) -> np.ndarray:
    """Diagonal of the spin operator s3 (x) t3 = diag(1,-1,-1,1) per site, for a BHZ (super)cell."""
    n_sites = hl.N // 4
    return np.tile(np.array([1.0, -1.0, -1.0, 1.0]), n_sites)


def spinful_bbh(mass: float = 1.0, delta: float = 0.5) -> HopList:
    """Spinful quadrupolar insulator of eq. 10 (orbital index 2*sigma + tau):
    sin kx s1(x)t3 + sin ky s2(x)t3 + (cos kx + cos ky + mass) s3(x)t3
    + delta (cos kx - cos ky) s0(x)t1.

    The last matrix is printed as s0(x)t0, which commutes with the chiral
    operator S = s0(x)t2 that the model is said to have and closes the gap at
    half filling; s0(x)t1 is the matrix that anticommutes with S and with the
    other three terms (the quadrupolar mass), and is used here.
    """
    m3 = np.kron(_S3, _S3)
    d = np.kron(_S0, _S1)
    blocks = {
        (0, 0): mass * m3,
        (1, 0): 0.5 * m3 + np.kron(_S1, _S3) / 2j + 0.5 * delta * d,
        (0, 1): 0.5 * m3 + np.kron(_S2, _S3) / 2j - 0.5 * delta * d,
    }
    return _from_blocks(4, 2, blocks, {"model": "spinful_bbh", "mass": mass, "delta": delta})


SPINFUL_BBH_SPIN = np.array([1.0, -1.0, 1.0, -1.0])   # diagonal of s0(x)t3 per site


def spinful_bbh_disordered(L: int, W: float, seed: Sequence[int]) -> HopList:
    """Spinful BBH on an L x L supercell with chiral-symmetric disorder
    w_s s0(x)t3 on every site, w_s ~ U[-W/2, W/2] (Sec. IV example)."""
    rng = np.random.default_rng(list(seed))
    eps = rng.uniform(-W / 2.0, W / 2.0, L * L)
    hl = supercell(spinful_bbh(), L, site_onsite=eps, onsite_weights=SPINFUL_BBH_SPIN)
    hl.meta.update({"W": W, "seed": list(seed)})
    return hl


def spinful_bbh_spin_diag(hl: HopList) -> np.ndarray:
    """Diagonal of the spin operator s0(x)t3 for a spinful-BBH (super)cell."""
    return np.tile(SPINFUL_BBH_SPIN, hl.N // 4)


def wannier_like(n_orb: int, seed: Sequence[int], r_max: float = 3.0,
                 decay: float = 1.5) -> HopList:
    """Synthetic many-orbital 'Wannier-like' model.

    Random Hermitian hoppings to every lattice vector with |R| <= r_max
    (Euclidean, cell units); T(R) = exp(-|R|/decay) (A + iB)/sqrt(2) with A, B
    standard normal n_orb x n_orb, T(-R) = T(R)^H, T(0) Hermitised.
    """
    rng = np.random.default_rng(list(seed))
    rmax = int(np.floor(r_max))
    vecs = [(a, b) for a in range(-rmax, rmax + 1) for b in range(-rmax, rmax + 1)
            if a * a + b * b <= r_max * r_max + 1e-12]
    blocks = {}
    for (a, b) in vecs:
        if (a, b) < (0, 0):
            continue
        amp = np.exp(-np.hypot(a, b) / decay)
        T = amp * (rng.standard_normal((n_orb, n_orb)) + 1j * rng.standard_normal((n_orb, n_orb))) / np.sqrt(2.0)
        if (a, b) == (0, 0):
            T = 0.5 * (T + T.conj().T)
        blocks[(a, b)] = T
    hl = _from_blocks(n_orb, 2, blocks, {"model": "wannier_like", "seed": list(seed),
                                         "n_R": len(vecs)})
    return hl


def concat_hops(hls: Sequence[HopList]) -> HopList:
    """Block-diagonal direct sum of several hopping lists (same dim)."""
    dim = hls[0].dim
    off = 0
    ii, jj, RR, tt = [], [], [], []
    for h in hls:
        assert h.dim == dim
        ii.append(h.i.astype(np.int64) + off)
        jj.append(h.j.astype(np.int64) + off)
        RR.append(h.R)
        tt.append(h.t)
        off += h.N
    hl = HopList(N=off, dim=dim, i=np.concatenate(ii).astype(np.int32),
                 j=np.concatenate(jj).astype(np.int32),
                 R=np.concatenate(RR).astype(np.int32).reshape(-1, dim),
                 t=np.concatenate(tt), meta={"model": "direct_sum"})
    hl.validate()
    return hl


def rotated_bhz(axis=(1.0, 0.0, 0.0), L: int = 1, W: float = 0.0, seed: Sequence[int] = (0,)) -> HopList:
    """BHZ (or its disordered L x L supercell) with the spin quantization axis
    turned from z to ``axis``: every hopping block conjugated by the spinor
    rotation exp(-i a/2 m.sigma) that takes z to the axis, in an interleaved
    spinor basis: BHZ orbital (site, s, t) becomes 2*(2*site + s) + b with
    b = 0 for the +1 eigenstate of the conserved BHZ spin s3 (x) t3 (b = s xor
    t). The conserved spin of the result is axis.sigma on every pair, not
    sigma_z."""
    base = supercell(bhz(), L, site_onsite=np.random.default_rng(list(seed)).uniform(-W / 2.0, W / 2.0, L * L)) \
        if L > 1 else bhz()
    n = np.asarray(axis, dtype=np.float64)
    n = n / np.linalg.norm(n)
    z = np.array([0.0, 0.0, 1.0])
    m = np.cross(z, n)
    a = np.arccos(np.clip(n @ z, -1.0, 1.0))
    if np.linalg.norm(m) < 1e-12:
        m = np.array([1.0, 0.0, 0.0])
    m = m / np.linalg.norm(m)
    msig = m[0] * _S1 + m[1] * _S2 + m[2] * _S3
    rot = np.cos(a / 2) * _S0 - 1j * np.sin(a / 2) * msig
    ns = base.N // 4
    perm = np.empty(base.N, dtype=np.int64)
    for s_ in range(ns):
        for sg in range(2):
            for tau in range(2):
                perm[4 * s_ + 2 * sg + tau] = 2 * (2 * s_ + sg) + (sg ^ tau)
    Rmat = np.kron(np.eye(base.N // 2), rot)
    keys = {}
    for e in range(base.nnz):
        keys.setdefault(tuple(int(x) for x in base.R[e]), []).append(e)
    ii, jj, RR, tt = [], [], [], []
    for R, es in keys.items():
        T = np.zeros((base.N, base.N), dtype=np.complex128)
        for e in es:
            T[perm[base.i[e]], perm[base.j[e]]] += base.t[e]
        T = Rmat @ T @ Rmat.conj().T
        a_, b_ = np.nonzero(np.abs(T) > 1e-15)
        ii.append(a_)
        jj.append(b_)
        RR.append(np.tile(np.array(R, dtype=np.int32), (a_.size, 1)))
        tt.append(T[a_, b_])
    hl = HopList(N=base.N, dim=2, i=np.concatenate(ii).astype(np.int32), j=np.concatenate(jj).astype(np.int32),
                 R=np.concatenate(RR).astype(np.int32).reshape(-1, 2), t=np.concatenate(tt),
                 meta={"model": "rotated_bhz", "axis": list(n), "L": L, "W": W})
    hl.validate()
    return hl


def write_tb(hl: HopList, path, lattice=None, degeneracy=None, header: str = "synthetic tight-binding model") -> None:
    """Write a hopping list in the Wannier90 ``_tb.dat`` layout: header,
    lattice (3 rows), num_wann, nrpts, degeneracies (15 per line), then per R
    a blank line, R (3 integers) and num_wann^2 lines 'm n Re Im' (1-based,
    m fastest) holding ndegen(R) * t(R)_{mn}, then the position section (the
    same R list, zeros). ``degeneracy(R)`` gives ndegen (default 1)."""
    lat = np.eye(3) if lattice is None else np.asarray(lattice, dtype=np.float64)
    N = hl.N
    blocks = {}
    for e in range(hl.nnz):
        R = tuple(int(x) for x in hl.R[e]) + (0,) * (3 - hl.dim)
        blocks.setdefault(R, np.zeros((N, N), dtype=np.complex128))[hl.i[e], hl.j[e]] += hl.t[e]
    for R in list(blocks):
        mR = tuple(-x for x in R)
        blocks.setdefault(mR, np.zeros((N, N), dtype=np.complex128))
    Rs = sorted(blocks)
    deg = [1 if degeneracy is None else int(degeneracy(R)) for R in Rs]
    with open(path, "w") as f:
        f.write(header + "\n")
        for row in lat:
            f.write(" ".join(f"{x:22.15e}" for x in row) + "\n")
        f.write(f"{N:12d}\n{len(Rs):12d}\n")
        for k in range(0, len(deg), 15):
            f.write("".join(f"{d:5d}" for d in deg[k:k + 15]) + "\n")
        for R, d in zip(Rs, deg):
            f.write("\n" + "".join(f"{x:5d}" for x in R) + "\n")
            T = blocks[R] * d
            for n_ in range(N):
                for m_ in range(N):
                    v = T[m_, n_]
                    f.write(f"{m_ + 1:5d}{n_ + 1:5d}   {v.real:23.16e} {v.imag:23.16e}\n")
        for R in Rs:
            f.write("\n" + "".join(f"{x:5d}" for x in R) + "\n")
            for n_ in range(N):
                for m_ in range(N):
                    f.write(f"{m_ + 1:5d}{n_ + 1:5d}   " + " ".join(["0.0"] * 6) + "\n")


def write_centres(centres: np.ndarray, path, atoms=()) -> None:
    """Wannier centres in the ``_centres.xyz`` layout (symbol X), then atoms."""
    c = np.asarray(centres, dtype=np.float64)
    with open(path, "w") as f:
        f.write(f"{len(c) + len(atoms)}\nWannier centres\n")
        for x in c:
            f.write(f"X {x[0]:17.8f}{x[1]:17.8f}{x[2]:17.8f}\n")
        for sym, x in atoms:
            f.write(f"{sym} {x[0]:17.8f}{x[1]:17.8f}{x[2]:17.8f}\n")


def kplane(n_par: int, n_perp: int, e_par=(1.0, 0.0, 0.0), e_perp=(0.0, 1.0, 0.0),
           k0=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Fractional k-points of a plane: kappa[i, j] = k0 + (j/n_par) e_par + (i/n_perp) e_perp.

    ``j`` runs along the Wilson loop (closed, n_par segments) and ``i`` over
    the transverse direction (n_perp points, half open). Returns float64
    [n_perp, n_par, 3].
    """
    e_par = np.asarray(e_par, dtype=np.float64)
    e_perp = np.asarray(e_perp, dtype=np.float64)
    k0 = np.asarray(k0, dtype=np.float64)
    j = np.arange(n_par, dtype=np.float64) / n_par
    i = np.arange(n_perp, dtype=np.float64) / n_perp
    return k0[None, None, :] + i[:, None, None] * e_perp[None, None, :] + j[None, :, None] * e_par[None, None, :]


def link_grid(cosines) -> np.ndarray:
    """A 2 x 2 grid of orthonormal bases (N = 2m, m = len(cosines)) whose links
    along the loop direction have the given singular values: U(i, 0) spans
    e_0 .. e_{m-1}, U(i, 1) has columns c_k e_k + sqrt(1 - c_k^2) e_{m+k}, so
    U(i, 1)^H U(i, 0) = diag(c); the links across the loop are identities.
    Returns (n_perp, n_par, N, m) complex128."""
    c = np.asarray(cosines, dtype=np.float64)
    m = c.size
    A = np.zeros((2 * m, m), dtype=np.complex128)
    A[np.arange(m), np.arange(m)] = 1.0
    B = np.zeros((2 * m, m), dtype=np.complex128)
    B[np.arange(m), np.arange(m)] = c
    B[m + np.arange(m), np.arange(m)] = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    return np.stack([np.stack([A, B]), np.stack([A, B])])


# ---------------------------------------------------------------- workload mixes
SERVED_TYPES = ("bhz8", "bhz12", "bhz16", "bhz24", "w96")


def served_types(n: int, seed) -> list:
    """Request types of a served stream of n requests: the five types
    (BHZ supercells L = 8, 12, 16, 24 and the 96-orbital model) equally
    often, in a seeded random order (each block of five holds every type once,
    so any prefix of the stream is balanced to within one request per type)."""
    rng = np.random.default_rng(list(seed))
    out = []
    while len(out) < n:
        out += [SERVED_TYPES[i] for i in rng.permutation(len(SERVED_TYPES))]
    return out[:n]


def served_model(kind: str, req: int) -> HopList:
    """The model of request number req of a served stream: a BHZ supercell
    with Anderson disorder of strength W ~ U[0, 4] (seeded [5, 1, req]), or
    the 96-orbital model (seeded [5, 2, req])."""
    if kind == "w96":
        return wannier_like(96, [5, 2, req])
    L = int(kind[3:])
    W = float(np.random.default_rng([5, 3, req]).uniform(0.0, 4.0))
    return bhz_disordered(L, W, [5, 1, req])


def uneven_systems(n: int = 64, sizes=(6, 8, 12, 16, 20), frac: float = 0.02) -> list:
    """Uneven batch of BHZ supercells: L drawn uniformly from sizes (seeded
    [4, 0]), round(frac L^2) vacancies each (seeded [4, 1, s]), no disorder."""
    Ls = np.random.default_rng([4, 0]).choice(np.asarray(sizes), size=n)
    return [bhz_vacancies(int(L), frac, [4, 1, s]) for s, L in enumerate(Ls)]
