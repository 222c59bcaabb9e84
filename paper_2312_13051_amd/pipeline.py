"""Whole-plane drivers over the C ABI (orchestration only, no arithmetic).

These chain the library calls the way the paper's functions are used:
``wsurf`` (hybrid Wannier centres over a plane, Sec. II), ``wnwl`` (nested
Wilson loop, Sec. III), ``wspinsurf`` (spin-resolved Wilson loop, Sec. IV)
``wflux`` / ``wspinflux`` (Berry flux per plaquette of the occupied space
or of its spin sectors, the coupling-matrix method of Sec. IV), and
``eig_planes`` / ``wnwl_planes`` (a family of parallel planes of a 3D model,
e.g. the nested loop against kz of Sec. III, in one batch).
Every step runs in the HIP library; torch only allocates device memory.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from . import _lib as L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise L.BerryError("berryhip needs a HIP GPU (torch.cuda is not available)")
    return torch


@dataclass
class EigGrid:
    """Selected eigenvectors of every k-point of a plane for n_sys systems.

    U has shape (n_sys * n_perp * n_par, m, ldu): matrix q is column-major N x m.
    evals: (n_mat, m + 2), status: (n_mat,) int32.
    """
    U: "object"
    evals: "object"
    status: "object"
    N: int
    m: int
    ldu: int
    n_sys: int
    n_par: int
    n_perp: int


def eig_grid(ctx: L.Context, plan: L.HkPlan, sys_first: int, n_sys: int, kappa_grid: np.ndarray, lo: int, hi: int,
             precision: int = L.BE_FP64, chunk: int = 4096) -> EigGrid:
    """build_hk + eigh_batched over a k-plane (n_perp, n_par, 3) for consecutive systems."""
    torch = _torch()
    n_perp, n_par = kappa_grid.shape[:2]
    N = plan.N[sys_first]
    m = hi - lo
    n_k = n_perp * n_par
    kap = torch.from_numpy(np.ascontiguousarray(kappa_grid.reshape(-1, 3), dtype=np.float64)).cuda()
    n_mat = n_sys * n_k
    ldu = N
    U = torch.empty((n_mat, max(m, 1), ldu), dtype=torch.complex128, device="cuda")
    ev = torch.empty((n_mat, m + 2), dtype=torch.float64, device="cuda")
    st = torch.empty(n_mat, dtype=torch.int32, device="cuda")
    cdt = torch.complex64 if L.c64_input(precision) else torch.complex128
    dt = L.BE_C64 if L.c64_input(precision) else L.BE_C128
    per = max(1, chunk // n_k)  # systems per chunk
    H = torch.empty((min(per, n_sys) * n_k, N, N), dtype=cdt, device="cuda")
    for s0 in range(0, n_sys, per):
        ns = min(per, n_sys - s0)
        ctx.build_hk(plan, sys_first + s0, ns, kap, H, N * N, N, dt)
        q0 = s0 * n_k
        ctx.eigh_batched(H, dt, N, N, N * N, ns * n_k, lo, hi, precision, ev[q0:], U[q0:], ldu, U.stride(0), st[q0:])
    return EigGrid(U, ev, st, N, m, ldu, n_sys, n_par, n_perp)


def wilson(ctx: L.Context, g: EigGrid, mode: int = L.BE_OVL_POLAR):
    torch = _torch()
    theta = torch.empty((g.n_sys, g.n_perp, max(g.m, 1)), dtype=torch.float64, device="cuda")
    phi = torch.empty((g.n_sys, g.n_perp), dtype=torch.float64, device="cuda")
    wind = torch.empty(g.n_sys, dtype=torch.int32, device="cuda")
    st = torch.empty(g.n_sys, dtype=torch.int32, device="cuda")
    ctx.wilson_loop(g.U, g.N, g.m, g.ldu, g.U.stride(0), g.n_sys, g.n_par, g.n_perp, mode, theta, phi, wind, st)
    return {"theta": theta[..., :g.m], "phi": phi, "winding": wind, "status": st}


def nested(ctx: L.Context, g: EigGrid, window=(0.0, 0.5), mode: int = L.BE_OVL_POLAR):
    torch = _torch()
    m = max(g.m, 1)
    nth = torch.empty((g.n_sys, g.n_par, m), dtype=torch.float64, device="cuda")
    p = torch.empty((g.n_sys, g.n_par), dtype=torch.float64, device="cuda")
    pm = torch.empty(g.n_sys, dtype=torch.float64, device="cuda")
    st = torch.empty(g.n_sys, dtype=torch.int32, device="cuda")
    s = ctx.nested_wilson(g.U, g.N, g.m, g.ldu, g.U.stride(0), g.n_sys, g.n_par, g.n_perp, mode, window[0], window[1],
                          nth, p, pm, st)
    return {"theta": nth, "s": s, "p": p, "p_mean": pm, "status": st}


def spin(ctx: L.Context, g: EigGrid, spin_diag, mode: int = L.BE_OVL_POLAR, precision: int = L.BE_FP64):
    """spin_diag: (n_sys, N) float64 (numpy or torch)."""
    torch = _torch()
    m = max(g.m, 1)
    sd = torch.as_tensor(np.asarray(spin_diag, dtype=np.float64).reshape(g.n_sys, g.N)).cuda()
    pso = torch.empty((g.n_sys, g.n_perp, g.n_par, m), dtype=torch.float64, device="cuda")
    tdn = torch.empty((g.n_sys, g.n_perp, m), dtype=torch.float64, device="cuda")
    tup = torch.empty((g.n_sys, g.n_perp, m), dtype=torch.float64, device="cuda")
    cdn = torch.empty(g.n_sys, dtype=torch.int32, device="cuda")
    cup = torch.empty(g.n_sys, dtype=torch.int32, device="cuda")
    cs = torch.empty(g.n_sys, dtype=torch.float64, device="cuda")
    st = torch.empty(g.n_sys, dtype=torch.int32, device="cuda")
    mdn = ctx.spin_resolved_wilson(g.U, g.N, g.m, g.ldu, g.U.stride(0), g.n_sys, g.n_par, g.n_perp, mode, sd, pso,
                                   tdn, tup, cdn, cup, cs, st, precision)
    return {"mu": pso, "theta_dn": tdn, "theta_up": tup, "m_dn": mdn, "C_dn": cdn, "C_up": cup, "C_s": cs,
            "status": st}


def flux(ctx: L.Context, g: EigGrid):
    """Berry flux through every plaquette of the grid: flux (n_sys, n_perp, n_par)."""
    torch = _torch()
    f = torch.empty((g.n_sys, g.n_perp, g.n_par), dtype=torch.float64, device="cuda")
    ch = torch.empty(g.n_sys, dtype=torch.int32, device="cuda")
    tot = torch.empty(g.n_sys, dtype=torch.float64, device="cuda")
    st = torch.empty(g.n_sys, dtype=torch.int32, device="cuda")
    ctx.plaquette_flux(g.U, g.N, g.m, g.ldu, g.U.stride(0), g.n_sys, g.n_par, g.n_perp, f, ch, tot, st)
    return {"flux": f, "chern": ch, "total": tot, "status": st}


def spin_flux(ctx: L.Context, g: EigGrid, spin_diag, precision: int = L.BE_FP64):
    """Berry flux maps of the spin-down and spin-up sectors of the occupied
    space; C_s = (C_up - C_dn)/2. spin_diag: (n_sys, N) float64."""
    torch = _torch()
    m = max(g.m, 1)
    n_k = g.n_perp * g.n_par
    sd = torch.as_tensor(np.asarray(spin_diag, dtype=np.float64).reshape(g.n_sys, g.N)).cuda()
    pso = torch.empty((g.n_sys, g.n_perp, g.n_par, m), dtype=torch.float64, device="cuda")
    V = torch.empty((g.n_sys * n_k, m, g.N), dtype=torch.complex128, device="cuda")
    st = torch.empty(g.n_sys, dtype=torch.int32, device="cuda")
    mdn = ctx.spin_sectors(g.U, g.N, g.m, g.ldu, g.U.stride(0), g.n_sys, n_k, sd, pso, V, g.N, V.stride(0), st,
                           precision)
    out = {"mu": pso, "m_dn": mdn, "status_pso": st}
    f = {k: torch.zeros((g.n_sys, g.n_perp, g.n_par), dtype=torch.float64, device="cuda") for k in ("dn", "up")}
    ch = {k: torch.zeros(g.n_sys, dtype=torch.int32, device="cuda") for k in ("dn", "up")}
    tot = {k: torch.zeros(g.n_sys, dtype=torch.float64, device="cuda") for k in ("dn", "up")}
    sst = {k: torch.zeros(g.n_sys, dtype=torch.int32, device="cuda") for k in ("dn", "up")}
    s0 = 0
    while s0 < g.n_sys:  # runs of systems with equal sector sizes
        s1 = s0 + 1
        while s1 < g.n_sys and mdn[s1] == mdn[s0]:
            s1 += 1
        for key, c0, ms in (("dn", 0, mdn[s0]), ("up", mdn[s0], g.m - mdn[s0])):
            ctx.plaquette_flux(V[s0 * n_k:, c0 if ms > 0 else 0:, :], g.N, ms, g.N, V.stride(0), s1 - s0, g.n_par, g.n_perp,
                               f[key][s0:], ch[key][s0:], tot[key][s0:], sst[key][s0:])
        s0 = s1
    out.update({"flux_dn": f["dn"], "flux_up": f["up"], "C_dn": ch["dn"], "C_up": ch["up"],
                "total_dn": tot["dn"], "total_up": tot["up"],
                "C_s": 0.5 * (ch["up"] - ch["dn"]).to(torch.float64),
                "status": st | sst["dn"] | sst["up"]})
    return out


def wsurf(ctx, hoplists: Sequence, kappa_grid, lo, hi, mode=L.BE_OVL_POLAR, precision=L.BE_FP64):
    """Hybrid WCCs over a plane for systems of equal N (paper's WSurf)."""
    plan = ctx.hk_plan(list(hoplists))
    g = eig_grid(ctx, plan, 0, len(hoplists), kappa_grid, lo, hi, precision)
    out = wilson(ctx, g, mode)
    out["eig"] = g
    return out


def wnwl(ctx, hoplists: Sequence, kappa_grid, lo, hi, window=(0.0, 0.5), mode=L.BE_OVL_POLAR, precision=L.BE_FP64):
    """Nested Wilson loop over a plane (paper's WNWL)."""
    plan = ctx.hk_plan(list(hoplists))
    g = eig_grid(ctx, plan, 0, len(hoplists), kappa_grid, lo, hi, precision)
    out = nested(ctx, g, window, mode)
    out["eig"] = g
    return out


def wspinsurf(ctx, hoplists: Sequence, spin_diag, kappa_grid, lo, hi, mode=L.BE_OVL_POLAR, precision=L.BE_FP64,
              chunk: int = 4096):
    """Spin-resolved WCCs over a plane (paper's WSpinSurf)."""
    plan = ctx.hk_plan(list(hoplists))
    g = eig_grid(ctx, plan, 0, len(hoplists), kappa_grid, lo, hi, precision, chunk)
    out = spin(ctx, g, spin_diag, mode, precision)
    out["eig"] = g
    return out


def wflux(ctx, hoplists: Sequence, kappa_grid, lo, hi, precision=L.BE_FP64):
    """Berry flux per plaquette of the bands [lo, hi) over a plane."""
    plan = ctx.hk_plan(list(hoplists))
    g = eig_grid(ctx, plan, 0, len(hoplists), kappa_grid, lo, hi, precision)
    out = flux(ctx, g)
    out["eig"] = g
    return out


def wspinflux(ctx, hoplists: Sequence, spin_diag, kappa_grid, lo, hi, precision=L.BE_FP64, chunk: int = 4096):
    """Spin-resolved Berry flux per plaquette (the spin-resolved coupling-matrix
    method of Sec. IV): flux maps and Chern numbers of both spin sectors."""
    plan = ctx.hk_plan(list(hoplists))
    g = eig_grid(ctx, plan, 0, len(hoplists), kappa_grid, lo, hi, precision, chunk)
    out = spin_flux(ctx, g, spin_diag, precision)
    out["eig"] = g
    return out


def eig_planes(ctx: L.Context, hoplist, kappa_planes: np.ndarray, lo: int, hi: int, precision: int = L.BE_FP64,
               chunk: int = 4096) -> EigGrid:
    """Selected eigenvectors on n_planes k-planes of one model
    (kappa_planes: (n_planes, n_perp, n_par, 3)) in one batch. The planes are
    diagonalized as one grid of n_planes * n_perp lines; since a U-grid stores
    matrix (s, i, j) at ((s n_perp + i) n_par + j), the result is returned as a
    grid of n_planes systems, one per plane, for any of the loop calls."""
    kp = np.asarray(kappa_planes, dtype=np.float64)
    n_planes, n_perp, n_par = kp.shape[:3]
    plan = ctx.hk_plan([hoplist])
    g = eig_grid(ctx, plan, 0, 1, kp.reshape(n_planes * n_perp, n_par, 3), lo, hi, precision, chunk)
    return EigGrid(g.U, g.evals, g.status, g.N, g.m, g.ldu, n_planes, n_par, n_perp)


def wnwl_planes(ctx, hoplist, kappa_planes, lo, hi, window=(0.0, 0.5), mode=L.BE_OVL_POLAR,
                precision=L.BE_FP64):
    """Nested Wilson loop on every plane of a family (paper's WNWL in a loop
    over kz): nested phases, p and p_mean per plane."""
    g = eig_planes(ctx, hoplist, kappa_planes, lo, hi, precision)
    out = nested(ctx, g, window, mode)
    out["eig"] = g
    return out
