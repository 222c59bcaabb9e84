#!/usr/bin/env python3
"""Benchmark of the Wilson-loop hot path on one MI355X.

Workload: BHZ model (eq. 7) on a 10 x 10 supercell (N = 400 orbitals) with
on-site Anderson disorder W in {0, 1, 2, 3}, 16 seeded realizations each
(64 systems), a 24 x 24 supercell k-grid, half filling (m = 200), and the
spin-resolved Wilson loop with S_z = diag(1, -1, -1, 1) per site. One step is
the whole hot path for all 64 systems: Bloch Hamiltonians, batched
eigensolver, projected spin operator and its eigensolver, sector overlaps,
polar factors, ordered products, eigenphases and windings. Inputs (packed
hopping lists, k-points) are resident on the device before timing starts.

Metric: Wilson-loop k-point solves per second (k-points of the grid taken
through the whole path per second of wall time).

Prints one JSON line. Also reports the dominant kernel's roofline (its
duration measured with HIP events recorded by the library around each of its
launches during the timed steps) and the FP64 CPU oracle's rate on a bounded
sample of the same workload (a baseline, not the target).
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synthetic as syn  # noqa: E402

METRIC = "Wilson-loop k-point solves/s at ≤1e-6 phase err vs FP64; p50/p99 latency"
METRIC_FLUX = "Berry-flux (plaquette) k-point solves/s at ≤1e-6 flux err vs FP64; p50/p99 latency"
L_SC, N_PAR, N_PERP = 10, 24, 24
W_VALUES = (0.0, 1.0, 2.0, 3.0)
REALIZATIONS = 16
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
NB = 32  # panel width of the Householder reduction


def systems():
    hls, tags = [], []
    for w_idx, W in enumerate(W_VALUES):
        for r in range(REALIZATIONS):
            hls.append(syn.bhz_disordered(L_SC, W, [3, w_idx, r]))
            tags.append((w_idx, r))
    return hls, tags


# ---------------------------------------------------------------- CPU oracle leg
def _oracle_line(args):
    """Spin-resolved Wilson loop of one transverse line with the FP64 oracle."""
    w_idx, r, i = args
    from oracle import berry as orc
    hl = syn.bhz_disordered(L_SC, W_VALUES[w_idx], [3, w_idx, r])
    kg = syn.kplane(N_PAR, N_PERP)
    m = hl.N // 2
    sd = syn.bhz_spin_diag(hl)
    ev, U, st = orc.eigh_grid(hl, kg[i], 0, m)
    vm, vp = [], []
    for j in range(N_PAR):
        mu, a, b = orc.spin_sectors(U[j], sd)
        vm.append(a)
        vp.append(b)
    out = []
    for V in (vm, vp):
        if min(x.shape[1] for x in V) != max(x.shape[1] for x in V):
            out.append(None)
            continue
        W, _ = orc.wilson_matrix(np.stack(V))
        out.append(orc.eigphases(W))
    return (w_idx, r, i, out[0], out[1])


def _oracle_strip(args):
    """Spin-resolved Berry flux of one row of plaquettes (k-point rows i and
    i + 1, all j) with the FP64 oracle: row 0 of the 2-row grid's maps."""
    w_idx, r, i = args
    from oracle import berry as orc
    hl = syn.bhz_disordered(L_SC, W_VALUES[w_idx], [3, w_idx, r])
    kg = syn.kplane(N_PAR, N_PERP)
    out = orc.spin_resolved_flux(hl, syn.bhz_spin_diag(hl), kg[[i, (i + 1) % N_PERP]], 0, hl.N // 2)
    if out["status"] & orc.PSO_GAP:
        return (w_idx, r, i, None, None)
    return (w_idx, r, i, out["flux_dn"][0], out["flux_up"][0])


def cpu_baseline(sample, workers, fn=_oracle_line):
    ctx = mp.get_context("spawn")
    old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        with ctx.Pool(workers) as pool:
            pool.map(fn, sample[:workers])  # warm the workers (imports)
            t0 = time.perf_counter()
            res = pool.map(fn, sample)
            dt = time.perf_counter() - t0
    finally:
        if old is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = old
        os.environ.pop("OPENBLAS_NUM_THREADS", None)
    return res, dt


# ---------------------------------------------------------------- algorithmic work
def hetrd_panel_bytes(N, n_mat, elem_bytes=16):
    """Algorithmic HBM bytes of all panel launches of one eigensolver call: the
    Hermitian matrix-vector product of each reflector column reads one
    triangle (diagonal included) of the trailing matrix, 16 B per c128
    element, 8 B per c64: sum_j e (N-j-1)(N-j)/2, about e N^3/6 per matrix."""
    return n_mat * sum(elem_bytes * (N - j - 1) * (N - j) // 2 for j in range(N - 1))


def eigh_gemm_flops(name, N, m, n_mat):
    """Algorithmic flops (8 per complex multiply-add) of the eigensolver's GEMMs."""
    P = (N + NB - 1) // NB
    if name == "her2k":   # Hermitian rank-2nb update, one triangle
        return n_mat * sum(8.0 * (N - p * NB - NB) ** 2 * NB for p in range(P) if N - p * NB - NB > 0)
    if name == "unmtr":   # X = V^H U, Y = T X (T triangular), U -= V Y
        tot = 0.0
        for p in range(P):
            p0 = p * NB
            nbp, K = min(NB, N - p0), N - p0 - 1
            if K > 0:
                tot += 16.0 * K * nbp * m + 4.0 * nbp * nbp * m
        return n_mat * tot
    raise KeyError(name)


def gemm_phase_flops(N, m, n_par, n_k_sys, m_dn):
    """Algorithmic GEMM flops per call-site tag for one pass over the systems
    (spin-resolved loop). m_dn: spin-down sector size per system."""
    nk = n_k_sys * len(m_dn)
    md = np.asarray(m_dn, dtype=np.float64)
    mu = m - md
    return {
        "her2k": eigh_gemm_flops("her2k", N, m, nk),
        "unmtr": eigh_gemm_flops("unmtr", N, m, nk),
        "pso": 4.0 * m * (m + 1) * N * nk,                 # U^H (S U), one triangle (Hermitian)
        "pso_her2k": eigh_gemm_flops("her2k", m, m, nk),   # eigensolver of P S P (order m, all bands)
        "pso_unmtr": eigh_gemm_flops("unmtr", m, m, nk),
        "spin_sector": 8.0 * N * m * m * nk,               # U [Q- Q+]
        "overlap": float(np.sum(8.0 * N * (md ** 2 + mu ** 2))) * n_k_sys,
        "chain": float(np.sum(8.0 * (md ** 3 + mu ** 3))) * (n_par - 1) / n_par * n_k_sys,
        "flux_links": 2.0 * float(np.sum(8.0 * N * (md ** 2 + mu ** 2))) * n_k_sys,   # both directions
    }


def det_phase_flops(m_dn, m, n_k_sys):
    """Algorithmic flops of the link determinants (LU, 8 flops per complex
    multiply-add, sum over k of (ms - k - 1)^2 updates): both sectors, both
    directions."""
    tot = 0.0
    for md in m_dn:
        for ms in (md, m - md):
            tot += 8.0 * sum((ms - k - 1) ** 2 for k in range(ms))
    return 2.0 * n_k_sys * tot


PANEL_SRC_BEGIN = "// ---------------------------------------------------------------- reductions"
PANEL_SRC_END = "// ---------------------------------------------------------------- tridiagonal solver"


def panel_source_digest(source):
    """sha256 of the panel kernel's section of the eigensolver source (its
    reductions and the kernel itself)."""
    import hashlib
    text = open(source).read()
    a, b = text.index(PANEL_SRC_BEGIN), text.index(PANEL_SRC_END)
    return hashlib.sha256(text[a:b].encode()).hexdigest()


def traffic_from_profile(path, source, precision):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3
    counter summary, if it was taken with the current kernel source."""
    try:
        text = open(path).read()
        sha = panel_source_digest(source)
    except (OSError, ValueError):
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("<!-- ") and ":" in line:
            k, v = line[5:].rstrip(" ->").split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != sha or vals.get("precision") != precision:
        return None
    return float(vals["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["spin_wilson", "spin_flux", "bbh_disorder", "choti_nested"],
                    default="spin_wilson",
                    help="spin_wilson: spin-resolved Wilson loops (the headline metric); spin_flux: spin-resolved "
                         "Berry flux per plaquette (coupling-matrix method) on the same systems and grid; "
                         "bbh_disorder: the disordered quadrupolar-insulator study (spinful BBH, 21x21 supercell, "
                         "20x20 plaquettes, W = 1 and 9); choti_nested: nested Wilson loop of the chiral HOTI on "
                         "21 kz planes of 100x100")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chunk-systems", type=int, default=8)
    ap.add_argument("--cpu-lines", type=int, default=32, help="oracle sample size (transverse lines)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="eigensolver precision (mixed: FP32 reduction/back-transformation, FP64 elsewhere; "
                         "its phases are checked against the FP64 oracle at 1e-6 rad). Default: mixed, except "
                         "fp64 for bbh_disorder (N = 1764, m = 882: the c64 Hamiltonian alone puts the summed "
                         "phases of 882 bands near 1e-6 rad)")
    ap.add_argument("--systems", type=int, default=0, help="profile a subset: first N systems only (0 = all 64)")
    ap.add_argument("--tune", action="append", default=[], metavar="KNOB=VALUE",
                    help="set a library tuning knob (be_tune_set) before timing")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run one plain device copy of this size (calibrates rocprof byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: berryhip has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.precision is None:
        args.precision = "fp64" if args.workload == "bbh_disorder" else "mixed"
    if args.workload in ("bbh_disorder", "choti_nested"):
        return main_study(args)

    hls, tags = systems()
    if args.systems:
        hls, tags = hls[:args.systems], tags[:args.systems]
    n_sys = len(hls)
    N = hls[0].N
    m = N // 2
    kg = syn.kplane(N_PAR, N_PERP)
    n_k = N_PAR * N_PERP

    # ---- CPU oracle on a bounded sample (before the GPU is touched)
    sample = []
    rng = np.random.default_rng([9, 9])
    for w_idx in range(len(W_VALUES)):
        for r in rng.choice(REALIZATIONS, size=2, replace=False):
            for i in rng.choice(N_PERP, size=max(1, args.cpu_lines // 8), replace=False):
                sample.append((w_idx, int(r), int(i)))
    flux_wl = args.workload == "spin_flux"
    if flux_wl:
        sample = sample[:max(1, len(sample) // 2)]
    cpu = None
    oracle_res = []
    if not args.no_cpu_baseline:
        workers = max(1, min(16, os.cpu_count() or 1, len(sample)))
        if flux_wl:
            oracle_res, cdt = cpu_baseline(sample, workers, _oracle_strip)
            cpu = {"value": len(sample) * N_PAR / cdt, "unit": "k-point solves/s", "cores": workers,
                   "kind": "oracle",
                   "sample": f"{len(sample)} rows of plaquettes ({len(sample) * N_PAR} plaquettes, "
                             f"{2 * len(sample) * N_PAR} eigensolves) of the same workload, NumPy/LAPACK FP64, "
                             f"one worker process per core, OMP_NUM_THREADS=1, wall {cdt:.2f} s"}
        else:
            oracle_res, cdt = cpu_baseline(sample, workers)
            cpu = {"value": len(sample) * N_PAR / cdt, "unit": "k-point solves/s", "cores": workers,
                   "kind": "oracle",
                   "sample": f"{len(sample)} transverse lines ({len(sample) * N_PAR} k-points) of the same "
                             f"workload, NumPy/LAPACK FP64, one worker process per core, OMP_NUM_THREADS=1, "
                             f"wall {cdt:.2f} s"}

    import torch
    from paper_2312_13051_amd import _lib as L
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    if args.copy_calibration_mb:
        nb = args.copy_calibration_mb << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = L.Context(0)
    tuning = {}
    for kv in args.tune:
        k, v = kv.split("=")
        ctx.tune_set(k, int(v))
        tuning[k] = int(v)
    plan = ctx.hk_plan(hls)
    kap = torch.from_numpy(np.ascontiguousarray(kg.reshape(-1, 3))).to(dev)
    spin = torch.from_numpy(np.stack([syn.bhz_spin_diag(h) for h in hls])).to(dev)
    cs = args.chunk_systems
    nmat = cs * n_k
    mixed = args.precision == "mixed"
    hdt, hcode = (torch.complex64, L.BE_C64) if mixed else (torch.complex128, L.BE_C128)
    prec = L.BE_MIXED_FP32 if mixed else L.BE_FP64
    H = torch.empty((nmat, N, N), dtype=hdt, device=dev)
    U = torch.empty((nmat, m, N), dtype=torch.complex128, device=dev)
    ev = torch.empty((nmat, m + 2), dtype=torch.float64, device=dev)
    est = torch.empty(nmat, dtype=torch.int32, device=dev)
    pso = torch.empty((n_sys, N_PERP, N_PAR, m), dtype=torch.float64, device=dev)
    tdn = torch.empty((n_sys, N_PERP, m), dtype=torch.float64, device=dev)
    tup = torch.empty((n_sys, N_PERP, m), dtype=torch.float64, device=dev)
    cdn = torch.empty(n_sys, dtype=torch.int32, device=dev)
    cup = torch.empty(n_sys, dtype=torch.int32, device=dev)
    csp = torch.empty(n_sys, dtype=torch.float64, device=dev)
    sst = torch.empty(n_sys, dtype=torch.int32, device=dev)
    eig_bad = torch.zeros(n_sys, dtype=torch.int32, device=dev)
    if flux_wl:
        V = torch.empty((nmat, m, N), dtype=torch.complex128, device=dev)
        fdn = torch.empty((n_sys, N_PERP, N_PAR), dtype=torch.float64, device=dev)
        fup = torch.empty((n_sys, N_PERP, N_PAR), dtype=torch.float64, device=dev)
        ftot = torch.empty((2, n_sys), dtype=torch.float64, device=dev)
        fst = torch.empty((3, n_sys), dtype=torch.int32, device=dev)
    mdn_all = [0] * n_sys
    chunk_lat = []

    def step(record=False):
        for s0 in range(0, n_sys, cs):
            ns = min(cs, n_sys - s0)
            t0 = time.perf_counter()
            ctx.build_hk(plan, s0, ns, kap, H, N * N, N, hcode)
            ctx.eigh_batched(H, hcode, N, N, N * N, ns * n_k, 0, m, prec, ev, U, N, U.stride(0), est)
            eig_bad[s0:s0 + ns] = est[:ns * n_k].view(ns, n_k).ne(0).any(dim=1).to(torch.int32)
            if flux_wl:
                md = ctx.spin_sectors(U, N, m, N, U.stride(0), ns, n_k, spin[s0:], pso[s0:], V, N, V.stride(0),
                                      fst[0, s0:], prec)
                a = 0
                while a < ns:  # runs of systems with equal sector sizes
                    b = a + 1
                    while b < ns and md[b] == md[a]:
                        b += 1
                    ctx.plaquette_flux(V[a * n_k:], N, md[a], N, V.stride(0), b - a, N_PAR, N_PERP,
                                       fdn[s0 + a:], cdn[s0 + a:], ftot[0, s0 + a:], fst[1, s0 + a:])
                    ctx.plaquette_flux(V[a * n_k:, md[a] if md[a] < m else 0:], N, m - md[a], N, V.stride(0),
                                       b - a, N_PAR, N_PERP, fup[s0 + a:], cup[s0 + a:], ftot[1, s0 + a:],
                                       fst[2, s0 + a:])
                    a = b
            else:
                md = ctx.spin_resolved_wilson(U, N, m, N, U.stride(0), ns, N_PAR, N_PERP, L.BE_OVL_POLAR,
                                              spin[s0:], pso[s0:], tdn[s0:], tup[s0:], cdn[s0:], cup[s0:], csp[s0:],
                                              sst[s0:], prec)
            mdn_all[s0:s0 + ns] = md
            if record:
                torch.cuda.synchronize()
                chunk_lat.append(time.perf_counter() - t0)

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        note(f"warmup step {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        note(f"timed step {k + 1}/{args.steps} issued")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    note(f"timed region {t1 - t0:.2f} s")
    prof = ctx.profile()
    ctx.profile_enable(False)
    step(record=True)  # latency of each chunk (systems finish together per chunk)
    torch.cuda.synchronize()

    total_k = n_sys * n_k
    sec = (t1 - t0) / args.steps
    value = total_k / sec

    # ---- dominant kernel and its roofline
    steps = args.steps
    dom = max(prof.items(), key=lambda kv: kv[1][0])
    name, (ms_tot, launches) = dom
    roof = {"kernel": name, "bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
            "traffic": None, "avg_launch_ms": round(ms_tot / launches, 4), "launches": launches}
    flops = gemm_phase_flops(N, m, N_PAR, n_k, mdn_all)
    fp32_tags = ("her2k", "unmtr", "pso_her2k", "pso_unmtr") if mixed else ()
    if name == "hetrd_panel":
        elem = 8 if mixed else 16
        byts = hetrd_panel_bytes(N, total_k, elem) * steps
        ach = byts / (ms_tot * 1e-3) / 1e9
        traffic = traffic_from_profile(os.path.join(ROOT, "profiles", f"hetrd_panel_bhz400_{args.precision}.md"),
                                       os.path.join(ROOT, "paper_2312_13051_amd", "csrc", "eigh.hip"), args.precision)
        roof.update({"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": round(byts / launches, 1)})
    elif name == "det_phase":
        fl = det_phase_flops(mdn_all, m, n_k) * steps
        ach = fl / (ms_tot * 1e-3) / 1e12
        roof.update({"bound": "alu", "achieved": round(ach, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ach / FP64_PEAK_TFLOPS, 4)})
    elif name in flops:
        pk = FP32_PEAK_TFLOPS if name in fp32_tags else FP64_PEAK_TFLOPS
        ach = flops[name] * steps / (ms_tot * 1e-3) / 1e12
        roof.update({"bound": "mfma", "achieved": round(ach, 2), "peak": pk, "unit": "TFLOP/s",
                     "frac": round(ach / pk, 4)})
    kernels = {k: {"ms_per_step": round(v[0] / steps, 2), "launches_per_step": v[1] // steps} for k, v in
               sorted(prof.items(), key=lambda kv: -kv[1][0])}
    # GEMM phases against the MFMA peak of their arithmetic type
    gemm = {}
    w_sum = t_sum = 0.0
    for tag, fl in flops.items():
        if tag not in prof:
            continue
        t = prof[tag][0] / steps * 1e-3
        pk = FP32_PEAK_TFLOPS if tag in fp32_tags else FP64_PEAK_TFLOPS
        gemm[tag] = {"tflops": round(fl / t / 1e12, 2), "peak": pk, "frac": round(fl / t / 1e12 / pk, 4)}
        w_sum += fl / (pk * 1e12)
        t_sum += t
    gemm_phases = {"per_tag": gemm, "frac_of_mfma_peak": round(w_sum / t_sum, 4) if t_sum else None,
                   "note": "algorithmic flops (one triangle for her2k and pso, 8 per complex multiply-add); "
                           "FP64 extras (polar, reorth) are timed but not counted"}

    # ---- phase error of the sampled lines against the FP64 oracle
    max_err = None
    gate_compared = gate_skipped = sector_mismatch = 0
    if oracle_res and flux_wl:
        fdn_h, fup_h = fdn.cpu().numpy(), fup.cpu().numpy()
        errs = []
        for (w_idx, r, i, a, b) in oracle_res:
            if a is None:
                continue
            s = w_idx * REALIZATIONS + r
            for g, ref in ((fdn_h[s, i], a), (fup_h[s, i], b)):
                errs.append(float(np.max(np.abs(np.mod(g - ref + np.pi, 2 * np.pi) - np.pi))))
        max_err = float(max(errs)) if errs else None
        gate_compared = len(errs)
        gate_skipped = sum(1 for x in oracle_res if x[3] is None)
    elif oracle_res:
        from tests.phase_metrics import phase_set_error
        tdn_h, tup_h = tdn.cpu().numpy(), tup.cpu().numpy()
        errs = []
        for (w_idx, r, i, a, b) in oracle_res:
            s = w_idx * REALIZATIONS + r
            md = mdn_all[s]
            for ref, got in ((a, tdn_h[s, i, :md]), (b, tup_h[s, i, :m - md])):
                if ref is None:        # the oracle's spin-sector size varies along the line
                    gate_skipped += 1
                elif ref.size != got.size:
                    sector_mismatch += 1
                else:
                    errs.append(phase_set_error(got, ref))
        max_err = float(max(errs)) if errs else None
        gate_compared = len(errs)

    if flux_wl:
        csp.copy_(0.5 * (cup - cdn).to(torch.float64))
        sst.copy_(fst[0] | fst[1] | fst[2])
    st = sst.cpu().numpy() | eig_bad.cpu().numpy()
    lat = np.array(chunk_lat) * 1e3
    out = {
        "metric": METRIC if not flux_wl else METRIC_FLUX,
        "value": round(value, 1),
        "unit": "k-point solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": "BHZ 10x10 supercell (N=400) with Anderson disorder W in {0,1,2,3} x 16 seeded "
                               "realizations, 24x24 supercell k-grid, half filling, " +
                               ("spin-resolved Berry flux per plaquette (coupling-matrix method, eig of P S_z P, "
                                "link determinants in both directions), " if flux_wl else
                                "spin-resolved Wilson loop (eig of P S_z P), ") + ("mixed path: FP32 Householder reduction and "
                               "back-transformation on MFMA, FP64 elsewhere" if mixed else "FP64 path"),
                   "systems": n_sys, "k_points": total_k, "N": N, "m": m, "chunk_systems": cs, "tuning": tuning},
        "roofline": roof,
        "gemm_phases": gemm_phases,
        "cpu_baseline": cpu,
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2), "p99": round(float(np.percentile(lat, 99)), 2),
                       "unit": f"per chunk of {cs} systems ({cs * n_k} k-points)"},
        ("flux_err_vs_fp64_oracle_rad" if flux_wl else "phase_err_vs_fp64_oracle_rad"): max_err,
        "phase_gate_1e-6_ok": (False if sector_mismatch else None if max_err is None else bool(max_err <= 1e-6)),
        "gate_lines": {"compared": gate_compared, "skipped_oracle_pso_gap": gate_skipped,
                       "sector_size_mismatch": sector_mismatch},
        "valid_systems": int((st == 0).sum()),
        "spin_chern_W0": [float(x) for x in csp.cpu().numpy()[:REALIZATIONS]][:4],
        "kernels": kernels,
    }
    print(json.dumps(out))


# ---------------------------------------------------------------- paper studies (secondary workloads)
BBH_L, BBH_GRID, BBH_W = 21, 20, (1.0, 9.0)
CHOTI_PLANES, CHOTI_GRID = 21, 100


def _oracle_bbh_corner(args):
    """Spin-resolved flux of one plaquette of the 21 x 21 spinful-BBH study
    with the FP64 oracle (its 2 x 2 corner grid: four eigensolves)."""
    w_idx, i, j = args
    from oracle import berry as orc
    hl = syn.spinful_bbh_disordered(BBH_L, BBH_W[w_idx], [7, w_idx])
    kg = syn.kplane(BBH_GRID, BBH_GRID)
    sub = kg[[i, (i + 1) % BBH_GRID]][:, [j, (j + 1) % BBH_GRID]]
    out = orc.spin_resolved_flux(hl, syn.spinful_bbh_spin_diag(hl), sub, 0, hl.N // 2)
    if out["status"] & orc.PSO_GAP:
        return (w_idx, i, j, None, None)
    return (w_idx, i, j, float(out["flux_dn"][0, 0]), float(out["flux_up"][0, 0]))


def _oracle_choti_plane(q):
    """Nested Wilson loop of one kz plane of the chiral-HOTI study with the FP64 oracle."""
    from oracle import berry as orc
    kz = np.linspace(0.0, 1.0, CHOTI_PLANES)[q]
    out = orc.nested_wilson(syn.choti(1.0), syn.kplane(CHOTI_GRID, CHOTI_GRID, k0=(0.0, 0.0, kz)), 0, 2)
    return (q, out["p"])


def main_study(args):
    """The disordered quadrupolar-insulator study (Sec. IV) or the chiral-HOTI
    nested loop against kz (Sec. III), timed like the headline workload."""
    bbh = args.workload == "bbh_disorder"
    workers = max(1, min(16, os.cpu_count() or 1))
    cpu, oracle_res = None, []
    if bbh:
        sample = [(w, int(i), int(j)) for w in range(2) for (i, j) in
                  np.random.default_rng([9, 10 + w]).integers(0, BBH_GRID, size=(max(1, workers // 2), 2))]
        fn, per = _oracle_bbh_corner, 4
        what = "plaquettes (each its 2x2 corner grid: 4 eigensolves of N=1764 and their PSO eigensolves)"
    else:
        sample = list(range(0, CHOTI_PLANES, max(1, CHOTI_PLANES // max(1, min(workers, 4)))))[:max(1, min(workers, 4))]
        fn, per = _oracle_choti_plane, CHOTI_GRID * CHOTI_GRID
        what = f"kz planes of {CHOTI_GRID}x{CHOTI_GRID} k-points (nested Wilson loop of each)"
    if not args.no_cpu_baseline:
        oracle_res, cdt = cpu_baseline(sample, min(workers, len(sample)), fn)
        cpu = {"value": len(sample) * per / cdt, "unit": "k-point solves/s", "cores": min(workers, len(sample)),
               "kind": "oracle", "sample": f"{len(sample)} {what}, NumPy/LAPACK FP64, one worker process per core, "
                                           f"OMP_NUM_THREADS=1, wall {cdt:.2f} s"}

    import torch
    from paper_2312_13051_amd import _lib as L
    from paper_2312_13051_amd import pipeline as PL
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    ctx = L.Context(0)
    mixed = args.precision == "mixed"
    prec = L.BE_MIXED_FP32 if mixed else L.BE_FP64
    if bbh:
        hls = [syn.spinful_bbh_disordered(BBH_L, W, [7, w]) for w, W in enumerate(BBH_W)]
        plan = ctx.hk_plan(hls)
        kg = syn.kplane(BBH_GRID, BBH_GRID)
        n_k = BBH_GRID * BBH_GRID
        N = hls[0].N
        m = N // 2
        sd = np.stack([syn.spinful_bbh_spin_diag(h) for h in hls])
        res = {}

        def step():
            for s in range(len(hls)):  # one supercell per eigensolver call
                g = PL.eig_grid(ctx, plan, s, 1, kg, 0, m, prec, chunk=n_k)
                res[s] = (g, PL.spin_flux(ctx, g, sd[s:s + 1], prec))
        total_k = len(hls) * n_k
    else:
        hl = syn.choti(1.0)
        kzs = np.linspace(0.0, 1.0, CHOTI_PLANES)
        kp = np.stack([syn.kplane(CHOTI_GRID, CHOTI_GRID, k0=(0.0, 0.0, kz)) for kz in kzs])
        N, m = hl.N, 2
        res = {}

        def step():
            g = PL.eig_planes(ctx, hl, kp, 0, m, prec, chunk=kp.shape[0] * CHOTI_GRID * CHOTI_GRID)
            res[0] = (g, PL.nested(ctx, g))
        total_k = CHOTI_PLANES * CHOTI_GRID * CHOTI_GRID

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        note(f"warmup step {w + 1}/{args.warmup} done")
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        note(f"timed step {k + 1}/{args.steps} issued")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile()
    ctx.profile_enable(False)
    lat = []
    for _ in range(2):
        a = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    sec = (t1 - t0) / args.steps
    steps = args.steps
    name, (ms_tot, launches) = max(prof.items(), key=lambda kv: kv[1][0])
    roof = {"kernel": name, "bound": "latency", "achieved": None, "peak": None, "unit": None, "frac": None,
            "traffic": None, "avg_launch_ms": round(ms_tot / launches, 4), "launches": launches}
    n_mat = total_k * steps
    if name == "hetrd_panel":
        byts = hetrd_panel_bytes(N, n_mat, 8 if mixed else 16)
        ach = byts / (ms_tot * 1e-3) / 1e9
        roof.update({"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": round(byts / launches, 1)})
    elif name in ("her2k", "unmtr"):
        fl = eigh_gemm_flops(name, N, m, n_mat)
        pk = FP32_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS
        ach = fl / (ms_tot * 1e-3) / 1e12
        roof.update({"bound": "mfma", "achieved": round(ach, 2), "peak": pk, "unit": "TFLOP/s",
                     "frac": round(ach / pk, 4)})
    kernels = {k: {"ms_per_step": round(v[0] / steps, 2), "launches_per_step": v[1] // steps} for k, v in
               sorted(prof.items(), key=lambda kv: -kv[1][0])}
    err = None
    extra = {}
    if bbh:
        errs = []
        for (w, i, j, a, b) in oracle_res:
            if a is None:
                continue
            f = res[w][1]
            errs.append(float(circ_dist(float(f["flux_dn"][0, i, j]), a)))
            errs.append(float(circ_dist(float(f["flux_up"][0, i, j]), b)))
        err = max(errs) if errs else None
        extra = {"spin_chern": {f"W={W}": float(res[w][1]["C_s"][0]) for w, W in enumerate(BBH_W)},
                 "status": {f"W={W}": int(res[w][1]["status"][0]) for w, W in enumerate(BBH_W)}}
        metric, cfg = METRIC_FLUX, {"workload": "spinful BBH (eq. 10) 21x21 supercell (N=1764, m=882) with chiral "
                                                "disorder w s0(x)t3, W in {1, 9}, one realization each, 20x20 "
                                                "plaquettes, spin-resolved Berry flux (s = s0(x)t3)",
                                    "systems": len(BBH_W), "k_points": total_k, "N": N, "m": m}
    else:
        p = res[0][1]["p"].cpu().numpy()
        errs = [float(np.max(circ_dist(2 * np.pi * p[q], 2 * np.pi * ref))) for (q, ref) in oracle_res]
        err = max(errs) if errs else None
        pm = res[0][1]["p_mean"].cpu().numpy()
        d = np.diff(np.r_[pm, pm[0]])
        d -= np.round(d)
        extra = {"nested_p_winding_vs_kz": round(float(d[:-1].sum()), 6)}
        metric, cfg = ("nested Wilson-loop k-point solves/s at ≤1e-6 phase err vs FP64",
                       {"workload": "chiral HOTI (eq. 9, Delta0 = 1), 21 kz planes in [0, 1] of 100x100 k-points, "
                                    "Wilson loop along kx, nested loop along ky", "planes": CHOTI_PLANES,
                        "k_points": total_k, "N": N, "m": m})
    out = {
        "metric": metric, "value": round(total_k / sec, 1), "unit": "k-point solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
        "config": cfg, "roofline": roof, "cpu_baseline": cpu,
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2), "p99": round(float(np.percentile(lat, 99)), 2),
                       "unit": "per step"},
        "err_vs_fp64_oracle_rad": err, "gate_1e-6_ok": None if err is None else bool(err <= 1e-6), **extra,
        "kernels": kernels,
    }
    print(json.dumps(out))


def circ_dist(a, b):
    return np.abs(np.mod(np.asarray(a) - np.asarray(b) + np.pi, 2 * np.pi) - np.pi)


if __name__ == "__main__":
    main()
