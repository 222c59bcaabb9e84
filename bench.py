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

PRECISION_TEXT = {
    "fp64": "FP64 path",
    "mixed": "mixed path: FP32 Householder reduction and back-transformation on MFMA, FP64 elsewhere",
    "refined": "refined mixed path: FP32 Householder reduction and back-transformation on MFMA for all bands, "
               "FP64 first-order correction of the occupied subspace from the other bands on MFMA, FP64 elsewhere",
    "bf16x": "split-bf16 mixed path: FP32 Householder panels, trailing updates and back-transformation as "
             "split-bf16 products on the bf16 matrix cores (three per real product, FP32 accumulation), FP64 "
             "elsewhere",
}
L_SC, N_PAR, N_PERP = 10, 24, 24
W_VALUES = (0.0, 1.0, 2.0, 3.0)
REALIZATIONS = 16
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 MFMA
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


def _warm_worker(_):
    """Imports of an oracle worker (timed outside the sample)."""
    from oracle import berry  # noqa: F401
    return 0


def cpu_baseline(sample, workers, fn=_oracle_line, warm_with_sample=True):
    ctx = mp.get_context("spawn")
    old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        with ctx.Pool(workers) as pool:
            if warm_with_sample:
                pool.map(fn, sample[:workers])  # warm the workers (imports, first calls)
            else:
                pool.map(_warm_worker, range(workers))
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


def served_gemm_flops(reqs, refined_code):
    """Algorithmic GEMM flops per call-site tag of a served stream of
    Wilson-loop requests (objects with N, m, n_k, kappa [n_perp, n_par, 3] and
    precision): the eigensolver's trailing updates and back-transformation
    (all N bands for the refined path, whose mixed pass diagonalizes the whole
    matrix), the overlaps U(k')^H U(k) and the ordered products."""
    out = {"her2k": 0.0, "unmtr": 0.0, "overlap": 0.0, "chain": 0.0}
    for r in reqs:
        me = r.N if r.precision == refined_code else r.m
        n_perp, n_par = r.kappa.shape[0], r.kappa.shape[1]
        out["her2k"] += eigh_gemm_flops("her2k", r.N, me, r.n_k)
        out["unmtr"] += eigh_gemm_flops("unmtr", r.N, me, r.n_k)
        out["overlap"] += 8.0 * r.N * r.m * r.m * r.n_k
        out["chain"] += 8.0 * float(r.m) ** 3 * (n_par - 1) * n_perp
    return out


def gemm_phase_summary(flops, prof_ms, fp32_tags, scale=1.0, bf16_tags=()):
    """Per tag: algorithmic flops over the timed milliseconds (prof_ms[tag],
    divided by scale), against the MFMA peak of the tag's arithmetic type; and
    the time-weighted fraction over all tags."""
    gemm = {}
    w_sum = t_sum = 0.0
    for tag, fl in flops.items():
        if tag not in prof_ms or fl <= 0:
            continue
        t = prof_ms[tag] / scale * 1e-3
        pk = BF16_PEAK_TFLOPS if tag in bf16_tags else FP32_PEAK_TFLOPS if tag in fp32_tags else FP64_PEAK_TFLOPS
        gemm[tag] = {"tflops": round(fl / t / 1e12, 2), "peak": pk, "frac": round(fl / t / 1e12 / pk, 4)}
        w_sum += fl / (pk * 1e12)
        t_sum += t
    return {"per_tag": gemm, "frac_of_mfma_peak": round(w_sum / t_sum, 4) if t_sum else None,
            "note": "algorithmic flops (one triangle for Hermitian outputs, 8 per complex multiply-add); FP64 "
                    "extras (polar, reorth) are timed but not counted"}


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
    ap.add_argument("--workload", choices=["served", "uneven", "spin_wilson", "spin_flux", "bbh_disorder",
                                           "choti_nested"],
                    default="served",
                    help="served: Poisson stream of Wilson-loop requests of mixed supercell sizes (BHZ L = 8..24 and "
                         "a 96-orbital model, 32x32 k-grids; the metric's own workload, with p50/p99 latency); "
                         "uneven: 64 vacancy supercells of five sizes, mixed and FP64 paths; "
                         "spin_wilson: spin-resolved Wilson loops of 64 disordered BHZ 10x10 supercells; spin_flux: spin-resolved "
                         "Berry flux per plaquette (coupling-matrix method) on the same systems and grid; "
                         "bbh_disorder: the disordered quadrupolar-insulator study (spinful BBH, 21x21 supercell, "
                         "20x20 plaquettes, W = 1 and 9); choti_nested: nested Wilson loop of the chiral HOTI on "
                         "21 kz planes of 100x100")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chunk-systems", type=int, default=8)
    ap.add_argument("--cpu-lines", type=int, default=32, help="oracle sample size (transverse lines)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "mixed", "refined", "bf16x"], default=None,
                    help="eigensolver precision (mixed: FP32 reduction/back-transformation, FP64 elsewhere; "
                         "refined: the mixed path for all bands, then an FP64 correction of the occupied "
                         "subspace; bf16x: the mixed path with split-bf16 products in the trailing updates and "
                         "the back-transformation, spin_wilson only; phases are checked against the FP64 oracle "
                         "at 1e-6 rad in every run). Default: mixed")
    ap.add_argument("--systems", type=int, default=0, help="profile a subset: first N systems only (0 = all 64)")
    ap.add_argument("--tune", action="append", default=[], metavar="KNOB=VALUE",
                    help="set a library tuning knob (be_tune_set) before timing")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run one plain device copy of this size (calibrates rocprof byte counters)")
    ap.add_argument("--requests", type=int, default=30, help="served: requests in the stream")
    ap.add_argument("--load", type=float, default=1.0,
                    help="served: arrival rate as a multiple of the one-request-at-a-time capacity")
    ap.add_argument("--lanes", type=int, default=2, help="served: GPU lanes (host threads with a stream each)")
    ap.add_argument("--hbm-gib", type=int, default=150, help="served: HBM budget of admitted requests (GiB)")
    ap.add_argument("--policy", choices=["fifo", "srpt"], default="srpt",
                    help="served: which admitted request's k-points go first (oldest, or least remaining work: "
                         "the default, measured to halve p50 latency at the same throughput)")
    ap.add_argument("--types", default=None, metavar="T1,T2",
                    help="served: only these request types (of bhz8, bhz12, bhz16, bhz24, w96), in the stream's order")
    ap.add_argument("--request-log", default=None, metavar="PATH",
                    help="served: append one JSON line per completed request of the stream to PATH")
    ap.add_argument("--graph-lanes", type=int, default=1,
                    help="uneven: lanes (context + stream) of the captured graph's size groups")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: berryhip has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.precision == "bf16x" and args.workload not in ("spin_wilson", "spin_flux"):
        raise SystemExit("--precision bf16x is measured on the spin_wilson and spin_flux workloads only")
    if args.workload == "uneven" and args.precision not in (None, "mixed"):
        print("[bench] the uneven workload times the mixed and the FP64 path on the same batch (value and "
              "fp64_value); --precision is not used", file=sys.stderr, flush=True)
    if args.precision is None:
        args.precision = "mixed"
    if args.workload in ("bbh_disorder", "choti_nested"):
        return main_study(args)
    if args.workload == "served":
        return main_served(args)
    if args.workload == "uneven":
        return main_uneven(args)

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
    copy_calibration(args.copy_calibration_mb)
    ctx = L.Context(0)
    tuning = {"table": ctx.tuning}
    for kv in args.tune:
        k, v = kv.split("=")
        ctx.tune_clear(k)  # one value for every order
        ctx.tune_set(k, int(v))
        tuning[k] = int(v)
    plan = ctx.hk_plan(hls)
    kap = torch.from_numpy(np.ascontiguousarray(kg.reshape(-1, 3))).to(dev)
    spin = torch.from_numpy(np.stack([syn.bhz_spin_diag(h) for h in hls])).to(dev)
    cs = args.chunk_systems
    nmat = cs * n_k
    # mixed: FP32 reduction and back-transformation; refined: the same for all
    # bands of an FP32 copy of the FP64 H, then the FP64 subspace correction
    mixed = args.precision in ("mixed", "refined", "bf16x")
    prec = {"fp64": L.BE_FP64, "mixed": L.BE_MIXED_FP32, "refined": L.BE_MIXED_FP32_REFINED,
            "bf16x": L.BE_MIXED_BF16X}[args.precision]
    hdt, hcode = (torch.complex64, L.BE_C64) if L.c64_input(prec) else (torch.complex128, L.BE_C128)
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
        pp = "mixed" if mixed else "fp64"  # the refined path runs the mixed path's panel kernel
        traffic = traffic_from_profile(os.path.join(ROOT, "profiles", f"hetrd_panel_bhz400_{pp}.md"),
                                       os.path.join(ROOT, "paper_2312_13051_amd", "csrc", "eigh.hip"), pp)
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
    bf16_tags = ("her2k", "unmtr", "pso_her2k", "pso_unmtr") if args.precision == "bf16x" else ()
    gemm_phases = gemm_phase_summary(flops, {k: v[0] for k, v in prof.items()}, fp32_tags, scale=steps,
                                     bf16_tags=bf16_tags)
    if bf16_tags:
        gemm_phases["note"] += ("; bf16x tags: FP32-equivalent flops against the dense bf16 peak (the split "
                                "takes three bf16 products per real product)")

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
        "dtype": ("bf16x3+f32+f64" if args.precision == "bf16x" else "f32+f64") if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": "BHZ 10x10 supercell (N=400) with Anderson disorder W in {0,1,2,3} x 16 seeded "
                               "realizations, 24x24 supercell k-grid, half filling, " +
                               ("spin-resolved Berry flux per plaquette (coupling-matrix method, eig of P S_z P, "
                                "link determinants in both directions), " if flux_wl else
                                "spin-resolved Wilson loop (eig of P S_z P), ") + PRECISION_TEXT[args.precision],
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
    mixed = args.precision in ("mixed", "refined")
    prec = {"fp64": L.BE_FP64, "mixed": L.BE_MIXED_FP32, "refined": L.BE_MIXED_FP32_REFINED}[args.precision]
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
                                                "plaquettes, spin-resolved Berry flux (s = s0(x)t3), " +
                                                PRECISION_TEXT[args.precision],
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

# ---------------------------------------------------------------- served stream (the metric's own workload)
SERVED_GRID = 32


def _served_request_model(kind, req):
    return syn.served_model(kind, req)


def _oracle_served_segment(args):
    """FP64 oracle on a segment of one transverse line of a served request:
    eigenvectors at n_pts consecutive k-points, the overlaps between them
    (polar), and, for a whole line, the Wilson phases. Returns (kind, req,
    n_pts, seconds, phases or None)."""
    kind, req, i, n_pts = args
    t0 = time.perf_counter()
    from oracle import berry as orc
    hl = _served_request_model(kind, req)
    kg = syn.kplane(SERVED_GRID, SERVED_GRID)[i]
    m = hl.N // 2
    ev, U, st = orc.eigh_grid(hl, kg[:n_pts], 0, m)
    th = None
    if n_pts == SERVED_GRID:
        W, _ = orc.wilson_matrix(U)
        th = orc.eigphases(W)
    else:
        for j in range(n_pts - 1):
            orc.polar_factor(U[j + 1].conj().T @ U[j])
    return (kind, req, n_pts, time.perf_counter() - t0, th)


def copy_calibration(mb: int):
    """One plain device copy of mb MiB (its FETCH_SIZE and WRITE_SIZE calibrate
    the byte counters of a rocprofv3 counter run); nothing when mb is 0."""
    if not mb:
        return
    import torch
    nb = mb << 20
    src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main_served(args):
    """Served stream: Poisson arrivals of Wilson-loop requests (BHZ supercells
    L in {8, 12, 16, 24} with W ~ U[0, 4], and the 96-orbital model), 32 x 32
    k-grids, continuous batching with HBM admission on two GPU lanes."""
    from collections import Counter
    n_req = args.requests
    if args.types:
        want = args.types.split(",")
        bad = [t for t in want if t not in syn.SERVED_TYPES]
        if bad:
            raise SystemExit(f"unknown served types {bad}; known: {', '.join(syn.SERVED_TYPES)}")
        kinds = [k for k in syn.served_types(n_req * len(syn.SERVED_TYPES), [5, 0]) if k in want][:n_req]
    else:
        kinds = syn.served_types(n_req, [5, 0])
    first = {}
    for q, k in enumerate(kinds):
        first.setdefault(k, q)
    workers = max(1, min(16, os.cpu_count() or 1))
    # ---- CPU oracle on a bounded sample (before the GPU is touched): whole
    # lines of the two smallest types (their phases also gate the GPU
    # results), line segments of bhz12 and bhz16; bhz24 is extrapolated from
    # bhz16 by the N^3 cost of dense diagonalization
    seg = {"w96": SERVED_GRID, "bhz8": SERVED_GRID, "bhz12": 6, "bhz16": 2}
    sample = [(k, first[k], 0, seg[k]) for k in seg if k in first]
    cpu, oracle_lines = None, {}
    if not args.no_cpu_baseline and sample:
        res, cdt = cpu_baseline(sample, min(workers, len(sample)), _oracle_served_segment, warm_with_sample=False)
        per_k = {}
        for kind, req, n_pts, secs, th in res:
            a = per_k.setdefault(kind, [0.0, 0])
            a[0] += secs
            a[1] += n_pts
            if th is not None:
                oracle_lines[kind] = th
        # single-core seconds per k-point of each type, and the mix's rate on
        # the pool (the stream's k-points over the pool's total core time)
        sec_k = {k: v[0] / v[1] for k, v in per_k.items()}
        if "bhz16" in sec_k:
            sec_k["bhz24"] = sec_k["bhz16"] * (2304 / 1024) ** 3
        cnt = Counter(kinds)
        core_s = sum(cnt[k] * SERVED_GRID * SERVED_GRID * sec_k[k] for k in cnt if k in sec_k)
        rate = sum(cnt[k] for k in cnt if k in sec_k) * SERVED_GRID * SERVED_GRID / core_s * workers
        cpu = {"value": rate, "unit": "k-point solves/s", "cores": workers, "kind": "oracle",
               "sample": "whole lines (32 k-points: eigenvectors, polar overlaps, Wilson phases) of one w96 and one "
                         "bhz8 request, line segments of 6 (bhz12) and 2 (bhz16) k-points; bhz24 extrapolated from "
                         "bhz16 by (2304/1024)^3; single-core seconds per k-point of each type "
                         f"({', '.join(f'{k}: {v:.3g}' for k, v in sorted(sec_k.items()))}) weighted by the "
                         f"stream's mix and scaled to {workers} worker processes (OMP_NUM_THREADS=1); pool wall "
                         f"{cdt:.1f} s",
               "cpu_model": _cpu_model(), "numpy": np.__version__}

    import torch
    from paper_2312_13051_amd import _lib as L
    from paper_2312_13051_amd import serve as S
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    mixed = args.precision in ("mixed", "refined")
    kg = syn.kplane(SERVED_GRID, SERVED_GRID)
    copy_calibration(args.copy_calibration_mb)

    def make(q):
        hl = _served_request_model(kinds[q], q)
        # mixed: the per-type choice (refined where the mixed path misses the gate)
        prec = {"mixed": S.served_precision(kinds[q]), "refined": L.BE_MIXED_FP32_REFINED,
                "fp64": L.BE_FP64}[args.precision]
        return S.Request(hoplist=hl, kappa=kg, lo=0, hi=hl.N // 2, kind=S.KIND_WILSON, precision=prec, tag=kinds[q])

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    ex = S.GpuExecutor(n_lanes=args.lanes)
    budget = int(args.hbm_gib) << 30

    def progress(ev):
        if ev["kind"] == "eig":
            note(f"lane {ev['lane']}: eigensolver N={ev['N']} k={ev['k_points']} {ev['t'] - ev['t0']:.2f} s")
        else:
            note(f"lane {ev['lane']}: request {ev['request']} ({ev['tag']}) done, latency {ev['latency']:.2f} s")
    # ---- warm-up and service times: one request of each type alone
    svc = {}
    for k in syn.SERVED_TYPES:
        if k not in first:
            continue
        eng = S.Engine(ex, hbm_budget=budget, on_event=progress)
        r = make(first[k])
        t0 = time.perf_counter()
        eng.submit(r)
        eng.run_until_idle()
        torch.cuda.synchronize()
        svc[k] = time.perf_counter() - t0
        if r.error is not None:
            raise r.error
        note(f"warm-up {k}: {svc[k]:.2f} s")
    cnt = Counter(kinds)
    mean_svc = sum(cnt[k] * svc[k] for k in cnt) / n_req
    capacity = 1.0 / mean_svc   # requests/s with one request in flight at a time
    rate = args.load * capacity
    # ---- the stream
    reqs = [make(q) for q in range(n_req)]
    arrivals = S.poisson_arrivals(rate, n_req, [5, 0])
    for lane_ctx, _ in ex.lanes:
        lane_ctx.profile_enable(True)
    eng = S.Engine(ex, hbm_budget=budget, on_event=progress, log_path=args.request_log, policy=args.policy)
    note(f"stream: {n_req} requests at {rate:.3f}/s ({args.load} x the one-at-a-time capacity)")
    wall = S.drive(eng, reqs, arrivals)
    torch.cuda.synchronize()
    prof = {}
    for lane_ctx, _ in ex.lanes:
        for name, (ms, n) in lane_ctx.profile().items():
            a = prof.setdefault(name, [0.0, 0])
            a[0] += ms
            a[1] += n
        lane_ctx.profile_enable(False)
    errs = [r for r in reqs if r.error is not None]
    if errs:
        raise errs[0].error
    t_first = min(r.t_submit for r in reqs)
    t_last = max(r.t_done for r in reqs)
    span = t_last - t_first
    total_k = sum(r.n_k for r in reqs)
    value = total_k / span
    lat = S.latency_stats(reqs)
    by_type = {k: S.latency_stats([r for r in reqs if r.tag == k]) for k in syn.SERVED_TYPES}
    note(f"stream done: {total_k} k-points in {span:.2f} s")

    # ---- phase error of sampled lines: oracle lines (small types), the GPU
    # FP64 path on the same line (large types)
    from paper_2312_13051_amd import pipeline as PL
    from tests.phase_metrics import phase_set_error
    gate = {}
    for k in syn.SERVED_TYPES:
        if k not in first:
            continue
        r = reqs[first[k]]
        got = r.result["theta"][0, 0, :r.m]
        if k in oracle_lines:
            gate[k] = {"vs": "oracle", "err": float(phase_set_error(got, oracle_lines[k]))}
        else:
            c0 = ex.lanes[0][0]
            g = PL.eig_grid(c0, c0.hk_plan([r.hoplist]), 0, 1, kg[:1], 0, r.m, L.BE_FP64)
            ref = PL.wilson(c0, g)["theta"][0, 0, :r.m].cpu().numpy()
            gate[k] = {"vs": "gpu_fp64", "err": float(phase_set_error(got, ref))}
    max_err = max((v["err"] for v in gate.values()), default=None)

    # ---- dominant kernel and its roofline over the stream
    name, (ms_tot, launches) = max(prof.items(), key=lambda kv: kv[1][0])
    roof = {"kernel": name, "bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
            "traffic": None, "avg_launch_ms": round(ms_tot / launches, 4), "launches": launches}
    if name == "hetrd_panel":
        byts = sum(hetrd_panel_bytes(r.N, r.n_k, 8 if mixed else 16) for r in reqs)
        ach = byts / (ms_tot * 1e-3) / 1e9
        roof.update({"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": round(byts / launches, 1),
                     "note": "durations of launches that may overlap with the other lane's work; the stream's "
                             "launches span several orders, so traffic per launch is given for the dominant "
                             "order's launches (counters of order-2304 requests) rather than for the mix"})
        prof24 = os.path.join(ROOT, "profiles", "hetrd_panel_served_bhz24_mixed.md")
        t24 = traffic_from_profile(prof24, os.path.join(ROOT, "paper_2312_13051_amd", "csrc", "eigh.hip"),
                                   "mixed") if mixed else None
        if t24 is not None:
            a24 = hetrd_panel_bytes(2304, 256, 8) / ((2304 + NB - 1) // NB)  # one panel of 256 matrices
            roof["order_2304_counters"] = {"profile": os.path.relpath(prof24, ROOT), "traffic_bytes_per_launch": t24,
                                           "algorithmic_bytes_per_launch": round(a24, 1),
                                           "traffic_over_algorithmic": round(t24 / a24, 3)}
    kernels = {k: {"ms": round(v[0], 1), "launches": v[1]} for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}
    gemm_phases = gemm_phase_summary(served_gemm_flops(reqs, L.BE_MIXED_FP32_REFINED),
                                     {k: v[0] for k, v in prof.items()}, ("her2k", "unmtr") if mixed else ())
    gemm_phases["note"] += "; launches of the two lanes may overlap, which lowers the apparent rates"
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "k-point solves/s", "n_gpus": 1,
        "steps": n_req, "warmup": len(svc), "ms_per_step": round(span / n_req * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": "served stream (Poisson arrivals) of Wilson-loop requests: BHZ supercells L in "
                               "{8, 12, 16, 24} (N = 256, 576, 1024, 2304) with Anderson disorder W ~ U[0, 4] and "
                               "a 96-orbital Wannier-like model (|R| <= 3, exp(-|R|/1.5) Gaussian hoppings), "
                               "equally mixed, 32x32 k-grid each, half filling, Wilson loop on all occupied bands, "
                               "HBM-admitted continuous batching on two GPU lanes, " +
                               (PRECISION_TEXT["mixed"] + " (refined mixed path for the 96-orbital model)"
                                if args.precision == "mixed" else PRECISION_TEXT[args.precision]),
                   "requests": n_req, "k_points": total_k, "types": dict(Counter(kinds)),
                   "arrival_rate_per_s": round(rate, 4), "load": args.load, "lanes": args.lanes, "policy": args.policy,
                   "hbm_budget_gib": args.hbm_gib},
        "roofline": roof,
        "gemm_phases": gemm_phases,
        "cpu_baseline": cpu,
        "latency_ms": {"p50": round(lat["p50_ms"], 1), "p99": round(lat["p99_ms"], 1), "unit": "per request",
                       "by_type": {k: {"p50": round(v["p50_ms"], 1), "p99": round(v["p99_ms"], 1), "n": v["n"]}
                                   for k, v in by_type.items() if v["n"]}},
        "service_s_alone": {k: round(v, 3) for k, v in svc.items()},
        "peak_admitted_gib": round(eng.peak_used / 2 ** 30, 1),
        "phase_err_vs_fp64_rad": gate, "phase_gate_1e-6_ok": None if max_err is None else bool(max_err <= 1e-6),
        "valid_requests": int(sum(1 for r in reqs if int(np.asarray(r.result["status"]).max()) == 0
                                  and not r.result["eig_status"])),
        # OR of the status words per request type (4 = WINDING_UNRESOLVED: the
        # phases stand, the grid does not resolve an integer winding)
        "status_by_type": {k: int(np.bitwise_or.reduce([int(np.bitwise_or.reduce(
            np.asarray(r.result["status"], dtype=np.int64).ravel())) for r in reqs if r.tag == k]))
            for k in syn.SERVED_TYPES if any(r.tag == k for r in reqs)},
        "kernels": kernels,
    }
    print(json.dumps(out))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# ---------------------------------------------------------------- uneven batch
UNEVEN_GRID = 16


def _oracle_uneven_line(args):
    """FP64 oracle Wilson phases of one transverse line of system s of the uneven batch."""
    s, i = args
    from oracle import berry as orc
    hl = syn.uneven_systems()[s]
    kg = syn.kplane(UNEVEN_GRID, UNEVEN_GRID)[i]
    ev, U, st = orc.eigh_grid(hl, kg, 0, hl.N // 2)
    W, _ = orc.wilson_matrix(U)
    return (s, i, orc.eigphases(W))


def main_uneven(args):
    """Uneven batch: 64 BHZ supercells L in {6, 8, 12, 16, 20} with 2 %
    vacancies (N = 140 ... 1568), 16 x 16 k-grids, Wilson loop on all occupied
    bands; the mixed path and the FP64 path on the same batch."""
    from collections import defaultdict
    hls = syn.uneven_systems()
    groups = defaultdict(list)
    for s, h in enumerate(hls):
        groups[h.N].append(s)
    sizes = sorted(groups)
    workers = max(1, min(16, os.cpu_count() or 1))
    # oracle: two lines of the first system of each of the three smallest sizes
    sample = [(groups[N][0], i) for N in sizes[:3] for i in (0, 7)]
    cpu, oracle_res = None, []
    if not args.no_cpu_baseline:
        oracle_res, cdt = cpu_baseline(sample, min(workers, len(sample)), _oracle_uneven_line, warm_with_sample=False)
        cpu = {"value": len(sample) * UNEVEN_GRID / cdt, "unit": "k-point solves/s", "cores": min(workers, len(sample)),
               "kind": "oracle", "sample": f"{len(sample)} transverse lines ({len(sample) * UNEVEN_GRID} k-points) of "
                                           f"the three smallest sizes (N = {sizes[:3]}), NumPy/LAPACK FP64, one worker "
                                           f"process per line, OMP_NUM_THREADS=1, wall {cdt:.2f} s",
               "cpu_model": _cpu_model(), "numpy": np.__version__}

    import torch
    from paper_2312_13051_amd import _lib as L
    from paper_2312_13051_amd import pipeline as PL
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    ctx = L.Context(0)
    kg = syn.kplane(UNEVEN_GRID, UNEVEN_GRID)
    n_k = UNEVEN_GRID * UNEVEN_GRID
    plans = {N: ctx.hk_plan([hls[s] for s in groups[N]]) for N in sizes}

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    def step(prec):
        out = {}
        hb = 8 if prec == L.BE_MIXED_FP32 else 16
        for N in sizes:
            ns = len(groups[N])
            chunk = max(n_k, min(ns * n_k, (16 << 30) // (N * N * hb) // n_k * n_k))
            g = PL.eig_grid(ctx, plans[N], 0, ns, kg, 0, N // 2, prec, chunk=chunk)
            out[N] = (None, PL.wilson(ctx, g))
            del g  # the eigenvectors of one size at a time (the N = 1568 group alone holds 65 GB)
        return out

    res, timing, profs = {}, {}, {}
    for pname, prec in (("mixed", L.BE_MIXED_FP32), ("fp64", L.BE_FP64)):
        for _ in range(args.warmup):
            step(prec)
            torch.cuda.synchronize()
        ctx.profile_enable(True)
        t0 = time.perf_counter()
        for k in range(args.steps):
            res[pname] = step(prec)
        torch.cuda.synchronize()
        timing[pname] = (time.perf_counter() - t0) / args.steps
        profs[pname] = ctx.profile()
        ctx.profile_enable(False)
        note(f"{pname}: {timing[pname]:.2f} s per step")
    total_k = len(hls) * n_k

    # ---- the mixed step as one HIP graph: the size groups on two lanes (a
    # library context and a stream each; groups dealt largest work first to
    # the less loaded lane), every buffer allocated beforehand; captured after
    # an eager run of the same body has sized the workspaces, then replayed.
    # The graph runs the Newton-Schulz loops' full schedules (converged
    # matrices skip the steps), so its phases equal the eager run's bit for bit.
    gprec, gdc, gcdt = L.BE_MIXED_FP32, L.BE_C64, torch.complex64
    kap = torch.from_numpy(np.ascontiguousarray(kg.reshape(-1, 3), dtype=np.float64)).cuda()
    nl = max(1, args.graph_lanes)
    lanes = [ctx] + [L.Context(0) for _ in range(nl - 1)]
    streams = [torch.cuda.Stream() for _ in range(nl)]
    work = {N: len(groups[N]) * N ** 3 for N in sizes}
    order = sorted(sizes, key=lambda n: -work[n])
    load, assign = [0] * nl, {}
    for N in order:
        k = int(np.argmin(load))
        assign[N] = k
        load[k] += work[N]
    lplans = {N: lanes[assign[N]].hk_plan([hls[s] for s in groups[N]]) for N in sizes}
    chunk_k = {N: max(n_k, min(len(groups[N]) * n_k, (4 << 30) // (N * N * 8) // n_k * n_k)) for N in sizes}
    gbuf = []
    for k in range(nl):
        Ns = [N for N in sizes if assign[N] == k]
        gbuf.append({"U": torch.empty(max(len(groups[N]) * n_k * (N // 2) * N for N in Ns), dtype=torch.complex128,
                                      device="cuda"),
                     "H": torch.empty(max(chunk_k[N] * N * N for N in Ns), dtype=gcdt, device="cuda"),
                     "ev": torch.empty(max(len(groups[N]) * n_k * (N // 2 + 2) for N in Ns), dtype=torch.float64,
                                       device="cuda"),
                     "st": torch.empty(max(len(groups[N]) * n_k for N in Ns), dtype=torch.int32, device="cuda")})
    gout = {N: {"theta": torch.empty((len(groups[N]), UNEVEN_GRID, N // 2), dtype=torch.float64, device="cuda"),
                "phi": torch.empty((len(groups[N]), UNEVEN_GRID), dtype=torch.float64, device="cuda"),
                "wind": torch.empty(len(groups[N]), dtype=torch.int32, device="cuda"),
                "st": torch.empty(len(groups[N]), dtype=torch.int32, device="cuda")} for N in sizes}

    def run_group(N):
        c, b = lanes[assign[N]], gbuf[assign[N]]
        ns, m = len(groups[N]), N // 2
        nmat = ns * n_k
        U = b["U"][:nmat * m * N].view(nmat, m, N)
        ev = b["ev"][:nmat * (m + 2)].view(nmat, m + 2)
        per = chunk_k[N] // n_k
        for s0 in range(0, ns, per):
            nsc = min(per, ns - s0)
            H = b["H"][:nsc * n_k * N * N].view(nsc * n_k, N, N)
            c.build_hk(lplans[N], s0, nsc, kap, H, N * N, N, gdc)
            q0 = s0 * n_k
            c.eigh_batched(H, gdc, N, N, N * N, nsc * n_k, 0, m, gprec, ev[q0:], U[q0:], N, U.stride(0),
                           b["st"][q0:])
        o = gout[N]
        c.wilson_loop(U, N, m, N, U.stride(0), ns, UNEVEN_GRID, UNEVEN_GRID, L.BE_OVL_POLAR, o["theta"], o["phi"],
                      o["wind"], o["st"])

    def body():
        cur = torch.cuda.current_stream()
        for s_ in streams:
            s_.wait_stream(cur)
        for N in order:
            with torch.cuda.stream(streams[assign[N]]):
                run_group(N)
        for s_ in streams:
            cur.wait_stream(s_)

    body()
    torch.cuda.synchronize()
    eager = {N: gout[N]["theta"].clone() for N in sizes}
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=cap):
        body()
    torch.cuda.synchronize()
    note("uneven step captured as one graph")
    graph.replay()
    torch.cuda.synchronize()
    graph_equal = all(torch.equal(gout[N]["theta"], eager[N]) for N in sizes)
    t0 = time.perf_counter()
    for k in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    timing["graph"] = (time.perf_counter() - t0) / args.steps
    note(f"graph: {timing['graph']:.2f} s per step (phases equal to the eager run's: {graph_equal})")
    # the line's value: the faster of the eager loop and the graph (when the
    # graph's phases equal the eager run's)
    tbest = min(timing["graph"], timing["mixed"]) if graph_equal else timing["mixed"]
    # gate: mixed against FP64 on every line; FP64 against the oracle's lines
    from tests.phase_metrics import phase_set_error
    err_mixed = 0.0
    for N in sizes:
        a = res["mixed"][N][1]["theta"].cpu().numpy()
        b = res["fp64"][N][1]["theta"].cpu().numpy()
        for s in range(a.shape[0]):
            for i in range(a.shape[1]):
                err_mixed = max(err_mixed, phase_set_error(a[s, i], b[s, i]))
    err_fp64 = 0.0
    for (s, i, th) in oracle_res:
        N = hls[s].N
        loc = groups[N].index(s)
        err_fp64 = max(err_fp64, phase_set_error(res["fp64"][N][1]["theta"][loc, i].cpu().numpy(), th))
    prof = profs["mixed"]
    name, (ms_tot, launches) = max(prof.items(), key=lambda kv: kv[1][0])
    roof = {"kernel": name, "bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
            "traffic": None, "avg_launch_ms": round(ms_tot / launches, 4), "launches": launches}
    if name == "hetrd_panel":
        byts = sum(hetrd_panel_bytes(N, len(groups[N]) * n_k, 8) for N in sizes) * args.steps
        ach = byts / (ms_tot * 1e-3) / 1e9
        roof.update({"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": round(byts / launches, 1)})
    st = np.concatenate([res["mixed"][N][1]["status"].cpu().numpy() for N in sizes])
    out = {
        "metric": METRIC, "value": round(total_k / tbest, 1), "unit": "k-point solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(tbest * 1e3, 2),
        "eager_value": round(total_k / timing["mixed"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "uneven batch: 64 BHZ L x L supercells, L drawn from {6, 8, 12, 16, 20}, 2 % vacancies "
                               "(N = 140, 252, 564, 1004, 1568), 16x16 k-grids, half filling, Wilson loop on all "
                               "occupied bands; mixed path (FP32 reduction and back-transformation) and FP64 path",
                   "systems": len(hls), "sizes": {str(N): len(groups[N]) for N in sizes}, "k_points": total_k},
        "fp64_value": round(total_k / timing["fp64"], 1), "mixed_over_fp64": round(timing["fp64"] / timing["mixed"], 3),
        "graph": {"value": round(total_k / timing["graph"], 1), "ms_per_step": round(timing["graph"] * 1e3, 2),
                  "lanes": nl, "groups_by_lane": {str(N): assign[N] for N in sizes},
                  "phases_equal_eager_bitwise": bool(graph_equal),
                  "note": "the mixed step captured once as one HIP graph (size groups dealt to the lanes, "
                          "largest work first) and replayed"},
        "roofline": roof, "cpu_baseline": cpu,
        "phase_err_mixed_vs_fp64_rad": err_mixed, "phase_err_fp64_vs_oracle_rad": err_fp64 if oracle_res else None,
        "phase_gate_1e-6_ok": bool(err_mixed <= 1e-6),
        "valid_systems": int((st == 0).sum()),
        "kernels_mixed": {k: {"ms_per_step": round(v[0] / args.steps, 2), "launches_per_step": v[1] // args.steps}
                          for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
