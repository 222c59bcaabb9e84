"""Autotuner for the eigensolver's per-order knobs.

For each matrix order and reduction precision it times one batched
eigensolver call for every panel kernel variant (each thread count the panel
kernel supports; for the FP32 reduction at 512 threads both loads-in-flight
forms), on the same matrices, best of a few runs, and keeps the fastest
setting. The result is a JSON tuning table: per knob ("hetrd_panel_threads",
"hetrd_panel_loads"), rows {"n_lo", "n_hi", "precision", "value"} whose order
ranges split at the midpoints between measured orders, plus the raw timings.
``Context.load_tuning`` applies a table.

    python -m paper_2312_13051_amd.tune --orders 128,256,400,576,800,1024,1568,2304 --out tuning.json

The matrices are random Hermitian ones (the kernels' work does not depend on
the values); the timed call is the library's ``be_eigh_batched`` with bands
[0, N/2).
"""
from __future__ import annotations

import argparse
import json
import time

from . import _lib as L

PANEL_THREADS = (256, 512, 1024)
PRECISIONS = {"fp64": L.BE_FP64, "mixed": L.BE_MIXED_FP32}
# (threads, loads in flight; 0: the variant's only form) timed per precision
VARIANTS = {"fp64": ((256, 0), (512, 0), (1024, 0)),
            "mixed": ((256, 0), (512, 4), (512, 8), (1024, 0))}


def variant_name(nt: int, loads: int) -> str:
    return f"{nt}" if loads == 0 else f"{nt}x{loads}"


def batch_for(N: int, n_cu: int = 256) -> int:
    """Matrices per timed call: about 6 GiB of c128 input, at most 1536, and
    at least one matrix per compute unit up to order 4096 (the eigensolver
    runs one workgroup per matrix: fewer matrices would time a partly idle
    device, where the thread counts rank differently), else 32."""
    floor = n_cu if N <= 4096 else 32
    return int(max(floor, min(1536, (6 << 30) // (16 * N * N))))


def time_eigh(ctx, N: int, precision: int, n_mat: int, reps: int = 2, seed: int = 0) -> float:
    """Best-of-reps seconds of one eigh_batched call on n_mat random Hermitian matrices."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    cdt = torch.complex64 if precision == L.BE_MIXED_FP32 else torch.complex128
    dcode = L.BE_C64 if precision == L.BE_MIXED_FP32 else L.BE_C128
    H0 = torch.randn((n_mat, N, N), dtype=cdt, device="cuda", generator=g)
    H0 = H0 + H0.transpose(1, 2).conj()
    H = torch.empty_like(H0)
    m = N // 2
    U = torch.empty((n_mat, max(m, 1), N), dtype=torch.complex128, device="cuda")
    ev = torch.empty((n_mat, m + 2), dtype=torch.float64, device="cuda")
    st = torch.empty(n_mat, dtype=torch.int32, device="cuda")
    best = float("inf")
    for _ in range(reps + 1):  # the first call also sizes the workspace
        H.copy_(H0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.eigh_batched(H, dcode, N, N, N * N, n_mat, 0, m, precision, ev, U, N, U.stride(0), st)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def autotune(ctx, orders, precisions=("mixed", "fp64"), reps: int = 2, log=print) -> dict:
    orders = sorted(set(int(n) for n in orders))
    bounds = [1] + [(a + b) // 2 + 1 for a, b in zip(orders, orders[1:])] + [1 << 30]
    rows, lrows, meas = [], [], []
    for pname in precisions:
        prec = PRECISIONS[pname]
        for i, N in enumerate(orders):
            n_mat = batch_for(N)
            t = {}
            for nt, loads in VARIANTS[pname]:
                ctx.tune_clear("hetrd_panel_threads")
                ctx.tune_clear("hetrd_panel_loads")
                ctx.tune_set("hetrd_panel_threads", nt)
                ctx.tune_set("hetrd_panel_loads", loads)
                t[(nt, loads)] = time_eigh(ctx, N, prec, n_mat, reps)
            best = min(t, key=t.get)
            rng = {"n_lo": bounds[i], "n_hi": bounds[i + 1] - 1, "precision": prec}
            rows.append(dict(rng, value=best[0]))
            both = [v for v in VARIANTS[pname] if v[0] == 512 and v[1]]
            if len(both) > 1:  # the faster form of the 512-thread kernel
                lrows.append(dict(rng, value=min(both, key=t.get)[1]))
            meas.append({"precision": pname, "N": N, "n_mat": n_mat,
                         "seconds": {variant_name(*k): round(v, 6) for k, v in t.items()},
                         "best": variant_name(*best)})
            log(f"[tune] {pname} N={N} ({n_mat} matrices): " +
                ", ".join(f"{variant_name(*k)} {v * 1e3:.1f} ms" for k, v in t.items()) +
                f" -> {variant_name(*best)}")
    ctx.tune_clear("hetrd_panel_threads")
    ctx.tune_clear("hetrd_panel_loads")
    return {"knobs": {"hetrd_panel_threads": rows, "hetrd_panel_loads": lrows}, "measurements": meas}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--orders", default="128,256,400,576,800,1024,1568,2304")
    ap.add_argument("--precisions", default="mixed,fp64")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    import torch
    ctx = L.Context(0)
    table = autotune(ctx, a.orders.split(","), a.precisions.split(","), a.reps,
                     log=lambda s: print(s, flush=True))
    table["device"] = torch.cuda.get_device_name(0)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"[tune] wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
