#!/usr/bin/env python3
"""Writes oracle_samples.json: FP64 oracle values at sampled points of the
large workloads, where the oracle takes minutes (every value comes from
oracle/ on seeded synthetic inputs; nothing from the GPU path).

bbh1764: spin-resolved Berry flux of single plaquettes of the spinful BBH
(eq. 10) 21 x 21 supercell with chiral disorder (N = 1764), W = 1 (seed
[7, 0]) and W = 9 (seed [7, 1]), 20 x 20 plaquette grid; the plaquettes
are the ones the flux benchmark samples (rng [9, 10 + w], 8 per W). Each is
the (0, 0) entry of the oracle's map on the 2 x 2 grid of its corners.

Run: python tests/golden/make_oracle_samples.py  (about 5 minutes on 8 cores)
"""
import json
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "oracle_samples.json")
BBH_L, BBH_GRID, BBH_W = 21, 20, (1.0, 9.0)


def bbh_plaquettes(w):
    """The plaquettes (i, j) sampled for disorder index w (as the benchmark)."""
    return [(int(i), int(j)) for i, j in np.random.default_rng([9, 10 + w]).integers(0, BBH_GRID, size=(8, 2))]


def _bbh_corner(args):
    w, i, j = args
    import synthetic as syn
    from oracle import berry as orc
    hl = syn.spinful_bbh_disordered(BBH_L, BBH_W[w], [7, w])
    kg = syn.kplane(BBH_GRID, BBH_GRID)
    sub = kg[[i, (i + 1) % BBH_GRID]][:, [j, (j + 1) % BBH_GRID]]
    out = orc.spin_resolved_flux(hl, syn.spinful_bbh_spin_diag(hl), sub, 0, hl.N // 2)
    rec = {"W": BBH_W[w], "seed": [7, w], "i": i, "j": j, "status": int(out["status"])}
    if not out["status"] & orc.PSO_GAP:
        rec.update({"m_dn": int(out["m_dn"]), "flux_dn": float(out["flux_dn"][0, 0]),
                    "flux_up": float(out["flux_up"][0, 0])})
    return rec


def main():
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    jobs = [(w, i, j) for w in range(len(BBH_W)) for (i, j) in bbh_plaquettes(w)]
    with mp.get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as pool:
        recs = pool.map(_bbh_corner, jobs)
    data = {"_about": "FP64 oracle values at sampled points of large workloads, written by "
                      "tests/golden/make_oracle_samples.py from oracle/ on seeded synthetic inputs.",
            "bbh1764_spin_flux": recs}
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)
    print(f"wrote {OUT}: {len(recs)} plaquettes")


if __name__ == "__main__":
    main()
