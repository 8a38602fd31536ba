"""Autotuner for the blocked one-sided Jacobi of the truncated split.

For every precision and bond-dimension bucket it builds an in-situ state (a
12-qubit brickwork of Haar gates with two-qubit depolarizing noise p = 0.01,
seed 0, run until the middle bonds sit at the bucket's chi_max), then times
the gates of the continuing brickwork on the middle sites with each candidate
(Jacobi block width 16 or 32 columns, 1 or 2 inner FP64 sweeps per block pair)
and keeps the fastest.  The result is a table of
(precision, chi_upto, block, inner) entries written as JSON; the binding
loads paper_2003_13163_amd/tuning.json when the library is first loaded and
hands every entry to mpo_set_default_tuning, so later handles of that
precision and bond cap use it.

    python -m paper_2003_13163_amd.autotune --out paper_2003_13163_amd/tuning.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

CANDIDATES = [(16, 1), (16, 2), (32, 1), (32, 2)]
BUCKETS = [64, 128, 256, 512, 1024]


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_candidates(pm, mi, torch, prec: str, chi: int, gates: int = 6, n: int = 12, p: float = 0.01):
    depth = 4 + int(np.ceil(np.log2(chi) / 2))           # enough time steps to saturate chi at the middle
    draws = mi.ginibre_draws(n, depth, seed=0)
    st = pm.Mpo(n, chi, "fp32" if prec != "fp64" else "fp64", "pauli")
    st.run_brickwork(depth, pm.build_superops(draws, p, "pauli"), chi, 1e-12, record=None)
    snap = st.export()
    dims = st.bond_dims()[0]
    st.close()
    mid = n // 2 - 1
    sites = [mid - 2 + 2 * (g % 3) + ((g // 3) % 2) for g in range(gates + 1)]
    sups = pm.build_superops(mi.ginibre_draws(n, 2 * gates + 2, seed=1)[: gates + 1], p, "pauli")
    out = {}
    for block, inner in CANDIDATES:
        st = pm.Mpo(n, chi, prec, "pauli")
        pm._check(pm.library().mpo_set_tuning(st._h, block, inner))
        st.import_state(snap)
        st.apply(sites[0], sups[0], chi, 1e-12)          # warmup: first moves and caches
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for g in range(1, gates + 1):
            st.apply(sites[g], sups[g], chi, 1e-12)
        torch.cuda.synchronize()
        out[f"{block}x{inner}"] = gates / (time.perf_counter() - t0)
        st.close()
    return out, max(dims)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--precisions", default="fp32,fp64,bf16x3")
    ap.add_argument("--buckets", default=",".join(map(str, BUCKETS)))
    ap.add_argument("--gates", type=int, default=6)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    import torch
    import mpo_inputs as mi
    import paper_2003_13163_amd as pm
    pm.library()
    entries, measured = [], {}
    for prec in a.precisions.split(","):
        for chi in (int(c) for c in a.buckets.split(",")):
            _log(f"autotune {prec} chi={chi}")
            rates, chi_reached = time_candidates(pm, mi, torch, prec, chi, a.gates)
            best = max(rates, key=rates.get)
            block, inner = (int(x) for x in best.split("x"))
            entries.append({"precision": prec, "chi_upto": chi, "block": block, "inner": inner})
            measured[f"{prec}/{chi}"] = {"updates_per_s": rates, "chi_reached": chi_reached, "best": best}
            _log(f"  {json.dumps(rates)} -> {best}")
    rec = {"entries": entries, "measured": measured,
           "command": "python -m paper_2003_13163_amd.autotune " + " ".join(argv or sys.argv[1:])}
    text = json.dumps(rec, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
