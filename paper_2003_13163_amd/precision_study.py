"""Precision-mode study on the large truncated workload: n = 64 qubits, Haar
U(4) gates with two-qubit depolarizing noise (Sec. II.B, Sec. III.B) in
brickwork order from |0...0>, chi_max = 1024, cutoff 1e-12, the same gates
(seed 0) for every mode and every p.  Each mode runs the whole circuit on the
GPU (gates ascending within a time step, or in snake order) and records, after the last
time step, the bond entropies (Sec. III.C), their maximum S_max, <Z_i> and
Tr rho (Sec. III.D).  The FP64 run is the
reference the reduced-precision modes are compared with.

    python -m paper_2003_13163_amd.precision_study run --mode fp32 --out r_fp32.json
    python -m paper_2003_13163_amd.precision_study compare r_fp64.json r_fp32.json ...
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def run(mode: str, n: int, depth: int, p: float, chi: int, seed: int, order: str = "ascending") -> dict:
    import torch
    import mpo_inputs as mi
    import paper_2003_13163_amd as pm
    pm.library()
    if not torch.cuda.is_available():
        raise SystemExit("the study runs on the GPU")
    draws = mi.ginibre_draws(n, depth, seed=seed)
    sup = pm.build_superops(draws, p, "pauli")
    st = pm.Mpo(n, chi, mode, "pauli")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, disc = 0, 0.0
    layers = mi.brickwork_sites(n, depth)
    for t in range(0, depth, 2):
        # two time steps per call (an odd then an even one, as a fresh brickwork
        # starts), so that progress can be reported; superops in the chosen
        # order, i.e. right to left within the even step under snake order
        steps = layers[t:t + 2]
        chunk = []
        for j, sites in enumerate(steps):
            blk = list(sup[g:g + len(sites)])
            chunk += blk[::-1] if (order == "snake" and j == 1) else blk
            g += len(sites)
        res = st.run_brickwork(len(steps), np.array(chunk), chi, 1e-12, record=None, order=order)
        disc += float(res["discarded"].sum())
        print(f"{mode} {order}: time steps {t + len(steps)}/{depth} done, "
              f"{time.perf_counter() - t0:.1f} s, max bond {max(st.bond_dims()[0])}",
              file=sys.stderr, flush=True)
    S = st.entropy(-1)
    Z, tr = st.expect_z_all()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dims = st.bond_dims()[0]
    st.close()
    return {"mode": mode, "order": order, "n": n, "depth": depth, "p": p, "chi_max": chi, "seed": seed,
            "cutoff": 1e-12, "gates": g, "seconds": dt, "S": S.tolist(), "S_max": float(S.max()),
            "Z": Z.tolist(), "trace": float(tr), "discarded_total": disc,
            "bond_dims": [int(d) for d in dims]}


def compare(paths: list[str]) -> dict:
    runs = [json.load(open(q)) for q in paths]
    ref = next((r for r in runs if r["mode"] == "fp64"), None)
    if ref is None:
        raise SystemExit("compare needs the fp64 run")
    table = []
    for r in runs:
        row = {"mode": r["mode"], "seconds": r["seconds"], "gates_per_s": r["gates"] / r["seconds"],
               "S_max": r["S_max"], "trace": r["trace"]}
        if r is not ref:
            row["dS_max"] = abs(r["S_max"] - ref["S_max"])
            row["max_abs_dS_bond"] = float(np.abs(np.array(r["S"]) - np.array(ref["S"])).max())
            row["max_abs_dZ"] = float(np.abs(np.array(r["Z"]) - np.array(ref["Z"])).max())
            row["rel_dtrace"] = abs(r["trace"] - ref["trace"]) / abs(ref["trace"])
        table.append(row)
    return {"workload": {k: ref[k] for k in ("n", "depth", "p", "chi_max", "seed", "cutoff", "gates")},
            "table": table}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--mode", required=True, choices=["fp64", "fp32", "bf16x3"])
    r.add_argument("--n", type=int, default=64)
    r.add_argument("--depth", type=int, default=48)
    r.add_argument("--p", type=float, default=0.01)
    r.add_argument("--chi", type=int, default=1024)
    r.add_argument("--seed", type=int, default=0)
    r.add_argument("--order", default="ascending", choices=["ascending", "snake"])
    r.add_argument("--out", required=True)
    c = sub.add_parser("compare")
    c.add_argument("files", nargs="+")
    a = ap.parse_args(argv)
    if a.cmd == "run":
        out = run(a.mode, a.n, a.depth, a.p, a.chi, a.seed, a.order)
        json.dump(out, open(a.out, "w"))
        print(json.dumps({k: out[k] for k in ("mode", "depth", "p", "seconds", "S_max", "trace")}),
              flush=True)
    else:
        print(json.dumps(compare(a.files), indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
