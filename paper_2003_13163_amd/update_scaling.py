"""Cost of the local update against the global one, per gate, versus n.

The paper's update (App. A) brings the whole chain back to the canonical
Gamma-lambda form after every gate, n - 1 SVDs per gate, O(n^2 D chi^3) for a
depth-D circuit; its "Note added" keeps the mixed canonical form and moves the
orthogonality centre locally, O(n D chi^3).  Both truncate the same Schmidt
values, so they give the same state.  This driver runs the same circuit both
ways on the GPU: the local update (ascending brickwork), and the global one
(every gate followed by a canonical sweep that recomputes the Schmidt values
at every bond), and reports seconds per gate and the largest difference of the
final bond entropies and <Z_i>.

    python -m paper_2003_13163_amd.update_scaling --n 8 16 32 --chi 64 --depth 8
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def measure(n: int, depth: int, p: float, chi: int, seed: int, prec: str) -> dict:
    import torch
    import mpo_inputs as mi
    import paper_2003_13163_amd as pm
    draws = mi.ginibre_draws(n, depth, seed=seed)
    sup = pm.build_superops(draws, p, "pauli")
    out = {"n": n, "depth": depth, "p": p, "chi_max": chi, "precision": prec, "gates": int(sup.shape[0])}
    # local update
    st = pm.Mpo(n, chi, prec, "pauli")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.run_brickwork(depth, sup, chi, 1e-12, record=None)
    torch.cuda.synchronize()
    out["local_s_per_gate"] = (time.perf_counter() - t0) / sup.shape[0]
    s_loc = st.entropy(-1)
    z_loc, _ = st.expect_z_all()
    st.close()
    # global update: a full canonical sweep (Schmidt values at every bond) after every gate
    st = pm.Mpo(n, chi, prec, "pauli")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = 0
    for t, sites in enumerate(mi.brickwork_sites(n, depth)):
        for s in sites:
            st.apply(s, sup[g], chi, 1e-12)
            st.entropy(-1)
            g += 1
        print(f"n={n} global: time step {t + 1}/{depth}, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    out["global_s_per_gate"] = (time.perf_counter() - t0) / sup.shape[0]
    s_glo = st.entropy(-1)
    z_glo, _ = st.expect_z_all()
    st.close()
    out["ratio"] = out["global_s_per_gate"] / out["local_s_per_gate"]
    out["max_abs_dS"] = float(np.abs(s_glo - s_loc).max())
    out["max_abs_dZ"] = float(np.abs(z_glo - z_loc).max())
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[8, 16, 32, 64])
    ap.add_argument("--depth", type=int, default=8)
    ap.add_argument("--p", type=float, default=0.01)
    ap.add_argument("--chi", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp64")
    a = ap.parse_args(argv)
    import paper_2003_13163_amd as pm
    pm.library()
    rows = [measure(n, a.depth, a.p, a.chi, a.seed, a.precision) for n in a.n]
    for r in rows:
        print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
