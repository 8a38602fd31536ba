"""Ensemble statistics of the MPO entanglement entropy (Sec. IV.A-B).

For each of N_s random circuit realizations (Haar U(4) gates plus two-qubit
depolarizing noise of rate p, brickwork from |0...0>), the bond entropies
S_l are recorded after every time step.  At each depth D the entropies are
averaged over the realizations, then maximised over l: S_max(D).  The optimal
depth D* maximises S_max(D) and S*_max = S_max(D*); the average Tr rho at D*
shows how much probability the bond-dimension cap kept (Sec. III.D, IV.B).

    python -m paper_2003_13163_amd.ensemble --p 0.15 --n 8 12 16 --chi 80 --depth 10
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def ensemble(n: int, p: float, chi: int, depth: int, samples: int, seed0: int,
             precision: str = "fp64", cutoff: float = 1e-12) -> dict:
    import mpo_inputs as mi
    import paper_2003_13163_amd as pm
    S = np.zeros((depth, n - 1))
    tr = np.zeros(depth)
    t0 = time.perf_counter()
    for i in range(samples):
        draws = mi.ginibre_draws(n, depth, seed=seed0 + i)
        st = pm.Mpo(n, chi, precision, "pauli")
        res = st.run_brickwork(depth, pm.build_superops(draws, p, "pauli"), chi, cutoff, record="all")
        st.close()
        S += res["S"]
        tr += res["trace"]
        print(f"n={n} p={p} chi={chi}: realization {i + 1}/{samples}, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    S /= samples
    tr /= samples
    smax = S.max(axis=1)
    d_star = int(np.argmax(smax)) + 1
    return {"n": n, "p": p, "chi_max": chi, "depth": depth, "samples": samples, "seed0": seed0,
            "precision": precision, "S_max_by_depth": smax.tolist(), "mean_trace_by_depth": tr.tolist(),
            "D_star": d_star, "S_star": float(smax[d_star - 1]), "trace_at_D_star": float(tr[d_star - 1]),
            "seconds": time.perf_counter() - t0}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--p", type=float, required=True)
    ap.add_argument("--n", type=int, nargs="+", default=[8])
    ap.add_argument("--chi", type=int, default=80)
    ap.add_argument("--depth", type=int, default=10)
    ap.add_argument("--samples", type=int, default=24)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--precision", default="fp64")
    a = ap.parse_args(argv)
    import torch  # noqa: F401
    import paper_2003_13163_amd as pm
    pm.library()
    for n in a.n:
        r = ensemble(n, a.p, a.chi, a.depth, a.samples, a.seed0, a.precision)
        print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
