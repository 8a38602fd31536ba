"""Ensemble statistics of the MPO entanglement entropy (Sec. IV.A-B).

For each of N_s random circuit realizations (Haar U(4) gates plus two-qubit
depolarizing noise of rate p, brickwork from |0...0>), the bond entropies
S_l are recorded after every time step; the realizations run together on the
batched path (mpo_batch_run, several streams).  At each depth D the entropies are
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


def ensemble_stats(S: np.ndarray, tr: np.ndarray) -> dict:
    """Statistics of Sec. IV.A-B from per-realization records: S (samples,
    depth, n-1) bond entropies and tr (samples, depth) Tr rho after every time
    step.  The entropies are averaged over the realizations, then maximised
    over the bond: S_max(D); D* = argmax S_max(D) (1-based), S*_max = S_max(D*)."""
    Sm = S.mean(axis=0)
    trm = tr.mean(axis=0)
    smax = Sm.max(axis=1)
    d_star = int(np.argmax(smax)) + 1
    return {"S_mean": Sm, "S_max_by_depth": smax.tolist(), "mean_trace_by_depth": trm.tolist(),
            "D_star": d_star, "S_star": float(smax[d_star - 1]), "trace_at_D_star": float(trm[d_star - 1])}


def ensemble(n: int, p: float, chi: int, depth: int, samples: int, seed0: int,
             precision: str = "fp64", cutoff: float = 1e-12, n_streams: int = 8) -> dict:
    """N_s = samples realizations (seeds seed0 .. seed0 + samples - 1) on the
    batched path: all of them in one mpo_batch_run over n_streams streams,
    observables after every time step."""
    import mpo_inputs as mi
    import paper_2003_13163_amd as pm
    t0 = time.perf_counter()
    circuits, sups = [], []
    for i in range(samples):
        circuits.append((n, depth, chi, cutoff))
        sups.append(pm.build_superops(mi.ginibre_draws(n, depth, seed=seed0 + i), p, "pauli"))
    out = pm.batch_run(circuits, sups, precision, "pauli", n_streams=min(n_streams, samples), record="all")
    S = np.stack([o["S"] for o in out])
    tr = np.stack([o["trace"] for o in out])
    st = ensemble_stats(S, tr)
    st.pop("S_mean")
    return {"n": n, "p": p, "chi_max": chi, "depth": depth, "samples": samples, "seed0": seed0,
            "precision": precision, **st, "seconds": time.perf_counter() - t0}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--p", type=float, required=True)
    ap.add_argument("--n", type=int, nargs="+", default=[8])
    ap.add_argument("--chi", type=int, default=80)
    ap.add_argument("--depth", type=int, default=10)
    ap.add_argument("--samples", type=int, default=24)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--streams", type=int, default=8)
    a = ap.parse_args(argv)
    import torch  # noqa: F401
    import paper_2003_13163_amd as pm
    pm.library()
    for n in a.n:
        r = ensemble(n, a.p, a.chi, a.depth, a.samples, a.seed0, a.precision, n_streams=a.streams)
        print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
