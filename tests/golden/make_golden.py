"""Write oracle-computed expected values for the larger parity cases.

Calls only oracle/ and mpo_inputs/ (the seeded draws).  Usage:
    python tests/golden/make_golden.py n32
writes tests/golden/oracle_n32_d32_p0.01_chi256.json: the truncating
single-circuit workload (n = 32 qubits, depth 32, two-qubit depolarizing
p = 0.01 after every Haar gate, chi_max = 256, cutoff 1e-12 on normalised
singular values, Pauli basis, seed 0), with S_b at every bond, <Z_i> and
Tr rho after every time step, and the discarded weight of every gate.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import mpo_inputs as mi  # noqa: E402
from oracle import gates, mpo  # noqa: E402


def n32():
    n, depth, p, chi, seed = 32, 32, 0.01, 256, 0
    draws = mi.ginibre_draws(n, depth, seed=seed)
    sup = gates.circuit_superops(draws, p, "pauli")
    t0 = time.time()
    res = mpo.run_brickwork(n, sup, mi.brickwork_sites(n, depth), chi, 1e-12, "pauli")
    out = {
        "workload": {"n": n, "depth": depth, "p": p, "chi_max": chi, "cutoff": 1e-12,
                     "basis": "pauli", "seed": seed},
        "made_by": "tests/golden/make_golden.py n32 (oracle only)",
        "oracle_seconds": time.time() - t0,
        "S": res["S"].tolist(), "Z": res["Z"].tolist(), "trace": res["trace"].tolist(),
        "discarded": res["discarded"].tolist(), "kept": res["kept"].tolist(),
    }
    path = os.path.join(HERE, "oracle_n32_d32_p0.01_chi256.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, "in", out["oracle_seconds"], "s")


if __name__ == "__main__":
    {"n32": n32}[sys.argv[1]]()
