"""Write the frozen-replay finite differences of the differentiation workload.

Calls only oracle/ and mpo_inputs/.  Workload: n = 32 qubits, depth 24, Haar
gates followed by two-qubit depolarizing p = 0.01, chi_max = 256, cutoff 1e-12
on normalised singular values, Pauli basis, seed 0; O = sum_i Tr[Z_i rho_D]
(unnormalised).  With the truncation projectors frozen at the oracle's forward
run (oracle/replay.py), central differences with step h = 1e-6 give
  * dO/dp, the superoperators rebuilt at p +- h (Sec. II.B, N2[p] after U);
  * dO/d eps along three unit directions D_k in superoperator space
    (mpo_inputs.gradient_directions(372, 3, seed=5)), M_g +- h D_k[g].
O is a polynomial of degree 372 in p (and in eps), so the h^2 term of a
central difference is not negligible at 1e-8 (about 3e-8 of dO/dp); the same
differences at 2h give the Richardson value (4 D(h) - D(2h)) / 3, whose error
is of order h^4.
Usage: python tests/golden/make_golden_adjoint.py
writes tests/golden/oracle_adjoint_n32_d24_p0.01_chi256.json.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import mpo_inputs as mi  # noqa: E402
from oracle import gates, replay  # noqa: E402


def main():
    n, depth, p, chi, seed, cutoff, h = 32, 24, 0.01, 256, 0, 1e-12, 1e-6
    draws = mi.ginibre_draws(n, depth, seed=seed)
    sup = gates.circuit_superops(draws, p, "pauli")
    layers = mi.brickwork_sites(n, depth)
    t0 = time.time()
    prefixes, m = replay.record_prefixes(n, sup, layers, chi, cutoff, "pauli")
    O_fwd = float(np.sum(m.expect_z_all()) * m.trace().real)
    print(f"forward {time.time() - t0:.0f} s, O = {O_fwd!r}, bonds {m.bond_dims()}", flush=True)

    def value(s):
        t1 = time.time()
        v = replay.frozen_replay_value(n, s, layers, prefixes, "pauli")
        print(f"  replay {time.time() - t1:.0f} s: {v!r}", flush=True)
        return v

    O_rep = value(sup)

    def central(f, step):
        return (f(step) - f(-step)) / (2 * step)

    def richardson(f):
        d1, d2 = central(f, h), central(f, 2 * h)
        return d1, (4 * d1 - d2) / 3

    dp, dp_r = richardson(lambda e: value(gates.circuit_superops(draws, p + e, "pauli")))
    dirs = mi.gradient_directions(len(sup), 3, seed=5)
    dd = [richardson(lambda e, d=d: value(sup + e * d)) for d in dirs]
    out = {"workload": {"n": n, "depth": depth, "p": p, "chi_max": chi, "seed": seed, "cutoff": cutoff,
                        "basis": "pauli", "observable": "sum_i Tr[Z_i rho_D]"},
           "h": h, "direction_seed": 5, "n_gates": len(sup),
           "O_forward": O_fwd, "O_replay": [O_rep.real, O_rep.imag],
           "dO_dp_fd": [dp.real, dp.imag],
           "dO_dp_richardson": [dp_r.real, dp_r.imag],
           "dO_ddir_fd": [[v[0].real, v[0].imag] for v in dd],
           "dO_ddir_richardson": [[v[1].real, v[1].imag] for v in dd],
           "seconds": time.time() - t0}
    path = os.path.join(HERE, "oracle_adjoint_n32_d24_p0.01_chi256.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
