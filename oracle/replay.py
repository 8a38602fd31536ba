"""Frozen-projector replay of a truncated brickwork run, in MPS form (test
infrastructure only).

With every truncation frozen at its forward value, gate g on sites (s, s+1) is
the linear map rho -> P_g M_g rho, P_g = (Phi_g Phi_g^dagger) (x) 1, where
Phi_g are the kept left Schmidt vectors at bond s (App. A truncation; the left
isometries of sites 0..s after the gate in the "Note added" update).  The
observable O = sum_i Tr[Z_i rho_D] is then linear in every M_g, and the value
of that frozen map at perturbed superoperators is what central finite
differences of the frozen-projector gradient are checked against.  adjoint.py
computes the same map on dense vectors (n <= 10); this module evaluates it on
an MPS, so it reaches the n = 32, depth 24, chi = 256 workload.

Recording.  In an ascending time step no gate touches sites left of its own
left site once it has been applied, so Phi_g (sites 0..s) is the prefix 0..s
of the state at the end of that time step: one prefix per time step is
recorded (record_prefixes).

Replay.  The replayed state R is an MPS in no particular gauge.  At gate g:
  1. theta' = M_g (R_s R_{s+1}), split again exactly by a QR (no truncation);
  2. P_g: with L_R the (4^{s+1} x r) matrix of sites 0..s of R,
     P_g R = Phi_g (Phi_g^dagger L_R) (rest), so sites 0..s of R become the
     recorded prefix and X = Phi_g^dagger L_R (k x r) is absorbed into site s+1.
X is an overlap of two MPS over sites 0..s.  After the first gate of a time
step, sites 0..s-2 of R already are that step's recorded prefix (set by the
previous projection of the same step), whose tensors are isometries, so the
overlap starts from the identity at bond s-2 and only sites s-1, s are
contracted: O(chi^3) per gate, one full overlap per time step.
"""
from __future__ import annotations

import numpy as np

from .gates import PAULI, dual_vector
from .mpo import MPO


def record_prefixes(n, superops, layers, chi_max, cutoff, basis="pauli"):
    """Forward truncated run (mpo.py, ascending order); per time step the site
    tensors 0..last of the state after its last gate (the frozen prefix) and the
    final MPO."""
    m = MPO(n, basis)
    prefixes = []
    g = 0
    for layer in layers:
        for s in layer:
            m.apply_gate(s, superops[g], chi_max, cutoff)
            g += 1
        last = layer[-1]
        prefixes.append([m.A[q].copy() for q in range(last + 1)])
    return prefixes, m


def _overlap_step(env, phi, r):
    """E'[a', b'] = sum_{a, I, b} conj(phi[a, I, a']) E[a, b] r[b, I, b'],
    as two matrix products: T = E r over b, then phi^dagger T over (a, I)."""
    a, d, x = phi.shape
    b, _, y = r.shape
    t = (env @ r.reshape(b, d * y)).reshape(a * d, y)
    return phi.reshape(a * d, x).conj().T @ t


def frozen_replay_value(n, superops, layers, prefixes, basis="pauli") -> complex:
    """O = sum_i Tr[Z_i rho_D] of the frozen linear map at the given
    (possibly perturbed) superoperators."""
    R = [a.copy() for a in MPO(n, basis).A]
    g = 0
    for t, layer in enumerate(layers):
        pre = prefixes[t]
        for j, s in enumerate(layer):
            # 1. noisy gate, exact split
            a, b = R[s], R[s + 1]
            chil, chir = a.shape[0], b.shape[2]
            th = (a.reshape(chil * 4, -1) @ b.reshape(b.shape[0], 4 * chir)).reshape(chil, 16, chir)
            th = np.einsum("ij,ajc->aic", np.asarray(superops[g]), th, optimize=True)
            q, r = np.linalg.qr(th.reshape(chil * 4, 4 * chir))
            R[s] = q.reshape(chil, 4, q.shape[1])
            R[s + 1] = r.reshape(r.shape[0], 4, chir)
            # 2. frozen projection onto the recorded prefix 0..s
            if j == 0:
                q0, env = 0, np.ones((1, 1), dtype=np.complex128)
            else:
                q0 = layer[j - 1] + 1          # sites 0..q0-1 already are the prefix
                env = np.eye(pre[q0 - 1].shape[2], dtype=np.complex128)
            for q in range(q0, s + 1):
                env = _overlap_step(env, pre[q], R[q])
            for q in range(s + 1):
                R[q] = pre[q]
            b1, d1, c1 = R[s + 1].shape
            R[s + 1] = (env @ R[s + 1].reshape(b1, d1 * c1)).reshape(env.shape[0], d1, c1)
            g += 1
    t_vec = dual_vector(PAULI[0], basis)
    z_vec = dual_vector(PAULI[3], basis)
    # <w|rho> = sum_i Tr[Z_i rho]: left environments with the trace vector, one
    # Z insertion per site, closed by right environments with the trace vector
    right = [None] * (n + 1)
    right[n] = np.ones(1, dtype=np.complex128)
    for s in range(n - 1, -1, -1):
        right[s] = np.einsum("aIb,I,b->a", R[s], t_vec, right[s + 1])
    left = np.ones(1, dtype=np.complex128)
    total = 0.0 + 0.0j
    for s in range(n):
        zl = np.einsum("a,aIb,I->b", left, R[s], z_vec)
        total += complex(zl @ right[s + 1])
        left = np.einsum("a,aIb,I->b", left, R[s], t_vec)
    return total
