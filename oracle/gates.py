"""Gate construction for the oracle (test infrastructure only).

Conventions:
  * two-qubit basis index 2*i1 + i2, the left qubit of the pair is the more
    significant one;
  * vectorised single-site index I = 2*i + i' for |i><i'| (Sec. III.A,
    merged index I_l = d*i_l + i'_l with d = 2);
  * superoperator element M[4*I1 + I2, 4*J1 + J2] =
    <i1 i2| M(|j1 j2><j1' j2'|) |i1' i2'>  (App. A, definition of M).
"""
from __future__ import annotations

import numpy as np

PAULI = np.array([
    [[1, 0], [0, 1]],
    [[0, 1], [1, 0]],
    [[0, -1j], [1j, 0]],
    [[1, 0], [0, -1]],
], dtype=np.complex128)


def haar_unitary(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Haar-random U(4) from one complex Ginibre draw.

    The paper samples Haar-random 4x4 unitaries (Sec. IV.A) without naming a
    method; this is QR of (re + i im)/sqrt(2) with the phases of R's diagonal
    moved into Q (Mezzadri, Notices AMS 54, 2007).
    """
    z = (np.asarray(re) + 1j * np.asarray(im)) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def unitary_superop(u: np.ndarray) -> np.ndarray:
    """Computational-basis superoperator of rho -> U rho U^dagger (App. A).

    M[(i1 i1')(i2 i2'), (j1 j1')(j2 j2')] = U[i1 i2, j1 j2] * conj(U[i1' i2', j1' j2']).
    """
    u4 = np.asarray(u, dtype=np.complex128).reshape(2, 2, 2, 2)  # [i1,i2,j1,j2]
    s = np.einsum("abcd,efgh->aebfcgdh", u4, u4.conj())
    return s.reshape(16, 16)


def depolarizing_superop(p: float) -> np.ndarray:
    """Computational-basis superoperator of N2[p] in its second form (Sec. II.B):
    rho -> (1 - 16p/15) rho + (16p/15) (I x I / 4) Tr rho."""
    q = 16.0 * p / 15.0
    t = np.zeros(16, dtype=np.complex128)
    for i1 in range(2):
        for i2 in range(2):
            t[4 * (2 * i1 + i1) + (2 * i2 + i2)] = 1.0
    return (1.0 - q) * np.eye(16, dtype=np.complex128) + (q / 4.0) * np.outer(t, t)


def noisy_gate_superop(u: np.ndarray, p: float) -> np.ndarray:
    """M = N2[p] . U, the unitary first and then the noise (Sec. III.B)."""
    return depolarizing_superop(p) @ unitary_superop(u)


def pauli_change() -> np.ndarray:
    """W[P, 2i+i'] = conj(sigma_P[i,i'])/sqrt(2): coefficients of an operator in
    the orthonormal basis sigma_P/sqrt(2) (Hilbert-Schmidt inner product)."""
    w = np.zeros((4, 4), dtype=np.complex128)
    for p in range(4):
        for i in range(2):
            for ip in range(2):
                w[p, 2 * i + ip] = np.conj(PAULI[p, i, ip]) / np.sqrt(2.0)
    return w


def to_pauli_basis(m: np.ndarray) -> np.ndarray:
    """(W x W) M (W x W)^dagger for a two-site superoperator."""
    ww = np.kron(pauli_change(), pauli_change())
    return ww @ m @ ww.conj().T


def site_vector(op: np.ndarray, basis: str) -> np.ndarray:
    """Coefficients of a single-qubit operator in the site basis."""
    flat = np.asarray(op, dtype=np.complex128).reshape(4)  # index 2i+i'
    if basis == "computational":
        return flat.copy()
    if basis == "pauli":
        return pauli_change() @ flat
    raise ValueError(basis)


def dual_vector(op: np.ndarray, basis: str) -> np.ndarray:
    """v[J] = Tr[op * B_J] for the site basis operators B_J, so that
    Tr[(op_1 x ... x op_n) rho] = contraction of the MPO with these vectors."""
    op = np.asarray(op, dtype=np.complex128)
    if basis == "computational":
        # B_{2i+i'} = |i><i'|  ->  Tr[op |i><i'|] = op[i', i]
        return np.array([op[ip, i] for i in range(2) for ip in range(2)])
    if basis == "pauli":
        return np.array([np.trace(op @ PAULI[p]) / np.sqrt(2.0) for p in range(4)])
    raise ValueError(basis)


def circuit_superops(draws: np.ndarray, p: float, basis: str = "pauli") -> np.ndarray:
    """All noisy-gate superoperators of a circuit, schedule order: (G,16,16)."""
    out = np.empty((draws.shape[0], 16, 16), dtype=np.complex128)
    for g in range(draws.shape[0]):
        m = noisy_gate_superop(haar_unitary(draws[g, 0], draws[g, 1]), p)
        out[g] = to_pauli_basis(m) if basis == "pauli" else m
    return out


def circuit_unitaries(draws: np.ndarray) -> np.ndarray:
    return np.stack([haar_unitary(d[0], d[1]) for d in draws])
