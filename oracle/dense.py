"""Brute-force dense evolution (test infrastructure only).

The plain definition the MPO method approximates: rho_D is the product of
the noisy gates applied to |0..0><0..0| (Sec. II.A), and every observable is
a function of rho_D.  Qubit 0 is the most significant bit of a basis index.
"""
from __future__ import annotations

import numpy as np

from .gates import PAULI


def initial_rho(n: int) -> np.ndarray:
    rho = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    rho[0, 0] = 1.0
    return rho


def apply_superop(rho: np.ndarray, n: int, s: int, m: np.ndarray) -> np.ndarray:
    """Apply a 16x16 computational-basis superoperator to qubits (s, s+1)."""
    t = rho.reshape((2,) * (2 * n))
    axes = [s, n + s, s + 1, n + s + 1]          # i_s, i'_s, i_{s+1}, i'_{s+1}
    t = np.moveaxis(t, axes, [0, 1, 2, 3])
    shp = t.shape
    t = (m @ t.reshape(16, -1)).reshape(shp)
    t = np.moveaxis(t, [0, 1, 2, 3], axes)
    return t.reshape(2 ** n, 2 ** n)


def embed(op2: np.ndarray, n: int, s: int) -> np.ndarray:
    """Full 2^n matrix of a two-qubit operator acting on qubits (s, s+1)."""
    return np.kron(np.kron(np.eye(2 ** s), op2), np.eye(2 ** (n - s - 2)))


def apply_noisy_gate_kraus(rho: np.ndarray, n: int, s: int, u: np.ndarray,
                           p: float) -> np.ndarray:
    """U rho U^dagger, then N2[p] in its first (Pauli-sum) form (Sec. II.B):
    (1-p) rho + p/15 sum_{P != II} P rho P.  Independent of any superoperator."""
    uf = embed(u, n, s)
    rho = uf @ rho @ uf.conj().T
    out = (1.0 - p) * rho
    for a in range(4):
        for b in range(4):
            if a == 0 and b == 0:
                continue
            pf = embed(np.kron(PAULI[a], PAULI[b]), n, s)
            out = out + (p / 15.0) * (pf @ rho @ pf)
    return out


def interleaved_vec(rho: np.ndarray, n: int) -> np.ndarray:
    """vec(rho) with site-major index (i_0 i'_0)(i_1 i'_1)... (Sec. III.A)."""
    t = rho.reshape((2,) * (2 * n))
    order = [k for s in range(n) for k in (s, n + s)]
    return t.transpose(order).reshape(-1)


def schmidt_values(rho: np.ndarray, n: int, bond: int) -> np.ndarray:
    """Singular values of vec(rho) across the cut after site `bond` (0-based)."""
    v = interleaved_vec(rho, n).reshape(4 ** (bond + 1), 4 ** (n - bond - 1))
    return np.linalg.svd(v, compute_uv=False)


def entropy_from_values(lam: np.ndarray) -> float:
    """MPO entanglement entropy (Sec. III.C): -sum w log2 w, w = lam^2/sum lam^2,
    with 0 log 0 = 0."""
    w = np.asarray(lam, dtype=np.float64) ** 2
    tot = w.sum()
    if tot <= 0.0:
        return 0.0
    w = w / tot
    w = w[w > 0.0]
    return float(-(w * np.log2(w)).sum())


def bond_entropies(rho: np.ndarray, n: int) -> np.ndarray:
    return np.array([entropy_from_values(schmidt_values(rho, n, b)) for b in range(n - 1)])


def expect_z(rho: np.ndarray, n: int) -> np.ndarray:
    """Tr[Z_i rho] / Tr[rho] for every qubit."""
    diag = np.real(np.diag(rho))
    tr = diag.sum()
    out = np.empty(n)
    for i in range(n):
        signs = np.array([1.0 - 2.0 * ((x >> (n - 1 - i)) & 1) for x in range(2 ** n)])
        out[i] = float((signs * diag).sum() / tr)
    return out


def run_dense(n: int, depth: int, superops: np.ndarray, layers: list[list[int]]):
    """Dense evolution with per-layer S_b, <Z_i>, Tr rho.  superops are in the
    computational basis and in schedule order."""
    rho = initial_rho(n)
    g = 0
    s_hist, z_hist, tr_hist = [], [], []
    for sites in layers:
        for s in sites:
            rho = apply_superop(rho, n, s, superops[g])
            g += 1
        s_hist.append(bond_entropies(rho, n))
        z_hist.append(expect_z(rho, n))
        tr_hist.append(float(np.real(np.trace(rho))))
    return rho, np.array(s_hist), np.array(z_hist), np.array(tr_hist)


# ----------------------------------------------------------------- pure states
def run_statevector(n: int, unitaries: np.ndarray, layers: list[list[int]]):
    """Noiseless evolution of |0..0> (p = 0), returning psi after every layer."""
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    g = 0
    out = []
    for sites in layers:
        for s in sites:
            t = psi.reshape(2 ** s, 4, 2 ** (n - s - 2))
            psi = np.einsum("ij,ajb->aib", unitaries[g], t).reshape(-1)
            g += 1
        out.append(psi.copy())
    return out


def vn_entropy_cut(psi: np.ndarray, n: int, bond: int) -> float:
    """Von Neumann entropy (bits) of qubits 0..bond of a pure state."""
    sv = np.linalg.svd(psi.reshape(2 ** (bond + 1), 2 ** (n - bond - 1)), compute_uv=False)
    p = sv ** 2
    p = p[p > 0]
    p = p / p.sum()
    return float(-(p * np.log2(p)).sum())
