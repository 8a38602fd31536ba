"""QR-centre-move + local truncated-SVD MPO simulator (test infrastructure only).

The density matrix is vectorised site by site (Sec. III.A) and held as an MPS
with physical dimension 4 (the MPO of Eq. "MPO"): A[s] has shape
(chi_{s-1}, 4, chi_s), outer bonds of dimension 1.  The state is kept in the
mixed canonical form: sites left of the centre are left isometries, sites
right of it are right isometries.  A noisy gate on (s, s+1) is applied the way
the "Note added" describes: move the centre to s by QR/LQ steps (no
truncation), contract the two sites, apply the 16x16 superoperator, split by a
truncated SVD.  Because both environments are orthonormal, that SVD is the
Schmidt decomposition of the whole state at bond s, which is what the paper's
global update (App. A) truncates as well.

Truncation rule (App. A keeps the largest chi singular values; a relative
cutoff is added): keep alpha iff alpha < chi_max and
lambda_alpha / ||lambda||_2 > cutoff, with the 2-norm over the full
pre-truncation spectrum, and keep at least one value.  No renormalisation:
Tr rho drops, which is the diagnostic of Sec. III.D.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.linalg

from .gates import PAULI, dual_vector, site_vector
from .dense import entropy_from_values


@dataclasses.dataclass
class TruncInfo:
    kept: int
    discarded_weight: float
    total_weight: float
    entropy: float


def svd(mat: np.ndarray):
    """Thin SVD: LAPACK gesdd, falling back to gesvd if it does not converge."""
    try:
        return np.linalg.svd(mat, full_matrices=False)
    except np.linalg.LinAlgError:
        return scipy.linalg.svd(mat, full_matrices=False, lapack_driver="gesvd")


def truncation_count(lam: np.ndarray, chi_max: int, cutoff: float) -> int:
    """Number of singular values kept (sorted descending input)."""
    norm = float(np.sqrt(np.sum(lam.astype(np.float64) ** 2)))
    if norm == 0.0:
        return 1
    k = int(np.count_nonzero(lam / norm > cutoff))
    return max(1, min(k, chi_max))


class MPO:
    """Vectorised density matrix in mixed canonical form."""

    def __init__(self, n: int, basis: str = "pauli", bits=None):
        if n < 2 or n % 2:
            raise ValueError("n must be even and >= 2 (Sec. II.A)")
        if basis not in ("pauli", "computational"):
            raise ValueError(basis)
        self.n = n
        self.basis = basis
        self.init_product(bits)

    # ------------------------------------------------------------- state setup
    def init_product(self, bits=None):
        """|x><x| product state, bond dimension 1 everywhere (Sec. IV.A uses x=0)."""
        bits = [0] * self.n if bits is None else list(bits)
        if len(bits) != self.n:
            raise ValueError("bits must have n entries")
        self.A = []
        for b in bits:
            op = np.zeros((2, 2), dtype=np.complex128)
            op[b, b] = 1.0
            self.A.append(site_vector(op, self.basis).reshape(1, 4, 1))
        self.centre = 0

    @classmethod
    def from_tensors(cls, tensors, basis="pauli"):
        """MPS from arbitrary tensors; brought into canonical form with centre 0."""
        obj = cls.__new__(cls)
        obj.n = len(tensors)
        obj.basis = basis
        obj.A = [np.array(t, dtype=np.complex128) for t in tensors]
        obj.centre = obj.n - 1
        obj.move_centre(0)
        return obj

    @classmethod
    def from_dense(cls, rho: np.ndarray, n: int, basis: str = "pauli"):
        """Exact MPO of a dense 2^n x 2^n operator by successive SVDs."""
        from .dense import interleaved_vec
        from .gates import pauli_change
        v = interleaved_vec(rho, n).reshape((4,) * n)
        if basis == "pauli":
            w = pauli_change()
            for s in range(n):
                v = np.moveaxis(np.tensordot(w, v, axes=([1], [s])), 0, s)
        tensors = []
        rest = v.reshape(1, -1)
        for s in range(n - 1):
            chil = rest.shape[0]
            mat = rest.reshape(chil * 4, -1)
            u, lam, vh = svd(mat)
            k = max(1, int(np.count_nonzero(lam > 1e-15 * max(lam[0], 1e-300))))
            tensors.append(u[:, :k].reshape(chil, 4, k))
            rest = lam[:k, None] * vh[:k]
        tensors.append(rest.reshape(rest.shape[0], 4, 1))
        obj = cls.__new__(cls)
        obj.n, obj.basis, obj.A, obj.centre = n, basis, tensors, n - 1
        return obj

    def bond_dims(self):
        return [self.A[s].shape[2] for s in range(self.n - 1)]

    # ----------------------------------------------------------- centre moves
    def _qr_right(self, s: int):
        """Centre s -> s+1: QR of A[s] as (chi_l*4) x chi_r (Note added)."""
        a = self.A[s]
        chil, _, chir = a.shape
        q, r = np.linalg.qr(a.reshape(chil * 4, chir))
        self.A[s] = q.reshape(chil, 4, q.shape[1])
        self.A[s + 1] = np.einsum("kb,bJc->kJc", r, self.A[s + 1])

    def _lq_left(self, s: int):
        """Centre s -> s-1: LQ of A[s] as chi_l x (4*chi_r), via QR of its adjoint."""
        a = self.A[s]
        chil, _, chir = a.shape
        q, r = np.linalg.qr(a.reshape(chil, 4 * chir).conj().T)
        self.A[s] = q.conj().T.reshape(q.shape[1], 4, chir)
        self.A[s - 1] = np.einsum("aIb,bk->aIk", self.A[s - 1], r.conj().T)

    def move_centre(self, target: int):
        if not 0 <= target < self.n:
            raise ValueError("centre out of range")
        while self.centre < target:
            self._qr_right(self.centre)
            self.centre += 1
        while self.centre > target:
            self._lq_left(self.centre)
            self.centre -= 1

    # ------------------------------------------------------------ gate update
    def apply_gate(self, s: int, m: np.ndarray, chi_max: int, cutoff: float) -> TruncInfo:
        """Apply a 16x16 superoperator (in this MPO's basis) to sites (s, s+1)."""
        if not 0 <= s < self.n - 1:
            raise ValueError("site out of range")
        if chi_max < 1 or not cutoff >= 0.0:
            raise ValueError("chi_max >= 1 and cutoff >= 0 required")
        m = np.asarray(m, dtype=np.complex128)
        if not np.all(np.isfinite(m)):
            raise FloatingPointError("non-finite superoperator")
        self.move_centre(s)
        a, b = self.A[s], self.A[s + 1]
        chil, chir = a.shape[0], b.shape[2]
        theta = np.einsum("aIb,bJc->aIJc", a, b)
        theta = np.einsum("IJKL,aKLc->aIJc", m.reshape(4, 4, 4, 4), theta)
        u, lam, vh = svd(theta.reshape(chil * 4, 4 * chir))
        k = truncation_count(lam, chi_max, cutoff)
        total = float(np.sum(lam ** 2))
        kept = lam[:k]
        self.A[s] = u[:, :k].reshape(chil, 4, k)
        self.A[s + 1] = (kept[:, None] * vh[:k]).reshape(k, 4, chir)
        self.centre = s + 1
        return TruncInfo(kept=k, discarded_weight=float(np.sum(lam[k:] ** 2)),
                         total_weight=total, entropy=entropy_from_values(kept))

    # ------------------------------------------------------- canonical sweep
    def schmidt_sweep(self) -> list[np.ndarray]:
        """Singular values at every bond from a fresh canonical sweep (R8 reading:
        after each time step).  Moves the centre to n-1 by QR, then walks left
        with SVDs, which leaves the centre at 0.  No truncation."""
        self.move_centre(self.n - 1)
        out = [None] * (self.n - 1)
        for s in range(self.n - 1, 0, -1):
            a = self.A[s]
            chil, _, chir = a.shape
            u, lam, vh = svd(a.reshape(chil, 4 * chir))
            out[s - 1] = lam
            self.A[s] = vh.reshape(vh.shape[0], 4, chir)
            self.A[s - 1] = np.einsum("aIb,bk->aIk", self.A[s - 1], u * lam[None, :])
        self.centre = 0
        return out

    def bond_entropies(self) -> np.ndarray:
        return np.array([entropy_from_values(l) for l in self.schmidt_sweep()])

    # ----------------------------------------------------------- observables
    def contract_product(self, vectors) -> complex:
        """Full contraction with one 4-vector per site (Sec. III.D)."""
        env = np.ones(1, dtype=np.complex128)
        for s in range(self.n):
            env = np.einsum("a,aIb,I->b", env, self.A[s], vectors[s])
        return complex(env[0])

    def trace(self) -> complex:
        v = dual_vector(PAULI[0], self.basis)
        return self.contract_product([v] * self.n)

    def pauli_expectation(self, codes) -> complex:
        """Tr[P rho] / Tr[rho] for a Pauli string given as codes 0..3 per site."""
        vecs = [dual_vector(PAULI[c], self.basis) for c in codes]
        return self.contract_product(vecs) / self.trace()

    def expect_z_all(self) -> np.ndarray:
        out = np.empty(self.n)
        for i in range(self.n):
            codes = [0] * self.n
            codes[i] = 3
            out[i] = self.pauli_expectation(codes).real
        return out

    def to_dense(self) -> np.ndarray:
        """Dense 2^n x 2^n operator (small n only)."""
        from .gates import pauli_change
        v = np.ones((1, 1), dtype=np.complex128)
        for s in range(self.n):
            v = np.einsum("xa,aIb->xIb", v, self.A[s]).reshape(-1, self.A[s].shape[2])
        v = v.reshape((4,) * self.n)
        if self.basis == "pauli":
            wi = pauli_change().conj().T
            for s in range(self.n):
                v = np.moveaxis(np.tensordot(wi, v, axes=([1], [s])), 0, s)
        t = v.reshape((2, 2) * self.n)
        order = [2 * s for s in range(self.n)] + [2 * s + 1 for s in range(self.n)]
        return t.transpose(order).reshape(2 ** self.n, 2 ** self.n)


def run_brickwork(n: int, superops: np.ndarray, layers, chi_max: int, cutoff: float,
                  basis: str = "pauli", record_layers=None):
    """Brickwork evolution (Sec. IV.A): gates of a time step applied in
    ascending site order; after every recorded time step, S_b at every bond,
    <Z_i> and Tr rho.  record_layers: None = every layer, else a set of
    0-based layer indices.  Returns a dict of arrays plus the final MPO."""
    mpo = MPO(n, basis)
    g = 0
    res = {"S": [], "Z": [], "trace": [], "layers": [], "kept": [], "discarded": [],
           "gate_entropy": []}
    for t, sites in enumerate(layers):
        for s in sites:
            info = mpo.apply_gate(s, superops[g], chi_max, cutoff)
            res["kept"].append(info.kept)
            res["discarded"].append(info.discarded_weight)
            res["gate_entropy"].append(info.entropy)
            g += 1
        if record_layers is None or t in record_layers:
            res["S"].append(mpo.bond_entropies())
            res["Z"].append(mpo.expect_z_all())
            res["trace"].append(mpo.trace().real)
            res["layers"].append(t)
    for key in res:
        res[key] = np.array(res[key])
    res["mpo"] = mpo
    return res
