"""The paper's global canonical update (App. A), test infrastructure only.

The vectorised state is held in the Gamma-lambda canonical form (Sec. III.A,
Eq. "MPO canonical form").  A noisy gate on sites (s, s+1) (0-based; the
paper's l = s+1) forms B = M (lambda Gamma lambda Gamma lambda), takes its
SVD, keeps the top values (same rule as mpo.py), and then restores the global
canonical form with SVD sweeps to the left (B_<-) and to the right (B_->),
dividing by the new lambda to recover Gamma (App. A, bulk and edge cases).
Used only to cross-check the QR-centre variant: both give the same truncated
state in exact arithmetic.  Singular values below `drop` relative to the
largest are removed before any division, since Gamma = W / lambda' is
undefined for zero lambda'.
"""
from __future__ import annotations

import numpy as np

from .gates import site_vector
from .mpo import svd, truncation_count, TruncInfo
from .dense import entropy_from_values


class VidalMPO:
    def __init__(self, n: int, basis: str = "pauli", drop: float = 1e-14):
        self.n, self.basis, self.drop = n, basis, drop
        op = np.zeros((2, 2), dtype=np.complex128)
        op[0, 0] = 1.0
        v = site_vector(op, basis)
        self.G = [v.reshape(1, 4, 1).copy() for _ in range(n)]
        self.lam = [np.ones(1) for _ in range(n - 1)]

    def _l(self, b: int) -> np.ndarray:
        return self.lam[b] if 0 <= b < self.n - 1 else np.ones(1)

    def _split(self, mat):
        u, lam, vh = svd(mat)
        r = max(1, int(np.count_nonzero(lam > self.drop * lam[0]))) if lam[0] > 0 else 1
        return u[:, :r], lam[:r], vh[:r]

    def apply_gate(self, s: int, m: np.ndarray, chi_max: int, cutoff: float) -> TruncInfo:
        n = self.n
        ga, gb = self.G[s], self.G[s + 1]
        la, lm, lb = self._l(s - 1), self._l(s), self._l(s + 1)
        theta = np.einsum("a,aIb,b,bJc,c->aIJc", la, ga, lm, gb, lb)
        theta = np.einsum("IJKL,aKLc->aIJc", np.asarray(m).reshape(4, 4, 4, 4), theta)
        chil, chir = theta.shape[0], theta.shape[3]
        u, lam, vh = svd(theta.reshape(chil * 4, 4 * chir))
        k = truncation_count(lam, chi_max, cutoff)
        info = TruncInfo(kept=k, discarded_weight=float(np.sum(lam[k:] ** 2)),
                         total_weight=float(np.sum(lam ** 2)),
                         entropy=entropy_from_values(lam[:k]))
        # the paper divides by lambda'; drop values that are numerically zero
        k = min(k, max(1, int(np.count_nonzero(lam[:k] > self.drop * lam[0]))))
        lp, v, w = lam[:k], u[:, :k], vh[:k]
        self.lam[s] = lp
        # ---- left part: Phi'[1..s]_beta = sum V_{(a,I),beta} Phi[1..s-1]_a |I>
        if s == 0:
            self.G[0] = v.reshape(1, 4, k)
        else:
            bl = (v * lp[None, :]).reshape(chil, 4 * k)          # (B_<-)
            v2, l2, w2 = self._split(bl)
            self.G[s] = (w2.reshape(-1, 4, k)) / lp[None, None, :]
            self.lam[s - 1] = l2
            carry, lcarry = v2, l2
            for j in range(s - 1, -1, -1):
                if j == 0:
                    self.G[0] = np.einsum("xIb,ba->xIa", self.G[0], carry)
                    break
                b2 = np.einsum("a,aIb,bk,k->aIk", self._l(j - 1), self.G[j], carry, lcarry)
                chia = b2.shape[0]
                v3, l3, w3 = self._split(b2.reshape(chia, -1))
                self.G[j] = w3.reshape(-1, 4, lcarry.size) / lcarry[None, None, :]
                self.lam[j - 1] = l3
                carry, lcarry = v3, l3
        # ---- right part: Phi'[s+1..n]_beta = sum W_{beta,(J,c)} |J> Phi[s+2..n]_c
        if s + 1 == n - 1:
            self.G[n - 1] = w.reshape(k, 4, 1)
        else:
            br = (lp[:, None] * w).reshape(k * 4, chir)          # (B_->)
            v2, l2, w2 = self._split(br)
            self.G[s + 1] = v2.reshape(k, 4, -1) / lp[:, None, None]
            self.lam[s + 1] = l2
            carry, lcarry = w2, l2
            for j in range(s + 2, n):
                if j == n - 1:
                    self.G[n - 1] = np.einsum("ab,bIx->aIx", carry, self.G[n - 1])
                    break
                b2 = np.einsum("k,kb,bIc,c->kIc", lcarry, carry, self.G[j], self._l(j))
                v3, l3, w3 = self._split(b2.reshape(lcarry.size * 4, -1))
                self.G[j] = v3.reshape(lcarry.size, 4, -1) / lcarry[:, None, None]
                self.lam[j] = l3
                carry, lcarry = w3, l3
        return info

    def bond_entropies(self) -> np.ndarray:
        return np.array([entropy_from_values(l) for l in self.lam])

    def to_tensors(self):
        """Left-canonical MPS tensors A[s] = lambda[s-1] Gamma[s] (last site
        carries its own Gamma only)."""
        return [self._l(s - 1)[:, None, None] * self.G[s] for s in range(self.n)]
