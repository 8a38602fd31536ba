"""Output probabilities and bit-string sampling from a vectorised MPO (test
infrastructure only; plain numpy complex128).

Sec. III.D of the paper: a computational-basis measurement of rho gives the
bit string x with probability P(x) = Tr[|x><x| rho], a contraction of the MPO
with one projector vector per site; summing over every x_l at every site gives
the total probability Tr rho, which falls below 1 under truncation.  Strings
are sampled dit by dit: the marginal of x_1 (every later site summed out), then
the conditional of x_2 given the drawn x_1, and so on, each conditional being a
ratio of two marginals.

Reading (the paper does not fix these, the GPU path follows the same rule):
- the caller supplies one uniform u in [0, 1) per site and sample; the dit
  drawn is 0 when u < P(0 | prefix) / (P(0 | prefix) + P(1 | prefix)), else 1;
- a truncated rho need not be positive, so a marginal can come out slightly
  negative: such a value is taken as 0 (and counted); if both candidates are
  0 the dit 0 is taken;
- the probability returned with a sample is P(x) of the whole string
  (unnormalised, i.e. of the truncated rho, not divided by Tr rho).
"""
from __future__ import annotations

import numpy as np

from .gates import dual_vector


def projector_vectors(basis: str):
    """Site vectors v_b with Tr[|b><b| B_J] = v_b[J], b = 0, 1, and their sum
    (the identity, which sums a site out)."""
    p0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
    p1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
    v0, v1 = dual_vector(p0, basis), dual_vector(p1, basis)
    return v0, v1, v0 + v1


def output_probability(mpo, bits) -> complex:
    """P(x) = Tr[|x><x| rho]: one vector-matrix product per site."""
    v0, v1, _ = projector_vectors(mpo.basis)
    env = np.ones(1, dtype=np.complex128)
    for s in range(mpo.n):
        env = np.einsum("a,aIb,I->b", env, mpo.A[s], v1 if bits[s] else v0)
    return complex(env[0])


def right_traces(mpo):
    """R[k][a]: sites k..n-1 contracted with the identity vector (summed
    out), R[n] = [1]."""
    _, _, vt = projector_vectors(mpo.basis)
    R = [None] * (mpo.n + 1)
    R[mpo.n] = np.ones(1, dtype=np.complex128)
    for s in range(mpo.n - 1, -1, -1):
        R[s] = np.einsum("aIb,I,b->a", mpo.A[s], vt, R[s + 1])
    return R


def sample(mpo, uniforms: np.ndarray, return_margin: bool = False):
    """Sequential conditional sampling of n_samples strings.

    uniforms: (n_samples, n) values in [0, 1).  Returns (bits (n_samples, n)
    uint8, P(x) of each sampled string, number of samples that met a negative
    marginal) and, with return_margin, per sample the smallest distance
    |u - P(0 | prefix)| over its draws (how close the sample came to a tie)."""
    u = np.asarray(uniforms, dtype=np.float64)
    ns, n = u.shape
    if n != mpo.n:
        raise ValueError("one uniform per site and sample")
    v0, v1, _ = projector_vectors(mpo.basis)
    R = right_traces(mpo)
    bits = np.zeros((ns, n), dtype=np.uint8)
    probs = np.zeros(ns)
    clamped = np.zeros(ns, dtype=bool)
    margin = np.full(ns, np.inf)
    for i in range(ns):
        env = np.ones(1, dtype=np.complex128)      # prefix contracted with its projectors
        for s in range(n):
            t0 = np.einsum("a,aIb,I->b", env, mpo.A[s], v0)
            t1 = np.einsum("a,aIb,I->b", env, mpo.A[s], v1)
            q0 = (t0 @ R[s + 1]).real                 # marginal of (prefix, 0)
            q1 = (t1 @ R[s + 1]).real                 # marginal of (prefix, 1)
            if q0 < 0.0 or q1 < 0.0:
                clamped[i] = True
            p0, p1 = max(q0, 0.0), max(q1, 0.0)
            x = 0 if (p0 + p1 == 0.0 or u[i, s] < p0 / (p0 + p1)) else 1
            if p0 + p1 > 0.0:
                margin[i] = min(margin[i], abs(u[i, s] - p0 / (p0 + p1)))
            bits[i, s] = x
            env = t1 if x else t0
        probs[i] = env[0].real
    if return_margin:
        return bits, probs, int(clamped.sum()), margin
    return bits, probs, int(clamped.sum())
