"""Reference gradient of a brickwork observable with frozen truncation projectors
(test infrastructure only).

Forward map.  The truncated MPO evolution (mpo.py) applies, at gate g on
sites (s, s+1), the noisy map M_g and then keeps the top-k left Schmidt
vectors at bond s (App. A truncation).  With the kept subspace frozen at its
forward value, that step is the linear map rho -> P_g M_g rho with
P_g = (Phi_g Phi_g^dagger) (x) 1, where the columns of Phi_g are the kept left
Schmidt vectors (the left-isometric part of the MPO, sites 0..s, after the
gate).  Exact re-gauging moves are identities.  The observable is
O = sum_i Tr[Z_i rho_D] = <w|rho_D> (unnormalised, so it is linear in rho).

Gradient.  O is linear in each M_g once the P's are frozen:
O = <lambda_g | M_g rho_{g-1}>, lambda_g = P_g mu_g, mu_{g-1} = M_g^dagger lambda_g,
mu_G = w, so dO/dM_g[IJ, KL] = sum over the other sites of
conj(lambda_g[.., I, J, ..]) rho_{g-1}[.., K, L, ..].

Everything here is a dense vector of length 4^n with the structured action of
P_g and M_g (n <= 10).
"""
from __future__ import annotations

import numpy as np

from .gates import PAULI, dual_vector
from .mpo import MPO


def mps_vector(tensors) -> np.ndarray:
    """Dense vec(rho) (index I_0 ... I_{n-1}, I_0 most significant)."""
    v = np.ones((1, 1), dtype=np.complex128)
    for a in tensors:
        v = np.einsum("xa,aIb->xIb", v, a).reshape(-1, a.shape[2])
    return v.reshape(-1)


def left_isometry(tensors, s) -> np.ndarray:
    """Sites 0..s contracted: a (4^{s+1} x chi_s) matrix."""
    v = np.ones((1, 1), dtype=np.complex128)
    for a in tensors[: s + 1]:
        v = np.einsum("xa,aIb->xIb", v, a).reshape(-1, a.shape[2])
    return v


def apply_local(vec, n, s, m):
    """M acting on the sites (s, s+1) of a dense vectorised operator."""
    t = vec.reshape(4 ** s, 16, 4 ** (n - s - 2))
    return np.einsum("ij,ajb->aib", m, t).reshape(-1)


def apply_projector(vec, n, s, phi):
    """(Phi Phi^dagger) (x) 1 with Phi acting on sites 0..s."""
    t = vec.reshape(4 ** (s + 1), -1)
    return (phi @ (phi.conj().T @ t)).reshape(-1)


def observable_vector(n, basis) -> np.ndarray:
    """w with <w|rho> = sum_i Tr[Z_i rho] (real in both bases)."""
    t = dual_vector(PAULI[0], basis)
    z = dual_vector(PAULI[3], basis)
    w = np.zeros(4 ** n, dtype=np.complex128)
    for i in range(n):
        v = np.ones(1, dtype=np.complex128)
        for j in range(n):
            v = np.kron(v, z if j == i else t)
        w += v
    return w.conj()      # stored so that <w|rho> = w.conj() @ rho = sum_i Tr[Z_i rho]


def record_forward(n, superops, layers, chi_max, cutoff, basis="pauli"):
    """Run the oracle MPO forward; return (gate sites, frozen Phi per gate, MPO)."""
    m = MPO(n, basis)
    sites, phis = [], []
    g = 0
    for layer in layers:
        for s in layer:
            m.apply_gate(s, superops[g], chi_max, cutoff)
            sites.append(s)
            phis.append(left_isometry(m.A, s))    # centre is at s+1: sites 0..s are isometries
            g += 1
    return sites, phis, m


def frozen_value(n, superops, sites, phis, basis="pauli"):
    """O of the frozen linear map for (possibly perturbed) superoperators."""
    rho = mps_vector(MPO(n, basis).A)
    for g, s in enumerate(sites):
        rho = apply_projector(apply_local(rho, n, s, superops[g]), n, s, phis[g])
    return complex(observable_vector(n, basis).conj() @ rho)


def frozen_gradient(n, superops, sites, phis, basis="pauli"):
    """(O, dO/dM_g for every gate) by the co-state recursion, dense."""
    rho = mps_vector(MPO(n, basis).A)
    rhos = [rho]
    for g, s in enumerate(sites):
        rho = apply_projector(apply_local(rho, n, s, superops[g]), n, s, phis[g])
        rhos.append(rho)
    w = observable_vector(n, basis)
    O = complex(w.conj() @ rhos[-1])
    mu = w
    grads = np.zeros((len(sites), 16, 16), dtype=np.complex128)
    for g in range(len(sites) - 1, -1, -1):
        s = sites[g]
        lam = apply_projector(mu, n, s, phis[g])
        a = lam.reshape(4 ** s, 16, 4 ** (n - s - 2))
        b = rhos[g].reshape(4 ** s, 16, 4 ** (n - s - 2))
        grads[g] = np.einsum("aib,ajb->ij", a.conj(), b)
        mu = apply_local(lam, n, s, superops[g].conj().T)
    return O, grads
