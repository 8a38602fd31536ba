"""torch.autograd.Function around mpo_adjoint_brickwork.

BrickworkObservable.apply(superops, n, depth, chi_max, cutoff, precision, basis)
returns O = sum_i Tr[Z_i rho_D] of the brickwork (Sec. II.A / IV.A) driven by
the given gate superoperators.  Its backward uses the library's hand-written
adjoint with the truncation projectors frozen at the forward point, so the
gradient is that of the linear map rho -> P_G M_G ... P_1 M_1 rho.  Build the
superoperators from parameters in torch (e.g. noisy_gate_superops_pauli) and
torch's own chain rule gives dO/dp.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Mpo, build_superop


class BrickworkObservable(torch.autograd.Function):
    @staticmethod
    def forward(ctx, superops, n, depth, chi_max, cutoff=1e-12, precision="fp64", basis="pauli"):
        sup = superops.detach().cpu().numpy()
        state = Mpo(n, chi_max, precision, basis)
        O, grads, _ = state.adjoint_brickwork(depth, sup.astype(np.complex128), chi_max, cutoff)
        state.close()
        ctx.is_complex = superops.is_complex()
        g = torch.from_numpy(grads)
        ctx.save_for_backward(g if ctx.is_complex else g.real.contiguous())
        return torch.tensor(O, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        # O = sum M * G is linear in M; for complex M torch wants conj(dO/dM)
        gm = g.conj() if ctx.is_complex else g
        return grad_out * gm, None, None, None, None, None, None


def unitary_ptms(draws: np.ndarray) -> torch.Tensor:
    """Pauli transfer matrices (real 16x16) of the Haar unitaries of each draw."""
    out = np.stack([build_superop(d[0], d[1], 0.0, "pauli")[0].real for d in draws])
    return torch.from_numpy(out)


def noisy_gate_superops_pauli(unitary_ptm: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    """M = N2[p] . U in the Pauli basis: N2[p] is diag(1, 1-16p/15, ...) (Sec. II.B)."""
    q = 16.0 * p / 15.0
    diag = torch.cat([torch.ones(1, dtype=torch.float64), (1.0 - q) * torch.ones(15, dtype=torch.float64)])
    return diag[None, :, None] * unitary_ptm
