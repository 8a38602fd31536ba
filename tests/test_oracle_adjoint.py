"""Pins for the frozen-projector reference gradient (oracle/adjoint.py).

Fixed by: the forward MPO evolution itself (the frozen linear map reproduces
the truncated state), the Euler identity of a map that is linear in each M_g,
exact central finite differences of the frozen map (linear, so they agree to
rounding), and the chain rule for the noise rate p of Sec. II.B.
"""
import numpy as np
import pytest

import mpo_inputs as mi
from oracle import adjoint, gates, mpo


def setup(n, depth, p, chi, seed, basis="pauli"):
    draws = mi.ginibre_draws(n, depth, seed=seed)
    sup = gates.circuit_superops(draws, p, basis)
    layers = mi.brickwork_sites(n, depth)
    sites, phis, m = adjoint.record_forward(n, sup, layers, chi, 1e-12, basis)
    return draws, sup, layers, sites, phis, m


@pytest.mark.parametrize("basis", ["pauli", "computational"])
def test_frozen_map_reproduces_forward(basis):
    n, depth, p, chi = 6, 5, 0.03, 6          # truncation active (exact needs 64)
    _, sup, _, sites, phis, m = setup(n, depth, p, chi, 3, basis)
    O = adjoint.frozen_value(n, sup, sites, phis, basis)
    z = m.expect_z_all() * m.trace().real
    assert abs(O - z.sum()) < 1e-12
    assert abs(O.imag) < 1e-12


def test_euler_identity_and_finite_differences():
    n, depth, p, chi = 6, 4, 0.02, 5
    _, sup, _, sites, phis, _ = setup(n, depth, p, chi, 7)
    O, grads = adjoint.frozen_gradient(n, sup, sites, phis)
    for g in range(len(sites)):
        assert abs(np.sum(sup[g] * grads[g]) - O) < 1e-12 * max(1.0, abs(O))
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(12):
        g = int(rng.integers(len(sites)))
        i, j = (int(x) for x in rng.integers(0, 16, 2))
        plus, minus = sup.copy(), sup.copy()
        plus[g, i, j] += h
        minus[g, i, j] -= h
        fd = (adjoint.frozen_value(n, plus, sites, phis) - adjoint.frozen_value(n, minus, sites, phis)) / (2 * h)
        assert abs(fd - grads[g, i, j]) < 1e-8 * max(1.0, abs(grads[g, i, j]))


def test_gradient_in_p_by_chain_rule():
    n, depth, p, chi = 6, 4, 0.05, 8
    draws, sup, _, sites, phis, _ = setup(n, depth, p, chi, 11)
    _, grads = adjoint.frozen_gradient(n, sup, sites, phis)
    us = gates.circuit_unitaries(draws)
    # dM/dp = (dS_N/dp) S_U, with dS_N/dp = (16/15)(-1 + t t^T / 4) (Sec. II.B second form)
    dsn = (gates.depolarizing_superop(1.0) - gates.depolarizing_superop(0.0)) / 1.0
    dO_dp = sum(np.sum(grads[g] * gates.to_pauli_basis(dsn @ gates.unitary_superop(us[g])))
                for g in range(len(sites)))
    h = 1e-6
    def O_at(q):
        s = np.stack([gates.to_pauli_basis(gates.noisy_gate_superop(u, q)) for u in us])
        return adjoint.frozen_value(n, s, sites, phis)
    fd = (O_at(p + h) - O_at(p - h)) / (2 * h)
    assert abs(fd - dO_dp) < 1e-7 * max(1.0, abs(dO_dp))
    assert abs(dO_dp.imag) < 1e-12


def test_one_gate_dO_dp_closed_form():
    # n = 2, one gate on |00>, no truncation: O = Tr[(Z1 + Z2) N(U rho U^dag)]
    # = (1 - 16p/15)(<Z1>_U + <Z2>_U), so dO/dp = -(16/15)(<Z1>_U + <Z2>_U)
    draws = mi.ginibre_draws(2, 1, seed=4)
    u = gates.haar_unitary(draws[0, 0], draws[0, 1])
    p = 0.1
    sup = gates.to_pauli_basis(gates.noisy_gate_superop(u, p))[None]
    sites, phis, _ = adjoint.record_forward(2, sup, [[0]], 16, 1e-14)
    _, grads = adjoint.frozen_gradient(2, sup, sites, phis)
    dsn = gates.depolarizing_superop(1.0) - gates.depolarizing_superop(0.0)
    dO_dp = np.sum(grads[0] * gates.to_pauli_basis(dsn @ gates.unitary_superop(u)))
    psi = u[:, 0]
    z1 = abs(psi[0]) ** 2 + abs(psi[1]) ** 2 - abs(psi[2]) ** 2 - abs(psi[3]) ** 2
    z2 = abs(psi[0]) ** 2 - abs(psi[1]) ** 2 + abs(psi[2]) ** 2 - abs(psi[3]) ** 2
    assert abs(dO_dp - (-16 / 15) * (z1 + z2)) < 1e-12
