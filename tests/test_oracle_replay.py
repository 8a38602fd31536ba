"""Pins for the frozen-projector replay in MPS form (oracle/replay.py).

Fixed by: the forward truncated run itself (at the forward superoperators the
frozen map reproduces sum_i Tr[Z_i rho_D] of the truncated state), the dense
frozen map of oracle/adjoint.py at perturbed superoperators (an independent
construction: explicit projectors on 4^(s+1)-dimensional left spaces), and
exactness of central differences of a map that is linear in each M_g (checked
against the dense co-state gradient).
"""
import numpy as np
import pytest

import mpo_inputs as mi
from oracle import adjoint, gates, replay


def _setup(n, depth, p, chi, seed, basis="pauli"):
    draws = mi.ginibre_draws(n, depth, seed=seed)
    sup = gates.circuit_superops(draws, p, basis)
    layers = mi.brickwork_sites(n, depth)
    return draws, sup, layers


@pytest.mark.parametrize("basis", ["pauli", "computational"])
def test_replay_reproduces_forward(basis):
    n, depth, p, chi = 8, 6, 0.03, 8          # truncation active (exact needs 256)
    _, sup, layers = _setup(n, depth, p, chi, 21, basis)
    prefixes, m = replay.record_prefixes(n, sup, layers, chi, 1e-12, basis)
    assert max(m.bond_dims()) == chi
    O = replay.frozen_replay_value(n, sup, layers, prefixes, basis)
    want = float(np.sum(m.expect_z_all()) * m.trace().real)
    assert abs(O - want) < 1e-12 * max(1.0, abs(want))


def test_replay_equals_dense_frozen_map_off_the_forward_point():
    n, depth, p, chi = 6, 5, 0.02, 5
    _, sup, layers = _setup(n, depth, p, chi, 5)
    prefixes, _ = replay.record_prefixes(n, sup, layers, chi, 1e-12)
    sites, phis, _ = adjoint.record_forward(n, sup, layers, chi, 1e-12)
    rng = np.random.default_rng(3)
    for _ in range(3):
        pert = sup + 0.05 * (rng.standard_normal(sup.shape) + 1j * rng.standard_normal(sup.shape))
        got = replay.frozen_replay_value(n, pert, layers, prefixes)
        want = adjoint.frozen_value(n, pert, sites, phis)
        assert abs(got - want) < 1e-12 * max(1.0, abs(want))


def test_replay_central_differences_match_dense_gradient():
    n, depth, p, chi = 6, 4, 0.02, 6
    _, sup, layers = _setup(n, depth, p, chi, 9)
    prefixes, _ = replay.record_prefixes(n, sup, layers, chi, 1e-12)
    sites, phis, _ = adjoint.record_forward(n, sup, layers, chi, 1e-12)
    _, grads = adjoint.frozen_gradient(n, sup, sites, phis)
    dirs = mi.gradient_directions(len(sup), 3, seed=1)
    h = 1e-6
    for d in dirs:
        fd = (replay.frozen_replay_value(n, sup + h * d, layers, prefixes)
              - replay.frozen_replay_value(n, sup - h * d, layers, prefixes)) / (2 * h)
        want = np.sum(grads * d)
        assert abs(fd - want) < 1e-8 * max(1.0, abs(want))


def test_gradient_directions_are_unit_and_seeded():
    a = mi.gradient_directions(10, 3, seed=4)
    b = mi.gradient_directions(10, 3, seed=4)
    assert a.shape == (3, 10, 16, 16) and np.array_equal(a, b)
    assert np.allclose(np.sum(a * a, axis=(1, 2, 3)), 1.0)
