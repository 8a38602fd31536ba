"""Pins for the oracle's gate construction (Sec. II.B, Sec. III.B, App. A).

Each check is fixed by something other than the oracle's own formula: the
defining action of the channel on a density matrix, the first (Pauli-sum) form
of the depolarizing channel, CPTP structure, Haar moments.
"""
import numpy as np
import pytest

import mpo_inputs as mi
from oracle import gates

RNG = np.random.default_rng(1234)


def rand_rho(dim, rng=RNG):
    x = rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))
    r = x @ x.conj().T
    return r / np.trace(r)


def vec2(rho):
    """Two-qubit operator -> 16-vector with index 4*(2 i1 + i1') + (2 i2 + i2')."""
    t = rho.reshape(2, 2, 2, 2)          # i1 i2 i1' i2'
    return t.transpose(0, 2, 1, 3).reshape(16)


def unvec2(v):
    return v.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)


def some_unitaries(k=50, seed=7):
    draws = mi.ginibre_draws(2, 2 * k, seed=seed)[: k]
    return [gates.haar_unitary(d[0], d[1]) for d in draws]


def test_haar_unitary_is_unitary():
    for u in some_unitaries():
        assert np.abs(u.conj().T @ u - np.eye(4)).max() < 1e-14


def test_haar_moments():
    # Haar U(4): E|U_ij|^2 = 1/4, E|U_ij|^4 = 2/(d(d+1)) = 1/10, E|Tr U|^2 = 1.
    rng = np.random.Generator(np.random.PCG64(99))
    n = 20000
    a2 = a4 = tr2 = 0.0
    for _ in range(n):
        u = gates.haar_unitary(rng.standard_normal((4, 4)), rng.standard_normal((4, 4)))
        m = np.abs(u) ** 2
        a2 += m.mean()
        a4 += (m ** 2).mean()
        tr2 += abs(np.trace(u)) ** 2
    # 5-sigma bands (per-sample std: |U|^2 ~ 0.19 / sqrt(16 correlated), |Tr U|^2 ~ 1)
    assert abs(a2 / n - 0.25) < 1e-12          # exact: rows are unit vectors
    assert abs(a4 / n - 0.1) < 5 * 0.09 / np.sqrt(n)
    assert abs(tr2 / n - 1.0) < 5 * 1.0 / np.sqrt(n)
    # without the phase fix the distribution is not Haar: E[U_00] would be biased
    # toward a positive real value; with it, the mean of U_00 vanishes
    rng = np.random.Generator(np.random.PCG64(5))
    mean00 = np.mean([gates.haar_unitary(rng.standard_normal((4, 4)),
                                         rng.standard_normal((4, 4)))[0, 0] for _ in range(4000)])
    assert abs(mean00) < 5 * 0.5 / np.sqrt(4000)


def test_unitary_superop_matches_conjugation():
    # the App. A definition: M acts on vec(rho) as rho -> U rho U^dagger
    for u in some_unitaries(10):
        rho = rand_rho(4)
        got = unvec2(gates.unitary_superop(u) @ vec2(rho))
        assert np.abs(got - u @ rho @ u.conj().T).max() < 1e-14


@pytest.mark.parametrize("p", [0.0, 0.02, 0.3, 15 / 16])
def test_depolarizing_two_forms_agree(p):
    # Sec. II.B gives N2[p] twice: Pauli-sum form and depolarized form
    rho = rand_rho(4)
    kraus = (1 - p) * rho
    for a in range(4):
        for b in range(4):
            if a or b:
                pp = np.kron(gates.PAULI[a], gates.PAULI[b])
                kraus = kraus + p / 15 * pp @ rho @ pp
    got = unvec2(gates.depolarizing_superop(p) @ vec2(rho))
    assert np.abs(got - kraus).max() < 1e-14


def test_trace_preserving_and_cp():
    t = vec2(np.eye(4))
    for u in some_unitaries(10):
        for p in (0.0, 0.01, 0.2):
            m = gates.noisy_gate_superop(u, p)
            assert np.abs(t.conj() @ m - t.conj()).max() < 1e-14
            # Choi matrix sum_{J,J'} M(|j><j'|) x |j><j'| must be PSD
            choi = np.zeros((16, 16), dtype=complex)
            for j in range(4):
                for jp in range(4):
                    e = np.zeros((4, 4), dtype=complex)
                    e[j, jp] = 1
                    choi += np.kron(unvec2(m @ vec2(e)), e)
            assert np.linalg.eigvalsh(choi).min() > -1e-13


def test_pauli_basis_ptm():
    for u in some_unitaries(10):
        for p in (0.0, 0.03):
            mp = gates.to_pauli_basis(gates.noisy_gate_superop(u, p))
            assert np.abs(mp.imag).max() < 1e-14                 # PTM is real
            assert np.abs(mp[0] - np.eye(16)[0]).max() < 1e-14    # trace preserving
            assert np.abs(mp[:, 0] - np.eye(16)[:, 0]).max() < 1e-14   # unital
    p = 0.07
    q = 16 * p / 15
    np.testing.assert_allclose(gates.to_pauli_basis(gates.depolarizing_superop(p)),
                               np.diag([1.0] + [1 - q] * 15), atol=1e-15)


def test_noise_commutes_with_unitary():
    for u in some_unitaries(5):
        a = gates.depolarizing_superop(0.05) @ gates.unitary_superop(u)
        b = gates.unitary_superop(u) @ gates.depolarizing_superop(0.05)
        assert np.abs(a - b).max() < 1e-14


def test_site_vectors():
    z0 = np.diag([1.0, 0.0]).astype(complex)
    np.testing.assert_allclose(gates.site_vector(z0, "computational"), [1, 0, 0, 0])
    np.testing.assert_allclose(gates.site_vector(z0, "pauli"), np.array([1, 0, 0, 1]) / np.sqrt(2), atol=1e-16)
    # dual vectors reproduce traces of products
    rho = rand_rho(2)
    for basis in ("pauli", "computational"):
        c = gates.site_vector(rho, basis)
        for p in range(4):
            assert abs(gates.dual_vector(gates.PAULI[p], basis) @ c
                       - np.trace(gates.PAULI[p] @ rho)) < 1e-14


def test_schedule_counts():
    # Sec. II.A: n/2 gates on odd steps, n/2-1 on even steps
    assert mi.n_gates(8, 8) == 28
    assert mi.n_gates(32, 32) == 496
    assert mi.n_gates(64, 48) == 1512
    lay = mi.brickwork_sites(6, 3)
    assert lay == [[0, 2, 4], [1, 3], [0, 2, 4]]
