"""Pins for the oracle's MPO simulator, dense evolution and the App. A cross-check.

Fixed by: brute-force dense evolution built from the Pauli-sum form of the
channel (never from a superoperator), pure-state simulation at p = 0, closed
form states the paper discusses, the Page value the paper prints, the
Hilbert-Schmidt error bound of truncation, and the paper's own global update.
"""
import json
import os

import numpy as np
import pytest

import mpo_inputs as mi
from oracle import dense, gates, mpo, vidal

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def circuit(n, depth, p, seed, basis):
    draws = mi.ginibre_draws(n, depth, seed=seed)
    return mi.brickwork_sites(n, depth), gates.circuit_superops(draws, p, basis), \
        gates.circuit_unitaries(draws)


def kraus_dense(n, layers, us, p):
    rho = dense.initial_rho(n)
    out = []
    g = 0
    for sites in layers:
        for s in sites:
            rho = dense.apply_noisy_gate_kraus(rho, n, s, us[g], p)
            g += 1
        out.append(rho.copy())
    return out


def test_dense_superop_matches_kraus():
    n, depth, p = 5 + 1, 5, 0.04
    layers, ms, us = circuit(n, depth, p, 11, "computational")
    rho, *_ = dense.run_dense(n, depth, ms, layers)
    assert np.abs(rho - kraus_dense(n, layers, us, p)[-1]).max() < 1e-14


@pytest.mark.parametrize("basis", ["pauli", "computational"])
@pytest.mark.parametrize("n,depth,p,seed", [(6, 6, 0.02, 0), (8, 8, 0.02, 0), (4, 7, 0.1, 3)])
def test_mpo_exact_regime_matches_dense(basis, n, depth, p, seed):
    # chi_max = 4^(n/2): no truncation; every S_b and <Z_i> after every layer
    layers, ms, us = circuit(n, depth, p, seed, basis)
    res = mpo.run_brickwork(n, ms, layers, 4 ** (n // 2), 1e-12, basis)
    rhos = kraus_dense(n, layers, us, p)
    s_ref = np.array([dense.bond_entropies(r, n) for r in rhos])
    z_ref = np.array([dense.expect_z(r, n) for r in rhos])
    assert np.abs(res["S"] - s_ref).max() < 1e-12
    assert np.abs(res["Z"] - z_ref).max() < 1e-12
    assert np.abs(res["trace"] - 1.0).max() < 1e-12
    assert np.abs(res["mpo"].to_dense() - rhos[-1]).max() < 1e-13


def test_bases_agree():
    n, depth, p = 6, 5, 0.05
    lp, mp_, _ = circuit(n, depth, p, 4, "pauli")
    _, mc, _ = circuit(n, depth, p, 4, "computational")
    a = mpo.run_brickwork(n, mp_, lp, 16, 1e-12, "pauli")
    b = mpo.run_brickwork(n, mc, lp, 16, 1e-12, "computational")
    assert np.abs(a["S"] - b["S"]).max() < 1e-11
    assert np.abs(a["Z"] - b["Z"]).max() < 1e-11


def test_pure_state_relation():
    # Sec. III.C: S_l(|psi><psi|) = 2 S_l(|psi>) at p = 0
    n, depth = 8, 6
    layers, ms, us = circuit(n, depth, 0.0, 21, "pauli")
    res = mpo.run_brickwork(n, ms, layers, 256, 1e-12, "pauli")
    psis = dense.run_statevector(n, us, layers)
    for t, psi in enumerate(psis):
        ref = [2 * dense.vn_entropy_cut(psi, n, b) for b in range(n - 1)]
        assert np.abs(res["S"][t] - ref).max() < 1e-11


def test_closed_form_states():
    n = 6
    dim = 2 ** n
    # product state: S = 0
    m = mpo.MPO(n)
    assert np.abs(m.bond_entropies()).max() < 1e-14
    # GHZ (Sec. III.B): MPS Schmidt values 1/sqrt2, MPO values their products
    g = np.zeros(dim, dtype=complex)
    g[0] = g[-1] = 1 / np.sqrt(2)
    lam_mps = GOLDEN["ghz_mps_lambda"]["value"]
    for basis in ("pauli", "computational"):
        mm = mpo.MPO.from_dense(np.outer(g, g.conj()), n, basis)
        for lam in mm.schmidt_sweep():
            top = np.sort(lam)[::-1][:4]
            np.testing.assert_allclose(top, [lam_mps ** 2] * 4, atol=1e-13)
            assert lam[4:].max(initial=0.0) < 1e-13
        np.testing.assert_allclose(mm.bond_entropies(), 2.0, atol=1e-12)
    # classical mixture of |00> and |11> (Sec. III.C): S = 1
    r = np.zeros((4, 4))
    r[0, 0] = r[3, 3] = 0.5
    mm = mpo.MPO.from_dense(r, 2)
    assert abs(mm.bond_entropies()[0] - GOLDEN["classical_mixture_entropy"]["value"]) < 1e-13
    # maximally mixed (Sec. III.C): S = 0 at every cut, Tr = 1, <Z> = 0
    mm = mpo.MPO.from_dense(np.eye(dim) / dim, n)
    assert np.abs(mm.bond_entropies() - GOLDEN["maximally_mixed_entropy"]["value"]).max() < 1e-12
    assert abs(mm.trace() - 1) < 1e-13
    assert np.abs(mm.expect_z_all()).max() < 1e-13


def test_one_gate_purity_closed_form():
    # rho' = (1-q) |psi><psi| + q I/4: sum lambda^2 = Tr rho'^2 in an orthonormal basis
    layers, ms, us = circuit(2, 1, 0.0, 5, "pauli")
    for p in (0.0, 0.01, 0.3):
        q = 16 * p / 15
        m = mpo.MPO(2)
        mat = gates.to_pauli_basis(gates.noisy_gate_superop(us[0], p))
        m.apply_gate(0, mat, 16, 1e-14)
        lam = m.schmidt_sweep()[0]
        purity = (1 - q) ** 2 + (1 - q) * q / 2 + q ** 2 / 4
        assert abs(np.sum(lam ** 2) - purity) < 1e-13
        if p == 0.0:
            psi = us[0][:, 0]
            assert abs(m.bond_entropies()[0] - 2 * dense.vn_entropy_cut(psi, 2, 0)) < 1e-12


def test_truncation_count_rule():
    lam = np.array([1.0, 0.5, 1e-6, 1e-13, 0.0])
    norm = np.linalg.norm(lam)
    assert mpo.truncation_count(lam, 10, 1e-12) == 3
    assert mpo.truncation_count(lam, 2, 1e-12) == 2
    assert mpo.truncation_count(lam, 10, 0.0) == 4
    assert mpo.truncation_count(lam, 10, 0.9) == 1
    assert mpo.truncation_count(np.zeros(3), 10, 1e-12) == 1
    # relative to the full-spectrum norm, strict '>'
    assert mpo.truncation_count(np.array([3.0, 4.0]), 5, 4.0 / 5.0) == 0 + 1


def test_truncation_error_bound():
    # unital channels and orthogonal projections do not increase the HS norm, so
    # ||rho_MPO - rho||_HS <= sum_g sqrt(discarded_g)
    n, depth, p = 6, 6, 0.01
    layers, ms, us = circuit(n, depth, p, 8, "pauli")
    res = mpo.run_brickwork(n, ms, layers, 6, 1e-12, "pauli")
    rho_exact = kraus_dense(n, layers, us, p)[-1]
    err = np.linalg.norm(res["mpo"].to_dense() - rho_exact)
    bound = np.sum(np.sqrt(res["discarded"]))
    assert res["discarded"].sum() > 1e-6          # truncation really active
    assert err <= bound * (1 + 1e-9)
    assert res["trace"][-1] < 1.0                  # Sec. III.D: Tr rho drops


@pytest.mark.parametrize("seed,chi", [(3, 12), (6, 20)])
def test_note_added_update_equals_appendix_a(seed, chi):
    # same lambda at every bond after every gate as the paper's global update
    n, depth = 10, 10
    layers, ms, _ = circuit(n, depth, 0.01, seed, "pauli")
    a, b = mpo.MPO(n), vidal.VidalMPO(n)
    g = 0
    for sites in layers:
        for s in sites:
            ia = a.apply_gate(s, ms[g], chi, 1e-10)
            ib = b.apply_gate(s, ms[g], chi, 1e-10)
            assert ia.kept == ib.kept
            assert abs(ia.discarded_weight - ib.discarded_weight) < 1e-12
            g += 1
            lam_a = a.schmidt_sweep()
            for bond in range(n - 1):
                la, lb = lam_a[bond], b.lam[bond]
                kk = min(la.size, lb.size)
                assert np.abs(la[:kk] - lb[:kk]).max() < 1e-11 * la[0]
                assert la[kk:].max(initial=0.0) < 1e-12 and lb[kk:].max(initial=0.0) < 1e-12


def test_invariants_under_truncation():
    n, depth = 12, 8
    layers, ms, _ = circuit(n, depth, 0.01, 2, "pauli")
    res = mpo.run_brickwork(n, ms, layers, 24, 1e-12, "pauli", record_layers={depth - 1})
    m = res["mpo"]
    lams = m.schmidt_sweep()
    w = [np.sum(l ** 2) for l in lams]
    assert np.ptp(w) < 1e-12 * w[0]               # sum lambda^2 = ||rho||_HS^2 at every bond
    rng = np.random.default_rng(0)
    for _ in range(5):                             # Hermiticity: Tr[P rho] real
        codes = rng.integers(0, 4, n)
        assert abs(m.pauli_expectation(codes).imag) < 1e-12


def test_large_depth_depolarizes():
    # Sec. IV.A: at large depth the state flows to I/2^n: S -> 0, <Z> -> 0, purity -> 2^-n
    n, depth, p = 6, 40, 0.2
    layers, ms, _ = circuit(n, depth, p, 1, "pauli")
    res = mpo.run_brickwork(n, ms, layers, 64, 1e-12, "pauli")
    assert res["S"][-1].max() < 1e-3
    assert res["S"][-1].max() < res["S"][2].max()
    assert np.abs(res["Z"][-1]).max() < 1e-3
    purity = np.sum(res["mpo"].schmidt_sweep()[0] ** 2)
    assert abs(purity * 2 ** n - 1) < 1e-2


def test_page_value_at_p0():
    # Sec. IV.A: at p = 0, n = 8 the mid-chain MPO entropy saturates at
    # 2 x S_{16,16} = 6.56 (24 circuits, large depth)
    n, depth = 8, 40
    page = sum(1.0 / k for k in range(17, 257)) - 15 / 32
    page_bits = page * np.log2(np.e)
    assert abs(page_bits - GOLDEN["page_half_chain_bits_n8"]["value"]) < 5e-3
    vals = []
    for seed in range(24):
        draws = mi.ginibre_draws(n, depth, seed=1000 + seed)
        psi = dense.run_statevector(n, gates.circuit_unitaries(draws), mi.brickwork_sites(n, depth))[-1]
        vals.append(2 * dense.vn_entropy_cut(psi, n, 3))
    assert abs(np.mean(vals) - GOLDEN["smax_p0_n8_large_depth"]["value"]) < 0.05
    # and the MPO oracle itself reaches it (two circuits, S_MPO = 2 S_vN exactly)
    for seed in range(2):
        draws = mi.ginibre_draws(n, 24, seed=1000 + seed)
        layers = mi.brickwork_sites(n, 24)
        res = mpo.run_brickwork(n, gates.circuit_superops(draws, 0.0, "pauli"), layers, 256,
                                1e-12, "pauli", record_layers={23})
        psi = dense.run_statevector(n, gates.circuit_unitaries(draws), layers)[-1]
        assert abs(res["S"][0][3] - 2 * dense.vn_entropy_cut(psi, n, 3)) < 1e-10
        assert abs(res["S"][0][3] - 6.56) < 0.3


def test_argument_errors():
    m = mpo.MPO(4)
    with pytest.raises(ValueError):
        m.apply_gate(3, np.eye(16), 4, 1e-12)
    with pytest.raises(ValueError):
        m.apply_gate(0, np.eye(16), 0, 1e-12)
    with pytest.raises(ValueError):
        m.apply_gate(0, np.eye(16), 4, float("nan"))
    with pytest.raises(FloatingPointError):
        bad = np.eye(16, dtype=complex)
        bad[0, 0] = np.inf
        m.apply_gate(0, bad, 4, 1e-12)
    with pytest.raises(ValueError):
        mpo.MPO(5)
