"""Pins of the oracle's output probabilities and sampler (Sec. III.D) against
the plain definition P(x) = Tr[|x><x| rho] on dense states, the total
probability, closed-form product states and the distribution of the draws."""
import numpy as np
import pytest

import mpo_inputs as mi
from oracle import dense, gates, mpo as omp, sampling

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _circuit(n, depth, p, basis, chi=256, cutoff=1e-12, seed=3):
    draws = mi.ginibre_draws(n, depth, seed=seed)
    sup = gates.circuit_superops(draws, p, basis)
    return omp.run_brickwork(n, sup, mi.brickwork_sites(n, depth), chi, cutoff, basis,
                             record_layers=set())["mpo"], draws


def _index(bits):
    return int("".join(str(int(b)) for b in bits), 2)


@pytest.mark.parametrize("basis", ["pauli", "computational"])
def test_probability_is_the_dense_diagonal(basis):
    n, depth, p = 6, 5, 0.03
    m, draws = _circuit(n, depth, p, basis)
    rho, _, _, _ = dense.run_dense(n, depth, gates.circuit_superops(draws, p, "computational"),
                                   mi.brickwork_sites(n, depth))
    for x in range(2 ** n):
        bits = [(x >> (n - 1 - k)) & 1 for k in range(n)]
        assert abs(sampling.output_probability(m, bits) - rho[x, x]) <= 1e-13


def test_probabilities_sum_to_the_trace_under_truncation():
    n = 8
    m, _ = _circuit(n, 6, 0.01, "pauli", chi=6)
    tot = sum(sampling.output_probability(m, [(x >> (n - 1 - k)) & 1 for k in range(n)])
              for x in range(2 ** n))
    tr = m.trace()
    assert tr.real < 1.0 - 1e-6          # truncation removed weight
    assert abs(tot - tr) <= 1e-12


def test_product_state_samples_are_deterministic():
    bits0 = [1, 0, 0, 1, 1, 0]
    for basis in ("pauli", "computational"):
        m = omp.MPO(6, basis, bits=bits0)
        u = mi.sampling_uniforms(50, 6, seed=1)
        bits, probs, clamped = sampling.sample(m, u)
        assert (bits == np.array(bits0)).all()
        assert np.allclose(probs, 1.0, atol=1e-14)
        assert clamped == 0


def test_sample_probabilities_match_the_contraction():
    m, _ = _circuit(6, 4, 0.02, "pauli")
    bits, probs, _ = sampling.sample(m, mi.sampling_uniforms(40, 6, seed=2))
    for b, pr in zip(bits, probs):
        assert abs(pr - sampling.output_probability(m, b).real) <= 1e-14


def test_first_dit_follows_its_marginal():
    # inverse-CDF rule: over a fine grid of u for the first site, the share of
    # draws giving x_1 = 0 is P(x_1 = 0) / Tr rho
    n = 4
    m, _ = _circuit(n, 4, 0.02, "pauli")
    grid = (np.arange(2000) + 0.5) / 2000
    u = np.full((grid.size, n), 0.5)
    u[:, 0] = grid
    bits, _, _ = sampling.sample(m, u)
    p0 = sum(sampling.output_probability(m, [0] + [(x >> (n - 2 - k)) & 1 for k in range(n - 1)])
             for x in range(2 ** (n - 1))).real / m.trace().real
    assert abs(np.mean(bits[:, 0] == 0) - p0) <= 1.0 / grid.size


def test_sampled_strings_follow_the_output_distribution():
    n, ns = 4, 20000
    m, _ = _circuit(n, 4, 0.02, "pauli")
    bits, _, _ = sampling.sample(m, mi.sampling_uniforms(ns, n, seed=5))
    freq = np.bincount([_index(b) for b in bits], minlength=2 ** n) / ns
    exact = np.array([sampling.output_probability(m, [(x >> (n - 1 - k)) & 1 for k in range(n)]).real
                      for x in range(2 ** n)]) / m.trace().real
    # total-variation distance; its spread over 16 outcomes at 20000 draws is about 0.01
    assert 0.5 * np.abs(freq - exact).sum() <= 0.03
