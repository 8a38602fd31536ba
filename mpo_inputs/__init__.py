"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds random draws and the brickwork schedule only; it performs
none of the simulation method's arithmetic (no Haar sampling step, no
superoperator, no contraction).  Both the oracle and the product build their
gates from the raw Gaussian draws produced here, each with its own code.

Workload shape (paper, Sec. II.A and Sec. IV.A): a chain of n qubits (n even),
depth D; odd time steps put a gate on every pair (0,1),(2,3),...; even steps
on (1,2),(3,4),...; gates within a step are listed in ascending site order.
Each gate consumes two independent 4x4 standard-normal blocks (real part,
imaginary part), drawn from numpy's PCG64 in the order
layer -> gate (ascending) -> real block -> imaginary block.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = ["brickwork_sites", "n_gates", "ginibre_draws", "CircuitSpec",
           "batch_specs", "batch_circuit", "sampling_uniforms", "gradient_directions"]


def brickwork_sites(n: int, depth: int) -> list[list[int]]:
    """Left site (0-based) of every gate, per time step (paper Sec. II.A)."""
    if n < 2 or n % 2:
        raise ValueError("n must be even and >= 2")
    if depth < 0:
        raise ValueError("depth must be >= 0")
    layers = []
    for t in range(1, depth + 1):
        first = 0 if t % 2 == 1 else 1
        layers.append(list(range(first, n - 1, 2)))
    return layers


def n_gates(n: int, depth: int) -> int:
    """ceil(D/2)*n/2 + floor(D/2)*(n/2-1) gates in a depth-D brickwork."""
    return ((depth + 1) // 2) * (n // 2) + (depth // 2) * (n // 2 - 1)


def ginibre_draws(n: int, depth: int, seed: int | None = None,
                  rng: np.random.Generator | None = None) -> np.ndarray:
    """Raw Gaussian draws for every gate: array (G, 2, 4, 4) float64.

    [:, 0] is the real block, [:, 1] the imaginary block, both i.i.d. N(0,1).
    Either a seed (fresh PCG64 stream) or a generator to continue is given.
    """
    g = n_gates(n, depth)
    if rng is None:
        if seed is None:
            raise ValueError("give seed or rng")
        rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((g, 2, 4, 4), dtype=np.float64)
    for k in range(g):
        out[k, 0] = rng.standard_normal((4, 4))
        out[k, 1] = rng.standard_normal((4, 4))
    return out


def sampling_uniforms(n_samples: int, n: int, seed: int) -> np.ndarray:
    """Uniform draws in [0, 1) for bit-string sampling: array (n_samples, n)
    float64, sample-major, from a fresh PCG64 stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random((n_samples, n))


@dataclasses.dataclass(frozen=True)
class CircuitSpec:
    """One random circuit instance of the batched workload."""
    seed: int
    n: int
    depth: int
    p: float
    chi_max: int


def batch_specs(count: int = 128, chi_choices=(64, 128, 256, 512)) -> list[CircuitSpec]:
    """Parameters of `count` independent circuits, circuit i drawn from PCG64(i).

    n uniform over the even numbers 16..96, depth uniform integer in [n/2, n],
    p uniform in [0.005, 0.03], chi_max uniform over `chi_choices`.  The gates
    of circuit i are then `ginibre_draws(n, depth, seed=i)`.
    """
    return [batch_circuit(i, chi_choices)[0] for i in range(count)]


def batch_circuit(i: int, chi_choices=(64, 128, 256, 512)):
    """(spec, draws) of circuit i: parameters first, then its gate draws,
    all from one PCG64(i) stream."""
    rng = np.random.Generator(np.random.PCG64(i))
    n = int(rng.integers(8, 49)) * 2
    depth = int(rng.integers(n // 2, n + 1))
    p = float(rng.uniform(0.005, 0.03))
    chi = int(chi_choices[int(rng.integers(0, len(chi_choices)))])
    spec = CircuitSpec(seed=i, n=n, depth=depth, p=p, chi_max=chi)
    return spec, ginibre_draws(n, depth, rng=rng)


def gradient_directions(n_gates: int, count: int, seed: int) -> np.ndarray:
    """Random directions in superoperator space for directional finite
    differences: array (count, n_gates, 16, 16) of i.i.d. N(0,1) float64, each
    direction scaled to unit Frobenius norm over all gates, from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.standard_normal((count, n_gates, 16, 16))
    return d / np.sqrt(np.sum(d * d, axis=(1, 2, 3)))[:, None, None, None]
