"""GPU output probabilities and bit-string sampling (Sec. III.D) against the
CPU oracle: P(x) = Tr[|x><x| rho] for every string of an exact n = 8 state,
the total probability, and sampled strings drawn with the same uniforms as the
oracle sampler (bit-identical wherever the draw is not within rounding of a
tie; the oracle runs its own MPO evolution of the same circuit)."""
import sys

import numpy as np
import pytest

import mpo_inputs as mi
from oracle import dense, gates, mpo as omp, sampling

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2003_13163_amd as pm
    pm.library()
    return pm


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_state(pm, n, depth, p, chi, prec="fp64", chi_cap=None, seed=11):
    draws = mi.ginibre_draws(n, depth, seed=seed)
    st = pm.Mpo(n, chi_cap or chi, prec, "pauli")
    st.run_brickwork(depth, pm.build_superops(draws, p, "pauli"), chi, 1e-12, record=None)
    return st, draws


def oracle_state(n, depth, p, chi, draws):
    sup = gates.circuit_superops(draws, p, "pauli")
    return omp.run_brickwork(n, sup, mi.brickwork_sites(n, depth), chi, 1e-12, "pauli",
                             record_layers=set())["mpo"]


def test_probabilities_exact_n8(pm):
    n, depth, p = 8, 6, 0.02
    say("case probabilities n8 exact fp64")
    st, draws = gpu_state(pm, n, depth, p, 256)
    rho, _, _, _ = dense.run_dense(n, depth, gates.circuit_superops(draws, p, "computational"),
                                   mi.brickwork_sites(n, depth))
    probs = np.array([st.probability([(x >> (n - 1 - k)) & 1 for k in range(n)])
                      for x in range(2 ** n)])
    err = np.abs(probs - np.diag(rho)).max()
    say(f"  max |P_gpu - P_dense| {err:.3e}  sum {probs.sum().real!r}")
    assert err <= 1e-13
    assert abs(probs.sum() - st.trace()) <= 1e-12
    st.close()


@pytest.mark.parametrize("n,depth,p,chi,prec,chi_cap,ns,ptol,tie", [
    (8, 6, 0.02, 256, "fp64", None, 500, 1e-10, 1e-9),     # exact regime
    (12, 8, 0.02, 16, "fp64", None, 500, 1e-10, 1e-9),     # truncated
    (8, 6, 0.02, 4, "fp64", 4, 2000, 1e-10, 1e-9),         # tiny scratch: many chunks
    (12, 8, 0.02, 16, "fp32", None, 500, 1e-4, 1e-4),      # FP32 state
])
def test_samples_match_oracle(pm, n, depth, p, chi, prec, chi_cap, ns, ptol, tie):
    say(f"case sampling n={n} depth={depth} chi={chi} {prec} samples={ns}")
    st, draws = gpu_state(pm, n, depth, p, chi, prec, chi_cap)
    ref = oracle_state(n, depth, p, chi, draws)
    u = mi.sampling_uniforms(ns, n, seed=7)
    bits, prob, clamped = st.sample(u)
    rbits, rprob, rclamped, margin = sampling.sample(ref, u, return_margin=True)
    clear = margin > tie
    same = (bits == rbits).all(axis=1)
    say(f"  {clear.sum()} clear of ties, mismatches among them {(~same & clear).sum()}, "
        f"clamped {clamped}/{rclamped}")
    assert clear.sum() >= 0.95 * ns
    assert same[clear].all()
    rel = np.abs(prob[same] - rprob[same]) / np.abs(rprob[same]).max()
    say(f"  max rel P(x) diff {rel.max():.3e}")
    assert rel.max() <= ptol
    # each reported probability is the contraction of its own string
    for i in range(0, ns, max(1, ns // 10)):
        assert abs(prob[i] - st.probability(bits[i]).real) <= ptol * abs(prob).max()
    st.close()


def test_sampling_rejects_bad_input(pm):
    st = pm.Mpo(4, 16, "fp64", "pauli")
    with pytest.raises(pm.MpoError):
        st.sample(np.full((3, 4), 1.0))
    with pytest.raises(pm.MpoError):
        st.probability([0, 2, 0, 0])
    bits, prob, clamped = st.sample(np.full((2, 4), 0.5))
    assert (bits == 0).all() and np.allclose(prob, 1.0) and clamped == 0   # |0000> is certain
    st.close()
