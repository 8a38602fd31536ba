"""GPU: the split's Hermitian eigen-solver (Householder tridiagonalisation,
divide and conquer, back-transformation; all FP64) through mpo_hermitian_eig,
against numpy's eigh, and the splits that start from it against the plain
Jacobi sweeps.

Bars: eigenvalues within 1e-12 ||G|| of numpy's (both are backward stable:
errors of a few eps ||G||), V unitary to 1e-12, and residual ||G V - V diag(w)||
at most 1e-12 ||G|| (max-abs entries).  Sizes cover single and several
32-column panels, ragged tails, a size that is not a power of two in the
divide-and-conquer tree, exact degeneracy (clusters the deflation must
rotate), rank deficiency (a zero cluster), a diagonal and the zero matrix.
"""
import sys

import numpy as np
import pytest

import mpo_inputs as mi
from oracle import gates, mpo as omp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2003_13163_amd as pm
    pm.library()
    return pm


@pytest.fixture(scope="module")
def handle(pm):
    st = pm.Mpo(2, 256, "fp64", "pauli")     # 4 chi_cap = 1024: eigen workspace for N <= 1024
    yield st
    st.close()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def hermitian_cases():
    rng = np.random.default_rng(7)
    out = []
    for N in (2, 3, 17, 33, 64, 65, 200, 513):
        X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
        out.append((f"random{N}", X @ X.conj().T))
    N = 300
    X = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) * np.logspace(0, -7, N)[None, :]
    out.append(("graded300", X.conj().T @ X))
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    ev = np.repeat([5.0, 1.0, 1e-3, 0.0], [40, 100, 80, 80])
    out.append(("degenerate300", (Q * ev) @ Q.conj().T))
    Xr = rng.standard_normal((N, 40)) + 1j * rng.standard_normal((N, 40))
    out.append(("rank40of300", Xr @ Xr.conj().T))
    out.append(("diagonal100", np.diag(rng.random(100)).astype(complex)))
    out.append(("zero64", np.zeros((64, 64), complex)))
    return out


@pytest.mark.parametrize("name,G", hermitian_cases(), ids=[c[0] for c in hermitian_cases()])
def test_hermitian_eig_matches_numpy(handle, name, G):
    G = 0.5 * (G + G.conj().T)
    N = G.shape[0]
    say(f"heev {name} N={N}")
    w, V = handle.hermitian_eig(G)
    ref = np.linalg.eigvalsh(G)
    scale = max(np.abs(ref).max(), 1e-300)
    assert np.all(np.diff(w) >= 0.0)
    assert np.abs(w - ref).max() <= 1e-12 * scale
    assert np.abs(V.conj().T @ V - np.eye(N)).max() <= 1e-12
    assert np.abs(G @ V - V * w[None, :]).max() <= 1e-12 * scale


def test_hermitian_eig_rejects_bad_input(pm, handle):
    with pytest.raises(pm.MpoError):
        handle.hermitian_eig(np.zeros((1, 1), complex))
    with pytest.raises(pm.MpoError):
        handle.hermitian_eig(np.zeros((1025, 1025), complex))
    bad = np.eye(8, dtype=complex)
    bad[3, 3] = np.nan
    with pytest.raises(pm.MpoError):
        handle.hermitian_eig(bad)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_eigen_start_matches_plain_sweeps(pm, prec):
    """A chi = 256 gate (theta' 1024 x 1024, at the default threshold) on an in-situ
    10-qubit state, split with and without the eigen start: same kept count,
    entropy, discarded weight and singular values (FP64 to 1e-12 relative,
    reduced modes to their Jacobi tolerance)."""
    n, depth, p, chi = 10, 8, 0.01, 256
    draws = mi.ginibre_draws(n, depth + 2, seed=3)
    sup = pm.build_superops(draws, p, "pauli")
    g = pm.n_schedule_gates(n, depth)
    st = pm.Mpo(n, chi, "fp64", "pauli")
    st.set_precond(0)
    st.run_brickwork(depth, sup[:g], chi, 1e-12, record=None)
    snap = st.export()
    st.close()
    res = {}
    for label, mc in (("plain", 0), ("eigen", 1024)):
        st = pm.Mpo(n, chi, prec, "pauli")
        st.import_state(snap)
        st.set_precond(mc)
        st.profile(True)
        info = st.apply(4, sup[g], chi, 1e-12)
        prof = st.profile_read()
        lam = st.singular_values(4)
        st.close()
        res[label] = (info, lam, prof["svd"])
        say(f"{prec} {label}: kept {info.kept} S {info.entropy:.12f} svd {prof['svd']}")
    (ip, lp, _), (ie, le, se) = res["plain"], res["eigen"]
    assert se["eigen_starts"] >= 1
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert ip.kept == ie.kept
    assert abs(ip.entropy - ie.entropy) <= (1e-11 if prec == "fp64" else 1e-5)
    assert abs(ip.discarded_weight - ie.discarded_weight) <= tol * ip.total_weight
    k = min(len(lp), len(le))
    assert np.abs(lp[:k] - le[:k]).max() <= tol * lp[0]


def test_eigen_start_gate_against_oracle(pm):
    """The same kind of gate in FP64 from the eigen start against the oracle's
    complex128 gesdd split: entropy, kept count, discarded weight, Schmidt values."""
    n, depth, p, chi = 10, 8, 0.01, 256
    draws = mi.ginibre_draws(n, depth + 2, seed=4)
    sup = pm.build_superops(draws, p, "pauli")
    g = pm.n_schedule_gates(n, depth)
    st = pm.Mpo(n, chi, "fp64", "pauli")
    st.run_brickwork(depth, sup[:g], chi, 1e-12, record=None)
    snap = st.export()
    st.profile(True)
    info = st.apply(4, sup[g], chi, 1e-12)
    starts = st.profile_read()["svd"]["eigen_starts"]
    lam = st.singular_values(4)
    st.close()
    nn, basis, centre, tensors = pm.snapshot_to_tensors(snap)
    m = omp.MPO.from_tensors(tensors, basis)
    ref = m.apply_gate(4, gates.circuit_superops(draws, p, "pauli")[g], chi, 1e-12)
    a5 = m.A[5]
    lam_ref = np.linalg.svd(a5.reshape(a5.shape[0], -1), compute_uv=False)
    say(f"eigen-start gate: S {info.entropy:.14f} oracle {ref.entropy:.14f} starts {starts}")
    assert starts >= 1
    assert info.kept == ref.kept
    assert abs(info.entropy - ref.entropy) <= 1e-10
    assert abs(info.discarded_weight - ref.discarded_weight) <= 1e-12 * ref.total_weight
    k = min(len(lam), len(lam_ref))
    assert np.abs(lam[:k] - lam_ref[:k]).max() <= 1e-11 * lam_ref[0]
