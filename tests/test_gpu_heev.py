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
import os
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


def graded_mps(n, dims, seed, decay):
    """Random MPS whose bond indices carry weights decaying geometrically by
    `decay` overall (a wide spread of Schmidt values, as truncated states have)."""
    rng = np.random.default_rng(seed)
    ts = []
    for s in range(n):
        cl = 1 if s == 0 else dims[s - 1]
        cr = 1 if s == n - 1 else dims[s]
        t = rng.standard_normal((cl, 4, cr)) + 1j * rng.standard_normal((cl, 4, cr))
        if cr > 1:
            t = t * np.logspace(0, np.log10(decay), cr)[None, None, :]
        ts.append(t / np.linalg.norm(t))
    return ts


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_qr_moves_preserve_state(pm, prec, tol):
    """Centre moves across bonds of dimension 200 (>= the Cholesky QR threshold)
    on a state whose bond weights span 12 orders of magnitude: Pauli
    expectations, the trace and the Schmidt values at the bonds must match the
    oracle's (QR moves of the same tensors), and the QR moves must agree with
    the SVD moves.  FP64 to 1e-12 relative, FP32 to its storage rounding."""
    n, dims = 8, [4, 16, 64, 200, 64, 16, 4]
    ts = graded_mps(n, dims, seed=21, decay=1e-6)
    ref = omp.MPO.from_tensors([t.copy() for t in ts], "pauli")
    strings = ["ZIIIIIII", "IIIZZIII", "XYIIIZIX", "IIIIIIIZ"]
    exp_ref = [complex(ref.contract_product([gates.dual_vector(gates.PAULI["IXYZ".index(ch)], "pauli")
                                             for ch in sgl])) for sgl in strings]
    tr_ref = ref.trace()
    lam_ref = ref.schmidt_sweep()[3]
    out = {}
    for label, qr_min in (("qr", 128), ("svd", 0)):
        os.environ["MPO_QR_MIN"] = str(qr_min)
        try:
            st = pm.Mpo(n, 256, prec, "pauli")
        finally:
            del os.environ["MPO_QR_MIN"]
        st.import_state(pm.tensors_to_snapshot(ts))
        for c in (7, 0, 5, 2, 4):
            st.canonicalize(c)
        tr = st.trace()
        ex = [st.expect(sgl) * tr for sgl in strings]
        lam = st.singular_values(3)
        st.close()
        out[label] = (tr, ex, lam)
        say(f"{prec} {label}: trace {tr} ({abs(tr - tr_ref) / abs(tr_ref):.2e})")
    for label in ("qr", "svd"):
        tr, ex, lam = out[label]
        scale = max(abs(e) for e in exp_ref)
        assert abs(tr - tr_ref) <= tol * abs(tr_ref)
        assert max(abs(a - b) for a, b in zip(ex, exp_ref)) <= tol * scale
        k = min(len(lam), len(lam_ref))
        assert np.abs(lam[:k] - lam_ref[:k]).max() <= tol * lam_ref[0]
