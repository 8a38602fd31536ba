"""Allocation-free observables (mpo_expect_z_all_noalloc) against the arena
entry point mpo_expect_z_all: the same transfer contraction with its
environments in the library's static device scratch instead of the handle's
arena.  Two calls in a row, the second on a smaller state, each compared with
the arena entry point (same kernels in the same order: bit-identical)."""
import ctypes

import numpy as np
import pytest

import mpo_inputs as mi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2003_13163_amd as pm
    lib = pm.library()
    lib.mpo_expect_z_all_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)]
    lib.mpo_expect_z_all_noalloc.restype = ctypes.c_int
    return pm


def _both(pm, st):
    lib = pm.library()
    n = st.n
    z_arena = np.zeros(n)
    tr_arena = ctypes.c_double()
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.mpo_expect_z_all(st._h, z_arena.ctypes.data_as(dp), ctypes.byref(tr_arena)) == 0
    z_static = np.full(n, np.nan)
    tr_static = ctypes.c_double(np.nan)
    rc = lib.mpo_expect_z_all_noalloc(st._h, z_static.ctypes.data_as(dp), ctypes.byref(tr_static))
    assert rc == 0, lib.mpo_last_error()
    return z_arena, tr_arena.value, z_static, tr_static.value


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_arena_entry_point_twice(pm, prec):
    cases = [(16, 10, 64, 0.02, 7), (8, 5, 16, 0.03, 8)]     # second call: smaller state
    for n, depth, chi, p, seed in cases:
        print(f"case noalloc {prec} n={n} depth={depth} chi={chi}", flush=True)
        st = pm.Mpo(n, chi, prec, "pauli")
        sup = pm.build_superops(mi.ginibre_draws(n, depth, seed=seed), p, "pauli")
        st.run_brickwork(depth, sup, chi, 1e-12, record=None)
        z_a, tr_a, z_s, tr_s = _both(pm, st)
        st.close()
        assert np.array_equal(z_a, z_s), np.abs(z_a - z_s).max()
        assert tr_a == tr_s
        assert 0.0 < tr_a <= 1.0 + 1e-9


def test_noalloc_rejects_states_beyond_the_scratch(pm):
    """n = 256 at chi_cap = 1024 needs about 9 MiB of environments, beyond the
    8 MiB static scratch: an arena error before any launch."""
    lib = pm.library()
    st = pm.Mpo(256, 1024, "fp32", "pauli")
    z = np.zeros(256)
    tr = ctypes.c_double()
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.mpo_expect_z_all_noalloc(st._h, z.ctypes.data_as(dp), ctypes.byref(tr)) == 2
    assert b"static scratch" in lib.mpo_last_error()
    st.close()
