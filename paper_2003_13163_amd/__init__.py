"""Python binding of libmpo: noisy 1D random-circuit simulation with MPOs on MI355X.

Argument marshalling only: every step of the simulation runs in the HIP
kernels of libmpo.so.  PyTorch supplies device memory (the arena) and the HIP
stream.  There is no CPU fallback: if the shared library is missing the import
of `libmpo` fails loudly.

Method: Noh, Jiang, Fefferman, "Efficient classical simulation of noisy random
quantum circuits in one dimension" (Quantum 4, 318, 2020).  Names follow the
C ABI declared in include/mpo.h.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

__all__ = ["MpoError", "TruncInfo", "Mpo", "build_superop", "build_superops", "library",
           "FP64", "FP32_MFMA", "BF16X3", "PAULI", "COMPUTATIONAL", "n_schedule_gates"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmpo.so")

FP64, FP32_MFMA, BF16X3 = 0, 1, 2
PAULI, COMPUTATIONAL = 0, 1
_ORDER = {"ascending": 0, "snake": 1}
_PREC = {"fp64": FP64, "fp32": FP32_MFMA, "fp32_mfma": FP32_MFMA, "bf16x3": BF16X3,
         FP64: FP64, FP32_MFMA: FP32_MFMA, BF16X3: BF16X3}
_BASIS = {"pauli": PAULI, "computational": COMPUTATIONAL, PAULI: PAULI, COMPUTATIONAL: COMPUTATIONAL}
_STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_ARENA", 3: "ERR_HIP", 4: "ERR_NUMERIC",
           5: "ERR_NOCONV", 6: "ERR_STATE"}


class MpoError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class _KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_longlong), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class _TruncInfo(ctypes.Structure):
    _fields_ = [("kept", ctypes.c_int), ("discarded_weight", ctypes.c_double),
                ("total_weight", ctypes.c_double), ("entropy", ctypes.c_double)]


@dataclasses.dataclass
class TruncInfo:
    kept: int
    discarded_weight: float
    total_weight: float
    entropy: float


_lib = None


def library() -> ctypes.CDLL:
    """Load libmpo.so (built in-tree by build.py); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: libmpo.so must bind to the HIP runtime torch has loaded (the
    # arena and the stream come from torch); loaded the other way round, the
    # process holds two runtimes and the library's pinned allocations fail
    import torch  # noqa: F401
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: run `python -m paper_2003_13163_amd.build` "
                          "(or __graft_entry__.build()) first; there is no CPU fallback")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    pd = ctypes.POINTER(ctypes.c_double)
    pi = ctypes.POINTER(ctypes.c_int)
    sig = {
        "mpo_workspace_bytes": [I, I, I, ctypes.POINTER(S)],
        "mpo_create": [I, I, I, I, P, S, P, ctypes.POINTER(P)],
        "mpo_destroy": [P],
        "mpo_init_product": [P, ctypes.c_char_p],
        "mpo_apply_2q_channel": [P, I, pd, I, D, ctypes.POINTER(_TruncInfo)],
        "mpo_canonicalize": [P, I],
        "mpo_bond_entropy": [P, I, pd],
        "mpo_singular_values": [P, I, pd, I, pi],
        "mpo_probability": [P, ctypes.c_char_p, pd, pd],
        "mpo_sample": [P, I, pd, ctypes.c_void_p, pd, pi],
        "mpo_expect_pauli": [P, ctypes.c_char_p, pd, pd],
        "mpo_trace": [P, pd, pd],
        "mpo_expect_z_all": [P, pd, pd],
        "mpo_bond_dims": [P, pi, pi],
        "run_brickwork": [P, I, pd, I, I, D, I, I, pd, pd, pd, pd],
        "mpo_export": [P, P, S, ctypes.POINTER(S)],
        "mpo_import": [P, P, S],
        "mpo_build_superop": [pd, pd, D, I, pd, pd],
        "mpo_batch_workspace_bytes": [P, I, I, I, ctypes.POINTER(S)],
        "mpo_batch_run": [P, I, pd, S, I, I, P, S, P, I, I, I, pd],
        "mpo_set_graphs": [P, I],
        "mpo_run_brickwork_vidal": [P, I, pd, I, I, D, pd, pd],
        "mpo_set_tuning": [P, I, I],
        "mpo_set_precond": [P, I],
        "mpo_hermitian_eig": [P, I, pd, pd, pd],
        "mpo_set_default_tuning": [I, I, I, I],
        "mpo_batch_result_doubles": [I, I, I],
        "mpo_adjoint_workspace_bytes": [I, I, I, I, I, ctypes.POINTER(S)],
        "mpo_adjoint_brickwork": [P, I, pd, I, I, D, I, P, S, pd, pd, pi],
        "mpo_profile_enable": [P, I],
        "mpo_profile_read": [P, ctypes.POINTER(_KernelStat), I, pi, ctypes.POINTER(ctypes.c_longlong)],
        "mpo_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = None if name == "mpo_destroy" else (ctypes.c_char_p if name == "mpo_last_error" else ctypes.c_int)
    _lib = lib
    _load_tuning(lib)
    return lib


_TUNING_PATH = os.path.join(_HERE, "tuning.json")


def _load_tuning(lib):
    """Hand the autotuner's table (tuning.json, if present) to the library."""
    import json
    try:
        with open(_TUNING_PATH) as f:
            entries = json.load(f).get("entries", [])
    except (OSError, ValueError):
        return
    for e in entries:
        _check(lib.mpo_set_default_tuning(_PREC[e["precision"]], int(e["chi_upto"]), int(e["block"]),
                                          int(e["inner"])))


def _check(status: int):
    if status != 0:
        raise MpoError(status, library().mpo_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_complex_pairs(m) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
    return a.view(np.float64)


def n_schedule_gates(n: int, depth: int) -> int:
    return ((depth + 1) // 2) * (n // 2) + (depth // 2) * (n // 2 - 1)


def build_superop(re, im, p: float, basis="pauli") -> tuple[np.ndarray, np.ndarray]:
    """Noisy Haar gate superoperator (16x16 complex) and its unitary (4x4) from
    one Ginibre draw, computed by the library's host code."""
    lib = library()
    re = np.ascontiguousarray(re, dtype=np.float64)
    im = np.ascontiguousarray(im, dtype=np.float64)
    out = np.zeros(512)
    u = np.zeros(32)
    _check(lib.mpo_build_superop(_dptr(re), _dptr(im), float(p), _BASIS[basis], _dptr(out), _dptr(u)))
    return out.view(np.complex128).reshape(16, 16), u.view(np.complex128).reshape(4, 4)


def build_superops(draws: np.ndarray, p: float, basis="pauli") -> np.ndarray:
    """Superoperators of a whole circuit from draws of shape (G, 2, 4, 4)."""
    out = np.empty((draws.shape[0], 16, 16), dtype=np.complex128)
    for g in range(draws.shape[0]):
        out[g] = build_superop(draws[g, 0], draws[g, 1], p, basis)[0]
    return out


class Mpo:
    """Vectorised density matrix of n qubits held on one GPU."""

    def __init__(self, n: int, chi_cap: int, precision="fp64", basis="pauli", device=None,
                 stream=None):
        import torch
        lib = library()
        self.n, self.chi_cap = n, chi_cap
        self.precision, self.basis = _PREC[precision], _BASIS[basis]
        nbytes = ctypes.c_size_t()
        _check(lib.mpo_workspace_bytes(n, chi_cap, self.precision, ctypes.byref(nbytes)))
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.arena = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._h = ctypes.c_void_p()
        _check(lib.mpo_create(n, chi_cap, self.precision, self.basis,
                              ctypes.c_void_p(self.arena.data_ptr()), nbytes.value,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            library().mpo_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- state
    def init_product(self, bits=None):
        buf = None if bits is None else bytes(int(b) for b in bits)
        if buf is not None and len(buf) != self.n:
            raise ValueError("bits must have n entries")
        _check(library().mpo_init_product(self._h, buf))

    def apply(self, site: int, superop, chi_max: int, cutoff: float = 1e-12, sync: bool = True):
        m = _as_complex_pairs(superop).reshape(-1)
        if m.size != 512:
            raise ValueError("superop must be 16x16 complex")
        info = _TruncInfo()
        _check(library().mpo_apply_2q_channel(self._h, site, _dptr(m), chi_max, float(cutoff),
                                              ctypes.byref(info) if sync else None))
        if sync:
            return TruncInfo(info.kept, info.discarded_weight, info.total_weight, info.entropy)
        return None

    def canonicalize(self, center: int):
        _check(library().mpo_canonicalize(self._h, center))

    def entropy(self, bond: int = -1):
        out = np.zeros(self.n - 1 if bond < 0 else 1)
        _check(library().mpo_bond_entropy(self._h, bond, _dptr(out)))
        return out if bond < 0 else float(out[0])

    def singular_values(self, bond: int) -> np.ndarray:
        out = np.zeros(4 * self.chi_cap)
        cnt = ctypes.c_int()
        _check(library().mpo_singular_values(self._h, bond, _dptr(out), out.size, ctypes.byref(cnt)))
        return out[: cnt.value].copy()

    def expect(self, pauli) -> complex:
        codes = [("IXYZ".index(c) if isinstance(c, str) else int(c)) for c in pauli]
        if len(codes) != self.n:
            raise ValueError("one Pauli code per site")
        re, im = ctypes.c_double(), ctypes.c_double()
        _check(library().mpo_expect_pauli(self._h, bytes(codes), ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    def trace(self) -> complex:
        re, im = ctypes.c_double(), ctypes.c_double()
        _check(library().mpo_trace(self._h, ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    def probability(self, bits) -> complex:
        """P(x) = Tr[|x><x| rho] of the held state (not divided by Tr rho)."""
        b = bytes(int(v) for v in bits)
        if len(b) != self.n:
            raise ValueError("one bit per site")
        re, im = ctypes.c_double(), ctypes.c_double()
        _check(library().mpo_probability(self._h, b, ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    def sample(self, uniforms):
        """Sequential conditional sampling with caller-supplied uniforms
        (n_samples x n, in [0, 1)).  Returns (bits uint8 (n_samples, n), P(x)
        of each string, number of samples that met a negative marginal)."""
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        if u.ndim != 2 or u.shape[1] != self.n:
            raise ValueError("uniforms must be (n_samples, n)")
        bits = np.zeros(u.shape, dtype=np.uint8)
        prob = np.zeros(u.shape[0])
        clamped = ctypes.c_int()
        _check(library().mpo_sample(self._h, u.shape[0], _dptr(u), bits.ctypes.data, _dptr(prob),
                                    ctypes.byref(clamped)))
        return bits, prob, clamped.value

    def expect_z_all(self):
        z = np.zeros(self.n)
        tr = ctypes.c_double()
        _check(library().mpo_expect_z_all(self._h, _dptr(z), ctypes.byref(tr)))
        return z, tr.value

    def bond_dims(self):
        dims = (ctypes.c_int * (self.n - 1))()
        c = ctypes.c_int()
        _check(library().mpo_bond_dims(self._h, dims, ctypes.byref(c)))
        return list(dims), c.value

    def export(self) -> bytes:
        used = ctypes.c_size_t()
        _check(library().mpo_export(self._h, None, 0, ctypes.byref(used)))
        buf = ctypes.create_string_buffer(used.value)
        _check(library().mpo_export(self._h, buf, used.value, ctypes.byref(used)))
        return buf.raw

    def import_state(self, data: bytes):
        buf = ctypes.create_string_buffer(data, len(data))
        _check(library().mpo_import(self._h, buf, len(data)))

    def adjoint_brickwork(self, depth: int, superops, chi_max: int, cutoff: float = 1e-12,
                          checkpoint_every: int = 0):
        """(O, dO/dM of every gate (G,16,16) complex, largest co-state bond) with the
        truncation projectors frozen; the state advances to the final one.
        checkpoint_every = K > 0 keeps the state every K time steps and recomputes
        one K-step segment at a time for the backward (0: the whole tape at once)."""
        import torch
        lib = library()
        sup = _as_complex_pairs(superops).reshape(-1)
        g = sup.size // 512
        nbytes = ctypes.c_size_t()
        _check(lib.mpo_adjoint_workspace_bytes(self.n, depth, chi_max, self.precision,
                                               int(checkpoint_every), ctypes.byref(nbytes)))
        work = torch.empty(nbytes.value, dtype=torch.uint8, device=self.arena.device)
        O = ctypes.c_double()
        grads = np.zeros(g * 512)
        comax = ctypes.c_int()
        _check(lib.mpo_adjoint_brickwork(self._h, depth, _dptr(sup), g, chi_max, float(cutoff),
                                         int(checkpoint_every), ctypes.c_void_p(work.data_ptr()), nbytes.value,
                                         ctypes.byref(O), _dptr(grads), ctypes.byref(comax)))
        del work
        return O.value, grads.view(np.complex128).reshape(g, 16, 16), comax.value

    def set_precond(self, min_cols: int):
        """Splits with at least min_cols columns start from the Gram eigenvectors (0 = never)."""
        _check(library().mpo_set_precond(self._h, int(min_cols)))

    def hermitian_eig(self, G):
        """Eigenvalues (ascending) and eigenvectors (columns) of a Hermitian matrix through
        the split's eigen-solver kernels (uses this handle's workspace)."""
        G = np.ascontiguousarray(np.asarray(G, dtype=np.complex128))
        N = G.shape[0]
        w = np.empty(N)
        V = np.empty((N, N), dtype=np.complex128)
        _check(library().mpo_hermitian_eig(self._h, N, _dptr(G.view(np.float64)), _dptr(w),
                                           _dptr(V.view(np.float64))))
        return w, V

    def set_graphs(self, on: bool = True):
        """Replay the Jacobi sweeps from captured HIP graphs (needs a non-null stream)."""
        _check(library().mpo_set_graphs(self._h, 1 if on else 0))

    # ------------------------------------------------------------- instrumentation
    def profile(self, on: bool = True):
        """Enable (and reset) per-kernel HIP-event timing on this handle's stream."""
        _check(library().mpo_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        stats = (_KernelStat * 32)()
        cnt = ctypes.c_int()
        svd = (ctypes.c_longlong * 6)()
        _check(library().mpo_profile_read(self._h, stats, 32, ctypes.byref(cnt), svd))
        out = {"kernels": {}, "svd": dict(zip(("splits", "sweeps", "rounds", "rotated_pairs", "eigen_starts",
                                               "gram_certified"), list(svd)))}
        for k in range(cnt.value):
            st = stats[k]
            out["kernels"][st.name.decode()] = {"launches": st.launches, "ms": st.ms,
                                                "flops": st.flops, "bytes": st.bytes}
        return out

    # ------------------------------------------------------------- evolution
    def run_brickwork(self, depth: int, superops, chi_max: int, cutoff: float = 1e-12,
                      record: str | None = "all", order: str = "ascending") -> dict:
        """Brickwork evolution; order "ascending" (every step from the left) or
        "snake" (even steps from the right; superops then list those steps'
        gates right to left)."""
        sup = _as_complex_pairs(superops).reshape(-1)
        g = sup.size // 512
        mask = {"all": 1, "last": 2, None: 0}[record]
        rows = depth if record == "all" else (1 if record == "last" else 0)
        S = np.zeros(max(rows, 1) * (self.n - 1))
        Z = np.zeros(max(rows, 1) * self.n)
        tr = np.zeros(max(rows, 1))
        disc = np.zeros(max(g, 1))
        _check(library().run_brickwork(self._h, depth, _dptr(sup), g, chi_max, float(cutoff),
                                       _ORDER[order], mask, _dptr(S), _dptr(Z), _dptr(tr), _dptr(disc)))
        return {"S": S[: rows * (self.n - 1)].reshape(rows, self.n - 1),
                "Z": Z[: rows * self.n].reshape(rows, self.n), "trace": tr[:rows],
                "discarded": disc[:g]}


    def run_brickwork_vidal(self, depth: int, superops, chi_max: int, cutoff: float = 1e-12) -> dict:
        """The paper's global Gamma-lambda update (App. A) from |0..0>: S_b after
        every time step (from the lambdas) and the discarded weight per gate."""
        sup = _as_complex_pairs(superops).reshape(-1)
        g = sup.size // 512
        S = np.zeros(max(depth, 1) * (self.n - 1))
        disc = np.zeros(max(g, 1))
        _check(library().mpo_run_brickwork_vidal(self._h, depth, _dptr(sup), g, chi_max, float(cutoff),
                                                 _dptr(S), _dptr(disc)))
        return {"S": S[: depth * (self.n - 1)].reshape(depth, self.n - 1), "discarded": disc[:g]}


class _BatchDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("depth", ctypes.c_int), ("chi_max", ctypes.c_int),
                ("cutoff", ctypes.c_double), ("gate_offset", ctypes.c_size_t),
                ("result_offset", ctypes.c_size_t)]


def batch_run(circuits, superops, precision="fp32", basis="pauli", n_streams=8, device=None,
              record="last", use_graph=False):
    """Evolve independent circuits concurrently (mpo_batch_run).

    circuits: list of (n, depth, chi_max, cutoff); superops: list of arrays
    (n_gates(n, depth), 16, 16) per circuit.  record: "last" (observables after
    the last time step) or "all" (after every time step).  use_graph: replay the
    Jacobi sweeps from captured HIP graphs (mpo_set_graphs).  Returns one dict per
    circuit with S (rows x (n-1) bond entropies), Z (rows x n), trace (rows),
    discarded (sum over gates) and max_bond; rows = 1 for "last"."""
    import torch
    lib = library()
    count = len(circuits)
    descs = (_BatchDesc * count)()
    mask = {"last": 2, "all": 1}[record]
    g_off, r_off = 0, 0
    for i, (n, depth, chi, cut) in enumerate(circuits):
        g = n_schedule_gates(n, depth)
        if superops[i].shape[0] != g:
            raise ValueError(f"circuit {i}: {superops[i].shape[0]} superoperators, {g} expected")
        descs[i] = _BatchDesc(n, depth, chi, float(cut), g_off, r_off)
        g_off += g
        r_off += lib.mpo_batch_result_doubles(n, depth, mask)
    sup = np.ascontiguousarray(np.concatenate([np.asarray(s, dtype=np.complex128).reshape(-1, 16, 16)
                                               for s in superops]))
    prec = _PREC[precision]
    nbytes = ctypes.c_size_t()
    dptr = ctypes.cast(descs, ctypes.c_void_p)
    _check(lib.mpo_batch_workspace_bytes(dptr, count, prec, n_streams, ctypes.byref(nbytes)))
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    arena = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    streams = [torch.cuda.Stream(device=dev) for _ in range(n_streams)]
    handles = (ctypes.c_void_p * n_streams)(*[s.cuda_stream for s in streams])
    res = np.zeros(max(r_off, 1))
    torch.cuda.synchronize(dev)
    _check(lib.mpo_batch_run(dptr, count, _dptr(sup.view(np.float64)), g_off, prec, _BASIS[basis],
                             ctypes.c_void_p(arena.data_ptr()), nbytes.value,
                             ctypes.cast(handles, ctypes.c_void_p), n_streams, 1 if use_graph else 0, mask,
                             _dptr(res)))
    out = []
    for i, (n, depth, chi, cut) in enumerate(circuits):
        rows = depth if (mask == 1 and depth > 0) else 1
        o = descs[i].result_offset
        S = res[o: o + rows * (n - 1)].reshape(rows, n - 1)
        Z = res[o + rows * (n - 1): o + rows * (2 * n - 1)].reshape(rows, n)
        tr = res[o + rows * (2 * n - 1): o + rows * 2 * n]
        tail = res[o + rows * 2 * n: o + rows * 2 * n + 2]
        if mask == 2:
            S, Z, tr = S[0], Z[0], float(tr[0])
        out.append({"S": S.copy(), "Z": Z.copy(), "trace": tr if mask == 2 else tr.copy(),
                    "discarded": tail[0], "max_bond": int(tail[1])})
    del arena
    return out


def snapshot_to_tensors(data: bytes):
    """Decode an exported snapshot into (n, basis, centre, list of (chi_l,4,chi_r) arrays)."""
    hdr = np.frombuffer(data, dtype=np.int64, count=4)
    n = int(hdr[1])
    dims = np.frombuffer(data, dtype=np.int64, count=n - 1, offset=32).tolist()
    off = 8 * (4 + n - 1)
    tensors = []
    for s in range(n):
        cl = 1 if s == 0 else dims[s - 1]
        cr = 1 if s == n - 1 else dims[s]
        cnt = cl * 4 * cr
        arr = np.frombuffer(data, dtype=np.complex128, count=cnt, offset=off).reshape(cl, 4, cr)
        tensors.append(arr.copy())
        off += cnt * 16
    return n, int(hdr[2]), int(hdr[3]), tensors


def tensors_to_snapshot(tensors, basis="pauli", centre=0) -> bytes:
    n = len(tensors)
    dims = [t.shape[2] for t in tensors[:-1]]
    hdr = np.array([0x4D504F31, n, _BASIS[basis], centre] + dims, dtype=np.int64)
    body = b"".join(np.ascontiguousarray(t, dtype=np.complex128).tobytes() for t in tensors)
    return hdr.tobytes() + body
