"""Python binding of libbpki (ctypes): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels.  If the built library is not
present the import of this module succeeds but every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbpki.so")

BPKI_FP64 = 0
BPKI_FP32 = 1


class BpkiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bpki error {code}: {msg}")
        self.code = code


class _Problem(C.Structure):
    _fields_ = [
        ("n_sites", C.c_int32), ("n_edges", C.c_int32),
        ("edges", C.POINTER(C.c_int32)), ("colour", C.POINTER(C.c_int32)),
        ("theta_h", C.c_double), ("depth", C.c_int32), ("chi", C.c_int32),
        ("precision", C.c_int32), ("bp_tol", C.c_double), ("bp_max_iter", C.c_int32),
        ("svd_cutoff", C.c_double), ("eig_cutoff", C.c_double),
        ("n_pauli", C.c_int32), ("pauli_offsets", C.POINTER(C.c_int32)),
        ("pauli_sites", C.POINTER(C.c_int32)), ("pauli_ops", C.POINTER(C.c_uint8)),
        ("record_every_step", C.c_int32), ("clifford_steps", C.c_int32),
    ]


class _Result(C.Structure):
    _fields_ = [
        ("z", C.POINTER(C.c_double)), ("pauli", C.POINTER(C.c_double)),
        ("bp_iters", C.POINTER(C.c_int32)), ("bp_residual", C.POINTER(C.c_double)),
        ("discarded", C.POINTER(C.c_double)), ("bond_entropy", C.POINTER(C.c_double)),
        ("bond_dims", C.POINTER(C.c_int32)), ("min_cut_gap", C.POINTER(C.c_double)),
        ("degenerate_cuts", C.POINTER(C.c_int32)),
    ]


class TestGemmDesc(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("M", "N", "K", "Mi", "Ni", "Ki")] + \
               [(n, C.c_int64) for n in ("a_mo", "a_mi", "a_ko", "a_ki", "b_ko", "b_ki", "b_no",
                                         "b_ni", "c_mo", "c_mi", "c_no", "c_ni", "a_b", "b_b",
                                         "c_b")] + \
               [(n, C.c_int32) for n in ("batch", "conjA", "conjB", "beta")] + \
               [("alpha_re", C.c_double), ("alpha_im", C.c_double), ("prec", C.c_int32),
                ("herm", C.c_int32), ("store32", C.c_int32)]


_lib = None


# bpki_alloc_fn / bpki_free_fn: (bytes, stream, user) -> device pointer; (ptr, stream, user)
AllocFn = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FreeFn = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


def load(path: str | None = None):
    """Load libbpki.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(path)
    P, R = C.POINTER(_Problem), C.POINTER(_Result)
    vp = C.c_void_p
    dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)
    sig = {
        "bpki_problem_defaults": (None, [P]),
        "bpki_create": (C.c_int, [C.POINTER(vp), C.c_int, vp, C.c_size_t]),
        "bpki_destroy": (None, [vp]),
        "bpki_set_allocator": (C.c_int, [vp, AllocFn, FreeFn, vp]),
        "bpki_last_error": (C.c_char_p, []),
        "bpki_validate": (C.c_int, [P]),
        "bpki_estimate_bytes": (C.c_int, [P, C.POINTER(C.c_size_t)]),
        "bpki_solve": (C.c_int, [vp, P, R]),
        "bpki_solve_noalloc": (C.c_int, [vp, P, R]),
        "bpki_submit": (C.c_int, [vp, P, R, C.POINTER(C.c_uint64)]),
        "bpki_poll": (C.c_int, [vp, C.c_uint64, C.POINTER(C.c_int)]),
        "bpki_wait": (C.c_int, [vp, C.c_uint64]),
        "bpki_cancel": (C.c_int, [vp, C.c_uint64]),
        "bpki_serving_config": (C.c_int, [vp, C.c_int]),
        "bpki_serving_packing": (C.c_int, [vp, C.c_int, C.c_int]),
        "bpki_ticket_times": (C.c_int, [vp, C.c_uint64, dp]),
        "bpki_ticket_pack_size": (C.c_int, [vp, C.c_uint64, ip]),
        "bpki_session_open": (C.c_int, [vp, P, C.POINTER(vp)]),
        "bpki_session_close": (None, [vp]),
        "bpki_session_sizes": (C.c_int, [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "bpki_session_get_state": (C.c_int, [vp, dp, dp, ip]),
        "bpki_session_set_state": (C.c_int, [vp, dp, dp, ip]),
        "bpki_session_apply_rx": (C.c_int, [vp]),
        "bpki_session_apply_layer": (C.c_int, [vp, C.c_int32, dp]),
        "bpki_session_layer_cuts": (C.c_int, [vp, ip, dp, dp]),
        "bpki_session_bp": (C.c_int, [vp, C.c_int32, ip, dp]),
        "bpki_session_bp_sweep": (C.c_int, [vp, dp]),
        "bpki_session_observe_z": (C.c_int, [vp, dp]),
        "bpki_session_observe_bond_entropy": (C.c_int, [vp, dp]),
        "bpki_session_vidal_gauge": (C.c_int, [vp, dp]),
        "bpki_session_bp_error": (C.c_int, [vp, C.c_int32, dp, dp]),
        "bpki_session_observe_pauli": (C.c_int, [vp, dp]),
        "bpki_session_step": (C.c_int, [vp, dp, ip, dp, dp]),
        "bpki_session_clifford_inverse_step": (C.c_int, [vp, dp, ip, dp, dp]),
        "bpki_session_last_timing": (C.c_int, [vp, dp]),
        "bpki_session_profile_read_prec": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_int64), dp,
                                                      dp]),
        "bpki_session_profile_read_kernel": (C.c_int, [vp, C.c_int32, C.c_int32,
                                                        C.POINTER(C.c_int64), dp, dp, dp,
                                                        C.POINTER(C.c_int64)]),
        "bpki_session_profile": (C.c_int, [vp, C.c_int]),
        "bpki_session_profile_read": (C.c_int, [vp, C.POINTER(C.c_int64), dp, dp,
                                                 C.POINTER(C.c_int64)]),
        "bpki_test_gemm": (C.c_int, [vp, C.POINTER(TestGemmDesc), C.c_int, dp, C.c_size_t, dp,
                                     C.c_size_t, dp, C.c_size_t]),
        "bpki_test_eigh": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, dp, dp, dp]),
        "bpki_test_gram_chol": (C.c_int, [vp, C.c_int, C.c_int, dp, C.c_double, dp, dp]),
        "bpki_test_mfma_rate": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, dp]),
        "bpki_test_bp_close": (C.c_int, [vp, C.c_int32, C.c_int, C.c_int, C.c_int32, C.c_int64,
                                         C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int, dp,
                                         dp, C.c_size_t, dp, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path == LIB_PATH or _lib is None:
        _lib = lib
    return lib


def exported_symbols() -> list[str]:
    return ["bpki_problem_defaults", "bpki_create", "bpki_destroy", "bpki_last_error",
            "bpki_validate", "bpki_estimate_bytes", "bpki_solve", "bpki_solve_noalloc",
            "bpki_submit", "bpki_poll",
            "bpki_wait", "bpki_cancel", "bpki_serving_config", "bpki_serving_packing",
            "bpki_ticket_times", "bpki_ticket_pack_size", "bpki_set_allocator",
            "bpki_session_open", "bpki_session_close",
            "bpki_session_sizes", "bpki_session_get_state", "bpki_session_set_state",
            "bpki_session_apply_rx", "bpki_session_apply_layer", "bpki_session_layer_cuts",
            "bpki_session_bp",
            "bpki_session_bp_sweep", "bpki_session_observe_z",
            "bpki_session_observe_bond_entropy", "bpki_session_vidal_gauge",
            "bpki_session_bp_error",
            "bpki_session_observe_pauli",
            "bpki_session_step", "bpki_session_clifford_inverse_step",
            "bpki_session_last_timing", "bpki_session_profile",
            "bpki_session_profile_read", "bpki_session_profile_read_prec",
            "bpki_session_profile_read_kernel", "bpki_test_gemm",
            "bpki_test_eigh", "bpki_test_gram_chol", "bpki_test_mfma_rate",
            "bpki_test_bp_close"]


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def _check(lib, rc: int) -> int:
    if rc < 0:
        raise BpkiError(rc, lib.bpki_last_error().decode())
    return rc


@dataclass
class ProblemSpec:
    """Host description of one circuit run (owns the arrays the C struct points into)."""
    n_sites: int
    edges: np.ndarray
    colour: np.ndarray | None
    theta: float
    depth: int
    chi: int
    precision: int = BPKI_FP64
    bp_tol: float = 1e-12
    bp_max_iter: int = 1000
    svd_cutoff: float = 1e-12
    eig_cutoff: float = 1e-12
    pauli: tuple = ()
    record_every_step: bool = True
    clifford_steps: int = 0         # steps of U(pi/2)^dagger after the depth steps
    bond_entropy: bool = False      # also return the entropy of every edge (result side)

    def to_c(self):
        keep = {}
        e = np.ascontiguousarray(np.asarray(self.edges, dtype=np.int32).reshape(-1))
        keep["e"] = e
        p = _Problem()
        p.n_sites = int(self.n_sites)
        p.n_edges = int(e.size // 2)
        p.edges = _ptr(e, C.c_int32)
        if self.colour is not None:
            c = np.ascontiguousarray(np.asarray(self.colour, dtype=np.int32))
            keep["c"] = c
            p.colour = _ptr(c, C.c_int32)
        p.theta_h = float(self.theta)
        p.depth = int(self.depth)
        p.chi = int(self.chi)
        p.precision = int(self.precision)
        p.bp_tol = float(self.bp_tol)
        p.bp_max_iter = int(self.bp_max_iter)
        p.svd_cutoff = float(self.svd_cutoff)
        p.eig_cutoff = float(self.eig_cutoff)
        p.record_every_step = 1 if self.record_every_step else 0
        p.clifford_steps = int(self.clifford_steps)
        if self.pauli:
            offs, sites, ops = [0], [], []
            for s, o in self.pauli:
                sites += [int(x) for x in s]
                ops += [int(x) for x in o]
                offs.append(len(sites))
            keep["po"] = np.array(offs, dtype=np.int32)
            keep["ps"] = np.array(sites, dtype=np.int32)
            keep["pp"] = np.array(ops, dtype=np.uint8)
            p.n_pauli = len(self.pauli)
            p.pauli_offsets = _ptr(keep["po"], C.c_int32)
            p.pauli_sites = _ptr(keep["ps"], C.c_int32)
            p.pauli_ops = _ptr(keep["pp"], C.c_uint8)
        return p, keep


def spec_from_lattice(lat, theta, depth, chi, **kw) -> ProblemSpec:
    return ProblemSpec(lat.n_sites, lat.edges, lat.colour, theta, depth, chi, **kw)


def torch_allocator(device: int = 0):
    """(alloc, free) for Context.set_allocator that take the memory from torch's caching allocator,
    on the library's stream (torch then reuses a returned block in that stream's order only)."""
    import torch

    def alloc(nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(nbytes, device, stream or 0)
        except torch.OutOfMemoryError:
            return None

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, free


class Context:
    """A device context (HIP device, stream, memory budget)."""

    def __init__(self, device: int = 0, stream: int | None = None, mem_budget: int = 0,
                 lib=None):
        self.lib = lib or load()
        h = C.c_void_p()
        _check(self.lib, self.lib.bpki_create(C.byref(h), device,
                                              C.c_void_p(stream) if stream else None,
                                              mem_budget))
        self.h = h

    def set_allocator(self, alloc, free):
        """Take the context's device memory from alloc(nbytes, stream) -> pointer (int, or None
        when there is none) and give it back with free(ptr, stream); streams are hipStream_t
        handles as ints (None for the null stream).  Before the first solve, session or submit.
        The callbacks run on the library's threads (serving slots included).  (None, None) keeps
        hipMalloc and hipFree."""
        if alloc is None and free is None:
            self._alloc_cb, self._free_cb = AllocFn(), FreeFn()       # NULL function pointers
        else:
            self._alloc_cb = AllocFn(lambda n, stream, user: alloc(n, stream))
            self._free_cb = FreeFn(lambda p, stream, user: free(p, stream))
        _check(self.lib, self.lib.bpki_set_allocator(self.h, self._alloc_cb, self._free_cb, None))

    def close(self):
        if self.h:
            self.lib.bpki_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- blocking solve ------------------------------------------------------------------
    def solve(self, spec: ProblemSpec) -> dict:
        p, keep = spec.to_c()
        out = _alloc_result(spec)
        r = _result_struct(out)
        rc = _check(self.lib, self.lib.bpki_solve(self.h, C.byref(p), C.byref(r)))
        out["status"] = rc
        return out

    def solve_noalloc(self, spec: ProblemSpec) -> dict:
        """bpki_solve on the library's static device scratch (no device allocation in the
        call); problems above its size are refused with -4."""
        p, keep = spec.to_c()
        out = _alloc_result(spec)
        r = _result_struct(out)
        rc = _check(self.lib, self.lib.bpki_solve_noalloc(self.h, C.byref(p), C.byref(r)))
        out["status"] = rc
        return out

    # -- serving ---------------------------------------------------------------------------
    def submit(self, spec: ProblemSpec):
        p, keep = spec.to_c()
        out = _alloc_result(spec)
        r = _result_struct(out)
        t = C.c_uint64()
        _check(self.lib, self.lib.bpki_submit(self.h, C.byref(p), C.byref(r), C.byref(t)))
        return Ticket(self, int(t.value), out, r, keep)

    def serving_config(self, slots: int):
        _check(self.lib, self.lib.bpki_serving_config(self.h, slots))

    def serving_packing(self, max_requests: int, max_chi: int = 32):
        """Cross-request packing limits (max_requests = 1 turns packing off)."""
        _check(self.lib, self.lib.bpki_serving_packing(self.h, max_requests, max_chi))

    def session(self, spec: ProblemSpec) -> "Session":
        return Session(self, spec)

    # -- test hooks ------------------------------------------------------------------------
    def test_gemm(self, desc: dict, A, B, Cm, nprob: int = 1):
        d = TestGemmDesc()
        defaults = dict(Mi=None, Ni=None, Ki=None, batch=1, conjA=0, conjB=0, beta=0,
                        alpha_re=1.0, alpha_im=0.0, prec=0, herm=0)
        full = {**defaults, **desc}
        for k in ("M", "N", "K"):
            if full.get(k + "i") is None:
                full[k + "i"] = full[k]
        for name, _ in TestGemmDesc._fields_:
            setattr(d, name, full.get(name, 0))
        A = np.ascontiguousarray(A, dtype=np.complex128)
        B = np.ascontiguousarray(B, dtype=np.complex128)
        Cm = np.ascontiguousarray(Cm, dtype=np.complex128).copy()
        dp = C.POINTER(C.c_double)
        _check(self.lib, self.lib.bpki_test_gemm(
            self.h, C.byref(d), nprob, A.ctypes.data_as(dp), A.size // nprob,
            B.ctypes.data_as(dp), B.size // nprob, Cm.ctypes.data_as(dp), Cm.size // nprob))
        return Cm

    def test_gram_chol(self, G: np.ndarray, cut: float = 1e-15):
        G = np.ascontiguousarray(G, dtype=np.complex128)
        nprob, n, _ = G.shape
        R = np.zeros((nprob, n, n), dtype=np.complex128)
        W = np.zeros((nprob, n, n), dtype=np.complex128)
        dp = C.POINTER(C.c_double)
        _check(self.lib, self.lib.bpki_test_gram_chol(self.h, n, nprob, G.ctypes.data_as(dp), cut,
                                                      R.ctypes.data_as(dp), W.ctypes.data_as(dp)))
        return R, W

    def test_mfma_rate(self, precision: int = 0, blocks: int = 1024, iters: int = 2000) -> float:
        """Achievable MFMA TFLOP/s (FP64 for precision 0, FP32 for 1) with no memory traffic."""
        out = C.c_double()
        _check(self.lib, self.lib.bpki_test_mfma_rate(self.h, precision, blocks, iters,
                                                      C.byref(out)))
        return out.value

    def test_bp_close(self, Y, T, M, rs: int, qs: int, cs: int, ss: int, precision: int = 0,
                      store32: int = 0, xdim: int | None = None, pair: int = 0):
        """Fused BP message at chi = 32 or 64, chi = M.shape[-1] (see bpki_testing.h): Y, T
        [nprob][elems], M [nprob][chi][chi] -> out [nprob][chi][chi]; xdim chi (degree 3, the
        default) or 1 (degree 2); pair = 1: Y conj(T) with no message applied (M gives chi only)."""
        Y = np.ascontiguousarray(Y, dtype=np.complex128)
        T = np.ascontiguousarray(T, dtype=np.complex128)
        M = np.ascontiguousarray(M, dtype=np.complex128)
        nprob, chi = Y.shape[0], M.shape[-1]
        out = np.zeros((nprob, chi, chi), dtype=np.complex128)
        dp = C.POINTER(C.c_double)
        _check(self.lib, self.lib.bpki_test_bp_close(
            self.h, chi, precision, store32, pair, rs, qs, cs, ss, chi if xdim is None else xdim,
            nprob,
            Y.ctypes.data_as(dp),
            T.ctypes.data_as(dp), Y.size // nprob, M.ctypes.data_as(dp), out.ctypes.data_as(dp)))
        return out

    def test_eigh(self, A: np.ndarray, ncols: int | None = None):
        """Eigenvalues (descending) and eigenvectors; with ncols only the leading ncols columns
        are computed from n = 32 up (the others stay zero)."""
        A = np.ascontiguousarray(A, dtype=np.complex128)
        nprob, n, _ = A.shape
        ev = np.zeros((nprob, n))
        V = np.zeros((nprob, n, n), dtype=np.complex128)
        dp = C.POINTER(C.c_double)
        _check(self.lib, self.lib.bpki_test_eigh(self.h, n, nprob, n if ncols is None else ncols,
                                                 A.ctypes.data_as(dp), ev.ctypes.data_as(dp),
                                                 V.ctypes.data_as(dp)))
        return ev, V


def _alloc_result(spec: ProblemSpec) -> dict:
    steps = spec.depth + spec.clifford_steps
    rows = steps if spec.record_every_step else 1
    return {
        "z": np.full((max(rows, 1), spec.n_sites), np.nan),
        "pauli": np.zeros(len(spec.pauli)),
        "bp_iters": np.zeros(max(steps, 1), dtype=np.int32),
        "bp_residual": np.zeros(max(steps, 1)),
        "discarded": np.zeros(max(steps, 1)),
        "bond_entropy": (np.full((max(rows, 1), int(np.asarray(spec.edges).size // 2)), np.nan)
                         if spec.bond_entropy else None),
        "bond_dims": np.zeros((max(rows, 1), int(np.asarray(spec.edges).size // 2)),
                              dtype=np.int32),
        "min_cut_gap": np.zeros(max(steps, 1)),
        "degenerate_cuts": np.zeros(max(steps, 1), dtype=np.int32),
    }


def _result_struct(out: dict) -> _Result:
    r = _Result()
    r.z = _ptr(out["z"], C.c_double)
    r.pauli = _ptr(out["pauli"], C.c_double) if out["pauli"].size else None
    r.bp_iters = _ptr(out["bp_iters"], C.c_int32)
    r.bp_residual = _ptr(out["bp_residual"], C.c_double)
    r.discarded = _ptr(out["discarded"], C.c_double)
    if out.get("bond_entropy") is not None:
        r.bond_entropy = _ptr(out["bond_entropy"], C.c_double)
    r.bond_dims = _ptr(out["bond_dims"], C.c_int32)
    r.min_cut_gap = _ptr(out["min_cut_gap"], C.c_double)
    r.degenerate_cuts = _ptr(out["degenerate_cuts"], C.c_int32)
    return r


class Ticket:
    def __init__(self, ctx, t, out, r, keep):
        self.ctx, self.t, self.out, self._r, self._keep = ctx, t, out, r, keep

    def poll(self) -> bool:
        d = C.c_int()
        _check(self.ctx.lib, self.ctx.lib.bpki_poll(self.ctx.h, self.t, C.byref(d)))
        return bool(d.value)

    def wait(self) -> dict:
        rc = _check(self.ctx.lib, self.ctx.lib.bpki_wait(self.ctx.h, self.t))
        self.out["status"] = rc
        return self.out

    def cancel(self):
        _check(self.ctx.lib, self.ctx.lib.bpki_cancel(self.ctx.h, self.t))

    def times(self):
        """(submitted, started, finished) host steady-clock seconds."""
        t = np.zeros(3)
        _check(self.ctx.lib, self.ctx.lib.bpki_ticket_times(self.ctx.h, self.t,
                                                            _ptr(t, C.c_double)))
        return t

    def pack_size(self) -> int:
        """Problems in the pack that ran this ticket (1 = alone, 0 = not started)."""
        n = C.c_int32()
        _check(self.ctx.lib, self.ctx.lib.bpki_ticket_pack_size(self.ctx.h, self.t, C.byref(n)))
        return int(n.value)


class Session:
    """Step-by-step access to one resident state (every phase of a Floquet step)."""

    def __init__(self, ctx: Context, spec: ProblemSpec):
        self.ctx, self.lib, self.spec = ctx, ctx.lib, spec
        p, self._keep = spec.to_c()
        self._p = p
        h = C.c_void_p()
        _check(self.lib, self.lib.bpki_session_open(ctx.h, C.byref(p), C.byref(h)))
        self.h = h
        te, me = C.c_size_t(), C.c_size_t()
        _check(self.lib, self.lib.bpki_session_sizes(h, C.byref(te), C.byref(me)))
        self.tensor_elems, self.message_elems = te.value, me.value

    def close(self):
        if self.h:
            self.lib.bpki_session_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_state(self):
        t = np.zeros(self.tensor_elems, dtype=np.complex128)
        m = np.zeros(self.message_elems, dtype=np.complex128)
        b = np.zeros(len(np.asarray(self.spec.edges).reshape(-1)) // 2, dtype=np.int32)
        dp = C.POINTER(C.c_double)
        _check(self.lib, self.lib.bpki_session_get_state(self.h, t.ctypes.data_as(dp),
                                                         m.ctypes.data_as(dp),
                                                         _ptr(b, C.c_int32)))
        return t, m, b

    def set_state(self, t, m, b=None):
        t = np.ascontiguousarray(t, dtype=np.complex128)
        m = np.ascontiguousarray(m, dtype=np.complex128)
        dp = C.POINTER(C.c_double)
        bb = None if b is None else np.ascontiguousarray(b, dtype=np.int32)
        _check(self.lib, self.lib.bpki_session_set_state(self.h, t.ctypes.data_as(dp),
                                                         m.ctypes.data_as(dp),
                                                         _ptr(bb, C.c_int32)))

    def apply_rx(self):
        _check(self.lib, self.lib.bpki_session_apply_rx(self.h))

    def apply_layer(self, colour: int) -> float:
        d = C.c_double()
        _check(self.lib, self.lib.bpki_session_apply_layer(self.h, colour, C.byref(d)))
        return d.value

    def layer_cuts(self):
        """Per edge, for the edges the last layer updated: (kept bond dimension, discarded
        weight, cut gap); -1 / NaN elsewhere."""
        ne = int(np.asarray(self.spec.edges).size // 2)
        k, d, g = np.zeros(ne, dtype=np.int32), np.zeros(ne), np.zeros(ne)
        _check(self.lib, self.lib.bpki_session_layer_cuts(self.h, _ptr(k, C.c_int32),
                                                          _ptr(d, C.c_double),
                                                          _ptr(g, C.c_double)))
        return k, d, g

    def bp(self, max_iter: int = 1000):
        it, r = C.c_int32(), C.c_double()
        rc = _check(self.lib, self.lib.bpki_session_bp(self.h, max_iter, C.byref(it),
                                                       C.byref(r)))
        return it.value, r.value, rc

    def bp_sweep(self) -> float:
        r = C.c_double()
        _check(self.lib, self.lib.bpki_session_bp_sweep(self.h, C.byref(r)))
        return r.value

    def observe_z(self) -> np.ndarray:
        z = np.zeros(self.spec.n_sites)
        _check(self.lib, self.lib.bpki_session_observe_z(self.h, _ptr(z, C.c_double)))
        return z

    def observe_bond_entropy(self) -> np.ndarray:
        """Entropy (bits) of the Schmidt weights of every edge, in edge order."""
        e = np.zeros(int(np.asarray(self.spec.edges).size // 2))
        _check(self.lib, self.lib.bpki_session_observe_bond_entropy(self.h, _ptr(e, C.c_double)))
        return e

    def vidal_gauge(self) -> np.ndarray:
        """Transform the state in place into the symmetric Vidal gauge; returns the bond weights
        S [n_edges, chi] (descending, unit 2-norm, zero-padded)."""
        lam = np.zeros((int(np.asarray(self.spec.edges).size // 2), int(self.spec.chi)))
        _check(self.lib, self.lib.bpki_session_vidal_gauge(self.h, _ptr(lam, C.c_double)))
        return lam

    def bp_error(self, edge: int):
        """BP error estimate on `edge` of a ring lattice (chi <= 16); leaves the state in the
        symmetric gauge.  Returns (error, singular values of the edge environment, unit norm)."""
        err = C.c_double()
        sp = np.zeros(int(self.spec.chi) ** 2)
        _check(self.lib, self.lib.bpki_session_bp_error(self.h, int(edge), C.byref(err),
                                                        _ptr(sp, C.c_double)))
        return err.value, sp

    def observe_pauli(self) -> np.ndarray:
        out = np.zeros(len(self.spec.pauli))
        _check(self.lib, self.lib.bpki_session_observe_pauli(
            self.h, _ptr(out, C.c_double) if out.size else None))
        return out

    def step(self, observe: bool = True):
        z = np.zeros(self.spec.n_sites) if observe else None
        it, r, d = C.c_int32(), C.c_double(), C.c_double()
        rc = _check(self.lib, self.lib.bpki_session_step(
            self.h, _ptr(z, C.c_double) if observe else None, C.byref(it), C.byref(r),
            C.byref(d)))
        return {"z": z, "bp_iters": it.value, "bp_residual": r.value, "discarded": d.value,
                "status": rc}

    def clifford_inverse_step(self, observe: bool = True):
        """One step of U(pi/2)^dagger (gates with exp(-i pi/4 ZZ) in descending colour, X
        rotations by -pi/2), BP, then <Z> if observe."""
        z = np.zeros(self.spec.n_sites) if observe else None
        it, r, d = C.c_int32(), C.c_double(), C.c_double()
        rc = _check(self.lib, self.lib.bpki_session_clifford_inverse_step(
            self.h, _ptr(z, C.c_double) if observe else None, C.byref(it), C.byref(r),
            C.byref(d)))
        return {"z": z, "bp_iters": it.value, "bp_residual": r.value, "discarded": d.value,
                "status": rc}

    def profile(self, enable: bool = True, stride: int = 1):
        """Bracket every `stride`-th GEMM launch with HIP events (off when enable is False)."""
        _check(self.lib, self.lib.bpki_session_profile(self.h, stride if enable else 0))

    def profile_read(self):
        n, ms, fl, a = C.c_int64(), C.c_double(), C.c_double(), C.c_int64()
        _check(self.lib, self.lib.bpki_session_profile_read(self.h, C.byref(n), C.byref(ms),
                                                            C.byref(fl), C.byref(a)))
        return {"launches": n.value, "ms": ms.value, "flops": fl.value,
                "all_launches": a.value}

    def profile_read_prec(self, prec: int):
        """The bracketed GEMM launches of one arithmetic (0 FP64, 1 FP32 MFMA)."""
        n, ms, fl = C.c_int64(), C.c_double(), C.c_double()
        _check(self.lib, self.lib.bpki_session_profile_read_prec(self.h, prec, C.byref(n),
                                                                 C.byref(ms), C.byref(fl)))
        return {"launches": n.value, "ms": ms.value, "flops": fl.value}

    def profile_read_kernel(self, kernel: int, prec: int = 0):
        """The bracketed launches of one kernel (0 gemm_kernel, 1 the fused BP closing
        bp_close_kernel, 2 gemm_stream_kernel) in one arithmetic (0 FP64, 1 FP32 MFMA): count,
        summed ms, algorithmic flops and algorithmic HBM bytes, and the count of all its
        launches."""
        n, ms, fl, by, al = C.c_int64(), C.c_double(), C.c_double(), C.c_double(), C.c_int64()
        _check(self.lib, self.lib.bpki_session_profile_read_kernel(
            self.h, kernel, prec, C.byref(n), C.byref(ms), C.byref(fl), C.byref(by),
            C.byref(al)))
        return {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value,
                "all_launches": al.value}

    def last_timing(self) -> np.ndarray:
        t = np.zeros(4)
        _check(self.lib, self.lib.bpki_session_last_timing(self.h, _ptr(t, C.c_double)))
        return t


def solve(lat, theta: float, depth: int, chi: int, ctx: Context | None = None, **kw) -> dict:
    """Convenience: one blocking solve on a lattice from ``paper_2306_14887_amd.lattice``."""
    own = ctx is None
    ctx = ctx or Context()
    try:
        return ctx.solve(spec_from_lattice(lat, theta, depth, chi, **kw))
    finally:
        if own:
            ctx.close()
