"""Host-side checks of the C ABI: the library loads, exports every symbol the headers declare,
validates problems and estimates memory without a device, and refuses to run without one."""
import os
import re

import numpy as np
import pytest

from paper_2306_14887_amd import bpki as B
from paper_2306_14887_amd import lattice as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libbpki.so not built")
    return B.load()


def _declared():
    names = set()
    for h in ("bpki.h", "bpki_testing.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"\b(bpki_[a-z_0-9]+)\s*\(", txt))
    return names


def test_exports_every_declared_symbol():
    lib = _lib()
    declared = _declared()
    assert len(declared) >= 20
    for n in sorted(declared):
        assert hasattr(lib, n), n
    assert declared == set(B.exported_symbols())


def _spec(lat, **kw):
    base = dict(theta=0.3, depth=2, chi=4)
    base.update(kw)
    return B.spec_from_lattice(lat, **base)


def _validate(spec):
    lib = _lib()
    p, keep = spec.to_c()
    return lib.bpki_validate(p)


def test_validate_accepts_lattices():
    for lat in (L.eagle(), L.hexagon_ring(), L.heavy_hex(3, 9), L.path(2)):
        assert _validate(_spec(lat)) == 0


def test_validate_error_codes():
    e = L.eagle()
    assert _validate(_spec(e, chi=0)) == -1
    assert _validate(_spec(e, chi=257)) == -1
    assert _validate(_spec(e, chi=256)) == 0                # no two degree-3 sites adjacent
    h = L.Lattice(6, np.array([[0, 1], [0, 2], [0, 3], [1, 4], [1, 5]], dtype=np.int32),
                  np.array([0, 1, 2, 1, 2], dtype=np.int32))
    assert _validate(_spec(h, chi=128)) == 0                 # degree-3 pair: 4 chi <= 512
    assert _validate(_spec(h, chi=129)) == -1
    assert _validate(_spec(e, depth=-1)) == -1
    assert _validate(_spec(e, theta=float("nan"))) == -1
    assert _validate(_spec(e, bp_max_iter=0)) == -1
    bad = L.Lattice(3, np.array([[0, 0], [1, 2]], dtype=np.int32), np.array([0, 1], np.int32))
    assert _validate(_spec(bad)) == -2                      # self loop
    dup = L.Lattice(3, np.array([[0, 1], [1, 0], [1, 2]], np.int32), np.array([0, 1, 2], np.int32))
    assert _validate(_spec(dup)) == -2                      # duplicate edge
    star = L.Lattice(5, np.array([[0, 1], [0, 2], [0, 3], [0, 4]], np.int32),
                     np.arange(4, dtype=np.int32))
    assert _validate(_spec(star)) == -2                     # degree 4
    iso = L.Lattice(3, np.array([[0, 1]], np.int32), np.array([0], np.int32))
    assert _validate(_spec(iso)) == -2                      # isolated site
    col = L.Lattice(3, np.array([[0, 1], [1, 2]], np.int32), np.array([0, 0], np.int32))
    assert _validate(_spec(col)) == -3                      # improper colouring
    # Pauli strings: op range, repeated site, clusters with more than one loop, loops at chi > 64
    r = L.hexagon_ring()
    assert _validate(_spec(r, pauli=[([0, 1], [1, 4])])) == -1
    assert _validate(_spec(r, pauli=[([0, 0], [1, 1])])) == -1
    assert _validate(_spec(r, pauli=[(list(range(12)), [3] * 12)])) == 0    # one loop
    assert _validate(_spec(r, chi=128, pauli=[(list(range(12)), [3] * 12)])) == -1
    hh = L.heavy_hex(3, 9)                                                    # two loops
    assert _validate(_spec(hh, pauli=[(list(range(hh.n_sites)), [3] * hh.n_sites)])) == -1
    assert _validate(_spec(r, pauli=[([0, 5], [3, 3])])) == -1               # disconnected
    assert _validate(_spec(r, pauli=[([0, 1, 2], [1, 2, 3])])) == 0


def test_null_colouring_uses_greedy():
    lib = _lib()
    e = L.eagle()
    spec = B.ProblemSpec(e.n_sites, e.edges, None, 0.3, 1, 4)
    p, keep = spec.to_c()
    assert lib.bpki_validate(p) == 0


def test_estimate_bytes_scales_like_chi_cubed():
    lib = _lib()
    import ctypes as C
    e = L.eagle()
    sizes = []
    for chi in (16, 32, 64):
        p, keep = _spec(e, chi=chi).to_c()
        b = C.c_size_t()
        assert lib.bpki_estimate_bytes(p, C.byref(b)) == 0
        sizes.append(b.value)
    assert sizes[0] < sizes[1] < sizes[2]
    # degree-3 tensors dominate: 36 sites of 2*chi^3 complex128
    assert sizes[2] > 36 * 2 * 64 ** 3 * 16


def test_create_without_device_fails_loudly():
    lib = _lib()
    import ctypes as C
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a device is present")
    except ImportError:
        pass
    h = C.c_void_p()
    rc = lib.bpki_create(C.byref(h), 0, None, 0)
    assert rc == -5
    assert b"HIP" in lib.bpki_last_error() or b"device" in lib.bpki_last_error()


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: --gpus N > 1 exits with status 2 and says why, before any
    device work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
