"""The allocation-free solve (bpki_solve_noalloc) against bpki_solve through the C ABI.

The entry point takes every device buffer from the library's static per-device scratch array, so
two calls in a row must each match the allocating solve of the same problem (the second one
smaller than the first, on memory that still holds the first call's contents), and a problem
larger than the array is refused with -4."""
import math

import numpy as np
import pytest

from paper_2306_14887_amd import lattice as L

pytestmark = pytest.mark.gpu
TOL = 1e-8          # FP64 parity tolerance of the path (the same kernels run in both entries)


def _same(a, b):
    assert a["status"] == b["status"]
    assert np.abs(a["z"] - b["z"]).max() < TOL
    assert a["pauli"].size == b["pauli"].size
    if a["pauli"].size:
        assert np.abs(a["pauli"] - b["pauli"]).max() < TOL
    assert np.array_equal(a["bp_iters"], b["bp_iters"])
    assert np.array_equal(a["bond_dims"], b["bond_dims"])
    assert np.abs(a["discarded"] - b["discarded"]).max() < TOL


def test_noalloc_matches_solve_twice_then_refuses_too_large():
    from paper_2306_14887_amd import bpki as B
    print("[noalloc] 29-qubit chi=16, then the 12-ring chi=4, then a too-large problem", flush=True)
    hh = L.heavy_hex(3, 9)
    ps = L.random_pauli_strings(hh, 3, seed=4, wmin=2, wmax=5)
    big = B.spec_from_lattice(hh, 0.9, 8, 16, pauli=[(p.sites, p.ops) for p in ps])
    small = B.spec_from_lattice(L.hexagon_ring(), math.pi / 4, 5, 4)
    with B.Context() as ctx:
        want_big, want_small = ctx.solve(big), ctx.solve(small)
        got_big = ctx.solve_noalloc(big)
        got_small = ctx.solve_noalloc(small)
        _same(got_big, want_big)
        _same(got_small, want_small)
        assert max(want_big["discarded"]) > 1e-6          # truncation active in the big one
        with pytest.raises(B.BpkiError) as ex:
            ctx.solve_noalloc(B.spec_from_lattice(L.eagle(), 0.5, 3, 32))
        assert ex.value.code == -4 and "scratch" in str(ex.value)
        # still usable after the refusal
        _same(ctx.solve_noalloc(small), want_small)
