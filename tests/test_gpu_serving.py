"""Serving (continuous batching) on the GPU: results are the same alone and in the mix,
admission respects the memory budget, cancellation and rejection work."""
import time

import numpy as np
import pytest

from paper_2306_14887_amd import lattice as L

pytestmark = pytest.mark.gpu


def _specs(n, seed=0, max_depth=6, max_chi=16):
    from paper_2306_14887_amd import bpki as B
    out = []
    for i, r in enumerate(L.serving_requests(n, seed=seed, rate=100.0)):
        lat = L.heavy_hex(r.rows, r.row_len)
        prec = B.BPKI_FP32 if i % 2 else B.BPKI_FP64
        tol = 1e-6 if prec else 1e-12
        out.append(B.spec_from_lattice(lat, r.theta, min(r.depth, max_depth), min(r.chi, max_chi),
                                       precision=prec, bp_tol=tol))
    return out


def test_same_alone_and_in_the_mix():
    from paper_2306_14887_amd import bpki as B
    print("[serving] 12 requests, 4 slots vs alone", flush=True)
    specs = _specs(12)
    with B.Context() as ctx:
        ctx.serving_config(4)
        tickets = [ctx.submit(s) for s in specs]
        mixed = [t.wait() for t in tickets]
    with B.Context() as ctx:
        for s, m in zip(specs, mixed):
            alone = ctx.solve(s)
            assert m["status"] == alone["status"]
            assert np.abs(m["z"] - alone["z"]).max() <= 1e-12


def test_budget_admission_and_overlap():
    from paper_2306_14887_amd import bpki as B
    import ctypes as C
    print("[serving] memory budget admission", flush=True)
    specs = _specs(6, seed=3)
    lib = B.load()
    sizes = []
    for s in specs:
        p, keep = s.to_c()
        b = C.c_size_t()
        assert lib.bpki_estimate_bytes(p, C.byref(b)) == 0
        sizes.append(b.value)
    budget = 2 * max(sizes)
    with B.Context(mem_budget=budget) as ctx:
        ctx.serving_config(6)
        tickets = [ctx.submit(s) for s in specs]
        while not all(t.poll() for t in tickets):
            time.sleep(0.002)
        times = [t.times() for t in tickets]
        outs = [t.wait() for t in tickets]
    assert all(o["status"] in (0, 1) for o in outs)
    # at every start time, the resident requests' estimates fit the budget
    for i, ti in enumerate(times):
        resident = [sizes[j] for j, tj in enumerate(times) if tj[1] <= ti[1] < tj[2]]
        assert sum(resident) <= budget or len(resident) == 1


def test_cancel_and_reject():
    from paper_2306_14887_amd import bpki as B
    print("[serving] cancel / reject", flush=True)
    e = L.eagle()
    with B.Context() as ctx:
        ctx.serving_config(1)
        long = ctx.submit(B.spec_from_lattice(e, 0.9, 20, 32))
        queued = ctx.submit(B.spec_from_lattice(e, 0.9, 20, 32))
        queued.cancel()
        long.cancel()
        for t in (long, queued):
            with pytest.raises(B.BpkiError) as ex:
                t.wait()
            assert ex.value.code == -6
    with B.Context(mem_budget=1024) as ctx:
        with pytest.raises(B.BpkiError) as ex:
            ctx.submit(B.spec_from_lattice(e, 0.9, 2, 8))
        assert ex.value.code == -4
