"""Serving (continuous batching) on the GPU: results are the same alone and in the mix,
packed requests match their solves alone, admission respects the memory budget, cancellation
and rejection work."""
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
        ctx.serving_packing(1)
        tickets = [ctx.submit(s) for s in specs]
        mixed = [t.wait() for t in tickets]
    with B.Context() as ctx:
        for s, m in zip(specs, mixed):
            alone = ctx.solve(s)
            assert m["status"] == alone["status"]
            assert np.abs(m["z"] - alone["z"]).max() <= 1e-12


def _pack_specs():
    """Eight requests that share a lattice, chi, precision and tolerances (so they pack): their
    own angles, depths, Pauli strings and recording modes."""
    from paper_2306_14887_amd import bpki as B
    lat = L.heavy_hex(3, 9)
    rng = np.random.default_rng(7)
    out = []
    for i in range(8):
        ps = L.random_pauli_strings(lat, 3, seed=200 + i, wmin=2, wmax=6)
        out.append(B.spec_from_lattice(lat, float(rng.uniform(0.0, 1.5)), int(rng.integers(1, 9)),
                                       8, pauli=[(p.sites, p.ops) for p in ps],
                                       record_every_step=int(i % 3 != 0),
                                       bond_entropy=i % 2 == 0))
    return out


def test_packed_requests_match_alone():
    """Queued requests on one lattice are packed into one solve on the union of their lattices;
    each member follows its own BP stopping point, so it matches its solve alone (to rounding)
    and, through it, the oracle."""
    from paper_2306_14887_amd import bpki as B
    from oracle import bp_tns as O
    print("[serving] packed requests vs alone", flush=True)
    specs = _pack_specs()
    with B.Context() as ctx:
        ctx.serving_config(1)
        ctx.serving_packing(16, 32)
        # a request on another lattice occupies the slot while the eight queue up; the deepest
        # request goes first so that it heads the pack (companions end no later than the head)
        blocker = ctx.submit(B.spec_from_lattice(L.heavy_hex(5, 11), 0.7, 6, 16))
        order = sorted(range(len(specs)), key=lambda i: -specs[i].depth)
        tickets = [None] * len(specs)
        for i in order:
            tickets[i] = ctx.submit(specs[i])
        blocker.wait()
        while not all(t.poll() for t in tickets):
            time.sleep(0.002)
        packs = [t.pack_size() for t in tickets]
        outs = [t.wait() for t in tickets]
    assert min(packs) == len(specs)
    with B.Context() as ctx:
        for s, o in zip(specs, outs):
            alone = ctx.solve(s)
            assert o["status"] == alone["status"] == 0
            assert np.abs(o["z"] - alone["z"]).max() < 1e-10
            assert np.abs(o["pauli"] - alone["pauli"]).max() < 1e-10
            d = s.depth
            assert np.abs(o["bp_iters"][:d] - alone["bp_iters"][:d]).max() <= 1
            assert np.abs(o["discarded"][:d] - alone["discarded"][:d]).max() < 1e-10
            if s.bond_entropy:
                assert np.abs(o["bond_entropy"] - alone["bond_entropy"]).max() < 1e-10
    lat = L.heavy_hex(3, 9)
    s, o = specs[1], outs[1]
    ref = O.solve(lat.n_sites, lat.edges, lat.colour, s.theta, s.depth, O.Options(chi=8),
                  pauli=s.pauli)
    assert np.abs(o["z"] - ref.z).max() < 1e-8
    assert np.abs(o["pauli"] - ref.pauli).max() < 1e-8


def test_requests_on_different_lattices_pack_together():
    """Queued requests with the same chi on lattices of 29, 65 and 127 qubits are packed into one
    solve on the union graph; each equals its solve alone (to rounding), bond dimensions included."""
    from paper_2306_14887_amd import bpki as B
    print("[serving] packing across lattices", flush=True)
    lats = [L.heavy_hex(3, 9), L.heavy_hex(5, 11), L.eagle(), L.heavy_hex(3, 9)]
    specs = [B.spec_from_lattice(lat, 0.5 + 0.2 * i, 6 - (i % 2), 8)
             for i, lat in enumerate(lats)]
    with B.Context() as ctx:
        ctx.serving_config(1)
        blocker = ctx.submit(B.spec_from_lattice(L.heavy_hex(5, 11), 0.7, 4, 16))
        order = sorted(range(len(specs)), key=lambda i: -specs[i].depth)
        tickets = [None] * len(specs)
        for i in order:
            tickets[i] = ctx.submit(specs[i])
        blocker.wait()
        while not all(t.poll() for t in tickets):
            time.sleep(0.002)
        packs = [t.pack_size() for t in tickets]
        outs = [t.wait() for t in tickets]
    assert min(packs) == len(specs)
    with B.Context() as ctx:
        for s, o in zip(specs, outs):
            alone = ctx.solve(s)
            assert o["status"] == alone["status"] == 0
            assert np.abs(o["z"] - alone["z"]).max() < 1e-10
            assert np.array_equal(o["bond_dims"], alone["bond_dims"])
            assert np.abs(o["discarded"] - alone["discarded"]).max() < 1e-10


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


def test_memory_estimate_bounds_the_device_footprint():
    """The admission estimate (bpki_estimate_bytes) bounds what a solve really holds on the device:
    the drop in free device memory (hipMemGetInfo) after opening a session and running two steps
    with every observable, workspaces included."""
    import ctypes as C

    from paper_2306_14887_amd import bpki as B
    print("[serving] memory estimate vs device footprint", flush=True)
    hip = C.CDLL("libamdhip64.so")
    free, total = C.c_size_t(), C.c_size_t()

    def free_bytes():
        assert hip.hipMemGetInfo(C.byref(free), C.byref(total)) == 0
        return free.value

    lib = B.load()
    cases = [(L.eagle(), 32), (L.heavy_hex(5, 11), 64), (L.infinite_cell(), 128),
             (L.infinite_cell(), 256), (L.hexagon_ring(), 16)]
    for lat, chi in cases:                   # a fresh context each: its workspaces start empty
        spec = B.spec_from_lattice(lat, 0.7, 2, chi, bond_entropy=True)
        p, keep = spec.to_c()
        est = C.c_size_t()
        assert lib.bpki_estimate_bytes(p, C.byref(est)) == 0
        with B.Context() as ctx:
            f0 = free_bytes()
            s = ctx.session(spec)
            s.step()
            s.step()
            s.observe_bond_entropy()
            s.vidal_gauge()
            used = f0 - free_bytes()
            s.close()
        print(f"  {lat.name} chi={chi}: estimate {est.value / 2**20:.0f} MiB, "
              f"used {used / 2**20:.0f} MiB", flush=True)
        assert used <= est.value, (lat.name, chi, used, est.value)
