"""The caller's device allocator (bpki_set_allocator): every device buffer of a solve, a session
and the serving slots comes from it and goes back to it, and the results equal those of a context
on hipMalloc."""
import threading

import numpy as np
import pytest

from paper_2306_14887_amd import lattice as L

pytestmark = pytest.mark.gpu


class _Counting:
    """Wraps (alloc, free), keeping the live pointers and their sizes; callable from any thread."""

    def __init__(self, alloc, free):
        self.a, self.f = alloc, free
        self.live = {}
        self.n_alloc = self.n_free = self.bad_free = 0
        self.streams = set()
        self.lock = threading.Lock()

    def alloc(self, n, stream):
        p = self.a(n, stream)
        with self.lock:
            self.n_alloc += 1
            self.streams.add(stream)
            if p:
                self.live[p] = n
        return p

    def free(self, p, stream):
        with self.lock:
            self.n_free += 1
            if self.live.pop(p, None) is None:
                self.bad_free += 1
        self.f(p, stream)


def _spec(seed=11, theta=0.8, depth=4, chi=16):
    from paper_2306_14887_amd import bpki as B
    lat = L.heavy_hex(3, 9)
    ps = L.random_pauli_strings(lat, 4, seed=seed, wmin=2, wmax=5)
    return B.spec_from_lattice(lat, theta, depth, chi, pauli=[(p.sites, p.ops) for p in ps],
                               bond_entropy=True)


def _same(a, b):
    assert a["status"] == b["status"] == 0
    assert np.abs(a["z"] - b["z"]).max() <= 1e-12
    assert np.abs(a["pauli"] - b["pauli"]).max() <= 1e-12
    assert np.abs(a["bond_entropy"] - b["bond_entropy"]).max() <= 1e-12
    assert np.array_equal(a["bp_iters"], b["bp_iters"])


def test_solve_on_torch_allocator_matches_hipmalloc():
    import torch
    from paper_2306_14887_amd import bpki as B
    print("[allocator] solve on torch's caching allocator vs hipMalloc", flush=True)
    spec = _spec()
    with B.Context() as ctx:
        ref = ctx.solve(spec)
    torch.cuda.synchronize(0)
    base = torch.cuda.memory_allocated(0)
    cnt = _Counting(*B.torch_allocator(0))
    ctx = B.Context()
    ctx.set_allocator(cnt.alloc, cnt.free)
    out = ctx.solve(spec)
    # the solve's own buffers went back; the context keeps its workspaces until it is destroyed
    assert cnt.n_alloc > cnt.n_free > 0 and cnt.bad_free == 0
    assert torch.cuda.memory_allocated(0) - base >= sum(cnt.live.values()) > 0
    assert len(cnt.streams) == 1 and None not in cnt.streams     # the context's own stream
    again = ctx.solve(spec)
    ctx.close()
    assert not cnt.live and cnt.bad_free == 0 and cnt.n_free == cnt.n_alloc
    assert torch.cuda.memory_allocated(0) == base
    _same(out, ref)
    _same(again, ref)


def test_allocator_only_before_device_memory():
    from paper_2306_14887_amd import bpki as B
    print("[allocator] refused once the context holds memory; both callbacks or neither",
          flush=True)
    with B.Context() as ctx:
        ctx.solve(_spec(depth=1, chi=4))
        with pytest.raises(B.BpkiError) as ex:
            ctx.set_allocator(*B.torch_allocator(0))
        assert ex.value.code == -1
    with B.Context() as ctx:
        lib = ctx.lib
        keep = B.AllocFn(lambda n, s, u: None)
        assert lib.bpki_set_allocator(ctx.h, keep, B.FreeFn(), None) == -1
        assert lib.bpki_set_allocator(None, B.AllocFn(), B.FreeFn(), None) == -1
        ctx.set_allocator(None, None)                                    # hipMalloc again
        out = ctx.solve(_spec(depth=1, chi=4))
        assert out["status"] == 0


def test_session_and_serving_slots_use_the_allocator():
    import torch
    from paper_2306_14887_amd import bpki as B
    print("[allocator] serving slots and a session on the caller's allocator", flush=True)
    specs = [_spec(seed=20 + i, theta=0.3 + 0.2 * i, depth=2 + i) for i in range(4)]
    with B.Context() as ctx:
        alone = [ctx.solve(s) for s in specs]
        s = ctx.session(specs[0])
        z_ref = [s.step()["z"] for _ in range(2)]
        s.close()
    torch.cuda.synchronize(0)
    base = torch.cuda.memory_allocated(0)
    cnt = _Counting(*B.torch_allocator(0))
    ctx = B.Context()
    ctx.set_allocator(cnt.alloc, cnt.free)
    ctx.serving_config(2)
    ctx.serving_packing(1)
    tickets = [ctx.submit(s) for s in specs]
    outs = [t.wait() for t in tickets]
    s = ctx.session(specs[0])
    z = [s.step()["z"] for _ in range(2)]
    s.close()
    ctx.close()
    assert not cnt.live and cnt.bad_free == 0 and cnt.n_free == cnt.n_alloc
    assert len(cnt.streams) >= 2                  # the slots' streams and the context's
    assert torch.cuda.memory_allocated(0) == base
    for o, a in zip(outs, alone):
        _same(o, a)
    for a, b in zip(z, z_ref):
        assert np.abs(a - b).max() <= 1e-12


def test_allocator_failures():
    """No memory from the allocator: the solve fails with -4 before any kernel runs; memory not
    aligned to 256 bytes goes back to the allocator and the solve fails with -5."""
    import torch
    from paper_2306_14887_amd import bpki as B
    print("[allocator] allocator out of memory / misaligned", flush=True)
    spec = _spec(depth=1, chi=4)
    calls = []
    ctx = B.Context()
    ctx.set_allocator(lambda n, s: calls.append(n), lambda p, s: calls.append(-1))
    with pytest.raises(B.BpkiError) as ex:
        ctx.solve(spec)
    assert ex.value.code == -4
    assert calls and all(n > 0 for n in calls)              # never asked to free NULL
    ctx.close()

    torch.cuda.synchronize(0)
    base = torch.cuda.memory_allocated(0)
    ta, tf = B.torch_allocator(0)
    given = {}

    def alloc(n, s):
        p = ta(n + 256, s)
        given[p + 16] = p
        return p + 16

    def free(p, s):
        tf(given.pop(p), s)

    ctx = B.Context()
    ctx.set_allocator(alloc, free)
    with pytest.raises(B.BpkiError) as ex:
        ctx.solve(spec)
    assert ex.value.code == -5
    ctx.close()
    assert not given
    assert torch.cuda.memory_allocated(0) == base


def test_serving_slot_recovers_after_allocation_failure():
    """A request whose memory the allocator refuses fails with -4, and the requests that the same
    serving slot takes afterwards still succeed (the slot replaces its backend once a job has
    left it in an error state) with the results of their solves alone."""
    import torch
    from paper_2306_14887_amd import bpki as B
    print("[allocator] serving slot after a refused allocation", flush=True)
    ta, tf = B.torch_allocator(0)
    limit = 8 << 20

    def alloc(n, s):
        return None if n > limit else ta(n, s)

    big = B.spec_from_lattice(L.eagle(), 0.5, 3, 32)
    small = [_spec(seed=20 + i, theta=0.3 + 0.2 * i, depth=3, chi=8) for i in range(3)]
    with B.Context() as ref_ctx:
        alone = [ref_ctx.solve(s) for s in small]
    torch.cuda.synchronize(0)
    base = torch.cuda.memory_allocated(0)
    ctx = B.Context()
    ctx.set_allocator(alloc, tf)
    ctx.serving_config(1)
    t_big = ctx.submit(big)
    with pytest.raises(B.BpkiError) as ex:
        t_big.wait()
    assert ex.value.code == -4
    outs = [ctx.submit(s).wait() for s in small]
    ctx.close()
    for o, a in zip(outs, alone):
        _same(o, a)
    torch.cuda.synchronize(0)
    assert torch.cuda.memory_allocated(0) == base
