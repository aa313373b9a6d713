"""HIP path against the FP64 oracle with truncation active (Methods, "The simple update
procedure": every gate keeps at most chi singular values).

* Whole 127-qubit runs (Fig. 1 lattice, 20 Floquet steps) against golden files written by
  tests/golden/make_eagle_goldens.py, which calls only the oracle: every <Z_v>(t) to 1e-8, the
  bond dimension of every edge after every step exactly, the discarded weight and the BP sweeps.
* One truncating gate layer at the benchmark size (127 qubits, chi = 64) from an identical state:
  per edge the kept bond dimension, the discarded weight, the cut gap, the new bond spectrum
  (the messages diag(S)/sum S) and <Z> afterwards.
* Per-step bond dimensions and discarded weights of smaller truncated runs against the oracle.
"""
import glob
import json
import math
import os

import numpy as np
import pytest

from oracle import bp_tns as O
from paper_2306_14887_amd import lattice as L

from ._state_io import to_flat

pytestmark = pytest.mark.gpu
TOL = 1e-8
GOLD = os.path.join(os.path.dirname(__file__), "golden")
GOLDEN_RUNS = sorted(glob.glob(os.path.join(GOLD, "eagle_chi*_theta*.json")))


@pytest.fixture(scope="module")
def ctx():
    from paper_2306_14887_amd import bpki as B
    c = B.Context()
    yield c
    c.close()


def _spec(lat, theta, depth, chi, **kw):
    from paper_2306_14887_amd import bpki as B
    return B.spec_from_lattice(lat, theta, depth, chi, **kw)


@pytest.mark.parametrize("path", GOLDEN_RUNS, ids=[os.path.basename(p)[:-5] for p in GOLDEN_RUNS])
def test_eagle_truncated_run_matches_oracle(ctx, path):
    """127 qubits, 20 steps, truncation from the step where the bonds saturate: every <Z_v>(t)
    within 1e-8 of the oracle, identical bond dimensions after every step, discarded weights to
    1e-8 (they are sums of Schmidt weights) and BP sweeps within one of the oracle's."""
    g = json.load(open(path))
    lat = L.eagle()
    assert np.array_equal(lat.edges, np.array(g["edges"])) and lat.colour.tolist() == g["colour"]
    print(f"[parity] eagle chi={g['chi']} theta={g['theta']:.4f} {g['depth']} steps vs golden",
          flush=True)
    out = ctx.solve(_spec(lat, g["theta"], g["depth"], g["chi"], bp_tol=g["bp_tol"],
                          bp_max_iter=g["bp_max_iter"], svd_cutoff=g["svd_cutoff"],
                          eig_cutoff=g["eig_cutoff"]))
    dz = np.abs(out["z"] - np.array(g["z"])).max(axis=1)
    print("  max |dZ| per step:", " ".join(f"{x:.1e}" for x in dz), flush=True)
    print("  sweeps gpu/oracle:", list(out["bp_iters"]), g["bp_iters"], flush=True)
    print("  degenerate cuts gpu/oracle:", list(out["degenerate_cuts"]), g["degenerate_cuts"],
          flush=True)
    assert np.array_equal(out["bond_dims"], np.array(g["bond_dims"]))
    assert np.abs(out["discarded"] - np.array(g["discarded"])).max() < TOL
    assert np.abs(out["bp_iters"] - np.array(g["bp_iters"])).max() <= 1
    assert list(out["degenerate_cuts"]) == g["degenerate_cuts"]
    assert dz.max() < TOL
    # truncation is active: bonds reach chi and the gates discard weight
    assert max(g["discarded"]) > 1e-6 and np.max(g["bond_dims"]) == g["chi"]


def _random_state(lat, chi, rng):
    net = O.Network(lat.n_sites, lat.edges, lat.colour)
    for v in range(net.n):
        d = len(net.nb[v])
        shape = (2,) + (chi,) * d
        net.T[v] = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / chi
    for k in list(net.M):
        X = rng.standard_normal((chi, chi)) + 1j * rng.standard_normal((chi, chi))
        M = X @ X.conj().T
        net.M[k] = M / np.trace(M)
    return net


def test_truncating_layer_identical_state_eagle_chi64(ctx):
    """One gate layer (colour 0, 54 edges) at 127 qubits and chi = 64 on an identical random
    full-bond state, so that every gate between sites of degree >= 2 truncates (two-site blocks
    of rank up to 2 chi): on a sample of 12 edges of every type, the same kept dimension,
    discarded weight, cut gap and bond spectrum as the oracle's simple_update, and the same <Z>
    afterwards on the sites of those edges.  The gates of one layer touch disjoint sites and read
    only messages on other edges, so each sampled edge is checked on its own."""
    from paper_2306_14887_amd import bpki as B
    print("[parity] eagle chi=64 truncating layer on identical state", flush=True)
    lat = L.eagle()
    chi = 64
    rng = np.random.default_rng(11)
    net = _random_state(lat, chi, rng)
    t, m, b = to_flat(net, chi)
    s = B.Session(ctx, _spec(lat, 0.4, 1, chi))
    s.set_state(t, m, b)
    d_gpu = s.apply_layer(0)
    kept, disc, gap = s.layer_cuts()
    _, m2, b2 = s.get_state()
    z_gpu = s.observe_z()
    s.close()
    opt = O.Options(chi=chi)
    layer = [e for e in range(lat.n_edges) if lat.colour[e] == 0]
    assert layer == [e for e in range(lat.n_edges) if kept[e] >= 0]
    deg = lat.degrees()
    kinds = {}
    for e in layer:
        kinds.setdefault(tuple(sorted(deg[lat.edges[e]])), []).append(e)
    assert set(kinds) == {(1, 3), (2, 2), (2, 3)}
    sample = kinds[(1, 3)][:1] + kinds[(2, 2)][:3] + kinds[(2, 3)][:8]
    want_k, want_d, want_g = {}, {}, {}
    for e in sample:
        u, v = net.edges[e]
        want_d[e] = net.simple_update(u, v, opt)
        want_k[e], want_g[e] = net.last_kept, net.last_cut_gap
    msgs = m2.reshape(-1, chi, chi)
    for e, (u, v) in enumerate(net.edges):
        if e not in layer:
            assert kept[e] == -1 and b2[e] == chi
            continue
        if e not in want_k:
            continue
        assert kept[e] == want_k[e] == b2[e]
        assert abs(disc[e] - want_d[e]) < 1e-12
        assert (math.isinf(gap[e]) and math.isinf(want_g[e])) or abs(gap[e] - want_g[e]) < 1e-10
        k = want_k[e]
        ref = np.diag(net.M[(u, v)]).real
        for j in (0, 1):
            got = msgs[2 * e + j]
            assert np.abs(np.diag(got)[:k].real - ref).max() < 1e-12
            assert np.abs(got - np.diag(np.diag(got))).max() == 0.0
            assert np.all(np.diag(got)[k:] == 0.0)
    assert abs(d_gpu - np.nansum(disc)) < 1e-12
    assert min(want_d[e] for e in kinds[(2, 3)][:8]) > 1e-3, "degree-3 gates truncate"
    for e in sample:
        for v in lat.edges[e]:
            assert abs(z_gpu[v] - net.expect_site(int(v), 3)) < 1e-10


@pytest.mark.parametrize("name,chi,theta,depth", [("heavy_hex_29", 8, 0.8, 8),
                                                  ("eagle", 4, 0.7, 6)])
def test_bond_dims_and_discarded_per_step(ctx, name, chi, theta, depth):
    """Truncated whole runs: the bond dimension of every edge after every step is the oracle's,
    and so is the discarded weight of every step."""
    lat = L.heavy_hex(3, 9) if name == "heavy_hex_29" else L.eagle()
    print(f"[parity] {name} chi={chi} bond dims and discarded per step", flush=True)
    out = ctx.solve(_spec(lat, theta, depth, chi))
    ref = O.solve(lat.n_sites, lat.edges, lat.colour, theta, depth, O.Options(chi=chi))
    assert np.array_equal(out["bond_dims"], ref.bond_dims)
    assert np.abs(out["discarded"] - np.array(ref.discarded)).max() < 1e-10
    assert max(ref.discarded) > 1e-3
    assert np.abs(out["z"] - ref.z).max() < TOL
    assert list(out["degenerate_cuts"]) == ref.degenerate_cuts
    g_ref = np.array(ref.min_cut_gap)
    fin = np.isfinite(g_ref)
    assert np.array_equal(np.isfinite(out["min_cut_gap"]), fin)
    assert np.abs(out["min_cut_gap"][fin] - g_ref[fin]).max() < 1e-9


def test_degenerate_cuts_counted_at_the_clifford_point(ctx):
    """theta_h = pi/2 on the 12-site ring with chi = 2: flat spectra, so once chi limits the
    bonds the cuts are degenerate; the result reports them like the oracle."""
    r = L.hexagon_ring()
    out = ctx.solve(_spec(r, math.pi / 2, 6, 2))
    ref = O.solve(r.n_sites, r.edges, r.colour, math.pi / 2, 6, O.Options(chi=2))
    assert out["degenerate_cuts"][0] == 0 and math.isinf(out["min_cut_gap"][0])
    assert max(out["degenerate_cuts"]) > 0
    assert np.array_equal(out["bond_dims"], ref.bond_dims)
