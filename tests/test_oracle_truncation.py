"""Pins of the oracle's truncation step against exact state vectors.

The truncation is the SVD of the gated two-site block cut back to at most chi singular values,
with the bond matrix returned as the new message (Methods, "The simple update procedure").  On a
tree, BP messages are the exact environments (Methods, "Belief propagation on a tensor network
state"), so when BP has converged before a gate, the SVD of the reduced two-site block is the
Schmidt decomposition of the whole state across the gated edge: the truncation must then keep
exactly the chi largest Schmidt weights of the exact state, discard the sum of the others, and
leave the state projected onto them.  These tests emulate that optimal truncation on a brute-force
state vector, gate by gate, independently of the tensor network.
"""
import math

import numpy as np
import pytest

from oracle import bp_tns as O
from paper_2306_14887_amd import lattice as L

CUT = 1e-12          # the default svd_cutoff, on Schmidt weights


class GateSV:
    """State vector with one ZZ gate at a time and the optimal truncation across a tree edge."""

    def __init__(self, n, edges):
        self.n = n
        self.edges = [tuple(map(int, e)) for e in np.asarray(edges).reshape(-1, 2)]
        self.psi = np.zeros((2,) * n, dtype=complex)
        self.psi[(0,) * n] = 1.0
        nb = [[] for _ in range(n)]
        for a, b in self.edges:
            nb[a].append(b)
            nb[b].append(a)
        self.nb = nb

    def rx(self, theta):
        c, s = math.cos(theta / 2), math.sin(theta / 2)
        R = np.array([[c, -1j * s], [-1j * s, c]])
        for q in range(self.n):
            self.psi = np.moveaxis(np.tensordot(R, self.psi, axes=([1], [q])), 0, q)

    def zz(self, u, v, sign=1.0):
        z = np.array([1.0, -1.0])
        ph = np.exp(1j * sign * math.pi / 4 * np.outer(z, z))
        shape = [1] * self.n
        shape[u], shape[v] = 2, 2
        if u < v:
            self.psi = self.psi * ph.reshape(shape)
        else:
            self.psi = self.psi * ph.T.reshape(shape)

    def side(self, u, v):
        """Sites on u's side of the tree once edge (u, v) is removed."""
        seen, stack = {u}, [u]
        while stack:
            x = stack.pop()
            for y in self.nb[x]:
                if (x, y) in ((u, v), (v, u)) or y in seen:
                    continue
                seen.add(y)
                stack.append(y)
        return sorted(seen)

    def schmidt(self, u, v):
        a = self.side(u, v)
        b = [q for q in range(self.n) if q not in a]
        m = np.transpose(self.psi, a + b).reshape(2 ** len(a), 2 ** len(b))
        return a, b, np.linalg.svd(m, full_matrices=False)

    def truncate(self, u, v, chi):
        """Project onto the chi largest Schmidt weights across (u, v) (those above CUT * p_1),
        renormalise.  Returns (kept weights normalised to sum 1, discarded fraction)."""
        a, b, (U, s, Vh) = self.schmidt(u, v)
        p = s ** 2
        k = min(chi, int(np.count_nonzero(p > CUT * p[0])))
        disc = float(p[k:].sum() / p.sum())
        m = (U[:, :k] * s[:k]) @ Vh[:k, :]
        m /= np.linalg.norm(m)
        t = m.reshape((2,) * self.n)
        self.psi = np.transpose(t, np.argsort(a + b))
        return p[:k] / p[:k].sum(), disc, k

    def z(self):
        pr = np.abs(self.psi) ** 2
        out = []
        for q in range(self.n):
            m = np.moveaxis(pr, q, 0).reshape(2, -1).sum(axis=1)
            out.append(m[0] - m[1])
        return np.array(out)


def _gate_order(lat):
    """Edges in the order the oracle applies them: ascending colour, edge-list order inside."""
    out = []
    for c in sorted(set(lat.colour.tolist())):
        out += [(int(u), int(v)) for e, (u, v) in enumerate(lat.edges) if lat.colour[e] == c]
    return out


TREES = [(11, 5, 2, 0.9), (12, 8, 3, 1.1), (13, 21, 2, 0.7)]


@pytest.mark.parametrize("n,seed,chi,theta", TREES)
def test_regauged_truncation_is_the_optimal_one_on_trees(n, seed, chi, theta):
    """BP before every gate: every gate keeps exactly the top-chi exact Schmidt weights of the
    state across its edge, its discarded weight is the dropped exact weight, and the state after
    every step is the state vector with each gate followed by the optimal truncation."""
    tr = L.random_tree(n, np.random.default_rng(seed))
    opt = O.Options(chi=chi, regauge_every_gate=True)
    net = O.Network(tr.n_sites, tr.edges, tr.colour)
    sv = GateSV(tr.n_sites, tr.edges)
    truncated = 0
    for _t in range(5):
        net.apply_rx(theta)
        sv.rx(theta)
        for u, v in _gate_order(tr):
            net.bp(opt.bp_tol, opt.bp_max_iter)
            d = net.simple_update(u, v, opt)
            sv.zz(u, v)
            w, d_ref, k = sv.truncate(u, v, chi)
            assert net.last_kept == k
            assert abs(d - d_ref) < 1e-12
            np.testing.assert_allclose(net.last_S ** 2, w, atol=1e-12)
            truncated += d_ref > 1e-6
        net.bp(opt.bp_tol, opt.bp_max_iter)
        z = np.array([net.expect_site(q, 3) for q in range(tr.n_sites)])
        assert np.abs(z - sv.z()).max() < 1e-10
    assert truncated >= 3, "the run must exercise the truncation"
    # the whole-run driver follows the same schedule when asked to regauge before every gate
    res = O.solve(tr.n_sites, tr.edges, tr.colour, theta, 5, opt)
    assert np.abs(res.z[-1] - z).max() < 1e-10


@pytest.mark.parametrize("n,seed,chi,theta", TREES)
def test_first_truncation_keeps_the_top_schmidt_weights(n, seed, chi, theta):
    """Default schedule (BP once per step): on a tree every gate up to and including the first
    truncating one sees exact environments, so that gate keeps the chi largest exact Schmidt
    weights and discards the rest; the run's state until then is the exact one."""
    tr = L.random_tree(n, np.random.default_rng(seed))
    opt = O.Options(chi=chi)
    net = O.Network(tr.n_sites, tr.edges, tr.colour)
    sv = GateSV(tr.n_sites, tr.edges)
    done = False
    for _t in range(8):
        net.apply_rx(theta)
        sv.rx(theta)
        for u, v in _gate_order(tr):
            d = net.simple_update(u, v, opt)
            sv.zz(u, v)
            w, d_ref, k = sv.truncate(u, v, chi)
            assert net.last_kept == k
            assert abs(d - d_ref) < 1e-12
            np.testing.assert_allclose(net.last_S ** 2, w, atol=1e-12)
            if d_ref > 1e-8:
                done = True
                break
        if done:
            break
        net.bp(opt.bp_tol, opt.bp_max_iter)
    assert done, "no gate truncated"


def test_bond_dimension_is_the_numerical_schmidt_rank():
    """Untruncated (chi above every rank) on a tree, each bond dimension equals the number of
    exact Schmidt weights above svd_cutoff times the largest, across that edge."""
    tr = L.random_tree(12, np.random.default_rng(4))
    theta = 0.35
    res = O.solve(tr.n_sites, tr.edges, tr.colour, theta, 4, O.Options(chi=64))
    sv = GateSV(tr.n_sites, tr.edges)
    for t in range(4):
        sv.rx(theta)
        for u, v in _gate_order(tr):
            sv.zz(u, v)
        for e, (u, v) in enumerate(tr.edges.tolist()):
            p = sv.schmidt(u, v)[2][1] ** 2
            assert res.bond_dims[t, e] == np.count_nonzero(p > CUT * p[0])
        assert res.min_cut_gap[t] == math.inf and res.degenerate_cuts[t] == 0
        assert np.abs(res.z[t] - sv.z()).max() < 1e-11


@pytest.mark.parametrize("lat_name,chi,theta,steps", [
    ("tree", 2, 0.9, 4), ("ring", 4, 0.8, 6), ("eagle", 4, 0.6, 3)])
def test_gate_message_is_the_bp_message_of_the_new_tensors(lat_name, chi, theta, steps):
    """After every gate, truncating or not, the message it writes on the edge, diag(S)/sum(S),
    is what the BP equation (Eq. "MessageTensorSelfConsistency") returns for the new tensors
    with the unchanged incoming messages, in both directions.  This holds only if S is split as
    sqrt(S) onto each side: S on one side would give diag(S^2) one way and the identity the
    other."""
    lat = {"tree": lambda: L.random_tree(11, np.random.default_rng(5)),
           "ring": L.hexagon_ring, "eagle": L.eagle}[lat_name]()
    opt = O.Options(chi=chi)
    net = O.Network(lat.n_sites, lat.edges, lat.colour)
    worst, truncated = 0.0, 0
    for _t in range(steps):
        net.apply_rx(theta)
        for u, v in _gate_order(lat):
            truncated += net.simple_update(u, v, opt) > 1e-8
            for a, b in ((u, v), (v, u)):
                worst = max(worst, float(np.abs(net.message(a, b, net.M) - net.M[(a, b)]).max()))
        net.bp(opt.bp_tol, opt.bp_max_iter)
    assert worst < 1e-9
    assert truncated > 0


def test_near_degenerate_cuts_are_counted_at_the_clifford_point():
    """At theta_h = pi/2 the Schmidt spectra are flat, so once chi limits the bonds every cut falls
    between equal singular values: the diagnostics report them (and none while untruncated)."""
    r = L.hexagon_ring()
    res = O.solve(r.n_sites, r.edges, r.colour, math.pi / 2, 6, O.Options(chi=2))
    assert res.degenerate_cuts[0] == 0 and res.min_cut_gap[0] == math.inf
    assert max(res.degenerate_cuts) > 0
    assert min(res.min_cut_gap) < O.DEGENERATE_GAP
