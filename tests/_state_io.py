"""Conversion between the oracle's tensor network and the library's exported state layout.

Exported layout (include/bpki.h, sessions): site tensors T_v[s][a_0]..[a_{d-1}] padded to chi
and concatenated over sites; messages [2E][chi][chi] with index 2e = edges[e,0] -> edges[e,1]
and 2e+1 the reverse.  Test infrastructure only.
"""
import numpy as np

from oracle import bp_tns as O


def to_flat(net: "O.Network", chi: int):
    ts = []
    for v in range(net.n):
        T = net.T[v]
        pad = np.zeros((2,) + (chi,) * (T.ndim - 1), dtype=complex)
        pad[tuple(slice(0, d) for d in T.shape)] = T
        ts.append(pad.reshape(-1))
    ms = []
    for u, v in net.edges:
        for a, b in ((u, v), (v, u)):
            M = net.M[(a, b)]
            pad = np.zeros((chi, chi), dtype=complex)
            pad[:M.shape[0], :M.shape[1]] = M
            ms.append(pad.reshape(-1))
    bonds = np.array([net.bond_dim(u, v) for u, v in net.edges], dtype=np.int32)
    return np.concatenate(ts), np.concatenate(ms), bonds


def from_flat(net: "O.Network", chi: int, tensors, messages, bonds):
    """Fill an oracle Network (same graph) from an exported state, trimming the padding."""
    off = 0
    bond = {}
    for e, (u, v) in enumerate(net.edges):
        bond[(u, v)] = bond[(v, u)] = int(bonds[e])
    for v in range(net.n):
        d = len(net.nb[v])
        size = 2 * chi ** d
        T = np.asarray(tensors[off:off + size]).reshape((2,) + (chi,) * d)
        off += size
        net.T[v] = T[(slice(None),) + tuple(slice(0, bond[(v, u)]) for u in net.nb[v])].copy()
    for e, (u, v) in enumerate(net.edges):
        k = int(bonds[e])
        for j, (a, b) in enumerate(((u, v), (v, u))):
            M = np.asarray(messages[(2 * e + j) * chi * chi:(2 * e + j + 1) * chi * chi])
            net.M[(a, b)] = M.reshape(chi, chi)[:k, :k].copy()
    return net


def message_list(net: "O.Network", chi: int):
    out = []
    for u, v in net.edges:
        for a, b in ((u, v), (v, u)):
            M = net.M[(a, b)]
            pad = np.zeros((chi, chi), dtype=complex)
            pad[:M.shape[0], :M.shape[1]] = M
            out.append(pad)
    return out


def contract_network(net, normalise=True):
    """Whole state vector of a (small) tensor network by one einsum over all bonds."""
    letters = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"
    el = {}
    for k, (u, v) in enumerate(net.edges):
        el[(u, v)] = el[(v, u)] = letters[k]
    phys = [letters[len(net.edges) + v] for v in range(net.n)]
    subs = [phys[v] + "".join(el[(v, u)] for u in net.nb[v]) for v in range(net.n)]
    psi = np.einsum(",".join(subs) + "->" + "".join(phys), *net.T, optimize=True).reshape(-1)
    return psi / np.linalg.norm(psi) if normalise else psi


def isometry_error(net, lam):
    """Eq. "IsometryDefinition": Gamma_v (T_v with S^{-1/2} removed from every leg), with S^2 on
    all legs but one, contracted with its conjugate is proportional to the identity on that
    leg.  Returns the largest deviation after dividing out the proportionality factor."""
    S = {}
    for (u, v), s in lam.items():
        S[(u, v)] = S[(v, u)] = s
    err = 0.0
    for v in range(net.n):
        G = net.T[v]
        for u in net.nb[v]:
            G = O.absorb(G, net.axis(v, u), np.diag(1.0 / np.sqrt(S[(v, u)])))
        for u in net.nb[v]:
            Y = G
            for w in net.nb[v]:
                if w != u:
                    Y = O.absorb(Y, net.axis(v, w), np.diag(S[(v, w)] ** 2).astype(complex))
            ax = net.axis(v, u)
            others = [a for a in range(G.ndim) if a != ax]
            I = np.tensordot(Y, G.conj(), axes=(others, others))
            c = np.trace(I) / I.shape[0]
            err = max(err, float(np.abs(I / c - np.eye(I.shape[0])).max()))
    return err
