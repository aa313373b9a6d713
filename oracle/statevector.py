"""Exact state-vector simulation of the kicked Ising circuit (test pins for the oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/bp_tns.py``).  This is the brute-force reference
the paper benchmarks against on small lattices (Fig. "smallheavyhexdynamics", Results)
and the exact light-cone simulation it quotes for 127 qubits at 5 steps (Results,
Fig. "comparison").  It knows nothing about tensor networks.

Qubit q is axis q of the state reshaped to (2,)*n; bit 0 is spin up, Z|0> = +|0>.
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np

_P = {
    1: np.array([[0, 1], [1, 0]], dtype=complex),
    2: np.array([[0, -1j], [1j, 0]], dtype=complex),
    3: np.array([[1, 0], [0, -1]], dtype=complex),
}


def _zvals(n: int) -> np.ndarray:
    """z[q, idx] = +1/-1 eigenvalue of Z_q on basis state idx (axis 0 most significant)."""
    idx = np.arange(2 ** n, dtype=np.int64)
    return np.stack([1 - 2 * ((idx >> (n - 1 - q)) & 1) for q in range(n)]).astype(np.int8)


class StateVector:
    def __init__(self, n: int, edges, zz_sign: float = 1.0):
        if n > 24:
            raise ValueError("state vector limited to 24 qubits")
        self.n = n
        self.psi = np.zeros(2 ** n, dtype=complex)
        self.psi[0] = 1.0
        z = _zvals(n)
        s = np.zeros(2 ** n, dtype=np.int64)
        for u, v in np.asarray(edges, dtype=np.int64).reshape(-1, 2).tolist():
            s += z[u].astype(np.int64) * z[v].astype(np.int64)
        # all two-site gates are diagonal and commute: their product is one phase
        self.zz_phase = np.exp(1j * zz_sign * math.pi / 4 * s)
        self.z = z

    def apply_rx(self, theta: float) -> None:
        c, s = math.cos(theta / 2), math.sin(theta / 2)
        R = np.array([[c, -1j * s], [-1j * s, c]], dtype=complex)
        psi = self.psi.reshape((2,) * self.n)
        for q in range(self.n):
            psi = np.moveaxis(np.tensordot(R, psi, axes=([1], [q])), 0, q)
        self.psi = psi.reshape(-1)

    def apply_zz(self) -> None:
        self.psi = self.psi * self.zz_phase

    def step(self, theta: float) -> None:
        """One Floquet step U(theta) = (ZZ layer)(RX layer)."""
        self.apply_rx(theta)
        self.apply_zz()

    def clifford_inverse_step(self) -> None:
        """One step of U(pi/2)^dagger = (RX layer at -pi/2)(ZZ layer)^dagger."""
        self.psi = self.psi * np.conj(self.zz_phase)
        self.apply_rx(-math.pi / 2)

    def expect_z(self) -> np.ndarray:
        p = np.abs(self.psi) ** 2
        return self.z.astype(float) @ p

    def expect_pauli(self, sites, ops) -> float:
        phi = self.psi.reshape((2,) * self.n)
        for q, o in zip(sites, ops):
            phi = np.moveaxis(np.tensordot(_P[int(o)], phi, axes=([1], [int(q)])), 0, int(q))
        return float(np.vdot(self.psi, phi.reshape(-1)).real)

    def norm(self) -> float:
        return float(np.linalg.norm(self.psi))


def run(n: int, edges, theta: float, depth: int, zz_sign: float = 1.0) -> np.ndarray:
    """<Z_v> after steps 1..depth: array [depth, n]."""
    sv = StateVector(n, edges, zz_sign)
    out = []
    for _ in range(depth):
        sv.step(theta)
        out.append(sv.expect_z())
    return np.array(out)


def ball(n: int, edges, v: int, radius: int) -> list[int]:
    nb = [[] for _ in range(n)]
    for a, b in np.asarray(edges).reshape(-1, 2).tolist():
        nb[a].append(b)
        nb[b].append(a)
    dist = {v: 0}
    dq = deque([v])
    while dq:
        x = dq.popleft()
        if dist[x] == radius:
            continue
        for y in nb[x]:
            if y not in dist:
                dist[y] = dist[x] + 1
                dq.append(y)
    return sorted(dist)


def light_cone_z(n: int, edges, v: int, theta: float, t: int) -> float:
    """Exact <Z_v> after t steps by simulating only the ball of radius t-1 around v.

    In the Heisenberg picture one Floquet step conjugates Z_v by the (diagonal, so
    commuting) ZZ layer and then the X rotations; each further step can only grow the
    support by one graph distance.  Gates outside the backward light cone cancel, so
    the circuit restricted to the induced subgraph on ball(v, t-1) gives the exact value.
    """
    if t == 0:
        return 1.0
    sub = ball(n, edges, v, max(t - 1, 0))
    idx = {q: i for i, q in enumerate(sub)}
    e_sub = [(idx[a], idx[b]) for a, b in np.asarray(edges).reshape(-1, 2).tolist()
             if a in idx and b in idx]
    sv = StateVector(len(sub), np.array(e_sub, dtype=np.int64).reshape(-1, 2))
    for _ in range(t):
        sv.step(theta)
    return float(sv.expect_z()[idx[v]])
