"""Pauli-string propagation at the Clifford point theta_h = pi/2 (test pins).

TEST INFRASTRUCTURE ONLY (see ``oracle/bp_tns.py``).

At theta_h = pi/2 every gate of U (Eq. "Propagator") is a Clifford gate, so conjugating a
Pauli string by U gives a single Pauli string with a phase (paper, "Measuring expectation
values").  This module builds the conjugation tables numerically from the 2x2 and 4x4 gate
matrices (no hand-written rules) and propagates strings through whole Floquet steps.
It gives (a) exact <Z_v>(t) at theta_h = pi/2 and theta_h = 0, and (b) the strings
U^n Z_i U^n^dagger used by the paper's extended-time-evolution identity.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

_P = [np.eye(2, dtype=complex),
      np.array([[0, 1], [1, 0]], dtype=complex),
      np.array([[0, -1j], [1j, 0]], dtype=complex),
      np.array([[1, 0], [0, -1]], dtype=complex)]


def _decompose(M: np.ndarray, basis: list[np.ndarray]):
    """Write M = phase * basis[k] (exactly one term); return (phase, k)."""
    d = M.shape[0]
    for k, B in enumerate(basis):
        c = np.trace(B.conj().T @ M) / d
        if abs(abs(c) - 1.0) < 1e-9:
            if np.allclose(M, c * B, atol=1e-9):
                ph = complex(np.round(c.real) + 1j * np.round(c.imag))
                return ph, k
    raise ValueError("not a Clifford image of a Pauli")


def _tables(theta: float, zz_sign: float):
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    R = np.array([[c, -1j * s], [-1j * s, c]], dtype=complex)
    D = np.diag([np.exp(1j * zz_sign * math.pi / 4 * za * zb)
                 for za in (1, -1) for zb in (1, -1)])
    basis2 = [np.kron(_P[a], _P[b]) for a in range(4) for b in range(4)]
    tab = {}
    for name, G in (("R", R), ("Rd", R.conj().T)):
        tab[name] = [_decompose(G @ _P[k] @ G.conj().T, _P) for k in range(4)]
    for name, G in (("D", D), ("Dd", D.conj().T)):
        t2 = []
        for a, b in itertools.product(range(4), range(4)):
            ph, k = _decompose(G @ basis2[4 * a + b] @ G.conj().T, basis2)
            t2.append((ph, divmod(k, 4)))
        tab[name] = t2
    return tab


class PauliString:
    def __init__(self, n: int, letters=None, phase: complex = 1.0):
        self.n = n
        self.l = np.zeros(n, dtype=np.int8) if letters is None else np.array(letters, np.int8)
        self.phase = complex(phase)

    @classmethod
    def single(cls, n: int, site: int, op: int) -> "PauliString":
        p = cls(n)
        p.l[site] = op
        return p

    def conj_1q(self, table, q: int) -> None:
        ph, k = table[int(self.l[q])]
        self.phase *= ph
        self.l[q] = k

    def conj_2q(self, table, a: int, b: int) -> None:
        ph, (ka, kb) = table[4 * int(self.l[a]) + int(self.l[b])]
        self.phase *= ph
        self.l[a], self.l[b] = ka, kb

    def expect_zero_state(self) -> float:
        """<0...0| P |0...0>: the phase if P has only I and Z letters, else 0."""
        if np.all((self.l == 0) | (self.l == 3)):
            return float(self.phase.real)
        return 0.0

    def support(self) -> dict:
        return {int(q): int(self.l[q]) for q in np.nonzero(self.l)[0]}


def heisenberg_step(p: PauliString, edges, tab) -> None:
    """P -> U^dagger P U with U = D R: first D^dagger P D, then R^dagger P R."""
    for a, b in edges:
        p.conj_2q(tab["Dd"], a, b)
    for q in range(p.n):
        p.conj_1q(tab["Rd"], q)


def schrodinger_step(p: PauliString, edges, tab) -> None:
    """P -> U P U^dagger with U = D R: first R P R^dagger, then D P D^dagger."""
    for q in range(p.n):
        p.conj_1q(tab["R"], q)
    for a, b in edges:
        p.conj_2q(tab["D"], a, b)


def z_expectations(n: int, edges, theta: float, depth: int, zz_sign: float = 1.0):
    """Exact <Z_v>(t), t = 1..depth, at a Clifford angle (theta in {0, pi/2})."""
    tab = _tables(theta, zz_sign)
    edges = [tuple(map(int, e)) for e in np.asarray(edges).reshape(-1, 2).tolist()]
    out = np.zeros((depth, n))
    for v in range(n):
        p = PauliString.single(n, v, 3)
        for t in range(depth):
            heisenberg_step(p, edges, tab)
            out[t, v] = p.expect_zero_state()
    return out


def pauli_expectation(n: int, edges, theta: float, depth: int, sites, ops,
                      zz_sign: float = 1.0) -> float:
    """Exact <psi(depth)| P |psi(depth)> at a Clifford angle."""
    tab = _tables(theta, zz_sign)
    edges = [tuple(map(int, e)) for e in np.asarray(edges).reshape(-1, 2).tolist()]
    p = PauliString(n)
    for s, o in zip(sites, ops):
        p.l[int(s)] = int(o)
    for _ in range(depth):
        heisenberg_step(p, edges, tab)
    return p.expect_zero_state()


def forward_string(n: int, edges, site: int, steps: int, theta: float = math.pi / 2,
                   zz_sign: float = 1.0) -> PauliString:
    """U^steps Z_site U^steps^dagger (the extended-time-evolution identity)."""
    tab = _tables(theta, zz_sign)
    edges = [tuple(map(int, e)) for e in np.asarray(edges).reshape(-1, 2).tolist()]
    p = PauliString.single(n, site, 3)
    for _ in range(steps):
        schrodinger_step(p, edges, tab)
    return p
