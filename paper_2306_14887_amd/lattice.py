"""Seeded input generators: heavy-hex lattices, gate-layer colourings, Pauli strings.

This module builds the *inputs* of a kicked-Ising circuit run (the lattice graph, a
proper edge colouring that fixes the order of the two-site gate layers, the
transverse-field angles and the Pauli strings to measure).  It holds none of the
method's arithmetic: it is shared by the HIP path, the CPU oracle's tests and the
benchmark, and it imports neither of them.

Lattice (paper, "Model and Ansatz" and Fig. 1): the heavy-hex lattice is a hexagonal
lattice with an extra qubit on every edge.  IBM Eagle's 127-qubit chip is 6x3
heavy hexagons plus two pendant qubits (13 and 113).  It is generated here as rows
of consecutively coupled qubits joined by "bridge" qubits: bridges sit at columns
0,4,8,... in even gaps and 2,6,10,... in odd gaps; the top row loses its last
column and the bottom row its first column (which leaves qubits 13 and 113 with
degree one), and a bridge whose row endpoint was dropped is omitted.  Qubits are
numbered row-major with each gap's bridges numbered right after the row above
the gap, which reproduces the Eagle numbering used by the paper's printed
Clifford identity (the weight-10 string X13,29,31 Y9,30 Z8,12,17,28,32).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Lattice:
    """An undirected graph with a proper edge colouring.

    ``edges`` is an (E, 2) int32 array of 0-based site pairs (u < v not required);
    ``colour`` is an (E,) int32 array; edges that share a site have different colours.
    """

    n_sites: int
    edges: np.ndarray
    colour: np.ndarray
    name: str = ""
    coords: dict = field(default_factory=dict)

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    def neighbours(self) -> list[list[int]]:
        nb: list[list[int]] = [[] for _ in range(self.n_sites)]
        for u, v in self.edges.tolist():
            nb[u].append(v)
            nb[v].append(u)
        return [sorted(x) for x in nb]

    def degrees(self) -> np.ndarray:
        return np.array([len(x) for x in self.neighbours()], dtype=np.int32)

    def n_colours(self) -> int:
        return int(self.colour.max()) + 1 if self.n_edges else 0


def greedy_colouring(n_sites: int, edges: np.ndarray) -> np.ndarray:
    """Greedy proper edge colouring over the edges sorted by (min, max) endpoint.

    Each edge takes the smallest colour not yet used by an edge at either endpoint.
    Returns colours in the order of ``edges``.
    """
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    order = sorted(range(len(edges)), key=lambda i: (min(edges[i]), max(edges[i])))
    used: list[set[int]] = [set() for _ in range(n_sites)]
    colour = np.full(len(edges), -1, dtype=np.int32)
    for i in order:
        u, v = int(edges[i, 0]), int(edges[i, 1])
        c = 0
        while c in used[u] or c in used[v]:
            c += 1
        colour[i] = c
        used[u].add(c)
        used[v].add(c)
    return colour


def heavy_hex(rows: int = 7, row_len: int = 15) -> Lattice:
    """Eagle-style heavy-hex lattice of ``rows`` rows of ``row_len`` qubits.

    rows=7, row_len=15 gives the 127-qubit, 144-edge Eagle lattice; (3, 9) gives
    29 qubits / 30 edges and (5, 11) gives 65 qubits / 72 edges.
    """
    if rows < 2 or row_len < 3:
        raise ValueError("need at least 2 rows of 3 qubits")
    # columns present in each row
    row_cols = []
    for r in range(rows):
        cols = list(range(row_len))
        if r == 0:
            cols = cols[:-1]
        if r == rows - 1:
            cols = cols[1:]
        row_cols.append(cols)
    ids: dict[tuple, int] = {}
    nid = 0
    bridges_in_gap = []
    for r in range(rows):
        for c in row_cols[r]:
            ids[("row", r, c)] = nid
            nid += 1
        if r < rows - 1:
            start = 0 if r % 2 == 0 else 2
            bcols = [c for c in range(start, row_len, 4)
                     if c in row_cols[r] and c in row_cols[r + 1]]
            bridges_in_gap.append(bcols)
            for c in bcols:
                ids[("bridge", r, c)] = nid
                nid += 1
    edges = []
    for r in range(rows):
        cols = row_cols[r]
        for a, b in zip(cols[:-1], cols[1:]):
            edges.append((ids[("row", r, a)], ids[("row", r, b)]))
    for r, bcols in enumerate(bridges_in_gap):
        for c in bcols:
            bq = ids[("bridge", r, c)]
            edges.append((ids[("row", r, c)], bq))
            edges.append((bq, ids[("row", r + 1, c)]))
    edges_a = np.array(sorted((min(e), max(e)) for e in edges), dtype=np.int32)
    colour = greedy_colouring(nid, edges_a)
    coords = {v: k for k, v in ids.items()}
    return Lattice(nid, edges_a, colour, name=f"heavyhex_{rows}x{row_len}", coords=coords)


def eagle() -> Lattice:
    """The 127-qubit / 144-edge IBM Eagle heavy-hex lattice."""
    lat = heavy_hex(7, 15)
    lat.name = "eagle127"
    return lat


def hexagon_ring() -> Lattice:
    """One heavy hexagon: the 12-qubit ring at the top-left of the Eagle lattice.

    Sites are the Eagle qubits 0-4, 15, 22-18, 14 relabelled 0..11 in ring order;
    each ring edge keeps the colour it has in the Eagle greedy colouring, which
    gives three gate layers on the ring.
    """
    e = eagle()
    ring = [0, 1, 2, 3, 4, 15, 22, 21, 20, 19, 18, 14]
    col = {(int(min(a, b)), int(max(a, b))): int(c)
           for (a, b), c in zip(e.edges.tolist(), e.colour.tolist())}
    edges, colours = [], []
    for i in range(12):
        a, b = ring[i], ring[(i + 1) % 12]
        edges.append((i, (i + 1) % 12))
        colours.append(col[(min(a, b), max(a, b))])
    return Lattice(12, np.array(edges, dtype=np.int32), np.array(colours, dtype=np.int32),
                   name="hexring12")


def heavy_hexagons(k: int) -> Lattice:
    """The first ``k`` (1, 2 or 3) heavy hexagons of the Eagle lattice's top row as a lattice of
    their own (the small systems of Fig. 2a-c): 12, 21 and 30 qubits.  Neighbouring hexagons share
    a side (a bridge qubit and its two row neighbours).  Sites are relabelled in increasing Eagle
    order and every edge keeps its Eagle colour."""
    if k not in (1, 2, 3):
        raise ValueError("k must be 1, 2 or 3")
    e = eagle()
    # top row columns 0..4k (qubits 0..4k), bridges of the first gap at columns 0, 4, .., 4k
    # (qubits 14 + j), second row columns 0..4k (qubits 18..18 + 4k)
    keep = list(range(4 * k + 1)) + [14 + j for j in range(k + 1)] + \
        [18 + c for c in range(4 * k + 1)]
    new = {q: i for i, q in enumerate(sorted(keep))}
    edges, colours = [], []
    for (a, b), c in zip(e.edges.tolist(), e.colour.tolist()):
        if a in new and b in new:
            edges.append((new[a], new[b]))
            colours.append(c)
    return Lattice(len(keep), np.array(edges, dtype=np.int32), np.array(colours, dtype=np.int32),
                   name=f"heavyhex{k}")


def ring(n: int) -> Lattice:
    """Periodic ring of ``n`` (even) sites with the alternating 2-colouring."""
    if n < 3:
        raise ValueError("ring needs >= 3 sites")
    edges = np.array([(i, (i + 1) % n) for i in range(n)], dtype=np.int32)
    if n % 2 == 0:
        colour = np.array([i % 2 for i in range(n)], dtype=np.int32)
    else:
        colour = greedy_colouring(n, edges)
    return Lattice(n, edges, colour, name=f"ring{n}")


def random_tree(n: int, rng: np.random.Generator, max_degree: int = 3) -> Lattice:
    """Uniformly grown random tree with maximum degree ``max_degree``."""
    deg = [0] * n
    edges = []
    for v in range(1, n):
        cand = [u for u in range(v) if deg[u] < max_degree]
        u = int(rng.choice(cand))
        edges.append((u, v))
        deg[u] += 1
        deg[v] += 1
    edges_a = np.array(edges, dtype=np.int32).reshape(-1, 2)
    return Lattice(n, edges_a, greedy_colouring(n, edges_a), name=f"tree{n}")


def path(n: int) -> Lattice:
    edges = np.array([(i, i + 1) for i in range(n - 1)], dtype=np.int32).reshape(-1, 2)
    return Lattice(n, edges, greedy_colouring(n, edges), name=f"path{n}")


# ---------------------------------------------------------------------------
# The infinite heavy-hex lattice: periodic cells
# ---------------------------------------------------------------------------

# Sites of one cell: the two degree-3 sites A, B of the underlying hexagonal lattice and one
# bridge C_d on each of its three bond directions d.
CELL_SITES = ("A", "B", "C0", "C1", "C2")
# Bridge C_d of cell r joins A(r) to B(r + shift[d]) (hexagonal lattice in brick-wall form).
_CELL_SHIFT = ((0, 0), (1, 0), (0, 1))


def heavy_hex_torus(l1: int, l2: int, derangement=(1, 2, 0)) -> Lattice:
    """Periodic heavy-hex lattice of l1 x l2 cells (5 sites, 6 edges per cell).

    Site 5 * (x * l2 + y) + k is CELL_SITES[k] of cell (x, y).  Edge A(r)-C_d(r) has colour d
    and edge C_d(r)-B(r + shift_d) colour derangement[d]: every site then sees distinct
    colours (the A legs by construction, the B legs because ``derangement`` is a bijection,
    the bridges because it has no fixed point), and the colouring is the same in every cell,
    so the gate layers commute with translations.  With l1 = l2 = 1 this is the paper's
    5-site unit cell ("Dynamics of the infinite heavy-hex lattice", Fig. 4): the quotient
    graph of the infinite lattice, a theta graph (A and B joined through the three bridges).
    BP on a quotient graph is BP on the infinite lattice restricted to translation-invariant
    messages, and a gate layer on it is the layer on every translate at once.
    """
    if l1 < 1 or l2 < 1:
        raise ValueError("need at least one cell in each direction")
    dr = tuple(int(c) for c in derangement)
    if sorted(dr) != [0, 1, 2] or any(dr[d] == d for d in range(3)):
        raise ValueError("derangement must be a fixed-point-free permutation of (0, 1, 2)")

    def site(x: int, y: int, k: int) -> int:
        return 5 * ((x % l1) * l2 + (y % l2)) + k

    edges, colour = [], []
    coords = {}
    for x in range(l1):
        for y in range(l2):
            for k in range(5):
                coords[site(x, y, k)] = (x, y, CELL_SITES[k])
            for d in range(3):
                sx, sy = _CELL_SHIFT[d]
                edges.append((site(x, y, 0), site(x, y, 2 + d)))
                colour.append(d)
                edges.append((site(x, y, 2 + d), site(x + sx, y + sy, 1)))
                colour.append(dr[d])
    name = "hhx_cell5" if l1 == l2 == 1 else f"hhx_torus{l1}x{l2}"
    return Lattice(5 * l1 * l2, np.array(edges, dtype=np.int32),
                   np.array(colour, dtype=np.int32), name=name, coords=coords)


def infinite_cell(derangement=(1, 2, 0)) -> Lattice:
    """The 5-site periodic unit cell of the infinite heavy-hex lattice (sites A, B, C0..C2)."""
    return heavy_hex_torus(1, 1, derangement)


# ---------------------------------------------------------------------------
# Pauli strings on connected clusters
# ---------------------------------------------------------------------------

@dataclass
class PauliString:
    sites: list[int]
    ops: list[int]          # 1 = X, 2 = Y, 3 = Z

    def label(self) -> str:
        return " ".join(f"{'IXYZ'[o]}{s}" for s, o in zip(self.sites, self.ops))


def induced_is_tree(sites: list[int], edges: np.ndarray) -> bool:
    s = set(sites)
    m = sum(1 for u, v in edges.tolist() if u in s and v in s)
    return m == len(sites) - 1          # connected by construction


def tree_cluster(lat: Lattice, weight: int, rng: np.random.Generator,
                 max_tries: int = 1000) -> list[int]:
    """Connected cluster of ``weight`` sites whose induced subgraph is a tree.

    Grown from a uniformly drawn seed site by repeatedly adding a uniformly drawn
    frontier site; a cluster whose induced subgraph has a cycle is rejected.
    """
    nb = lat.neighbours()
    for _ in range(max_tries):
        seed = int(rng.integers(lat.n_sites))
        cl = [seed]
        inset = {seed}
        ok = True
        while len(cl) < weight:
            frontier = sorted({u for v in cl for u in nb[v] if u not in inset})
            if not frontier:
                ok = False
                break
            u = int(frontier[int(rng.integers(len(frontier)))])
            cl.append(u)
            inset.add(u)
        if ok and induced_is_tree(cl, lat.edges):
            return sorted(cl)
    raise RuntimeError("could not draw a tree cluster")


def random_pauli_strings(lat: Lattice, count: int, seed: int,
                         wmin: int = 3, wmax: int = 17) -> list[PauliString]:
    """``count`` strings: weight ~ U{wmin..wmax}, tree cluster, ops ~ U{X,Y,Z}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        w = int(rng.integers(wmin, wmax + 1))
        sites = tree_cluster(lat, w, rng)
        ops = [int(o) for o in rng.integers(1, 4, size=w)]
        out.append(PauliString(sites, ops))
    return out


def pauli_csr(strings: list[PauliString]):
    """CSR arrays (offsets, sites, ops) for the C-ABI."""
    offs = [0]
    sites: list[int] = []
    ops: list[int] = []
    for p in strings:
        sites += list(p.sites)
        ops += list(p.ops)
        offs.append(len(sites))
    return (np.array(offs, dtype=np.int32), np.array(sites, dtype=np.int32),
            np.array(ops, dtype=np.uint8))


# ---------------------------------------------------------------------------
# Workload parameter draws
# ---------------------------------------------------------------------------

def theta_grid_config1() -> list[float]:
    """theta_h in {0, 0.2, ..., 1.4, pi/2}."""
    return [round(0.2 * i, 10) for i in range(8)] + [math.pi / 2]


def theta_draw(n: int = 8, seed: int = 2306) -> list[float]:
    """``n`` angles uniform in [0, pi/2] from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return [float(x) for x in rng.uniform(0.0, math.pi / 2, size=n)]


@dataclass
class ServeRequest:
    rows: int
    row_len: int
    theta: float
    depth: int
    chi: int
    arrival: float


def serving_requests(n: int = 256, seed: int = 0, rate: float = 1.0) -> list[ServeRequest]:
    """Serving workload: lattices from {(3,9),(5,11),(7,15)}, theta ~ U[0,pi/2],
    depth ~ U{1..20}, chi ~ U{8,16,32,64}, Poisson arrivals at ``rate`` per second."""
    rng = np.random.default_rng(seed)
    shapes = [(3, 9), (5, 11), (7, 15)]
    chis = [8, 16, 32, 64]
    t = 0.0
    out = []
    for _ in range(n):
        r, c = shapes[int(rng.integers(3))]
        th = float(rng.uniform(0.0, math.pi / 2))
        d = int(rng.integers(1, 21))
        chi = chis[int(rng.integers(4))]
        t += float(rng.exponential(1.0 / rate))
        out.append(ServeRequest(r, c, th, d, chi, t))
    return out
