"""FP64 CPU oracle: BP-approximated tensor network simulation of the kicked Ising circuit.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or link this
module: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP path.

What it computes (arXiv 2306.14887, Tindall, Fishman, Stoudenmire, Sels):

* The circuit (Eq. "Propagator"): one Floquet step is
  U(theta_h) = prod_<v,v'> exp(+i pi/4 Z_v Z_v') . prod_v exp(-i theta_h X_v / 2),
  the X rotations acting first; the state after n steps is U^n |0...0> (Eq. "State").
* The state is a tensor network on the lattice graph (Fig. 1): one tensor per site with
  a physical leg of dimension 2 and one virtual leg per neighbour.  It is kept in an
  arbitrary gauge together with belief-propagation (BP) message tensors, which the
  Methods show to be equivalent to working in the Vidal gauge.
* The X rotations are applied exactly ("State ansatz").
* Each two-site gate is applied by the reduced-tensor simple update in the BP gauge
  (Methods, "The simple update procedure", Fig. "SimpleUpdate" steps i-v): the square
  roots of the incoming messages are absorbed on the environment legs, each side is
  QR-isolated, the gate is applied to the two R factors, the block is SVD-truncated to at
  most chi singular values, the inverse square roots are absorbed back, and the message
  on the updated edge becomes the SVD bond matrix.
* After every Floquet step the network is regauged by BP (Methods, "Belief propagation
  on a tensor network state", Eq. "MessageTensorSelfConsistency"): each directed message
  is the contraction of the site tensor, its conjugate and all other incoming messages,
  iterated to a fixed point.
* Single-site expectation values use the rank-one BP environment (Eq. "SingleSIte");
  Pauli strings on a cluster whose induced subgraph is a tree are contracted exactly
  inside the cluster with BP messages on the cut legs.
* Bond entanglement entropy (Eq. "EntanglementEntropy"): the Schmidt weights of an edge
  are the spectrum of the two messages that meet on it (Network.bond_spectrum).
* The explicit Vidal gauge (Methods, "The Vidal gauge"): the gauge transformation built from
  the messages (Network.vidal_gauge), equivalent to the message form in exact arithmetic.
* The BP error estimate (Eq. "BPErrorEstimate"): the index of separability of the exactly
  contracted edge environment in the symmetric gauge (Network.bp_error; small networks).
* The infinite lattice ("Dynamics of the infinite heavy-hex lattice", Fig. 4) is its
  periodic unit cell given as a graph: BP on the 5-site quotient graph is BP on the
  infinite lattice with translation-invariant messages, so nothing here is specific to it.

Readings where the paper is silent (all mirrored by the HIP path):
  message normalisation: unit trace; singular values: unit 2-norm;
  BP schedule: sweeps by vertex class (the two sides of a bipartite lattice, else a greedy
  vertex colouring; see Network.bp_sweep), warm-started from the current messages, residual =
  max over directed edges of the Frobenius norm of the change, stop when < tol;
  extended time evolution (U(pi/2)^dagger steps): gates exp(-i pi/4 ZZ) in descending
  colour, then X rotations by -pi/2;
  truncation: keep min(chi, #{sigma_i^2 > eps_svd * sigma_1^2}) singular values (the cutoff
  acts on the Schmidt weights sigma^2, which is what an FP64 Gram-matrix eigensolver resolves);
  message square roots: eigenvalues clipped at 0; inverse square roots keep eigenvalues
  > eps_eig * lambda_max; gate layers: ascending colour of a proper edge colouring;
  entropy: s = -sum_i p_i log2 p_i with the minus sign the printed formula lacks, over the
  chi weights of one bond (not chi^2), normalised to sum 1.

Conventions: the legs of the tensor of site v are (physical, then neighbours in
ascending site id).  A message M[a_ket, a_bra] carries the ket index first.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Pauli operators, 1 = X, 2 = Y, 3 = Z
PAULI = {
    0: np.eye(2, dtype=complex),
    1: np.array([[0, 1], [1, 0]], dtype=complex),
    2: np.array([[0, -1j], [1j, 0]], dtype=complex),
    3: np.array([[1, 0], [0, -1]], dtype=complex),
}


def rx_matrix(theta: float) -> np.ndarray:
    """exp(-i theta X / 2) (Eq. "Propagator")."""
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=complex)


def zz_gate_phases(sign: float = 1.0) -> np.ndarray:
    """Diagonal of exp(+i pi/4 Z Z) as g[s_v, s_w] (Eq. "Propagator"); Z|0> = |0>."""
    g = np.empty((2, 2), dtype=complex)
    for a in range(2):
        for b in range(2):
            za, zb = 1 - 2 * a, 1 - 2 * b
            g[a, b] = np.exp(1j * sign * math.pi / 4 * za * zb)
    return g


def absorb(T: np.ndarray, axis: int, X: np.ndarray) -> np.ndarray:
    """Contract leg ``axis`` of T with the row index of X: T'[..b..] = sum_a T[..a..] X[a, b]."""
    return np.moveaxis(np.tensordot(T, X, axes=([axis], [0])), -1, axis)


def msg_sqrt(M: np.ndarray, eps_eig: float):
    """Hermitian square root X = M^{1/2} and pseudo-inverse square root X+ of a message.

    Used to absorb the BP environment onto the environment legs before the gate and to
    remove it afterwards (Eq. "SymmetricTensor"; Fig. "SimpleUpdate" steps iv-v).
    """
    H = 0.5 * (M + M.conj().T)
    lam, W = np.linalg.eigh(H)
    lam = np.clip(lam, 0.0, None)
    lmax = lam.max() if lam.size else 0.0
    sq = np.sqrt(lam)
    inv = np.where(lam > eps_eig * lmax, 1.0 / np.where(sq > 0, sq, 1.0), 0.0)
    X = (W * sq) @ W.conj().T
    Xp = (W * inv) @ W.conj().T
    return X, Xp


def contract_greedy(tensors):
    """Contract a list of (array, labels) over all shared labels, pairwise, always taking the
    pair whose result is smallest (pieces without shared labels are joined by outer products).
    Returns a one-element list.  Plain and exact; for the small networks of the diagnostics."""
    tensors = list(tensors)
    while len(tensors) > 1:
        best = None
        for i in range(len(tensors)):
            for j in range(i + 1, len(tensors)):
                li, lj = tensors[i][1], tensors[j][1]
                common = [x for x in li if x in lj]
                if not common:
                    continue
                size = 1
                for t_, l_ in ((tensors[i][0], li), (tensors[j][0], lj)):
                    for dim, lab in zip(t_.shape, l_):
                        if lab not in common:
                            size *= dim
                if best is None or size < best[0]:
                    best = (size, i, j, common)
        if best is None:                       # disconnected pieces: outer product
            best = (0, 0, 1, [])
        _, i, j, common = best
        (A, la), (B, lb) = tensors[i], tensors[j]
        C = np.tensordot(A, B, axes=([la.index(x) for x in common], [lb.index(x) for x in common]))
        lc = [x for x in la if x not in common] + [x for x in lb if x not in common]
        tensors = [t for k_, t in enumerate(tensors) if k_ not in (i, j)] + [(C, lc)]
    return tensors


@dataclass
class Options:
    chi: int
    bp_tol: float = 1e-12
    bp_max_iter: int = 1000
    svd_cutoff: float = 1e-12
    eig_cutoff: float = 1e-12
    zz_sign: float = 1.0            # +1: exp(+i pi/4 ZZ) as printed in Eq. "Propagator"
    # BP to convergence before every gate (the costly "most accurate" schedule the Methods
    # mention; the default regauges once per Floquet step).  Tests only: on a tree it makes
    # every truncation the optimal one of the current state across that edge.
    regauge_every_gate: bool = False


class Network:
    """Site tensors and directed BP messages of a tensor network state on a graph."""

    def __init__(self, n_sites: int, edges, colour=None):
        edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
        self.n = int(n_sites)
        self.edges = [(int(u), int(v)) for u, v in edges.tolist()]
        self.colour = (np.zeros(len(self.edges), dtype=np.int64) if colour is None
                       else np.asarray(colour, dtype=np.int64))
        nb = [[] for _ in range(self.n)]
        for u, v in self.edges:
            nb[u].append(v)
            nb[v].append(u)
        self.nb = [sorted(x) for x in nb]
        # |0...0> as a bond-dimension-1 network (Eq. "State": all spins up)
        self.T = []
        for v in range(self.n):
            t = np.zeros((2,) + (1,) * len(self.nb[v]), dtype=complex)
            t[(0,) + (0,) * len(self.nb[v])] = 1.0
            self.T.append(t)
        self.M = {}
        for u, v in self.edges:
            self.M[(u, v)] = np.ones((1, 1), dtype=complex)
            self.M[(v, u)] = np.ones((1, 1), dtype=complex)

    def axis(self, v: int, u: int) -> int:
        """Leg of T_v that points at neighbour u."""
        return 1 + self.nb[v].index(u)

    def bond_dim(self, u: int, v: int) -> int:
        return self.T[u].shape[self.axis(u, v)]

    # -- state evolution ---------------------------------------------------------------
    def apply_rx(self, theta: float) -> None:
        """Exact single-site rotation on every physical leg (first factor of U)."""
        R = rx_matrix(theta)
        for v in range(self.n):
            self.T[v] = np.tensordot(R, self.T[v], axes=([1], [0]))

    def _isolate(self, x: int, y: int, eps_eig: float):
        """Absorb sqrt(messages) on the environment legs of x, then QR-isolate the bond.

        Returns (Q or None, R[r, s, b], layout) with A = Q R, where A is the matricised
        tensor with rows = environment legs and columns = (physical, bond to y).
        """
        T = self.T[x]
        ax_y = self.axis(x, y)
        env_axes, Xp = [], {}
        Tt = T
        for i, u in enumerate(self.nb[x]):
            if u == y:
                continue
            ax = 1 + i
            X, Xpinv = msg_sqrt(self.M[(u, x)], eps_eig)
            Tt = absorb(Tt, ax, X)
            Xp[ax] = Xpinv
            env_axes.append(ax)
        perm = env_axes + [0, ax_y]
        A = np.transpose(Tt, perm)
        env_shape = A.shape[:len(env_axes)]
        rows = int(np.prod(env_shape)) if env_shape else 1
        d_e = T.shape[ax_y]
        A = A.reshape(rows, 2 * d_e)
        if rows > 2 * d_e:
            Q, R = np.linalg.qr(A, mode="reduced")
        else:
            Q, R = None, A
        layout = (perm, env_shape, env_axes, Xp)
        return Q, R.reshape(R.shape[0], 2, d_e), layout

    def _rebuild(self, x: int, Q, Rn: np.ndarray, layout) -> None:
        """T~' = Q R'; then remove the environment with the inverse square roots."""
        perm, env_shape, env_axes, Xp = layout
        r, _, k = Rn.shape
        B = Rn.reshape(r, 2 * k)
        if Q is not None:
            B = Q @ B
        B = B.reshape(tuple(env_shape) + (2, k))
        inv = np.argsort(perm)
        Tn = np.transpose(B, inv)
        for ax in env_axes:
            Tn = absorb(Tn, ax, Xp[ax])
        self.T[x] = Tn

    def simple_update(self, v: int, w: int, opt: Options) -> float:
        """Apply exp(+i pi/4 Z_v Z_w) on edge (v, w); returns the discarded weight."""
        Qv, Rv, lay_v = self._isolate(v, w, opt.eig_cutoff)
        Qw, Rw, lay_w = self._isolate(w, v, opt.eig_cutoff)
        g = zz_gate_phases(opt.zz_sign)
        theta = np.einsum("isb,jtb->isjt", Rv, Rw) * g[None, :, None, :]
        rv, rw = Rv.shape[0], Rw.shape[0]
        mat = theta.reshape(rv * 2, rw * 2)
        U, sig, Vh = np.linalg.svd(mat, full_matrices=False)
        if sig.size == 0 or sig[0] <= 0.0:
            raise FloatingPointError("simple update: zero two-site block")
        # truncation to at most chi: the Schmidt weights are p_i = sigma_i^2; weights below
        # svd_cutoff * p_1 are dropped as numerically zero
        p = sig ** 2
        above = int(np.count_nonzero(p > opt.svd_cutoff * p[0]))
        k = min(opt.chi, above)
        discarded = float(np.sum(p[k:])) / float(np.sum(p))
        S = sig[:k] / np.linalg.norm(sig[:k])
        # diagnostics of the cut: when chi (not the cutoff) sets k, the gap between the last
        # kept and the first dropped singular value relative to sigma_1 (a near-zero gap makes
        # the kept subspace ill-determined)
        self.last_kept = k
        self.last_cut_gap = float((sig[k - 1] - sig[k]) / sig[0]) if above > k else math.inf
        self.last_S = S
        sq = np.sqrt(S)
        Rv_new = (U[:, :k] * sq[None, :]).reshape(rv, 2, k)
        Rw_new = (sq[:, None] * Vh[:k, :]).reshape(k, rw, 2).transpose(1, 2, 0)
        self._rebuild(v, Qv, Rv_new, lay_v)
        self._rebuild(w, Qw, Rw_new, lay_w)
        Mnew = np.diag(S / S.sum()).astype(complex)
        self.M[(v, w)] = Mnew
        self.M[(w, v)] = Mnew.copy()
        return discarded

    # -- belief propagation --------------------------------------------------------------
    def message(self, v: int, w: int, M: dict) -> np.ndarray:
        """M'_{v->w} = sum T_v (prod_{u != w} M_{u->v}) conj(T_v), unit trace
        (Eq. "MessageTensorSelfConsistency")."""
        T = self.T[v]
        Y = T
        for i, u in enumerate(self.nb[v]):
            if u == w:
                continue
            Y = absorb(Y, 1 + i, M[(u, v)])
        ax = self.axis(v, w)
        others = [a for a in range(T.ndim) if a != ax]
        out = np.tensordot(Y, T.conj(), axes=(others, others))
        # Divide by the complex trace: the result has trace exactly 1.  (Dividing by the
        # real part only would leave a common phase of the messages undamped; it grows
        # by a factor degree-1 at every site and destabilises the sweep.)
        tr = np.trace(out)
        if not (tr.real > 0.0) or not np.isfinite(tr):
            raise FloatingPointError(f"BP: non-positive message trace on {v}->{w}")
        return out / tr

    def vertex_classes(self) -> list:
        """Site classes of the BP sweep: the two sides of a bipartite graph (breadth-first
        2-colouring, each connected component started at its smallest site, which takes class
        0), otherwise the greedy proper vertex colouring in increasing site id."""
        cls = [-1] * self.n
        bip = True
        for s in range(self.n):
            if cls[s] >= 0:
                continue
            cls[s] = 0
            queue = [s]
            while queue:
                x = queue.pop(0)
                for y in self.nb[x]:
                    if cls[y] < 0:
                        cls[y] = 1 - cls[x]
                        queue.append(y)
                    elif cls[y] == cls[x]:
                        bip = False
        if not bip:
            cls = [-1] * self.n
            for v in range(self.n):
                used = {cls[u] for u in self.nb[v] if cls[u] >= 0}
                c = 0
                while c in used:
                    c += 1
                cls[v] = c
        return cls

    def bp_sweep(self):
        """One sweep of Eq. "MessageTensorSelfConsistency", class by class: all messages sent by
        the sites of one vertex class are recomputed from the current messages (the sites of a
        class are not adjacent, so their updates are independent) and replace them before the
        next class.  On a bipartite graph this advances the message fixed-point iteration by two
        of its synchronous steps per sweep.  Returns the largest Frobenius change."""
        if not hasattr(self, "_classes"):
            self._classes = self.vertex_classes()
        res = 0.0
        for c in range(max(self._classes) + 1 if self.n else 0):
            new = {}
            for v in range(self.n):
                if self._classes[v] != c:
                    continue
                for w in self.nb[v]:
                    m = self.message(v, w, self.M)
                    res = max(res, float(np.linalg.norm(m - self.M[(v, w)])))
                    new[(v, w)] = m
            self.M.update(new)
        return res

    def bp(self, tol: float, max_iter: int):
        it, res = 0, math.inf
        while it < max_iter:
            res = self.bp_sweep()
            it += 1
            if res < tol:
                break
        return it, res

    # -- observables ---------------------------------------------------------------------
    def site_density(self, v: int) -> np.ndarray:
        """rho[s, s'] = sum T_v[s] (prod_u M_{u->v}) conj(T_v[s']) (Eq. "SingleSIte")."""
        Y = self.T[v]
        for i, u in enumerate(self.nb[v]):
            Y = absorb(Y, 1 + i, self.M[(u, v)])
        legs = list(range(1, Y.ndim))
        return np.tensordot(Y, self.T[v].conj(), axes=(legs, legs))

    def expect_site(self, v: int, op: int) -> float:
        rho = self.site_density(v)
        val = np.trace(PAULI[op] @ rho) / np.trace(rho)
        return float(val.real)

    def expect_pauli_cluster(self, sites, ops) -> float:
        """<P> of a Pauli string on any connected cluster, loops included: the cluster's norm
        network (operators on the ket, every leg leaving the cluster closed with its incoming BP
        message) is contracted exactly, Re(<P>_BP / <I>_BP).  On a tree cluster this is
        expect_pauli; a cluster that is the whole lattice is the exact expectation in the state.
        """
        sites = [int(x) for x in sites]
        opmap = {x: int(o) for x, o in zip(sites, ops)}
        cset = set(sites)

        def value(with_ops: bool) -> complex:
            tensors = []
            for w in sites:
                O = PAULI[opmap[w]] if with_ops else PAULI[0]
                Y = np.tensordot(O, self.T[w], axes=([1], [0]))
                out_legs = []
                for i, x in enumerate(self.nb[w]):
                    if x in cset:
                        out_legs.append(1 + i)
                    else:
                        Y = absorb(Y, 1 + i, self.M[(x, w)])
                closed = [a for a in range(Y.ndim) if a not in out_legs]   # physical + cut legs
                N = np.tensordot(Y, self.T[w].conj(), axes=(closed, closed))
                k = len(out_legs)
                perm = [q for i in range(k) for q in (i, k + i)]
                dims = [self.T[w].shape[a] ** 2 for a in out_legs]
                N = np.transpose(N, perm).reshape(dims) if k else N
                labels = [(min(w, self.nb[w][a - 1]), max(w, self.nb[w][a - 1])) for a in out_legs]
                tensors.append((N, labels))
            return complex(np.asarray(contract_greedy(tensors)[0][0]))

        return float((value(True) / value(False)).real)

    def expect_pauli(self, sites, ops) -> float:
        """<P> of a Pauli string on a cluster whose induced subgraph is a tree.

        The cluster is contracted exactly; every leg that leaves the cluster is closed
        with the incoming BP message.  Returns Re(<P>_BP / <I>_BP).
        """
        sites = [int(s) for s in sites]
        opmap = {s: int(o) for s, o in zip(sites, ops)}
        cset = set(sites)
        inner = [(u, v) for (u, v) in self.edges if u in cset and v in cset]
        if len(inner) != len(sites) - 1:
            raise ValueError("Pauli cluster must induce a tree")
        root = sites[0]

        def value(with_ops: bool) -> complex:
            def env(v: int, parent) -> np.ndarray:
                O = PAULI[opmap[v]] if with_ops else PAULI[0]
                # fold the operator onto the ket: T'[s] = sum_s' O[s, s'] T[s'] gives
                # sum T' conj(T) = sum_{s,s'} O[s,s'] T[s'] conj(T[s]) = <O> contribution
                Y = np.tensordot(O, self.T[v], axes=([1], [0]))
                for i, u in enumerate(self.nb[v]):
                    if u == parent:
                        continue
                    E = env(u, v) if u in cset else self.M[(u, v)]
                    Y = absorb(Y, 1 + i, E)
                legs = [a for a in range(Y.ndim)
                        if parent is None or a != self.axis(v, parent)]
                return np.tensordot(Y, self.T[v].conj(), axes=(legs, legs))
            return complex(env(root, None))

        return float((value(True) / value(False)).real)

    def bond_spectrum(self, v: int, w: int) -> np.ndarray:
        """Schmidt weights p_i = lambda_i^2 of the bond (v, w) under the BP approximation,
        descending, unit sum (the bond tensor spectrum of Eq. "EntanglementEntropy").

        Cutting the edge splits the BP-contracted norm into the two messages that meet on it:
        <psi|psi> = sum_{a,a'} M_{v->w}[a, a'] M_{w->v}[a, a'] = Tr(M_{v->w} M_{w->v}^T), and in
        the Vidal gauge both messages are the diagonal bond matrix, so the squared bond
        weights are the eigenvalues of M_{v->w} M_{w->v}^T (real and >= 0 for the positive
        semidefinite messages: rounding below zero is clipped).  Exact on a tree without
        truncation.
        """
        P = self.M[(v, w)] @ self.M[(w, v)].T
        lam = np.clip(np.linalg.eigvals(P).real, 0.0, None)
        s = lam.sum()
        if not s > 0.0:
            raise FloatingPointError(f"bond ({v}, {w}): zero norm")
        return np.sort(lam / s)[::-1]

    def vidal_gauge(self, cutoff: float = 1e-12) -> dict:
        """Bring the state into the symmetric Vidal gauge with the BP messages (Methods, "The
        Vidal gauge": the messages define the gauge transformation that makes every grouping of
        Eq. "IsometryPropertyDefinition" an isometry, Eq. "IsometryDefinition").

        For an edge (u, v) let X = M_{u->v}^{1/2}, Y = M_{v->u}^{1/2}.  The state across the
        edge is L R^T with Gram matrices L^H L = M_{u->v}^T and R^H R = M_{v->u}^T, so
        L = Q_L X^T and R = Q_R Y^T with isometric Q's, and the SVD X^T Y = U S V^H gives the
        Schmidt form (Q_L U) S (Q_R conj V)^T.  Inserting the identity X^{T+} U S V^H Y^{+}
        (on the supports, up to a positive factor) on the bond and splitting S symmetrically,
        leg u->v of T_u absorbs P_u = X^{T+} U W and leg v->u of T_v absorbs
        P_v = Y^{T+} conj(V) W with W = (S / sum S)^{1/2}, the root of the new unit-trace message:
        a state already in this gauge then gets P = 1 (the transform is idempotent and keeps the
        tensors' scale).  S is normalised to unit 2-norm and singular values whose Schmidt weight
        s_i^2 is <= cutoff * s_1^2 are dropped.  The new messages are the BP fixed point diag(S) / sum S.  Returns
        {(u, v): S} in edge order.
        """
        lam, P = {}, {}
        for u, v in self.edges:
            X, Xp = msg_sqrt(self.M[(u, v)], cutoff)
            Y, Yp = msg_sqrt(self.M[(v, u)], cutoff)
            U, sv, Vh = np.linalg.svd(X.T @ Y)
            keep = sv ** 2 > cutoff * sv[0] ** 2          # Schmidt weights, as in the truncation
            U, sv, Vh = U[:, keep], sv[keep], Vh[keep, :]
            sv = sv / np.linalg.norm(sv)
            lam[(u, v)] = sv
            w = np.sqrt(sv / sv.sum())
            P[(u, v)] = Xp.T @ (U * w[None, :])
            P[(v, u)] = Yp.T @ (Vh.T * w[None, :])
        for v in range(self.n):
            for u in self.nb[v]:
                self.T[v] = absorb(self.T[v], self.axis(v, u), P[(v, u)])
        for (u, v), sv in lam.items():
            D = np.diag(sv / sv.sum()).astype(complex)
            self.M[(u, v)] = D
            self.M[(v, u)] = D.copy()
        return lam

    def edge_environment(self, u: int, v: int) -> np.ndarray:
        """The norm network <psi|psi> with edge (u, v) cut and everything else contracted exactly
        (Methods, "Estimating the error of BP for general tensor networks", Fig.
        "EdgeEnvironment"): a (d*d) x (d*d) matrix, rows the (ket, bra) pair of the cut on u's
        side, columns on v's side, d the bond dimension.  Small networks only: every site first
        becomes its norm tensor N_w = sum_s T_w[s] (x) conj(T_w[s]) (one leg of dimension d_e^2
        per neighbour), then pairs of tensors are contracted greedily (smallest result first).
        """
        tensors = []
        for w in range(self.n):
            T = self.T[w]
            k = T.ndim - 1
            N = np.tensordot(T, T.conj(), axes=([0], [0]))          # legs ket..., bra...
            perm = [x for i in range(k) for x in (i, k + i)]          # (ket_i, bra_i) adjacent
            N = np.transpose(N, perm).reshape([T.shape[1 + i] ** 2 for i in range(k)])
            labels = []
            for x in self.nb[w]:
                if {w, x} == {u, v}:
                    labels.append(("cut", w))
                else:
                    labels.append(("bond", min(w, x), max(w, x)))
            tensors.append((N, labels))
        tensors = contract_greedy(tensors)
        E, labels = tensors[0]
        E = np.transpose(E, [labels.index(("cut", u)), labels.index(("cut", v))])
        return E

    def bp_error(self, u: int, v: int, cutoff: float = 1e-12):
        """BP error estimate on edge (u, v) (Eq. "BPErrorEstimate"): 1 - sqrt(l_1^2 / sum l_i^2)
        over the singular values l_i of the edge environment, taken in the symmetric gauge (the
        state is first brought into it with vidal_gauge, which the paper prescribes for
        consistency).  Returns (error, singular values normalised to unit 2-norm)."""
        self.vidal_gauge(cutoff)
        sv = np.linalg.svd(self.edge_environment(u, v), compute_uv=False)
        sv = sv / np.linalg.norm(sv)
        return float(1.0 - math.sqrt(sv[0] ** 2)), sv

    def bond_entropy(self, v: int, w: int) -> float:
        """s = -sum_i p_i log2 p_i over the Schmidt weights of the bond (Eq.
        "EntanglementEntropy", read with the minus sign and the sum over the chi weights)."""
        p = self.bond_spectrum(v, w)
        p = p[p > 0.0]
        return float(-np.sum(p * np.log2(p)))


# A chi-limited cut whose gap (sigma_chi - sigma_{chi+1}) / sigma_1 is below this is counted as
# near-degenerate: rounding can then move the kept subspace.
DEGENERATE_GAP = 1e-10


@dataclass
class Result:
    z: np.ndarray                       # [depth, n_sites] (or [1, n_sites])
    pauli: np.ndarray                   # [n_pauli] at the final step
    bp_iters: list = field(default_factory=list)
    bp_residual: list = field(default_factory=list)
    discarded: list = field(default_factory=list)
    converged: bool = True
    entropy: np.ndarray | None = None   # [rows, n_edges] bond entropies (bits) when asked for
    bond_dims: np.ndarray | None = None  # [rows, n_edges] bond dimension of every edge
    min_cut_gap: list = field(default_factory=list)      # per step, min over chi-limited cuts
    degenerate_cuts: list = field(default_factory=list)  # per step, cuts with gap < DEGENERATE_GAP


def solve(n_sites: int, edges, colour, theta: float, depth: int, opt: Options,
          pauli=(), record_every_step: bool = True, net: Network | None = None,
          clifford_steps: int = 0, entropy: bool = False) -> Result:
    """Run ``depth`` Floquet steps and measure (Eq. "State"; Methods).

    Each step: exact X rotations, then the simple-update gate layers in ascending
    colour, then BP to convergence, then <Z_v> for every site.
    ``clifford_steps`` further steps apply U(pi/2)^dagger (the extended time evolution of
    "Measuring expectation values"): since U = (ZZ gates)(X rotations), its adjoint applies
    the gates exp(-i pi/4 ZZ) first (descending colour, the forward order mirrored), then the
    X rotations by -pi/2; BP and <Z_v> follow as after a forward step.
    ``pauli`` is a sequence of (sites, ops) evaluated after the final step.
    ``entropy``: also record the bond entropy of every edge (``Network.bond_entropy``) on
    the same steps as <Z_v>.
    """
    if net is None:
        net = Network(n_sites, edges, colour)
    colours = sorted(set(int(c) for c in net.colour.tolist()))
    inv = Options(chi=opt.chi, bp_tol=opt.bp_tol, bp_max_iter=opt.bp_max_iter,
                  svd_cutoff=opt.svd_cutoff, eig_cutoff=opt.eig_cutoff, zz_sign=-opt.zz_sign)
    steps = depth + clifford_steps
    zs, iters, resid, disc, ents, dims, gaps, degen = [], [], [], [], [], [], [], []
    converged = True
    for _t in range(steps):
        dsum, gmin, ndeg = 0.0, math.inf, 0

        def gate(u, v, o):
            nonlocal dsum, gmin, ndeg
            if opt.regauge_every_gate:
                net.bp(opt.bp_tol, opt.bp_max_iter)
            dsum += net.simple_update(u, v, o)
            gmin = min(gmin, net.last_cut_gap)
            ndeg += net.last_cut_gap < DEGENERATE_GAP

        if _t < depth:
            net.apply_rx(theta)
            for c in colours:
                for e, (u, v) in enumerate(net.edges):
                    if int(net.colour[e]) == c:
                        gate(u, v, opt)
        else:
            for c in reversed(colours):
                for e, (u, v) in enumerate(net.edges):
                    if int(net.colour[e]) == c:
                        gate(u, v, inv)
            net.apply_rx(-math.pi / 2)
        it, res = net.bp(opt.bp_tol, opt.bp_max_iter)
        converged &= res < opt.bp_tol
        iters.append(it)
        resid.append(res)
        disc.append(dsum)
        gaps.append(gmin)
        degen.append(ndeg)
        if record_every_step or _t == steps - 1:
            zs.append([net.expect_site(v, 3) for v in range(net.n)])
            dims.append([net.bond_dim(u, v) for u, v in net.edges])
            if entropy:
                ents.append([net.bond_entropy(u, v) for u, v in net.edges])
    if steps == 0:
        zs.append([1.0] * net.n)
        dims.append([1] * len(net.edges))
        ents.append([0.0] * len(net.edges))
    pv = np.array([net.expect_pauli(s, o) for s, o in pauli], dtype=float)
    return Result(np.array(zs, dtype=float), pv, iters, resid, disc, converged,
                  np.array(ents, dtype=float) if entropy else None,
                  np.array(dims, dtype=np.int64), gaps, degen)
