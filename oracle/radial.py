"""CPU oracle of the three-phase radialization (Section V).

TEST INFRASTRUCTURE ONLY: the tests and the package smoke check use this;
the product path never does.

Steps, in the paper's order:

* The Kron-reduced network of a kept set (eq. Y_kron: the Schur complement
  that eliminates every other node, with the pseudo-inverse on present
  phases).  Two kept nodes are connected when their 3x3 block of Y_Kron has
  a nonzero entry (Lemma 2: the pattern is that of a single-phase network
  with the same topology).
* Its maximal cliques (the reduced network of a radial one is an
  edge-disjoint union of maximal cliques; a clique of three or more nodes
  is a mesh).
* For every maximal clique of three or more nodes: the sub-tree of the
  original feeder that spans the clique's nodes, and its nodes of degree 3
  or more (critical nodes).  The radialized kept set is the kept set plus
  every critical node.
* Injections are not reassigned (critical nodes carry none), so the
  radialized and the meshed reduced networks give the same voltages at the
  kept nodes.
"""
from __future__ import annotations

import numpy as np


def full_Y(f):
    """Dense admittance matrix over present node-phases and the index map
    (node, phase) -> row (-1 on absent phases)."""
    parent, phase = np.asarray(f["parent"]), np.asarray(f["phase"])
    n = len(parent)
    idx = -np.ones((n, 3), dtype=np.int64)
    k = 0
    for i in range(n):
        for p in range(3):
            if (int(phase[i]) >> p) & 1:
                idx[i, p] = k
                k += 1
    Y = np.zeros((k, k), dtype=np.complex128)
    Yd, Yo = np.asarray(f["Y_diag"]), np.asarray(f["Y_off"])

    def put(i, j, B):
        for a in range(3):
            for b in range(3):
                if idx[i, a] >= 0 and idx[j, b] >= 0:
                    Y[idx[i, a], idx[j, b]] += B[a, b]

    for i in range(n):
        put(i, i, Yd[i])
        if i > 0:
            put(i, int(parent[i]), Yo[i])
            put(int(parent[i]), i, Yo[i].T)
    return Y, idx


def kron(Y, idx, kept):
    """Y_Kron = Y_KK - Y_KR pinv(Y_RR) Y_RK over the kept nodes' rows."""
    kept = np.asarray(kept, bool)
    K = np.concatenate([idx[i][idx[i] >= 0] for i in np.flatnonzero(kept)])
    R = np.concatenate([idx[i][idx[i] >= 0] for i in np.flatnonzero(~kept)] + [np.zeros(0, np.int64)])
    if len(R) == 0:
        return Y[np.ix_(K, K)], K
    return Y[np.ix_(K, K)] - Y[np.ix_(K, R)] @ np.linalg.pinv(Y[np.ix_(R, R)]) @ Y[np.ix_(R, K)], K


def kron_adjacency(f, kept, Y=None, idx=None, rtol=1e-10):
    """Kept nodes joined in the Kron-reduced network: {i: set of j}."""
    if Y is None:
        Y, idx = full_Y(f)
    Yk, K = kron(Y, idx, kept)
    nodes = [int(i) for i in np.flatnonzero(np.asarray(kept, bool))]
    rows = {}
    at = 0
    for i in nodes:
        c = int((idx[i] >= 0).sum())
        rows[i] = slice(at, at + c)
        at += c
    scale = np.abs(Yk).max()
    adj = {i: set() for i in nodes}
    for a, i in enumerate(nodes):
        for j in nodes[a + 1:]:
            if np.abs(Yk[rows[i], rows[j]]).max() > rtol * scale:
                adj[i].add(j)
                adj[j].add(i)
    return adj


def maximal_cliques(adj):
    """Every maximal clique of an undirected graph (Bron-Kerbosch)."""
    out = []

    def grow(R, P, X):
        if not P and not X:
            out.append(sorted(R))
            return
        for v in sorted(P):
            grow(R | {v}, P & adj[v], X & adj[v])
            P = P - {v}
            X = X | {v}

    grow(set(), set(adj), set())
    return out


def spanning_subtree(parent, nodes):
    """Edges (child, parent) of the smallest sub-tree of the feeder that holds
    `nodes`: the union of their paths to their common ancestor."""
    def path(v):
        p = [v]
        while parent[p[-1]] >= 0:
            p.append(int(parent[p[-1]]))
        return p

    paths = [path(v) for v in nodes]
    common = set(paths[0])
    for p in paths[1:]:
        common &= set(p)
    top = max(common, key=lambda v: len(path(v)))  # the deepest common ancestor
    edges = set()
    for p in paths:
        for v in p:
            if v == top:
                break
            edges.add((v, int(parent[v])))
    return edges


def radialize(f, kept):
    """(radialized kept set, critical nodes, maximal cliques of 3+ nodes)."""
    parent = np.asarray(f["parent"])
    kept = np.asarray(kept, bool)
    cliques = [c for c in maximal_cliques(kron_adjacency(f, kept)) if len(c) >= 3]
    critical = set()
    for c in cliques:
        deg = {}
        for a, b in spanning_subtree(parent, c):
            deg[a] = deg.get(a, 0) + 1
            deg[b] = deg.get(b, 0) + 1
        critical |= {v for v, d in deg.items() if d >= 3 and not kept[v]}
    out = kept.copy()
    out[sorted(critical)] = True
    return out, sorted(critical), cliques


def reduced_voltages(f, kept, Iagg):
    """Voltages of the kept nodes from the Kron-reduced network with the
    slack held at V0 and injections Iagg[S, n, 3] (zero at nodes that carry
    none); absent phases are zero."""
    Y, idx = full_Y(f)
    kept = np.asarray(kept, bool)
    assert kept[0]
    Yk, K = kron(Y, idx, kept)
    nodes = [int(i) for i in np.flatnonzero(kept)]
    pos = {}
    at = 0
    for i in nodes:
        for p in range(3):
            if idx[i, p] >= 0:
                pos[(i, p)] = at
                at += 1
    s_rows = [pos[(0, p)] for p in range(3) if idx[0, p] >= 0]
    o_rows = [r for r in range(at) if r not in s_rows]
    V0 = np.asarray(f["V0"], dtype=np.complex128)[[p for p in range(3) if idx[0, p] >= 0]]
    S = Iagg.shape[0]
    V = np.zeros((S, len(f["parent"]), 3), dtype=np.complex128)
    for l in range(S):
        I = np.array([Iagg[l, i, p] for i in nodes for p in range(3) if idx[i, p] >= 0])
        rhs = I[o_rows] - Yk[np.ix_(o_rows, s_rows)] @ V0
        x = np.linalg.solve(Yk[np.ix_(o_rows, o_rows)], rhs)
        full = np.zeros(at, dtype=np.complex128)
        full[o_rows] = x
        full[s_rows] = V0
        for (i, p), r in pos.items():
            V[l, i, p] = full[r]
    return V
