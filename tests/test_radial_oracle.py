"""Pins of the radialization oracle (Section V).

The oracle takes the paper's route (dense Kron reduction, maximal cliques,
spanning sub-trees, degree-3 nodes); these tests check it against a
hand-derived star (the paper's Fig. 4 situation), a chain, Lemma 2 (the
three-phase pattern equals the single-phase one), an independent
characterisation of critical nodes by tree directions, radiality of the
result, and the voltage equivalence the paper states.
"""
import numpy as np
import pytest

import oracle
from oracle import greedy as G
from oracle import radial as RA
from synth_feeders import make_feeder
from test_oracle import hand_feeder


def line_feeder(parent, phase=None):
    n = len(parent)
    phase = [7] * n if phase is None else phase
    z = np.array([[0.3 + 1.0j, 0.1 + 0.4j, 0.1 + 0.4j], [0.1 + 0.4j, 0.3 + 1.0j, 0.1 + 0.4j],
                  [0.1 + 0.4j, 0.1 + 0.4j, 0.3 + 1.0j]]) * 0.01
    zs = [None] + [z * (1 + 0.1 * i) for i in range(1, n)]
    return hand_feeder(parent, phase, zs, np.zeros((1, n, 3)))


def edges(adj):
    return {(min(i, j), max(i, j)) for i in adj for j in adj[i]}


def test_star_by_hand():
    """0-1-2-3 with 3 -> 4, 3 -> 5; keeping 0, 1, 4, 5 meshes 1, 4, 5 (node 3
    has degree 3); node 3 is the critical node and the result is a tree."""
    f = line_feeder([-1, 0, 1, 2, 3, 3])
    kept = np.array([1, 1, 0, 0, 1, 1], bool)
    adj = RA.kron_adjacency(f, kept)
    assert edges(adj) == {(0, 1), (1, 4), (1, 5), (4, 5)}
    assert sorted(map(tuple, RA.maximal_cliques(adj))) == [(0, 1), (1, 4, 5)]
    out, crit, cliques = RA.radialize(f, kept)
    assert crit == [3] and cliques == [[1, 4, 5]]
    assert edges(RA.kron_adjacency(f, out)) == {(0, 1), (1, 3), (3, 4), (3, 5)}


def test_chain_needs_nothing():
    f = line_feeder([-1, 0, 1, 2, 3])
    kept = np.array([1, 0, 1, 0, 1], bool)
    out, crit, cliques = RA.radialize(f, kept)
    assert crit == [] and cliques == []
    assert edges(RA.kron_adjacency(f, kept)) == {(0, 2), (2, 4)}


def directions_rule(parent, kept):
    """Reduced nodes with three or more tree directions that reach a kept
    node through reduced nodes only (breadth-first search per direction)."""
    n = len(parent)
    nb = [[] for _ in range(n)]
    for v in range(1, n):
        nb[v].append(int(parent[v]))
        nb[int(parent[v])].append(v)
    out = []
    for c in range(n):
        if kept[c]:
            continue
        k = 0
        for d in nb[c]:
            seen, todo, hit = {c}, [d], False
            while todo and not hit:
                u = todo.pop()
                if u in seen:
                    continue
                seen.add(u)
                if kept[u]:
                    hit = True
                else:
                    todo.extend(nb[u])
            k += hit
        if k >= 3:
            out.append(c)
    return out


def kept_sets(seed):
    """A random kept set and the super-nodes of an Algorithm 1 search."""
    f = make_feeder("c2", seed, n=40, snapshots=1, kappa=1.0)
    rng = np.random.default_rng(seed)
    keep = rng.random(f["n"]) < 0.4
    keep[0] = True
    V, I, _, _ = oracle.powerflow(f)
    sup, _, _ = G.greedy(f, V, I, e_bar=3e-4)
    ks = np.zeros(f["n"], bool)
    ks[np.unique(sup)] = True
    return f, V, I, sup, [keep, ks]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lemma2_pattern_matches_single_phase(seed):
    """The three-phase Kron pattern equals that of the single-phase network
    with the same topology (unit line admittances)."""
    f, _, _, _, sets = kept_sets(seed)
    n = f["n"]
    z1 = np.zeros((3, 3), complex)
    z1[0, 0] = 1.0
    f1 = hand_feeder(f["parent"], [1] * n, [None] + [z1] * (n - 1), np.zeros((1, n, 3)), V0=[1, 0, 0])
    for kept in sets:
        assert edges(RA.kron_adjacency(f, kept)) == edges(RA.kron_adjacency(f1, kept))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_radialization(seed):
    """Critical nodes equal the reduced nodes with three or more directions
    to kept nodes; the radialized pattern is a tree; and the kept nodes'
    voltages from the meshed and the radialized reduced networks equal each
    other and the full network's (injections not reassigned)."""
    f, V, I, sup, sets = kept_sets(seed)
    for k_i, kept in enumerate(sets):
        out, crit, cliques = RA.radialize(f, kept)
        assert crit == directions_rule(f["parent"], kept)
        adj = RA.kron_adjacency(f, out)
        assert len(edges(adj)) == int(out.sum()) - 1
        # connected
        seen, todo = set(), [0]
        while todo:
            u = todo.pop()
            if u not in seen:
                seen.add(u)
                todo.extend(adj[u])
        assert len(seen) == int(out.sum())
        if k_i == 1:
            Iagg = G.aggregate(I, sup)
        else:
            s = np.zeros(f["n"], int)
            for v in range(f["n"]):
                s[v] = v if kept[v] else s[f["parent"][v]]
            Iagg = G.aggregate(I, s)
        Vm = RA.reduced_voltages(f, kept, Iagg)
        Vr = RA.reduced_voltages(f, out, Iagg)
        Vf = G.Network(f).solve(Iagg)
        k = np.flatnonzero(kept)
        pres = G.Network(f).present[k]
        np.testing.assert_allclose(Vr[:, k][:, pres], Vm[:, k][:, pres], rtol=0, atol=1e-11)
        np.testing.assert_allclose(Vm[:, k][:, pres], Vf[:, k][:, pres], rtol=0, atol=1e-11)
