"""Pins of the Algorithm 1 (greedy single-move search) oracle.

Each test checks the oracle against something other than itself: a
hand-derived three-bus case, the power flow's own solution, the Kron
elimination route of the C oracle, and invariants of the search.
"""
import numpy as np
import pytest

import oracle
from oracle import greedy as G
from synth_feeders import make_feeder
from test_oracle import hand_feeder


def three_bus(z1, z2, I1, I2, V0=1.0):
    """Single-phase (phase a) line 0 - 1 - 2 with branch impedances z1, z2
    and injections I1, I2; V^ is the exact fixed-current solution."""
    Z1 = np.zeros((3, 3), complex)
    Z2 = np.zeros((3, 3), complex)
    Z1[0, 0], Z2[0, 0] = z1, z2
    f = hand_feeder([-1, 0, 1], [1, 1, 1], [None, Z1, Z2], np.zeros((1, 3, 3)), V0=[V0, 0, 0])
    V1 = V0 + z1 * (I1 + I2)
    V2 = V1 + z2 * I2
    Vhat = np.zeros((1, 3, 3), complex)
    Ihat = np.zeros((1, 3, 3), complex)
    Vhat[0, :, 0] = [V0, V1, V2]
    Ihat[0, 1:, 0] = [I1, I2]
    return f, Vhat, Ihat


def test_three_bus_candidates_by_hand():
    """Candidate set, moved currents, voltage copies and SMICE of every move
    on a three-bus line, derived by hand (V = V0 + sum of path impedance
    times downstream injection)."""
    z1, z2, I1, I2, V0 = 0.01 + 0.02j, 0.03 + 0.01j, -0.5 + 0.1j, -0.3 - 0.05j, 1.0
    f, Vhat, Ihat = three_bus(z1, z2, I1, I2, V0)
    V1, V2 = Vhat[0, 1, 0], Vhat[0, 2, 0]
    net = G.Network(f)
    sup = np.arange(3)
    cands = G.candidates(f["parent"], f["phase"], sup)
    # edge (1, 0): node 1 up into the slack; the slack never moves.
    # edge (2, 1): node 2 up into 1 (id 4), node 1 down into 2 (id 5)
    assert cands == [(2, 0, 1), (4, 1, 2), (5, 2, 1)]
    sm, em = G.score(net, Vhat, Ihat, sup, cands, e_bar=1.0)
    # id 2: I1 served at the slack, node 1 copies V0
    V2a = V0 + (z1 + z2) * I2
    e1a, e2a = abs(abs(V1) - abs(V0)), abs(abs(V2) - abs(V2a))
    # id 4: I2 moves to node 1 (V1 unchanged), node 2 copies V1
    e2b = abs(abs(V2) - abs(V1))
    # id 5: I1 moves to node 2, node 1 copies the new V2
    V2c = V0 + (z1 + z2) * (I1 + I2)
    e1c, e2c = abs(abs(V1) - abs(V2c)), abs(abs(V2) - abs(V2c))
    want_sm = [e1a + e2a, e2b, max(e1c, e2c)]
    want_em = [max(e1a, e2a), e2b, max(e1c, e2c)]
    np.testing.assert_allclose(sm, want_sm, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(em, want_em, rtol=1e-12, atol=1e-15)
    # feasibility: a bound between the values makes the larger ones infinite
    bound = sorted(want_em)[1]
    sm2, _ = G.score(net, Vhat, Ihat, sup, cands, e_bar=bound)
    assert np.isinf(sm2[np.array(want_em) > bound]).all()
    # the whole search on this line: smallest SMICE first
    sup_f, steps, err = G.greedy(f, Vhat, Ihat, e_bar=1.0)
    assert steps[0]["cand"] == cands[int(np.argmin(want_sm))][0]
    assert len(steps) == 2 and len(set(sup_f.tolist())) == 1


def test_solve_reproduces_power_flow():
    """With every node its own super-node, the full-network solve at the
    power flow's injections gives back the power flow's voltages (pins the
    assembly of Y: block placement, transposes, slack handling)."""
    for seed in (0, 1):
        f = make_feeder("c2", seed, n=80, snapshots=2)
        V, I, st, _ = oracle.powerflow(f)
        net = G.Network(f)
        np.testing.assert_allclose(net.solve(I), V, rtol=0, atol=1e-11)
        assert G.evaluate(f, V, I, np.arange(f["n"])).max() < 1e-11


@pytest.mark.parametrize("seed", [0, 2, 5])
def test_aggregated_solve_equals_kron_route(seed):
    """For assignments to the nearest kept ancestor, the aggregated-current
    full-network solve with voltage copies (Algorithm 1) equals the C
    oracle's route through the Kron-reduced network (Section IV states the
    two give the same super-node voltages), and so do the per-scenario
    errors."""
    f = make_feeder("c2", seed, n=60, snapshots=3)
    V, I, _, _ = oracle.powerflow(f)
    rng = np.random.default_rng(seed)
    keep = (rng.random(f["n"]) < 0.5).astype(np.uint8)
    keep[0] = 1
    sup = np.zeros(f["n"], int)
    for v in range(f["n"]):  # parents precede children in these feeders
        assert v == 0 or f["parent"][v] < v
        sup[v] = v if keep[v] else sup[f["parent"][v]]
    net = G.Network(f)
    Vc = net.solve(G.aggregate(I, sup))[:, sup, :]
    Vc = np.where(net.present, Vc, 0)
    np.testing.assert_allclose(Vc, oracle.candidate_voltages(f, I, keep), rtol=0, atol=1e-11)
    err, _ = oracle.final_errors(f, V, I, keep)
    np.testing.assert_allclose(G.evaluate(f, V, I, sup), err, rtol=0, atol=1e-11)


def test_scenario_sum_reading():
    """SMICE over scenarios is the sum of the per-scenario SMICE: a feeder
    with its one scenario duplicated scores every candidate twice as high,
    with the same largest error and the same decisions."""
    f1 = make_feeder("c2", 3, n=40, snapshots=1)
    V, I, _, _ = oracle.powerflow(f1)
    V2, I2 = np.concatenate([V, V]), np.concatenate([I, I])
    net = G.Network(f1)
    sup = np.arange(f1["n"])
    cands = G.candidates(f1["parent"], f1["phase"], sup)
    s1, e1 = G.score(net, V, I, sup, cands, e_bar=0.003)
    s2, e2 = G.score(net, V2, I2, sup, cands, e_bar=0.003)
    np.testing.assert_allclose(s2, 2 * s1, rtol=1e-13)
    np.testing.assert_array_equal(e2, e1)


@pytest.mark.parametrize("seed,e_bar", [(0, 3e-4), (1, 1e-3), (4, 3e-3)])
def test_search_invariants(seed, e_bar):
    """One super-node fewer per step; every applied move was feasible and is
    a valid candidate of its state (adjacent clusters, phases of r within
    s's, the slack never moved); SMICE >= the largest error; clusters stay
    connected; the final errors respect the bound; the search stops only
    when no candidate is feasible."""
    f = make_feeder("c2", seed, n=50, snapshots=2, kappa=1.0)
    V, I, _, _ = oracle.powerflow(f)
    sup, steps, err = G.greedy(f, V, I, e_bar=e_bar)
    n = f["n"]
    parent, phase = f["parent"], f["phase"]
    s_state = np.arange(n)
    for k, st in enumerate(steps):
        assert (st["cand"], st["s"], st["r"]) in G.candidates(parent, phase, s_state)
        assert st["r"] != 0 and st["emax"] <= e_bar and st["smice"] >= st["emax"]
        s_state = np.where(s_state == st["r"], st["s"], s_state)
        assert len(set(s_state.tolist())) == n - k - 1
    np.testing.assert_array_equal(s_state, sup)
    # clusters are connected: every member's path to its super stays in the cluster
    for x in range(n):
        a, b = x, sup[x]
        anc_a, anc_b = [a], [b]
        while anc_a[-1] > 0:
            anc_a.append(int(parent[anc_a[-1]]))
        while anc_b[-1] > 0:
            anc_b.append(int(parent[anc_b[-1]]))
        w = next(u for u in anc_a if u in anc_b)
        path = anc_a[:anc_a.index(w) + 1] + anc_b[:anc_b.index(w)]
        assert all(sup[u] == sup[x] for u in path)
    assert err.max() <= e_bar
    net = G.Network(f)
    cands = G.candidates(parent, phase, sup)
    sm, _ = G.score(net, V, G.aggregate(I, sup), sup, cands, e_bar)
    assert not np.isfinite(sm).any()
