"""Three-phase radialization (Section V) on the GPU against the oracle: the
radialized kept set (bit-exact), the number of critical nodes, the edges of
the radial reduced network, and the voltage equivalence of the radialized
network with the full one."""
import sys

import numpy as np
import pytest

import oracle
from oracle import greedy as G
from oracle import radial as RA
from synth_feeders import extreme_scenarios, hourly_feeder, make_feeder
from test_radial_oracle import directions_rule

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def okr():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2510_19608_amd as okr
    okr.lib()
    return okr


def nearest_kept_parent(parent, kept):
    kp = np.full(len(parent), -1)
    for v in range(1, len(parent)):  # parents precede children in these feeders
        p = int(parent[v])
        kp[v] = p if kept[p] else kp[p]
    return kp


def check(okr, f, sup):
    kept = np.zeros(f["n"], bool)
    kept[np.unique(sup)] = True
    want, crit, cliques = RA.radialize(f, kept)
    Gr = okr.Greedy(f)
    try:
        out = Gr.radialize(sup)
    finally:
        Gr.close()
    np.testing.assert_array_equal(out["kept_radial"].astype(bool), want)
    assert out["n_critical"] == len(crit)
    np.testing.assert_array_equal(out["kept_parent"], nearest_kept_parent(f["parent"], want))
    assert out["dv_radial"] <= 1e-12
    if crit:
        assert out["dv_meshed"] > 1e-9
    else:
        assert out["dv_meshed"] <= 1e-12
    return out, crit


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_radialize_matches_oracle(okr, seed):
    """Super-nodes of an Algorithm 1 search and a random kept set (nearest
    kept ancestor clusters) on 40-node feeders."""
    _say(f"radialize seed={seed}")
    f = make_feeder("c2", seed, n=40, snapshots=2, kappa=1.0)
    V, I, _, _ = oracle.powerflow(f)
    sup, _, _ = G.greedy(f, V, I, e_bar=3e-4)
    n_crit = [check(okr, f, sup)[1]]
    rng = np.random.default_rng(seed)
    keep = rng.random(f["n"]) < 0.4
    keep[0] = True
    s = np.zeros(f["n"], int)
    for v in range(f["n"]):
        s[v] = v if keep[v] else s[f["parent"][v]]
    n_crit.append(check(okr, f, s)[1])
    assert any(len(c) for c in n_crit)


def test_radialize_1000_node_search(okr):
    """The 1000-node Algorithm 1 reduction: critical nodes by the tree
    direction rule, radial voltages equal to the full network's."""
    f = extreme_scenarios(hourly_feeder("c2", 0, n=1000))
    out = okr.greedy(f, e_bar=1e-3)
    _say(f"radialize 1000-node: {out['n_kept']} super-nodes")
    Gr = okr.Greedy(f)
    try:
        r = Gr.radialize(out["super"])
    finally:
        Gr.close()
    kept = np.zeros(f["n"], bool)
    kept[np.unique(out["super"])] = True
    crit = directions_rule(f["parent"], kept)
    want = kept.copy()
    want[crit] = True
    np.testing.assert_array_equal(r["kept_radial"].astype(bool), want)
    assert r["n_critical"] == len(crit) > 0
    assert r["dv_radial"] <= 1e-12 < r["dv_meshed"]


def test_radialize_degenerate_assignments(okr):
    """Nothing reduced (no clique, nothing critical), and everything in the
    slack's cluster (a single kept node: no clique either)."""
    f = make_feeder("c2", 1, n=40, snapshots=1)
    for sup in (np.arange(f["n"]), np.zeros(f["n"], int)):
        out, crit = check(okr, f, sup)
        assert crit == [] and out["n_critical"] == 0
        assert out["dv_radial"] <= 1e-12 and out["dv_meshed"] <= 1e-12
