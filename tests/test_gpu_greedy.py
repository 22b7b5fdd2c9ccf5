"""The greedy single-move search (Algorithm 1) and the fixed-reduction
evaluation on the GPU, against the oracle: every applied move (candidate id,
super-nodes, SMICE, largest error), the final assignment and the final
errors; at 1000 nodes, the first move among all candidates and the
termination state."""
import sys

import numpy as np
import pytest

import oracle
from oracle import greedy as G
from synth_feeders import extreme_scenarios, hourly_feeder, make_feeder

pytestmark = pytest.mark.gpu

TOL = 1e-9


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


def same_steps(got, want):
    assert [(s["cand"], s["s"], s["r"]) for s in got] == [(s["cand"], s["s"], s["r"]) for s in want]
    # absolute, like every other error comparison: the two load flows stop at
    # 1e-13, so SMICE (a sum over clusters) differs by up to about n * 1e-13
    np.testing.assert_allclose([s["smice"] for s in got], [s["smice"] for s in want], rtol=0, atol=TOL)
    np.testing.assert_allclose([s["emax"] for s in got], [s["emax"] for s in want], rtol=0, atol=TOL)
    assert [s["n_cand"] for s in got] == [s["n_cand"] for s in want]
    assert [s["n_feasible"] for s in got] == [s["n_feasible"] for s in want]


@pytest.mark.parametrize("incremental", [False, True])
@pytest.mark.parametrize("n,S,seed,kappa,e_bar", [
    (30, 1, 0, 1.0, 3e-3), (40, 2, 1, 1.0, 3e-4), (60, 2, 2, 1.0, 1e-3), (80, 2, 3, 0.25, 3e-3),
    (100, 2, 4, 1.0, 1e-3)])
def test_every_step_matches_oracle(okr, n, S, seed, kappa, e_bar, incremental):
    """Whole searches on small feeders, in both scoring forms (every node of
    every candidate, or only the clusters a move can change): the same moves
    in the same order, the same SMICE and errors, the same final assignment
    and errors."""
    _say(f"greedy n={n} S={S} seed={seed} kappa={kappa} e_bar={e_bar} incremental={incremental}")
    f = make_feeder("c2", seed, n=n, snapshots=S, kappa=kappa)
    V, I, _, _ = oracle.powerflow(f)
    sup, steps, err = G.greedy(f, V, I, e_bar=e_bar)
    if any(s["ambiguous"] for s in steps):
        pytest.skip("a near-tie within the ambiguity margin in the oracle's search")
    out = okr.greedy(f, e_bar=e_bar, incremental=incremental)
    assert out["incremental"] == incremental
    same_steps(out["steps"], steps)
    np.testing.assert_array_equal(out["super"], sup)
    np.testing.assert_allclose(out["err_per_snapshot"], err, rtol=0, atol=TOL)
    assert out["n_kept"] == n - len(steps)
    assert not any(s["ambiguous"] for s in out["steps"])


def test_given_vhat_and_move_cap(okr):
    """With V^ passed in (no load flow) and a cap on the moves, the search is
    the first moves of the uncapped one."""
    f = make_feeder("c2", 5, n=50, snapshots=2, kappa=1.0)
    V, I, _, _ = oracle.powerflow(f)
    sup, steps, err = G.greedy(f, V, I, e_bar=1e-3, max_iter=7)
    out = okr.greedy(f, e_bar=1e-3, vhat=V, max_iter=7)
    same_steps(out["steps"], steps)
    np.testing.assert_array_equal(out["super"], sup)
    np.testing.assert_allclose(out["err_per_snapshot"], err, rtol=0, atol=TOL)


@pytest.mark.parametrize("n,seed", [(60, 0), (150, 1)])
def test_robustness_evaluation(okr, n, seed):
    """Section VI robustness study: reduce with the highest- and lowest-loaded
    of 168 hourly scenarios, then score that reduction over all 168; every
    hour's largest error equals the oracle's."""
    _say(f"greedy robustness n={n} seed={seed}")
    fh = hourly_feeder("c2", seed, n=n, kappa=1.0)
    f2 = extreme_scenarios(fh)
    V, I, _, _ = oracle.powerflow(f2)
    sup, steps, _ = G.greedy(f2, V, I, e_bar=1e-3)
    out = okr.greedy(f2, e_bar=1e-3)
    np.testing.assert_array_equal(out["super"], sup)
    err, mx = okr.evaluate_assignment(fh, out["super"])
    Vh, Ih, _, _ = oracle.powerflow(fh)
    want = G.evaluate(fh, Vh, Ih, sup)
    np.testing.assert_allclose(err, want, rtol=0, atol=TOL)
    assert mx == err.max()


def test_evaluate_rejects_bad_assignments(okr):
    """okr_greedy_evaluate refuses assignments that are not clusterings: a
    cluster in two pieces, a node assigned to a node that is itself
    assigned elsewhere."""
    f = make_feeder("c2", 0, n=30, snapshots=1)
    sup = np.arange(30)
    bad = sup.copy()
    bad[5] = 29  # {5, 29}: node 5's parent is outside the cluster, and so is 29's
    with pytest.raises(okr.OkrError) as e:
        okr.evaluate_assignment(f, bad)
    assert e.value.code == okr.OKR.E_ARG
    bad = sup.copy()
    bad[3] = 4   # 4 is not a super-node once it is assigned to the slack
    bad[4] = 0
    with pytest.raises(okr.OkrError) as e:
        okr.evaluate_assignment(f, bad)
    assert e.value.code == okr.OKR.E_ARG


@pytest.mark.parametrize("incremental", [False, True])
def test_1000_node_first_move_and_termination(okr, incremental):
    """1000-node feeder with its two extreme scenarios (the Table III workload
    shape), both scoring forms: the first move is the oracle's choice among
    all ~2000 candidates with the oracle's SMICE, and at the end no candidate
    is feasible in the oracle's scoring of the final state."""
    fh = hourly_feeder("c2", 0, n=1000)
    f = extreme_scenarios(fh)
    V, I, _, _ = oracle.powerflow(f)
    e_bar = f["e_bar"]
    _say(f"greedy 1000-node: GPU run, incremental={incremental}")
    out = okr.greedy(f, e_bar=e_bar, incremental=incremental)
    assert out["incremental"] == incremental
    assert out["n_steps"] > 0 and out["max_err"] <= e_bar
    net = G.Network(f)
    sup0 = np.arange(f["n"])
    cands = G.candidates(f["parent"], f["phase"], sup0)
    _say(f"greedy 1000-node: oracle scores {len(cands)} first-move candidates")
    sm, em = G.score(net, V, I, sup0, cands, e_bar)
    pick, amb = G.select(cands, sm, em, e_bar, 1e-11, 1e-13)
    assert not amb
    first = out["steps"][0]
    assert (first["cand"], first["s"], first["r"]) == cands[pick]
    np.testing.assert_allclose(first["smice"], sm[pick], rtol=0, atol=TOL)
    assert first["n_cand"] == len(cands)
    _say("greedy 1000-node: oracle scores the final state")
    supf = out["super"]
    cf = G.candidates(f["parent"], f["phase"], supf)
    smf, emf = G.score(net, V, G.aggregate(I, supf), supf, cf, e_bar)
    assert not np.isfinite(smf).any()
    np.testing.assert_allclose(out["err_per_snapshot"], G.evaluate(f, V, I, supf, net=net), rtol=0, atol=TOL)


def test_scoring_forms_agree_at_3000_nodes(okr):
    """Where both forms fit (S * n = 6000), the incremental scoring makes the
    same moves as scoring every node, with the same SMICE (the forms differ
    only in summation order), on a 3000-node feeder."""
    f = extreme_scenarios(hourly_feeder("c2", 1, n=3000))
    _say("greedy 3000-node: both scoring forms")
    a = okr.greedy(f, e_bar=f["e_bar"])
    b = okr.greedy(f, e_bar=f["e_bar"], incremental=True)
    assert not a["incremental"] and b["incremental"]
    assert a["n_steps"] > 100
    same_steps(b["steps"], a["steps"])
    np.testing.assert_array_equal(b["super"], a["super"])
    np.testing.assert_allclose(b["err_per_snapshot"], a["err_per_snapshot"], rtol=0, atol=TOL)


@pytest.mark.parametrize("incremental", [False, True])
def test_graph_replay_equals_stream_launches(okr, incremental):
    """Without timing, full batches of 32 iterations replay one captured
    graph; with timing every launch goes to the stream.  Both give the same
    moves, bit for bit, over many replays with host synchronisations
    between them."""
    f = extreme_scenarios(hourly_feeder("c2", 2, n=300))
    Gr = okr.Greedy(f)
    try:
        a = Gr.run(f["e_bar"], incremental=incremental)
        b = Gr.run(f["e_bar"], timing=True, incremental=incremental)
    finally:
        Gr.close()
    assert a["n_steps"] > 64
    assert [(s["cand"], s["s"], s["r"]) for s in a["steps"]] == [(s["cand"], s["s"], s["r"]) for s in b["steps"]]
    assert [s["smice"] for s in a["steps"]] == [s["smice"] for s in b["steps"]]
    np.testing.assert_array_equal(a["super"], b["super"])
    np.testing.assert_array_equal(a["err_per_snapshot"], b["err_per_snapshot"])


def test_edge_cases(okr):
    """Degenerate inputs: a two-node feeder (one candidate), a single node
    (nothing to do), a bound no move meets (nothing reduced), the largest
    scenario count (64) and one above it (refused)."""
    f2 = make_feeder("c2", 0, n=2, snapshots=1)
    V, I, _, _ = oracle.powerflow(f2)
    sup, steps, err = G.greedy(f2, V, I, e_bar=1.0)
    out = okr.greedy(f2, e_bar=1.0)
    same_steps(out["steps"], steps)
    assert out["n_steps"] == 1 and out["n_kept"] == 1 and list(out["super"]) == [0, 0]
    f1 = make_feeder("c2", 0, n=1, snapshots=1)
    out = okr.greedy(f1, e_bar=1.0)
    assert out["n_steps"] == 0 and out["n_kept"] == 1 and out["max_err"] == 0.0
    f = make_feeder("c2", 3, n=40, snapshots=2)
    out = okr.greedy(f, e_bar=1e-14)
    assert out["n_steps"] == 0 and list(out["super"]) == list(range(40))
    f64 = make_feeder("c2", 4, n=30, snapshots=64)
    V, I, _, _ = oracle.powerflow(f64)
    sup, steps, err = G.greedy(f64, V, I, e_bar=1e-3, max_iter=5)
    out = okr.greedy(f64, e_bar=1e-3, max_iter=5)
    same_steps(out["steps"], steps)
    f65 = make_feeder("c2", 4, n=30, snapshots=65)
    with pytest.raises(okr.OkrError) as e:
        okr.greedy(f65, e_bar=1e-3)
    assert e.value.code == okr.OKR.E_UNSUPPORTED
