"""Full-size parity where the error bound binds: the 1000-node (24
snapshots), 6000-node (96 snapshots) and 8400-node (288 snapshots) workloads
at e_bar = 1e-4 / 7e-5, where a quarter or more of the segments choose a mask
below their top level, so each arg-min is decided among many candidates (the
candidate-tile rescan of the arg-min, the mixed-precision shortlists and the
surrogate's second ranking stage and fallback all run).

Expected decisions, kept counts and final errors come from
tests/golden/make_golden.py (oracle only); per-mask scores are compared on
sampled masks, each scored by the oracle at the state the golden decisions
leave.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from synth_feeders import dfs_preorder, make_feeder

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-9
# (workload, golden file): every case here has a committed golden
CASES = [("c2", "oracle_c2_seed0_ebar1e-4.json"), ("c3", "oracle_c3_seed0_ebar7e-5.json")]
if os.path.exists(os.path.join(HERE, "golden", "oracle_c4_seed0_ebar7e-5.json")):
    CASES.append(("c4", "oracle_c4_seed0_ebar7e-5.json"))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def golden(fname):
    with open(os.path.join(HERE, "golden", fname)) as fh:
        return json.load(fh)


def seg_sizes(f, nseg):
    seg = np.asarray(f["segment"])
    return [int((seg == g).sum()) for g in range(nseg)]


@pytest.mark.parametrize("cfg,fname", CASES)
def test_binding_golden_is_not_degenerate(cfg, fname):
    """The golden decisions are spread over the levels: at least a quarter of
    the segments choose a mask below the top level, and none is a near-tie."""
    G = golden(fname)
    f = make_feeder(cfg, 0, e_bar=G["e_bar"])
    ks = seg_sizes(f, len(G["segments"]))
    below = sum(1 for k, s in zip(ks, G["segments"]) if s["popcount"] < k)
    assert below >= 0.25 * len(ks), (below, len(ks))
    assert not any(s["ambiguous"] for s in G["segments"])
    assert G["status"] == 0


@pytest.fixture(scope="module")
def okr():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2510_19608_amd as okr
    okr.lib()
    return okr


def check_against_golden(out, G):
    got = [s["mask"] for s in out["segments"]]
    want = [s["mask"] for s in G["segments"]]
    assert got == want
    assert int(out["n_kept"]) == G["n_kept"]
    for s, d in zip(out["segments"], G["segments"]):
        assert abs(s["e_loc"] - d["e_loc"]) < TOL
        assert not s["ambiguous"]
    np.testing.assert_allclose(out["err_per_snapshot"], G["err_per_snapshot"], rtol=0, atol=TOL)


FORMS = [dict(), dict(graph=True), dict(lanes=1), dict(precision="factored", graph=True),
         dict(precision="mixed", graph=True)]


@pytest.mark.gpu
@pytest.mark.parametrize("cfg,fname", CASES)
@pytest.mark.parametrize("form", range(len(FORMS)))
def test_binding_decisions(okr, cfg, fname, form):
    kw = FORMS[form]
    _say(f"{cfg} binding bound {kw}")
    G = golden(fname)
    f = make_feeder(cfg, 0, e_bar=G["e_bar"])
    out = okr.reduce_feeder(f, want_vhat=False, **kw)
    check_against_golden(out, G)
    if kw.get("precision") == "mixed":
        assert sum(s["n_refined"] for s in out["segments"]) > len(G["segments"])  # shortlists beyond the winners


@pytest.mark.gpu
@pytest.mark.parametrize("cfg,fname", CASES)
def test_binding_sampled_masks(okr, cfg, fname):
    """Every mask's FP64 score is dumped; for three segments below their top
    level, the winner, masks of the winner's level and above, and random
    masks are compared with the oracle at the golden state."""
    _say(f"{cfg} binding bound sampled masks")
    G = golden(fname)
    f = make_feeder(cfg, 0, e_bar=G["e_bar"])
    out = okr.reduce_feeder(f, dump=True, want_vhat=False)
    check_against_golden(out, G)
    V, I, st, _ = oracle.powerflow(f)
    assert st == 0
    pre = dfs_preorder(f["parent"])
    nseg = len(G["segments"])
    ks = seg_sizes(f, nseg)
    below = [g for g in range(nseg) if G["segments"][g]["popcount"] < ks[g]]
    picks = sorted({below[0], below[len(below) // 2], below[-1]})
    rng = np.random.default_rng(11)
    keep = np.ones(f["n"], np.uint8)
    for g in range(nseg):
        order = [int(v) for v in pre if f["segment"][v] == g]
        if g in picks:
            e, s, k = out["scores"][g]
            win = G["segments"][g]["mask"]
            pc = np.array([bin(m).count("1") for m in range(1 << k)])
            at_level = np.flatnonzero(pc >= G["segments"][g]["popcount"])
            masks = np.unique(np.concatenate([rng.choice(at_level, min(6, len(at_level)), replace=False),
                                              rng.integers(0, 1 << k, 4), [0, (1 << k) - 1, win]]))
            ref = oracle.score_masks(f, V, I, keep, g, masks.astype(np.uint32))
            np.testing.assert_allclose(e[masks], ref["e_loc"], rtol=0, atol=TOL)
            fin = np.isfinite(ref["slack_loc"])
            np.testing.assert_allclose(s[masks][fin], ref["slack_loc"][fin], rtol=0, atol=TOL)
            # the winner is feasible, everything above its level is not
            assert ref["feasible"][masks == win][0]
            above = pc[masks] > G["segments"][g]["popcount"]
            assert not np.any(ref["feasible"][above])
        for j, v in enumerate(order):
            if G["segments"][g]["mask"] >> j & 1:
                keep[v] = 0


@pytest.mark.gpu
def test_binding_surrogate_second_stage_and_fallback(okr):
    """A network that predicts every mask infeasible with top_k = 1: the first
    ranking stage finds no predicted-feasible mask, the second stage ranks
    every mask, the top-1 is the all-ones mask; where it is infeasible the
    search falls back to full enumeration.  Either way each decision is the
    exhaustive one, so the run reproduces the golden decisions."""
    import torch
    from paper_2510_19608_amd import surrogate
    _say("c2 binding bound surrogate top_k=1 constant network")
    cfg, fname = CASES[0]
    G = golden(fname)
    f = make_feeder(cfg, 0, e_bar=G["e_bar"])
    params = surrogate.init_params(0)
    params.zero_()
    params[surrogate.OFF_B3] = 10.0  # ln error 10: far above ln(e_bar)
    torch.cuda.synchronize()
    out = okr.reduce_feeder(f, want_vhat=False, surrogate=params, top_k=1)
    check_against_golden(out, G)
    ks = seg_sizes(f, len(G["segments"]))
    fallback = [s["n_scored"] > s["n_refined"] for s in out["segments"]]
    below = [d["popcount"] < k for d, k in zip(G["segments"], ks)]
    assert fallback == below
