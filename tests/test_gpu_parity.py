"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Decisions (chosen masks) must match bit for bit; per-mask errors, band
slacks, scenario voltages, Y_Kron blocks and final errors within 1e-9 p.u.
"""
import sys

import numpy as np
import pytest

import oracle
from synth_feeders import dfs_preorder, make_feeder

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


def oracle_run(f):
    V, I, st, _ = oracle.powerflow(f)
    assert st == 0
    keep, dec, st = oracle.search(f, V, I)
    return V, I, keep, dec, st


def check_outputs(f, out, V, I, keep, dec, exact_gap=True):
    got = [s["mask"] for s in out["segments"]]
    want = [d["mask"] for d in dec]
    amb = [d["ambiguous"] for d in dec]
    assert not any(amb), "oracle flags a near-tie; pick another seed"
    assert got == want
    assert [bool(s["ambiguous"]) for s in out["segments"]] == amb
    np.testing.assert_array_equal(out["kept"], keep)
    # scenario voltages
    np.testing.assert_allclose(out["Vhat"], V, rtol=0, atol=1e-12)
    # final per-snapshot error over every node
    err, _ = oracle.final_errors(f, V, I, keep)
    np.testing.assert_allclose(out["err_per_snapshot"], err, rtol=0, atol=TOL)
    # Y_Kron blocks of the final reduced network
    kp, Ykd, Yko, extra = oracle.kron_blocks(f, keep)
    assert extra == 0
    np.testing.assert_array_equal(out["kept_parent"], kp)
    scale = np.abs(Ykd).max()
    np.testing.assert_allclose(out["Yk_diag"], Ykd, rtol=0, atol=1e-9 * scale)
    np.testing.assert_allclose(out["Yk_off"], Yko, rtol=0, atol=1e-9 * scale)
    # chosen masks' errors and the decisions' margins
    for s, d in zip(out["segments"], dec):
        assert abs(s["e_loc"] - d["e_loc"]) < TOL
        if exact_gap:
            assert (np.isinf(s["key_gap"]) and np.isinf(d["key_gap"])) or abs(s["key_gap"] - d["key_gap"]) < TOL
        else:  # over the FP64-rescored masks only: at least the exact margin
            assert s["key_gap"] >= d["key_gap"] - TOL


@pytest.mark.parametrize("seed,e_bar", [(s, e) for s in range(6) for e in (3e-3, 3e-4, 1e-4)])
def test_c1_decisions_and_outputs(okr, seed, e_bar):
    _say(f"c1 seed={seed} e_bar={e_bar}")
    f = make_feeder("c1", seed, e_bar=e_bar)
    V, I, keep, dec, st = oracle_run(f)
    out = okr.reduce_feeder(f)
    check_outputs(f, out, V, I, keep, dec)


def _level_errors(f, V, I, level):
    nodes = [int(v) for v in dfs_preorder(f["parent"]) if f["segment"][v] == 0]
    masks = np.array([m for m in range(1 << len(nodes)) if bin(m).count("1") == level], np.uint32)
    sc = oracle.score_masks(f, V, I, np.ones(f["n"], np.uint8), 0, masks)
    return masks, sc


@pytest.mark.parametrize("precision", ["fp64", "factored", "mixed"])
def test_ambiguity_flags_match_the_oracle(okr, precision):
    """Decisions placed on a boundary on purpose: e_bar on the all-nodes
    mask's error, and tie_tol on the gap between the two best masks of the
    chosen level.  Both sides flag the segment (and agree 1e-12 away from
    the boundary, where neither flags and the decisions are equal)."""
    cases = []
    f = make_feeder("c1", 0, n=20, n_eligible=8, seg_size=(8, 8))
    V, I, _, _ = oracle.powerflow(f)
    masks, sc = _level_errors(f, V, I, 8)
    e_all = float(sc["e_loc"][0])
    for shift in (0.0, 1e-12):
        cases.append((dict(f, e_bar=e_all + shift), {}))
    f = make_feeder("c1", 1, n=20, n_eligible=8, seg_size=(8, 8), e_bar=1e-4)
    V, I, _, _ = oracle.powerflow(f)
    _, dec, _ = oracle.search(f, V, I)
    masks, sc = _level_errors(f, V, I, dec[0]["popcount"])
    e = np.sort(sc["e_loc"][sc["feasible"]])
    for shift in (0.0, 1e-12, -1e-12):
        cases.append((f, dict(tie_tol=float(e[1] - e[0]) + shift)))
    flags = []
    for fc, kw in cases:
        _say(f"ambiguity case {kw} e_bar={fc['e_bar']} {precision}")
        V, I, _, _ = oracle.powerflow(fc)
        keep, dec, st = oracle.search(fc, V, I, **kw)
        out = okr.reduce_feeder(fc, precision=precision, **kw)
        assert bool(out["segments"][0]["ambiguous"]) == dec[0]["ambiguous"]
        if not dec[0]["ambiguous"]:
            assert out["segments"][0]["mask"] == dec[0]["mask"]
        flags.append(dec[0]["ambiguous"])
    assert flags == [True, False, True, False, False]


@pytest.mark.parametrize("seed", [0, 3])
def test_c1_every_mask_matches_oracle(okr, seed):
    """All 4,096 candidates of the 30-bus case: per-mask error and band slack
    over the affected nodes, element by element."""
    _say(f"c1 all masks seed={seed}")
    f = make_feeder("c1", seed, e_bar=3e-4)
    out = okr.reduce_feeder(f, dump=True)
    V, I, _, _ = oracle.powerflow(f)
    keep = np.ones(f["n"], np.uint8)
    e, s, k = out["scores"][0]
    ref = oracle.score_masks(f, V, I, keep, 0, np.arange(1 << k))
    np.testing.assert_allclose(e, ref["e_loc"], rtol=0, atol=TOL)
    fin = np.isfinite(ref["slack_loc"])
    np.testing.assert_allclose(s[fin], ref["slack_loc"][fin], rtol=0, atol=TOL)
    assert (s[~fin] > 1e300).all()


@pytest.mark.parametrize("seed,e_bar,band", [(1, 3e-4, None), (2, 1e-4, None), (4, 3e-3, 2e-4),
                                             (5, 2e-4, None), (6, 3e-4, 5e-4), (7, 3e-3, 5e-5)])
def test_multisegment_cumulative_state(okr, seed, e_bar, band):
    """Small feeders split into several segments: each segment is scored
    against the state the earlier decisions left; every mask of every segment
    is compared with the oracle at that state.  With `band`, v_min sits that
    far below the lowest full-network voltage so the band binds."""
    _say(f"multiseg seed={seed} e_bar={e_bar} band={band}")
    f = make_feeder("c1", seed, n=40, n_eligible=None, seg_size=(4, 7), snapshots=3,
                    scale=(0.3, 1.0), e_bar=e_bar)
    if band is not None:
        V, _, _, _ = oracle.powerflow(f)
        pres = np.array([[(int(m) >> p) & 1 for p in range(3)] for m in f["phase"]], bool)
        f = dict(f, v_min=float(np.abs(V)[:, pres].min()) - band)
    V, I, keep_final, dec, st = oracle_run(f)
    if st == oracle.W_BASE_OUT_OF_BAND:
        pytest.skip("base network outside the band for this seed")
    out = okr.reduce_feeder(f, dump=True)
    check_outputs(f, out, V, I, keep_final, dec)
    keep = np.ones(f["n"], np.uint8)
    for g, d in enumerate(dec):
        e, s, k = out["scores"][g]
        ref = oracle.score_masks(f, V, I, keep, g, np.arange(1 << k))
        np.testing.assert_allclose(e, ref["e_loc"], rtol=0, atol=TOL)
        fin = np.isfinite(ref["slack_loc"])
        np.testing.assert_allclose(s[fin], ref["slack_loc"][fin], rtol=0, atol=TOL)
        nodes = [int(v) for v in np.nonzero(f["segment"] == g)[0]]
        from synth_feeders import dfs_preorder
        order = [int(v) for v in dfs_preorder(f["parent"]) if f["segment"][v] == g]
        for j, v in enumerate(order):
            if d["mask"] >> j & 1:
                keep[v] = 0


@pytest.mark.parametrize("seed,e_bar", [(0, 3e-3), (1, 3e-3), (0, 3e-4)])
def test_c2_full_size(okr, seed, e_bar):
    """1000-node, 24-snapshot workload in the benchmark's launch configuration:
    every decision, final outputs, and sampled masks of sampled segments."""
    _say(f"c2 seed={seed} e_bar={e_bar}")
    f = make_feeder("c2", seed, e_bar=e_bar)
    V, I, keep_final, dec, st = oracle_run(f)
    out = okr.reduce_feeder(f, dump=True)
    check_outputs(f, out, V, I, keep_final, dec)
    rng = np.random.default_rng(seed)
    keep = np.ones(f["n"], np.uint8)
    from synth_feeders import dfs_preorder
    pre = dfs_preorder(f["parent"])
    for g, d in enumerate(dec):
        if g % 11 == 0 or g == len(dec) - 1:
            e, s, k = out["scores"][g]
            masks = np.unique(np.concatenate([[0, (1 << k) - 1], rng.integers(0, 1 << k, size=24)]))
            ref = oracle.score_masks(f, V, I, keep, g, masks)
            np.testing.assert_allclose(e[masks], ref["e_loc"], rtol=0, atol=TOL)
            fin = np.isfinite(ref["slack_loc"])
            np.testing.assert_allclose(s[masks][fin], ref["slack_loc"][fin], rtol=0, atol=TOL)
        order = [int(v) for v in pre if f["segment"][v] == g]
        for j, v in enumerate(order):
            if d["mask"] >> j & 1:
                keep[v] = 0


def test_base_out_of_band_warns(okr):
    f = make_feeder("c1", 0, v_min=0.999)
    out = okr.reduce_feeder(f)
    assert out["status"] == okr.OKR.W_BASE_OUT_OF_BAND
    assert out["n_kept"] == f["n"] and all(s["mask"] == 0 for s in out["segments"])


def test_vhat_given_matches_powerflow_run(okr):
    f = make_feeder("c1", 2, e_bar=3e-4)
    V, I, _, _ = oracle.powerflow(f)
    a = okr.reduce_feeder(f)
    b = okr.reduce_feeder(f, vhat=a["Vhat"])
    assert [s["mask"] for s in a["segments"]] == [s["mask"] for s in b["segments"]]
    np.testing.assert_allclose(a["err_per_snapshot"], b["err_per_snapshot"], rtol=0, atol=1e-15)


def test_input_errors_are_reported(okr):
    f = make_feeder("c1", 1)
    g = dict(f, Y_off=f["Y_off"].copy())
    g["Y_off"][1, 0, 1] += 1e-3  # asymmetric block (node 1 is three-phase)
    with pytest.raises(okr.OkrError) as ei:
        okr.reduce_feeder(g)
    assert ei.value.code == okr.OKR.E_UNSUPPORTED
    g = dict(f, Y_diag=f["Y_diag"].copy())
    pres = np.array([(int(f["phase"][3]) >> p) & 1 for p in range(3)], float)
    g["Y_diag"][3] += np.diag(pres) * 0.5  # a shunt on the present phases
    with pytest.raises(okr.OkrError) as ei:
        okr.reduce_feeder(g)
    assert ei.value.code == okr.OKR.E_UNSUPPORTED
    g = dict(f, S_load=f["S_load"] * 400.0)  # load flow diverges
    with pytest.raises(okr.OkrError) as ei:
        okr.reduce_feeder(g)
    assert ei.value.code == okr.OKR.E_PF_DIVERGED


def test_scoring_sqrt_is_correctly_rounded(okr):
    """The scoring kernel's square root (rsq seed + Newton-Raphson) against
    libm on |V|^2-range arguments and a wide range: at most 1 ulp, exact for
    nearly all."""
    import ctypes
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(0.5, 1.5, 500_000), np.exp(rng.uniform(-40, 40, 100_000))])
    dx = torch.from_numpy(x).cuda()
    dy = torch.empty_like(dx)
    L = okr.lib()
    L.okr_selftest_sqrt.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    assert L.okr_selftest_sqrt(dx.data_ptr(), dy.data_ptr(), len(x), None) == 0
    torch.cuda.synchronize()
    y = dy.cpu().numpy()
    ref = np.sqrt(x)
    ulp = np.abs(y - ref) / np.spacing(ref)
    assert ulp.max() <= 1.0
    assert (ulp == 0).mean() > 0.999


def test_graph_replay_matches_stream_run(okr):
    """The whole search captured as one hipGraph and replayed gives the same
    decisions and outputs as the plain stream launch, on every replay, with
    other GPU work and host synchronisations between replays."""
    import torch
    f = make_feeder("c2", 1, e_bar=3e-4)
    ref = okr.reduce_feeder(f)
    R = okr.Reducer(f, graph=True)
    try:
        for rep in range(3):
            R.run(replan=False)
            torch.cuda.synchronize()
            out = R.result()
            assert [s["mask"] for s in out["segments"]] == [s["mask"] for s in ref["segments"]]
            np.testing.assert_array_equal(out["super"], ref["super"])
            np.testing.assert_array_equal(out["err_per_snapshot"], ref["err_per_snapshot"])
            np.testing.assert_array_equal(out["Yk_diag"], ref["Yk_diag"])
            x = torch.randn(1 << 20, device="cuda")
            (x * 2).sum().item()
    finally:
        R.close()


MIXED_DELTA = 1e-8


@pytest.mark.parametrize("name,seed,e_bar,band", [("c1", 0, 3e-4, None), ("c1", 3, 1e-4, None),
                                                  ("c1", 5, 3e-3, None), ("ms", 1, 3e-4, None),
                                                  ("ms", 4, 3e-3, 2e-4), ("ms", 6, 3e-4, 5e-4),
                                                  ("c2", 0, 3e-3, None), ("c2", 0, 3e-4, None)])
def test_mixed_precision_decisions_equal_fp64(okr, name, seed, e_bar, band):
    """FP32 screening + FP64 refinement of the shortlist: identical decisions
    and outputs to the FP64 path and the oracle; the FP32 error stays within
    the shortlist bound."""
    _say(f"mixed {name} seed={seed} e_bar={e_bar} band={band}")
    if name == "ms":
        f = make_feeder("c1", seed, n=40, n_eligible=None, seg_size=(4, 7), snapshots=3,
                        scale=(0.3, 1.0), e_bar=e_bar)
    else:
        f = make_feeder(name, seed, e_bar=e_bar)
    if band is not None:
        V, _, _, _ = oracle.powerflow(f)
        pres = np.array([[(int(m) >> p) & 1 for p in range(3)] for m in f["phase"]], bool)
        f = dict(f, v_min=float(np.abs(V)[:, pres].min()) - band)
    V, I, keep, dec, st = oracle_run(f)
    a = okr.reduce_feeder(f, precision="fp64")
    b = okr.reduce_feeder(f, precision="mixed")
    check_outputs(f, b, V, I, keep, dec, exact_gap=False)
    assert [s["mask"] for s in a["segments"]] == [s["mask"] for s in b["segments"]]
    for sa, sb in zip(a["segments"], b["segments"]):
        assert sa["e_loc"] == sb["e_loc"]  # the decision's error is the FP64 value
        assert sb["fp32_dev"] <= MIXED_DELTA
    np.testing.assert_array_equal(a["Yk_diag"], b["Yk_diag"])
    np.testing.assert_array_equal(a["err_per_snapshot"], b["err_per_snapshot"])


@pytest.mark.parametrize("name,seed,e_bar", [("c1", 2, 3e-4), ("c2", 1, 3e-3)])
def test_fp32_screening_error_bound(okr, name, seed, e_bar):
    """Every mask's FP32 difference-form error and band slack against the FP64
    kernel's, for masks with e64 <= 2 e_bar: within the shortlist bound."""
    f = make_feeder(name, seed, e_bar=e_bar)
    a = okr.reduce_feeder(f, precision="fp64", dump=True)
    b = okr.reduce_feeder(f, precision="mixed", dump=True)
    worst_e = worst_s = 0.0
    for g in range(len(a["segments"])):
        e64, s64, _ = a["scores"][g]
        e32, s32, _ = b["scores"][g]
        sel = e64 <= 2 * e_bar
        worst_e = max(worst_e, np.abs(e32[sel] - e64[sel]).max(initial=0.0))
        fin = sel & np.isfinite(s64)
        worst_s = max(worst_s, np.abs(s32[fin] - s64[fin]).max(initial=0.0))
    _say(f"fp32 screening worst |de| = {worst_e:.3e}, |dslack| = {worst_s:.3e}")
    assert worst_e <= MIXED_DELTA and worst_s <= MIXED_DELTA


def test_autotuned_launch_shape_gives_identical_results(okr):
    """Tuning the scoring launch (snapshot groups per segment size) changes
    only the schedule: decisions, per-segment errors and outputs are the same
    as with the default shape, on the tuning call and after it."""
    import torch
    _say("autotune c2 seed 2")
    f = make_feeder("c2", 2, e_bar=3e-4)
    ref = okr.reduce_feeder(f, want_vhat=False)
    R = okr.Reducer(f)
    try:
        for autotune in (True, False, False):
            R.run(replan=False, autotune=autotune)
            torch.cuda.synchronize()
            out = R.result()
            assert [s["mask"] for s in out["segments"]] == [s["mask"] for s in ref["segments"]]
            assert [s["e_loc"] for s in out["segments"]] == [s["e_loc"] for s in ref["segments"]]
            np.testing.assert_array_equal(out["err_per_snapshot"], ref["err_per_snapshot"])
            np.testing.assert_array_equal(out["Yk_diag"], ref["Yk_diag"])
    finally:
        R.close()


@pytest.mark.parametrize("cfg,lanes,precision,graph", [("c2", 4, "fp64", False), ("c3", 8, "fp64", True),
                                                       ("c3", 8, "mixed", False), ("c2", 8, "mixed", True)])
def test_concurrent_lanes_give_identical_results(okr, cfg, lanes, precision, graph):
    """Independent segments searched together (chunks of up to `lanes`
    segments per launch, level by level) give bit-identical decisions,
    per-segment errors and outputs to one segment per launch, in stream
    launches and in the captured graph."""
    _say(f"lanes {cfg} seed 3 lanes={lanes} {precision} graph={graph}")
    f = make_feeder(cfg, 3)
    ref = okr.reduce_feeder(f, lanes=1, precision=precision, want_vhat=False)
    out = okr.reduce_feeder(f, lanes=lanes, precision=precision, graph=graph, want_vhat=False)
    assert [s["mask"] for s in out["segments"]] == [s["mask"] for s in ref["segments"]]
    assert [s["e_loc"] for s in out["segments"]] == [s["e_loc"] for s in ref["segments"]]
    np.testing.assert_array_equal(out["err_per_snapshot"], ref["err_per_snapshot"])
    np.testing.assert_array_equal(out["Yk_diag"], ref["Yk_diag"])
    np.testing.assert_array_equal(out["kept"], ref["kept"])


def _method_flops_brute(f, keep, g, S):
    """Per-candidate work of segment g by brute force over its masks: 2|phi|
    per reduced node and hop to its super-node, 8|phi|^2 + 2|phi| per edge
    carrying a moved current, 2|phi| per segment node, 10 per node-phase of
    the affected region, 18 per reduced node per candidate."""
    parent, phase, seg = f["parent"], f["phase"], f["segment"]
    ph = lambda v: bin(int(phase[v])).count("1")
    nodes = [int(v) for v in dfs_preorder(parent) if seg[v] == g]
    k = len(nodes)
    tops = []
    for e in nodes:
        c = e
        while parent[c] >= 0 and (seg[parent[c]] == g or not keep[parent[c]]):
            c = int(parent[c])
        tops.append(c)
    order = dfs_preorder(parent)
    pos = {int(v): i for i, v in enumerate(order)}
    size = np.ones(len(parent), int)
    for v in order[::-1]:
        if parent[v] >= 0:
            size[parent[v]] += size[v]
    omega = set()
    for t in tops:
        omega.update(int(u) for u in order[pos[t]:pos[t] + size[t]])
    const = 10 * sum(ph(u) for u in omega) + 2 * sum(ph(e) for e in nodes)
    tot = 0.0
    for m in range(1 << k):
        red = {nodes[j] for j in range(k) if m >> j & 1}
        carry, hop = set(), 0.0
        for r in red:
            c, h = r, 0
            while True:
                carry.add(c)
                h += 1
                p = int(parent[c])
                if p < 0 or (p not in red and keep[p] and seg[p] != g) or (seg[p] == g and p not in red):
                    break
                c = p
            hop += 2 * ph(r) * h
        tot += (hop + sum(8 * ph(c) ** 2 + 2 * ph(c) for c in carry) + const) * S + 18 * len(red)
    return tot


def test_algorithmic_flop_count():
    """The library's per-segment algorithmic flop count (exact mask averages,
    chain by chain) equals a brute force over every mask of every segment."""
    import paper_2510_19608_amd as okr
    f = make_feeder("c1", 5, n=40, n_eligible=None, seg_size=(3, 7), snapshots=2)
    out = okr.reduce_feeder(f, want_vhat=False, timing=True)
    keep = np.ones(f["n"], bool)
    for g, s in enumerate(out["segments"]):
        want = _method_flops_brute(f, keep, g, 2)
        assert abs(s["flops"] - want) <= 1e-9 * want, (g, s["flops"], want)
        nodes = [int(v) for v in dfs_preorder(f["parent"]) if f["segment"][v] == g]
        for j, v in enumerate(nodes):
            if s["mask"] >> j & 1:
                keep[v] = False


@pytest.mark.parametrize("seed", [0, 3])
def test_mixed_reruns_fp64_past_its_bound(okr, seed):
    """With the assumed FP32 bound set below the measured deviation, every
    segment whose shortlist shows a larger deviation is scored again in FP64
    over every mask; the decisions stay the FP64 path's and the oracle's."""
    _say(f"mixed with a 1e-15 bound, ms seed={seed}")
    f = make_feeder("c1", seed, n=40, n_eligible=None, seg_size=(4, 7), snapshots=3, scale=(0.3, 1.0), e_bar=2e-4)
    V, I, keep, dec, st = oracle_run(f)
    b = okr.reduce_feeder(f, precision="mixed", mixed_delta=1e-15)
    check_outputs(f, b, V, I, keep, dec, exact_gap=False)
    rerun = [s for s in b["segments"] if s["fp32_dev"] > 1e-15]
    assert rerun, "no segment exceeded the bound"
    for s in rerun:
        assert s["n_refined"] >= (1 << s["k"])
        want = next(d["key_gap"] for d in dec if d["segment"] == s["segment"])  # exact again after the re-run
        assert (np.isinf(want) and np.isinf(s["key_gap"])) or abs(s["key_gap"] - want) < TOL


@pytest.mark.parametrize("secondary", ["maxerr", "smice"])
def test_whole_call_against_the_oracle_entry(okr, secondary):
    """The library's reduce_feeder against the oracle's one-call reduction
    (okr_oracle_reduce_feeder) on a feeder of several segments: the same
    result fields, element by element."""
    _say(f"whole call vs oracle entry, {secondary}")
    f = make_feeder("c1", 2, n=40, n_eligible=None, seg_size=(4, 7), snapshots=3, scale=(0.3, 1.0), e_bar=3e-4)
    ref = oracle.reduce_feeder(f, secondary=secondary)
    out = okr.reduce_feeder(f, secondary=secondary)
    assert not any(s["ambiguous"] for s in ref["segments"])
    for key in ("mask", "popcount", "ambiguous", "k"):
        assert [s[key] for s in out["segments"]] == [s[key] for s in ref["segments"]]
    for a, b in zip(out["segments"], ref["segments"]):
        assert abs(a["e_loc"] - b["e_loc"]) < TOL and abs(a["e_min"] - b["e_min"]) < TOL
        if secondary == "smice":
            assert abs(a["smice_rise"] - b["smice_rise"]) < 1e-10
    np.testing.assert_array_equal(out["super"], ref["super"])
    np.testing.assert_array_equal(out["kept_parent"], ref["kept_parent"])
    assert out["n_kept"] == ref["n_kept"]
    np.testing.assert_allclose(out["err_per_snapshot"], ref["err_per_snapshot"], rtol=0, atol=TOL)
    np.testing.assert_allclose(out["Vhat"], ref["Vhat"], rtol=0, atol=1e-12)
    scale = np.abs(ref["Yk_diag"]).max()
    np.testing.assert_allclose(out["Yk_diag"], ref["Yk_diag"], rtol=0, atol=1e-9 * scale)
    np.testing.assert_allclose(out["Yk_off"], ref["Yk_off"], rtol=0, atol=1e-9 * scale)
