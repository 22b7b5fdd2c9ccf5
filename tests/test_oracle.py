"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, an independent dense NumPy implementation (numpy.linalg.pinv Kron and
dense solves), invariants of Kron reduction, and hand-derived values.
"""
import itertools

import numpy as np
import pytest

import dense_check as dc
from synth_feeders import make_feeder


def tiny(seed, n=10, seg=(3, 5), **kw):
    return make_feeder("c1", seed, n=n, n_eligible=None, seg_size=seg, **kw)


def hand_feeder(parent, phase, zs, loads, V0=None):
    """Feeder dict from explicit branch impedances zs[i] (3x3, i >= 1) and
    consumed powers loads[l][i][p]."""
    n = len(parent)
    Yo = np.zeros((n, 3, 3), complex)
    Yd = np.zeros((n, 3, 3), complex)
    for i in range(1, n):
        idx = [p for p in range(3) if phase[i] >> p & 1]
        y = np.zeros((3, 3), complex)
        y[np.ix_(idx, idx)] = np.linalg.inv(np.asarray(zs[i])[np.ix_(idx, idx)])
        Yo[i] = -y
        Yd[i] += y
        Yd[parent[i]] += y
    S = np.asarray(loads, complex)
    return dict(n=n, parent=np.asarray(parent, np.int32), phase=np.asarray(phase, np.uint8),
                segment=np.full(n, -1, np.int32), Y_diag=Yd, Y_off=Yo, S_load=S,
                V0=np.exp(-2j * np.pi / 3 * np.arange(3)) if V0 is None else np.asarray(V0, complex),
                e_bar=0.003, v_min=0.95, v_max=1.05)


# ---------------------------------------------------------------- pinv ----

def test_pinv_is_moore_penrose_on_present_phases(oracle_lib):
    rng = np.random.default_rng(0)
    for mask in range(1, 8):
        idx = [p for p in range(3) if mask >> p & 1]
        A = np.zeros((3, 3), complex)
        B = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
        B = B + B.T + 4 * np.eye(3)
        A[np.ix_(idx, idx)] = B[np.ix_(idx, idx)]
        got = oracle_lib.pinv3(A, mask)
        np.testing.assert_allclose(got, np.linalg.pinv(A), rtol=0, atol=1e-13)


# ------------------------------------------------------------ power flow --

def test_two_bus_closed_form(oracle_lib):
    """Single-phase two-bus feeder: |V2|^4 - (|V0|^2 - 2(RP+XQ))|V2|^2
    + (R^2+X^2)(P^2+Q^2) = 0, high-voltage root."""
    R, X, P, Q = 0.02, 0.05, 0.8, 0.3
    z = np.zeros((3, 3), complex)
    z[0, 0] = R + 1j * X
    f = hand_feeder([-1, 0], [7, 1], [None, z], [[[0, 0, 0], [P + 1j * Q, 0, 0]]])
    V, I, st, it = oracle_lib.powerflow(f)
    assert st == 0
    b = 1.0 - 2 * (R * P + X * Q)
    c = (R * R + X * X) * (P * P + Q * Q)
    v2sq = (b + np.sqrt(b * b - 4 * c)) / 2
    assert abs(abs(V[0, 1, 0]) - np.sqrt(v2sq)) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_power_balance_residual(oracle_lib, seed):
    """The converged library satisfies V o conj(Y V) = -S_load at every
    non-slack node-phase, with Y assembled densely from the input blocks."""
    f = make_feeder("c1", seed)
    V, I, st, it = oracle_lib.powerflow(f)
    assert st == 0
    Y = dc.dense_Y(f)
    pres = dc.present(f)
    for l in range(V.shape[0]):
        v = V[l].reshape(-1)
        sinj = v * np.conj(Y @ v)
        res = (sinj + f["S_load"][l].reshape(-1))[3:][pres[3:]]
        assert np.abs(res).max() < 1e-10
        # returned injections equal Y V^ off the slack
        np.testing.assert_allclose((Y @ v)[3:][pres[3:]], I[l].reshape(-1)[3:][pres[3:]],
                                   rtol=0, atol=1e-10)


@pytest.mark.parametrize("seed", [0, 4])
def test_powerflow_agrees_with_newton(oracle_lib, seed):
    """A second solver of the same load flow: Newton-Raphson (analytic
    Jacobian of the complex power mismatch, in rectangular coordinates) on the
    dense Y, started from the flat profile, reaches the oracle's sweep
    solution."""
    f = make_feeder("c1", seed, snapshots=2)
    V, I, st, it = oracle_lib.powerflow(f)
    assert st == 0
    Y = dc.dense_Y(f)
    pres = dc.present(f)
    unk = np.nonzero(pres & (np.arange(len(pres)) >= 3))[0]
    Yuu, Yus = Y[np.ix_(unk, unk)], Y[np.ix_(unk, [0, 1, 2])]
    for l in range(V.shape[0]):
        S = f["S_load"][l].reshape(-1)[unk]
        v = np.tile(f["V0"], f["n"])[unk].astype(complex)
        for _ in range(30):
            i_net = Yuu @ v + Yus @ f["V0"]
            F = v * np.conj(i_net) + S                     # injected = -consumed
            if np.abs(F).max() < 1e-14:
                break
            # dF = dv conj(i) + v conj(Y dv): real 2m x 2m system in (Re dv, Im dv)
            m = len(unk)
            A = np.diag(np.conj(i_net))                    # coefficient of dv
            B = np.diag(v) @ np.conj(Yuu)                  # coefficient of conj(dv)
            J = np.block([[(A + B).real, -(A - B).imag], [(A + B).imag, (A - B).real]])
            d = np.linalg.solve(J, -np.concatenate([F.real, F.imag]))
            v = v + d[:m] + 1j * d[m:]
        np.testing.assert_allclose(v, V[l].reshape(-1)[unk], rtol=0, atol=1e-11)


def test_powerflow_reports_divergence(oracle_lib):
    f = make_feeder("c1", 0)
    f = dict(f, S_load=f["S_load"] * 400.0)
    _, _, st, _ = oracle_lib.powerflow(f)
    assert st == -5


# ------------------------------------------------------- Kron reduction --

def random_keep(rng, n, p=0.5):
    keep = (rng.random(n) > p).astype(np.uint8)
    keep[0] = 1
    return keep


@pytest.mark.parametrize("seed", range(6))
def test_kron_blocks_match_dense_pinv(oracle_lib, seed):
    """Y_Kron from block elimination equals the dense Schur complement with
    numpy's pseudo-inverse; it stays symmetric and Laplacian (no shunts)."""
    f = tiny(seed, n=11)
    rng = np.random.default_rng(seed)
    elig = f["eligible"].astype(bool)
    for _ in range(4):
        keep = np.ones(f["n"], np.uint8)
        keep[elig & (rng.random(f["n"]) < 0.6)] = 0
        kp, Ykd, Yko, extra = oracle_lib.kron_blocks(f, keep)
        Yk, K = dc.dense_kron(f, keep)
        kept = [i for i in range(f["n"]) if keep[i]]
        pos = {i: j for j, i in enumerate(kept)}
        for i in kept:
            np.testing.assert_allclose(Ykd[i], Yk[3 * pos[i]:3 * pos[i] + 3, 3 * pos[i]:3 * pos[i] + 3],
                                       rtol=0, atol=1e-9 * np.abs(Yk).max())
            if i > 0:
                j = kp[i]
                np.testing.assert_allclose(Yko[i], Yk[3 * pos[i]:3 * pos[i] + 3, 3 * pos[j]:3 * pos[j] + 3],
                                           rtol=0, atol=1e-9 * np.abs(Yk).max())
        # eligible nodes have at most one child: the reduction stays radial
        assert extra == 0
        np.testing.assert_allclose(Yk, Yk.T, rtol=0, atol=1e-9 * np.abs(Yk).max())
        # Y_Kron (1 (x) v) = 0 for any phase vector v restricted to each node's phases
        v = np.array([1.0, 0.3 - 0.2j, -0.7 + 0.1j])
        pres = dc.present(f).reshape(f["n"], 3)
        vec = np.concatenate([v * pres[i] for i in kept])
        assert np.abs(Yk @ vec).max() < 1e-8 * np.abs(Yk).max()


def test_lemma2_pattern_equals_single_phase_kron(oracle_lib):
    """Lemma 2: the block pattern of three-phase Kron equals the pattern of
    the single-phase Kron reduction of the same topology, also for a node of
    degree 3 whose elimination creates a clique (Section V)."""
    parent = [-1, 0, 1, 1, 1, 2]
    phase = [7, 7, 7, 7, 7, 7]
    rng = np.random.default_rng(3)
    zs = [None]
    for i in range(1, 6):
        a = rng.uniform(0.5, 1.5, size=(3, 3)) * (0.01 + 0.03j)
        zs.append(a + a.T + np.eye(3) * (0.02 + 0.06j))
    f = hand_feeder(parent, phase, zs, np.zeros((1, 6, 3)))
    for keep in itertools.product([0, 1], repeat=5):
        keep = np.array((1,) + keep, np.uint8)
        Yk, K = dc.dense_kron(f, keep)
        # scalar Laplacian with unit weights, same topology
        L = np.zeros((6, 6))
        for i in range(1, 6):
            p = parent[i]
            L[i, i] += 1; L[p, p] += 1; L[i, p] -= 1; L[p, i] -= 1
        k = [i for i in range(6) if keep[i]]
        r = [i for i in range(6) if not keep[i]]
        Lk = L[np.ix_(k, k)] - (L[np.ix_(k, r)] @ np.linalg.pinv(L[np.ix_(r, r)]) @ L[np.ix_(r, k)] if r else 0)
        for a, b in itertools.product(range(len(k)), repeat=2):
            blk = Yk[3 * a:3 * a + 3, 3 * b:3 * b + 3]
            assert (np.abs(blk).max() > 1e-12) == (abs(Lk[a, b]) > 1e-12)


def test_series_chain_and_leaf_closed_forms(oracle_lib):
    """Eliminating the middle node of 0-a-b gives the series branch
    -(z_a + z_b)^-1; eliminating a leaf removes its branch (Section II.B)."""
    rng = np.random.default_rng(7)
    zs = [None]
    for _ in range(3):
        a = rng.uniform(0.5, 1.5, size=(3, 3)) * (0.01 + 0.03j)
        zs.append(a + a.T + np.eye(3) * (0.02 + 0.06j))
    # 0 - 1 - 2, and a leaf 3 hanging off 2; node 2 is two-phase (a, b)
    phase = [7, 7, 3, 1]
    zs[2] = zs[2] * np.outer([1, 1, 0], [1, 1, 0])
    zs[3] = zs[3] * np.outer([1, 0, 0], [1, 0, 0])
    f = hand_feeder([-1, 0, 1, 2], phase, zs, np.zeros((1, 4, 3)))
    kp, Ykd, Yko, extra = oracle_lib.kron_blocks(f, np.array([1, 0, 1, 0], np.uint8))
    zeq = (zs[1] + zs[2])[:2, :2]
    want = np.zeros((3, 3), complex)
    want[:2, :2] = -np.linalg.inv(zeq)
    assert kp[2] == 0
    np.testing.assert_allclose(Yko[2], want, rtol=1e-12, atol=1e-9)
    # after removing leaf 3 and node 1, node 2's self block is the series admittance only
    np.testing.assert_allclose(Ykd[2], -want, rtol=1e-12, atol=1e-9)


# ---------------------------------------------------- candidate voltages --

@pytest.mark.parametrize("seed", range(6))
def test_candidate_voltages_match_dense_routes(oracle_lib, seed):
    """V^c from the oracle equals (a) the dense pinv Kron route and (b) the
    full-network solve Y V^c = I^c, for random kept sets."""
    f = tiny(seed, n=11, snapshots=2, scale=(0.3, 1.0))
    V, I, st, _ = oracle_lib.powerflow(f)
    assert st == 0
    rng = np.random.default_rng(100 + seed)
    for _ in range(5):
        keep = random_keep(rng, f["n"])
        got = oracle_lib.candidate_voltages(f, I, keep)
        a = dc.vc_kron_route(f, I, keep)
        b = dc.vc_full_route(f, I, keep)
        np.testing.assert_allclose(got, a, rtol=0, atol=1e-12)
        np.testing.assert_allclose(got, b, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_zero_injection_invariant(oracle_lib, seed):
    """Kron reduction preserves kept-node voltages when the reduced nodes carry
    no injection (Section II.C): zero their loads, reduce them, compare."""
    f = tiny(seed, n=12, snapshots=3, scale=(0.3, 1.0))
    rng = np.random.default_rng(seed)
    keep = random_keep(rng, f["n"], 0.4)
    S = f["S_load"].copy()
    S[:, keep == 0, :] = 0
    f = dict(f, S_load=S)
    V, I, st, _ = oracle_lib.powerflow(f)
    assert st == 0
    Vc = oracle_lib.candidate_voltages(f, I, keep)
    np.testing.assert_allclose(Vc[:, keep == 1], V[:, keep == 1], rtol=0, atol=1e-12)


def test_hand_example_three_node_chain(oracle_lib):
    """Single-phase chain 0-a-b with fixed load currents L_a, L_b:
    reduce b -> V^c_a = V^_a, V^c_b = V^_a; reduce a -> V^c_a = V0,
    V^c_b = V0 - (z_a + z_b) L_b; reduce both -> V0 everywhere."""
    za, zb = 0.01 + 0.03j, 0.02 + 0.05j
    zs = [None] + [np.diag([z, 0, 0]) for z in (za, zb)]
    f = hand_feeder([-1, 0, 1], [7, 1, 1], zs, [[[0, 0, 0], [0.3 + 0.1j, 0, 0], [0.5 + 0.2j, 0, 0]]])
    V, I, st, _ = oracle_lib.powerflow(f)
    assert st == 0
    La, Lb = -I[0, 1, 0], -I[0, 2, 0]
    V0 = f["V0"][0]
    Va = V0 - za * (La + Lb)
    Vb = Va - zb * Lb
    assert abs(V[0, 1, 0] - Va) < 1e-12 and abs(V[0, 2, 0] - Vb) < 1e-12
    Vc = oracle_lib.candidate_voltages(f, I, np.array([1, 1, 0], np.uint8))[0, :, 0]
    assert abs(Vc[1] - Va) < 1e-12 and abs(Vc[2] - Va) < 1e-12
    Vc = oracle_lib.candidate_voltages(f, I, np.array([1, 0, 1], np.uint8))[0, :, 0]
    assert abs(Vc[1] - V0) < 1e-12 and abs(Vc[2] - (V0 - (za + zb) * Lb)) < 1e-12
    Vc = oracle_lib.candidate_voltages(f, I, np.array([1, 0, 0], np.uint8))[0, :, 0]
    assert abs(Vc[1] - V0) < 1e-12 and abs(Vc[2] - V0) < 1e-12


# --------------------------------------------------------------- search --

@pytest.mark.parametrize("secondary", ["maxerr", "smice"])
@pytest.mark.parametrize("seed,e_bar", [(0, 3e-4), (1, 1e-4), (2, 3e-4), (3, 1e-3), (4, 2e-4), (5, 3e-3)])
def test_search_matches_dense_brute_force(oracle_lib, seed, e_bar, secondary):
    """Every mask of every segment of a tiny feeder, scored with the dense
    full-network route, picks the same aggregation as the oracle, under
    either selection key."""
    f = tiny(seed, n=11, snapshots=2, scale=(0.3, 1.0), e_bar=e_bar)
    V, I, st, _ = oracle_lib.powerflow(f)
    keep_b, masks_b = dc.brute_search(f, V, I, secondary=secondary)
    for mode in (0, 1):
        keep, dec, st = oracle_lib.search(f, V, I, mode=mode, secondary=secondary)
        assert st == 0
        assert [d["mask"] for d in dec] == masks_b
        assert not any(d["ambiguous"] for d in dec)
        np.testing.assert_array_equal(keep, keep_b)


def test_masks_leave_errors_outside_omega_unchanged(oracle_lib):
    """Omega_g holds every node whose error can depend on the mask: outside it
    the candidate voltages equal those of the empty mask."""
    f = make_feeder("c1", 1, seg_size=(6, 6), n_eligible=None, snapshots=2, scale=(0.3, 1.0))
    V, I, st, _ = oracle_lib.powerflow(f)
    keep = np.ones(f["n"], np.uint8)
    rng = np.random.default_rng(0)
    nseg = int(f["segment"].max()) + 1
    for g in range(nseg):
        om = dc.omega(f, keep, g)
        nodes = dc.seg_nodes(f, g)
        base = oracle_lib.candidate_voltages(f, I, keep)
        for m in rng.integers(0, 1 << len(nodes), size=4):
            keep2 = keep.copy()
            for j, v in enumerate(nodes):
                if m >> j & 1:
                    keep2[v] = 0
            Vc = oracle_lib.candidate_voltages(f, I, keep2)
            np.testing.assert_allclose(Vc[:, ~om], base[:, ~om], rtol=0, atol=1e-13)
        # cumulative state: reduce the odd-positioned nodes of this segment
        for j, v in enumerate(nodes):
            if j % 2:
                keep[v] = 0


def test_omega_under_cumulative_state_is_what_masks_touch(oracle_lib):
    """Omega_g against a cumulative state (Algorithm 1's "assign previously
    reduced"): the oracle's region equals, node for node, the set found by
    experiment -- every node whose physical voltage (full-network solve with
    aggregated currents) or super-node changes under some single-node mask of
    the segment.  Earlier segments' reductions sit above later segments'
    chains on these deep-lateral feeders, so the region must climb through
    already-reduced nodes.  The oracle's e_loc is then the error maximum over
    exactly that set (dense route)."""
    climbs = 0
    rng = np.random.default_rng(11)
    for seed in range(8):
        f = make_feeder("c1", seed, n=24, n_eligible=None, seg_size=(2, 3), snapshots=2,
                        scale=(0.3, 1.0), p_deep=0.6)
        V, I, st, _ = oracle_lib.powerflow(f)
        assert st == 0
        keep = np.ones(f["n"], np.uint8)
        for g in range(int(f["segment"].max()) + 1):
            nodes = dc.seg_nodes(f, g)
            om = oracle_lib.omega(f, keep, g)
            ob, dmin_in, dmax_out = dc.omega_behavioural(f, I, keep, nodes)
            assert dmin_in > 1e-9 and dmax_out < 1e-13  # the experiment separates cleanly
            np.testing.assert_array_equal(om, ob)
            # a reduced node sits above a chain of this segment: the region
            # reaches above the segment's own topmost nodes
            tops = {v for v in nodes if f["segment"][f["parent"][v]] != g}
            if any(not keep[f["parent"][v]] for v in tops):
                climbs += 1
            masks = np.unique(np.concatenate([[0, (1 << len(nodes)) - 1],
                                              rng.integers(0, 1 << len(nodes), 3)])).astype(np.uint32)
            got = oracle_lib.score_masks(f, V, I, keep, g, masks)
            for q, m in enumerate(masks):
                keep2 = keep.copy()
                for j, v in enumerate(nodes):
                    if m >> j & 1:
                        keep2[v] = 0
                ref = dc.score(f, V, I, keep2, ob)
                assert abs(got["e_loc"][q] - ref["e_loc"]) < 1e-12
                assert abs(got["slack_loc"][q] - ref["slack_loc"]) < 1e-12 or \
                    (np.isinf(got["slack_loc"][q]) and np.isinf(ref["slack_loc"]))
            if (seed + g) % 3:  # cumulative state: reduce the whole segment
                for v in nodes:
                    keep[v] = 0
    assert climbs >= 10


def _dense_level_scores(f, V, I, level):
    """Dense-route (e_loc, feasible) of every mask of segment 0 at `level`,
    from the full state."""
    nodes = dc.seg_nodes(f, 0)
    keep = np.ones(f["n"], np.uint8)
    om = dc.omega(f, keep, 0)
    rows = []
    for m in range(1 << len(nodes)):
        if bin(m).count("1") != level:
            continue
        keep2 = keep.copy()
        for j, v in enumerate(nodes):
            if m >> j & 1:
                keep2[v] = 0
        sc = dc.score(f, V, I, keep2, om)
        rows.append((m, sc["e_loc"], sc["feasible"]))
    return rows


@pytest.mark.parametrize("seed", [0, 3])
def test_ambiguity_flag_at_the_e_bar_boundary(oracle_lib, seed):
    """A segment is flagged when a mask at the chosen level or above lies
    within amb_tol of the e_bar boundary: with e_bar set to the all-nodes
    mask's error (dense route) the flag is raised; 1e-12 away it is not."""
    f = make_feeder("c1", seed, n=20, n_eligible=8, seg_size=(8, 8))
    V, I, st, _ = oracle_lib.powerflow(f)
    assert st == 0
    k = len(dc.seg_nodes(f, 0))
    (m_all, e_all, _), = _dense_level_scores(f, V, I, k)
    for shift, want in ((0.0, True), (1e-12, False), (-1e-12, False)):
        keep, dec, st = oracle_lib.search(dict(f, e_bar=e_all + shift), V, I)
        assert st == 0
        assert dec[0]["ambiguous"] == want, (shift, dec[0])
    # just above the bound the all-nodes mask is feasible and wins outright
    _, dec, _ = oracle_lib.search(dict(f, e_bar=e_all + 1e-12), V, I)
    assert dec[0]["mask"] == m_all


def test_ambiguity_flag_at_the_tie_boundary(oracle_lib):
    """A segment is flagged when a feasible mask at the chosen level lies
    within amb_tol of e_min + tie_tol.  Place tie_tol on the gap between the
    two best masks of the level (dense route): flagged; 1e-12 wider: the two
    tie, the lower mask wins, no flag; 1e-12 narrower: the best one wins."""
    f = make_feeder("c1", 1, n=20, n_eligible=8, seg_size=(8, 8), e_bar=1e-4)
    V, I, st, _ = oracle_lib.powerflow(f)
    keep, dec, st = oracle_lib.search(f, V, I)
    assert st == 0 and not dec[0]["ambiguous"]
    level = dec[0]["popcount"]
    rows = sorted((e, m) for m, e, feas in _dense_level_scores(f, V, I, level) if feas)
    assert len(rows) >= 2
    (e1, m1), (e2, m2) = rows[0], rows[1]
    assert dec[0]["mask"] == m1
    gap = e2 - e1
    assert gap > 1e-11  # room for the three placements below
    _, dec, _ = oracle_lib.search(f, V, I, tie_tol=gap)
    assert dec[0]["ambiguous"]
    _, dec, _ = oracle_lib.search(f, V, I, tie_tol=gap + 1e-12)
    assert not dec[0]["ambiguous"] and dec[0]["mask"] == min(m1, m2)
    _, dec, _ = oracle_lib.search(f, V, I, tie_tol=gap - 1e-12)
    assert not dec[0]["ambiguous"] and dec[0]["mask"] == m1


def test_exact_tie_lower_mask_wins(oracle_lib):
    """Two feasible masks at the chosen level share their error (the dense
    route agrees to rounding): they tie, the lower mask is chosen, and the
    segment is not flagged (the tie is exact, far from the tie boundary)."""
    f = make_feeder("c1", 1, n=20, n_eligible=8, seg_size=(8, 8), e_bar=5e-5)
    V, I, st, _ = oracle_lib.powerflow(f)
    keep, dec, st = oracle_lib.search(f, V, I)
    assert st == 0
    level = dec[0]["popcount"]
    rows = sorted((e, m) for m, e, feas in _dense_level_scores(f, V, I, level) if feas)
    (e1, m1), (e2, m2) = rows[0], rows[1]
    assert e2 - e1 < 1e-15 and (len(rows) == 2 or rows[2][0] - e1 > 1e-9)
    assert dec[0]["mask"] == min(m1, m2) and max(m1, m2) != min(m1, m2)
    assert not dec[0]["ambiguous"]


def test_superposition_over_non_interacting_chains(oracle_lib):
    """Fixed currents make candidate voltages linear in the moved currents:
    for two segment nodes whose affected regions are disjoint, reducing both
    changes every voltage by the sum of the two single changes, and the error
    over the segment's region is the larger of the two single errors."""
    pairs = 0
    for seed in range(4):
        f = make_feeder("c1", seed, n=24, n_eligible=None, seg_size=(6, 6), snapshots=2,
                        scale=(0.3, 1.0))
        V, I, st, _ = oracle_lib.powerflow(f)
        assert st == 0
        keep = np.ones(f["n"], np.uint8)
        nodes = dc.seg_nodes(f, 0)
        regions = [dc.omega_behavioural(f, I, keep, [v])[0] for v in nodes]
        base = oracle_lib.candidate_voltages(f, I, keep)
        for a in range(len(nodes)):
            for b in range(a + 1, len(nodes)):
                if (regions[a] & regions[b]).any():
                    continue
                pairs += 1
                single = []
                for v in (nodes[a], nodes[b]):
                    k2 = keep.copy()
                    k2[v] = 0
                    single.append(oracle_lib.candidate_voltages(f, I, k2) - base)
                k2 = keep.copy()
                k2[nodes[a]] = k2[nodes[b]] = 0
                both = oracle_lib.candidate_voltages(f, I, k2) - base
                np.testing.assert_allclose(both, single[0] + single[1], rtol=0, atol=1e-13)
                sc = oracle_lib.score_masks(f, V, I, keep, 0,
                                            np.array([1 << a, 1 << b, (1 << a) | (1 << b)], np.uint32))
                assert abs(sc["e_loc"][2] - max(sc["e_loc"][0], sc["e_loc"][1])) < 1e-14
    assert pairs >= 20


def test_empty_mask_scores_the_cumulative_state(oracle_lib):
    """The empty mask changes nothing: its error is the error of the state the
    earlier segments left (dense route), about the load flow's residual for
    the first segment."""
    f = make_feeder("c1", 4, n=24, n_eligible=None, seg_size=(3, 3), snapshots=2, scale=(0.3, 1.0),
                    p_deep=0.6)
    V, I, st, _ = oracle_lib.powerflow(f)
    keep = np.ones(f["n"], np.uint8)
    for g in range(int(f["segment"].max()) + 1):
        nodes = dc.seg_nodes(f, g)
        sc = oracle_lib.score_masks(f, V, I, keep, g, np.array([0], np.uint32))
        ref = dc.score(f, V, I, keep, np.ones(f["n"], bool))
        assert abs(sc["e_glob"][0] - ref["e_glob"]) < 1e-13
        if g == 0:
            assert sc["e_glob"][0] < 1e-12
        for v in nodes[::2]:
            keep[v] = 0
    assert ref["e_glob"] > 1e-6  # the later states carry real errors


def test_base_out_of_band_warns_and_reduces_nothing(oracle_lib):
    f = make_feeder("c1", 0, v_min=0.999)
    V, I, st, _ = oracle_lib.powerflow(f)
    keep, dec, st = oracle_lib.search(f, V, I)
    assert st == oracle_lib.W_BASE_OUT_OF_BAND
    assert keep.all() and all(d["mask"] == 0 for d in dec)


def test_score_masks_agrees_with_dense_scores(oracle_lib):
    f = tiny(2, n=11, snapshots=2, scale=(0.3, 1.0), e_bar=3e-4)
    V, I, _, _ = oracle_lib.powerflow(f)
    keep = np.ones(f["n"], np.uint8)
    nodes = dc.seg_nodes(f, 0)
    masks = np.arange(1 << len(nodes))
    got = oracle_lib.score_masks(f, V, I, keep, 0, masks)
    om = dc.omega(f, keep, 0)
    for q, m in enumerate(masks):
        keep2 = keep.copy()
        for j, v in enumerate(nodes):
            if m >> j & 1:
                keep2[v] = 0
        ref = dc.score(f, V, I, keep2, om)
        for key in ("e_glob", "e_loc", "slack_glob", "slack_loc"):
            assert abs(got[key][q] - ref[key]) < 1e-12
        assert got["feasible"][q] == ref["feasible"]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_key_gap_is_the_runner_up_margin(oracle_lib, seed):
    """The search's decision margin equals the one read off the per-mask
    scores of every mask (a separate route through score_masks): the smallest
    error of a feasible mask of the chosen level outside the tie window,
    minus the smallest error of that level."""
    import oracle
    f = make_feeder("c1", seed, e_bar=3e-4)
    V, I, st, _ = oracle.powerflow(f)
    keep, dec, st = oracle.search(f, V, I)
    k = dec[0]["k"]
    ref = oracle.score_masks(f, V, I, np.ones(f["n"], np.uint8), 0, np.arange(1 << k))
    pc = np.array([bin(m).count("1") for m in range(1 << k)])
    lvl = (pc == dec[0]["popcount"]) & ref["feasible"].astype(bool)
    e = ref["e_loc"][lvl]
    emin = e.min()
    outside = e[e > emin + 1e-11]
    want = (outside.min() - emin) if outside.size else np.inf
    got = dec[0]["key_gap"]
    assert (np.isinf(want) and np.isinf(got)) or got == want
    assert got >= 0.0


# ---------------------------------------------------------------- SMICE --

def _leaf_pairs(f):
    """(leaf, parent) pairs with the parent off the slack."""
    par = f["parent"]
    nch = np.bincount(par[1:], minlength=f["n"])
    return [(int(i), int(par[i])) for i in range(1, f["n"]) if nch[i] == 0 and par[i] > 0]


def _leaf_err(V, r, s, phase_r):
    """Per snapshot: the largest over r's phases of ||V^_r| - |V^_s||, the
    error of leaf r once its load moves to s (nothing else moves: every other
    node shares its whole root path with s, so the moved current changes no
    other voltage, and s's own voltage stays V^_s)."""
    ph = [p for p in range(3) if phase_r >> p & 1]
    return np.abs(np.abs(V[:, r, ph]) - np.abs(V[:, s, ph])).max(axis=1)


def test_smice_closed_forms(oracle_lib):
    """SMICE (Algorithm 1, MICE of Section II.C) on reductions whose errors are
    fixed by the load-flow voltages alone: nothing reduced -> 0 (the full
    network reproduces V^); one leaf into its parent -> the sum over snapshots
    of the leaf's error; two sibling leaves into their common parent -> one
    cluster, the sum of their per-snapshot maximum; two leaves under different
    parents -> two clusters, the sum of both."""
    f = make_feeder("c1", 3)
    V, I, st, _ = oracle_lib.powerflow(f)
    assert st == 0
    pairs = _leaf_pairs(f)
    by_parent = {}
    for r, s in pairs:
        by_parent.setdefault(s, []).append(r)
    sib = next(v for v in by_parent.values() if len(v) >= 2)[:2]
    r1, r2 = sib
    s12 = int(f["parent"][r1])
    ra, rb = next((a, b) for (a, sa) in pairs for (b, sb) in pairs if sa != sb and a < b)
    keep = np.ones(f["n"], np.uint8)

    def smice_of(nodes, masks):
        seg = np.full(f["n"], -1, np.int32)
        seg[sorted(nodes)] = 0
        return oracle_lib.score_masks(dict(f, segment=seg), V, I, keep, 0, np.asarray(masks, np.uint32))["smice"]

    e1 = _leaf_err(V, r1, s12, f["phase"][r1])
    e2 = _leaf_err(V, r2, s12, f["phase"][r2])
    lo, hi = sorted((r1, r2))   # bit j = j-th segment node in DFS preorder (children in index order)
    sm = smice_of([r1, r2], [0, 1, 2, 3])
    assert abs(sm[0]) < 1e-12
    elo, ehi = (e1, e2) if lo == r1 else (e2, e1)
    np.testing.assert_allclose(sm[1:], [elo.sum(), ehi.sum(), np.maximum(e1, e2).sum()], rtol=1e-9, atol=1e-13)
    assert np.maximum(e1, e2).sum() < e1.sum() + e2.sum() - 1e-9   # one cluster, not two
    ea = _leaf_err(V, ra, int(f["parent"][ra]), f["phase"][ra])
    eb = _leaf_err(V, rb, int(f["parent"][rb]), f["phase"][rb])
    sm = smice_of([ra, rb], [3])
    np.testing.assert_allclose(sm, [ea.sum() + eb.sum()], rtol=1e-9, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_smice_scores_and_rise_match_dense(oracle_lib, seed):
    """Per-mask SMICE of the oracle equals the dense full-network route's on
    every mask of the first segment of a tiny feeder, and each decision's
    SMICE rise is the chosen mask's SMICE minus mask 0's at that state."""
    f = tiny(seed, n=11, snapshots=2, scale=(0.3, 1.0), e_bar=3e-4)
    V, I, st, _ = oracle_lib.powerflow(f)
    keep = np.ones(f["n"], np.uint8)
    k = int((f["segment"] == 0).sum())
    nodes = dc.seg_nodes(f, 0)
    om = dc.omega(f, keep, 0)
    got = oracle_lib.score_masks(f, V, I, keep, 0, np.arange(1 << k))["smice"]
    for m in range(1 << k):
        keep2 = keep.copy()
        for j in range(k):
            if m >> j & 1:
                keep2[nodes[j]] = 0
        assert abs(got[m] - dc.score(f, V, I, keep2, om)["smice"]) < 1e-12
    keep_s, dec, st = oracle_lib.search(f, V, I, secondary="smice")
    state = np.ones(f["n"], np.uint8)
    for d in dec:
        sc = oracle_lib.score_masks(f, V, I, state, d["segment"], np.array([0, d["mask"]], np.uint32))
        assert abs(d["smice_rise"] - (sc["smice"][1] - sc["smice"][0])) < 1e-12
        for j, v in enumerate(dc.seg_nodes(f, d["segment"])):
            if d["mask"] >> j & 1:
                state[v] = 0


def test_smice_key_changes_decisions(oracle_lib):
    """The two keys differ somewhere: on the 30-bus feeders at a bound that
    binds, some segment's SMICE choice is not its smallest-maximum-error
    choice, and it never has a larger SMICE nor a smaller maximum error."""
    differ = 0
    for seed in range(8):
        f = make_feeder("c1", seed, e_bar=3e-4)
        V, I, st, _ = oracle_lib.powerflow(f)
        _, dm, _ = oracle_lib.search(f, V, I)
        _, ds, _ = oracle_lib.search(f, V, I, secondary="smice")
        if dm[0]["mask"] != ds[0]["mask"] and dm[0]["popcount"] == ds[0]["popcount"]:
            differ += 1
            keep = np.ones(f["n"], np.uint8)
            sc = oracle_lib.score_masks(f, V, I, keep, 0, np.array([dm[0]["mask"], ds[0]["mask"]], np.uint32))
            assert sc["smice"][1] <= sc["smice"][0] + 1e-9
            assert sc["e_loc"][0] <= sc["e_loc"][1] + 1e-11
    assert differ >= 2


# ------------------------------------------------- one-call reduction --

@pytest.mark.parametrize("secondary", ["maxerr", "smice"])
def test_one_call_reduction_composes_the_pinned_steps(oracle_lib, secondary):
    """okr_oracle_reduce_feeder equals its steps called one by one (load
    flow, search, final errors, Kron blocks), and with the scenario voltages
    given instead of the load flow it reaches the same reduction."""
    f = make_feeder("c1", 2, n=40, n_eligible=None, seg_size=(4, 7), snapshots=3, scale=(0.3, 1.0), e_bar=3e-4)
    out = oracle_lib.reduce_feeder(f, secondary=secondary)
    V, I, st, _ = oracle_lib.powerflow(f)
    keep, dec, st = oracle_lib.search(f, V, I, secondary=secondary)
    assert out["status"] == st == 0
    assert [s["mask"] for s in out["segments"]] == [d["mask"] for d in dec]
    assert [s["smice_rise"] for s in out["segments"]] == [d["smice_rise"] for d in dec]
    np.testing.assert_array_equal(out["kept"], keep)
    np.testing.assert_array_equal(out["super"], dc.super_of(f["parent"], keep))
    err, _ = oracle_lib.final_errors(f, V, I, keep)
    np.testing.assert_array_equal(out["err_per_snapshot"], err)
    assert out["max_err"] == err.max() and out["n_kept"] == int(keep.sum())
    kp, Ykd, Yko, _ = oracle_lib.kron_blocks(f, keep)
    np.testing.assert_array_equal(out["kept_parent"], kp)
    np.testing.assert_array_equal(out["Yk_diag"], Ykd)
    np.testing.assert_array_equal(out["Vhat"], V)
    given = oracle_lib.reduce_feeder(f, vhat=V, secondary=secondary)
    assert [s["mask"] for s in given["segments"]] == [d["mask"] for d in dec]
    np.testing.assert_allclose(given["err_per_snapshot"], err, rtol=0, atol=1e-13)
