"""CPU FP64 oracle of Algorithm 1 (Section IV): the greedy search that reduces
one node per iteration, scoring every single assignment move.

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg use this; the product path never does.

What is computed, step by step, in the order of Algorithm 1:

* State: the assignment (every node's super-node, ``sup``; a super-node is
  its own super) and the aggregated injections ``I = A I^`` (each super-node
  carries the sum of its cluster's injections).
* Candidates (the set A of Algorithm 1): every ordered pair (s, r) of
  super-nodes that are adjacent in the reduced network (an original edge
  joins their clusters; Lambda after contraction) with phi(r) a subset of
  phi(s).  Both directions of every such edge are candidates.  The slack's
  cluster is never the one that moves (its voltage is the fixed source).
* Each candidate, independently (the parallel block of Algorithm 1):
  r's cluster current moves to s (I_s += I_r, I_r = 0), the full network is
  solved with the slack held at V0 (``solve I^c = Y V^c``), every reduced
  node takes its super-node's voltage (r's cluster now has super s), the
  phase-to-phase error e = ||V^| - |V^c|| is formed, and the candidate is
  feasible when max e <= e_bar; its SMICE is the sum over clusters of the
  cluster's largest member error (MICE).
* The feasible candidate with the smallest SMICE is applied (cluster merge,
  aggregated-current update); the search stops when no candidate is
  feasible.

Readings where the paper is silent (also listed with the design notes):

* SMICE over several loading scenarios is the sum over scenarios of each
  scenario's SMICE (MICE taken per scenario over members and phases).
* Candidates are numbered by the original edge that joins the two clusters:
  edge (x, parent(x)) gives id 2x for the child-side cluster moving up and
  2x + 1 for the parent-side cluster moving down.  SMICE values within
  ``tie_tol`` of the minimum tie; the lowest id wins.
* An iteration is flagged ambiguous when a feasible candidate's SMICE lies
  within ``amb_tol`` of the tie threshold, or an active candidate's largest
  error lies within ``amb_tol`` of e_bar.

The full-network solve uses one LU factorisation of the non-slack block of Y
(Y does not change during the search; only the injections do) and one
back-substitution per candidate and scenario.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class Network:
    """Dense admittance matrix over present node-phases (Section II.A: Y_ii
    diagonal blocks, Y_{i,parent(i)} off-diagonal blocks and their
    transposes) with the slack's rows split off and the rest factorised."""

    def __init__(self, f):
        parent = np.asarray(f["parent"])
        phase = np.asarray(f["phase"])
        n = len(parent)
        self.n = n
        self.parent = parent
        self.phase = phase
        self.present = np.array([[(int(phase[i]) >> p) & 1 for p in range(3)] for i in range(n)], bool)
        idx = -np.ones((n, 3), dtype=np.int64)
        k = 0
        for i in range(n):
            for p in range(3):
                if self.present[i, p]:
                    idx[i, p] = k
                    k += 1
        self.idx = idx
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
        slack = idx[0][idx[0] >= 0]
        rest = np.setdiff1d(np.arange(k), slack)
        self.slack_cols, self.rest = slack, rest
        self.Ynn = Y[np.ix_(rest, rest)]
        self.Yn0 = Y[np.ix_(rest, slack)]
        self.lu = sla.lu_factor(self.Ynn)
        self.V0 = np.asarray(f["V0"], dtype=np.complex128)[self.present[0]]
        # flat index -> (node, phase) of the non-slack unknowns
        self.flat = np.array([(i * 3 + p) for i in range(n) for p in range(3) if self.present[i, p] and i > 0])

    def solve(self, I):
        """Voltages for injections I[..., n, 3] with the slack at V0: the
        non-slack block of Y V = I (Algorithm 1's full-network solve)."""
        lead = I.shape[:-2]
        Iflat = I.reshape(-1, self.n * 3)[:, self.flat]           # [B, m]
        rhs = Iflat.T - (self.Yn0 @ self.V0)[:, None]              # [m, B]
        Vn = sla.lu_solve(self.lu, rhs)                            # [m, B]
        V = np.zeros((Iflat.shape[0], self.n * 3), dtype=np.complex128)
        V[:, self.flat] = Vn.T
        V[:, 0:3][:, self.present[0]] = self.V0
        return V.reshape(*lead, self.n, 3)


def candidates(parent, phase, sup):
    """Candidate moves (id, s, r) in increasing id (see the module notes)."""
    out = []
    for x in range(1, len(parent)):
        a, b = int(sup[x]), int(sup[parent[x]])
        if a == b:
            continue
        for d, (r, s) in enumerate(((a, b), (b, a))):
            if r == 0:
                continue
            if int(phase[r]) & ~int(phase[s]):
                continue
            out.append((2 * x + d, s, r))
    return out


def errors(net, Vhat, V, sup):
    """e[l, x, p] = ||V^| - |V^c|| with V^c_x = V_sup(x) (reduced nodes take
    their super-node's voltage); zero on absent phases."""
    Vc = V[..., np.asarray(sup), :]
    e = np.abs(np.abs(Vhat) - np.abs(Vc))
    return np.where(net.present, e, 0.0)


def smice(e, sup, n):
    """Sum over scenarios and clusters of each cluster's largest member error
    (MICE of Algorithm 1)."""
    per_node = e.max(axis=-1)                                      # [S, n]
    mice = np.zeros((e.shape[0], n))
    for x in range(n):
        mice[:, sup[x]] = np.maximum(mice[:, sup[x]], per_node[:, x])
    return mice.sum()


def score(net, Vhat, Iagg, sup, cands, e_bar):
    """SMICE (inf when infeasible) and largest error of every candidate."""
    n = net.n
    if not cands:
        return np.zeros(0), np.zeros(0)
    Ic = np.repeat(Iagg[None], len(cands), axis=0)                 # [C, S, n, 3]
    for c, (_, s, r) in enumerate(cands):
        Ic[c, :, s] += Ic[c, :, r]
        Ic[c, :, r] = 0
    V = net.solve(Ic)
    sm = np.empty(len(cands))
    em = np.empty(len(cands))
    for c, (_, s, r) in enumerate(cands):
        sup2 = np.where(sup == r, s, sup)
        e = errors(net, Vhat, V[c], sup2)
        em[c] = e.max()
        sm[c] = smice(e, sup2, n) if em[c] <= e_bar else np.inf
    return sm, em


def select(cands, sm, em, e_bar, tie_tol, amb_tol):
    """Index of the chosen candidate (or None) and the ambiguity flag."""
    feas = np.isfinite(sm)
    amb = bool(np.any(np.abs(em - e_bar) <= amb_tol))
    if not feas.any():
        return None, amb
    m = sm[feas].min()
    thr = m + tie_tol
    pick = int(np.flatnonzero(feas & (sm <= thr))[0])  # candidates are in increasing id
    amb = amb or bool(np.any(feas & (np.abs(sm - thr) <= amb_tol)))
    return pick, amb


def greedy(f, Vhat, Ihat, e_bar=None, tie_tol=1e-11, amb_tol=1e-13, max_iter=None):
    """Run Algorithm 1.  Returns (sup, steps, err_per_snapshot): the final
    assignment, one record per applied move, and the final largest error per
    scenario."""
    net = Network(f)
    n = net.n
    e_bar = f["e_bar"] if e_bar is None else e_bar
    sup = np.arange(n)
    Iagg = np.array(Ihat, dtype=np.complex128, copy=True)
    steps = []
    while max_iter is None or len(steps) < max_iter:
        cands = candidates(net.parent, net.phase, sup)
        if not cands:
            break
        sm, em = score(net, Vhat, Iagg, sup, cands, e_bar)
        pick, amb = select(cands, sm, em, e_bar, tie_tol, amb_tol)
        if pick is None:
            break
        cid, s, r = cands[pick]
        sup = np.where(sup == r, s, sup)
        Iagg[:, s] += Iagg[:, r]
        Iagg[:, r] = 0
        steps.append(dict(cand=cid, s=s, r=r, smice=float(sm[pick]), emax=float(em[pick]), ambiguous=amb,
                          n_cand=len(cands), n_feasible=int(np.isfinite(sm).sum())))
    err = evaluate(f, Vhat, Ihat, sup, net=net)
    return sup, steps, err


def aggregate(Ihat, sup):
    """I = A I^: each super-node carries its cluster's injections."""
    Iagg = np.zeros_like(Ihat)
    for x in range(len(sup)):
        Iagg[:, sup[x]] += Ihat[:, x]
    return Iagg


def evaluate(f, Vhat, Ihat, sup, net=None):
    """Largest error per scenario of a fixed assignment (the robustness
    evaluation of Section VI: a reduction found on some scenarios, scored on
    others)."""
    net = Network(f) if net is None else net
    V = net.solve(aggregate(np.asarray(Ihat, dtype=np.complex128), np.asarray(sup)))
    e = errors(net, Vhat, V, np.asarray(sup))
    return e.reshape(e.shape[0], -1).max(axis=1)
