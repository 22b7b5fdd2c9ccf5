"""Dense NumPy brute-force checker used to pin the oracle on tiny feeders.

Independent of the oracle's C code: it assembles the full 3n x 3n nodal
admittance matrix (Section II.A), forms Y_Kron with numpy's Moore-Penrose
pseudo-inverse on the whole Y_RR block (eq. Y_kron, with the absent-phase
zero rows and columns left in, as the paper's footnote describes), and solves
with numpy's dense solver.  A second route solves the full network
Y V^c = I^c directly (Algorithm 1's solve step).
"""
import numpy as np


def present(f):
    ph = np.asarray(f["phase"])
    return np.array([[(int(m) >> p) & 1 for p in range(3)] for m in ph], dtype=bool).reshape(-1)


def dense_Y(f):
    n = f["n"]
    Y = np.zeros((3 * n, 3 * n), dtype=np.complex128)
    for i in range(n):
        Y[3 * i:3 * i + 3, 3 * i:3 * i + 3] = f["Y_diag"][i]
    for i in range(1, n):
        p = int(f["parent"][i])
        Y[3 * i:3 * i + 3, 3 * p:3 * p + 3] = f["Y_off"][i]
        Y[3 * p:3 * p + 3, 3 * i:3 * i + 3] = f["Y_off"][i].T
    return Y


def super_of(parent, keep):
    n = len(parent)
    sup = np.arange(n)
    for i in range(n):
        v = i
        while not keep[v]:
            v = int(parent[v])
        sup[i] = v
    return sup


def dense_kron(f, keep):
    """Y_Kron over all 3 phases of the kept nodes (absent phases as zero rows)."""
    Y = dense_Y(f)
    n = f["n"]
    K = np.concatenate([np.arange(3 * i, 3 * i + 3) for i in range(n) if keep[i]])
    R = [np.arange(3 * i, 3 * i + 3) for i in range(n) if not keep[i]]
    if not R:
        return Y[np.ix_(K, K)], K
    R = np.concatenate(R)
    Yk = Y[np.ix_(K, K)] - Y[np.ix_(K, R)] @ np.linalg.pinv(Y[np.ix_(R, R)]) @ Y[np.ix_(R, K)]
    return Yk, K


def aggregate(f, Ihat, keep):
    sup = super_of(f["parent"], keep)
    Iagg = np.zeros_like(Ihat)
    for i in range(f["n"]):
        Iagg[:, sup[i]] += Ihat[:, i]
    return Iagg, sup


def vc_kron_route(f, Ihat, keep):
    """V^c via Y_Kron V_K = I^c_K with the slack fixed (eq. Ik-YkVk)."""
    n = f["n"]
    pres = present(f)
    Iagg, sup = aggregate(f, Ihat, keep)
    Yk, K = dense_kron(f, keep)
    pos = {int(q): j for j, q in enumerate(K)}
    unk = [pos[q] for q in K if q >= 3 and pres[q]]
    slack = [pos[q] for q in range(3)]
    S = Ihat.shape[0]
    Vc = np.zeros((S, n, 3), dtype=np.complex128)
    for l in range(S):
        Ivec = Iagg[l].reshape(-1)[K]
        rhs = Ivec[unk] - Yk[np.ix_(unk, slack)] @ f["V0"]
        Vu = np.linalg.solve(Yk[np.ix_(unk, unk)], rhs)
        VK = np.zeros(3 * n, dtype=np.complex128)
        VK[:3] = f["V0"]
        for j, u in enumerate(unk):
            VK[K[u]] = Vu[j]
        VK = VK.reshape(n, 3)
        for i in range(n):
            Vc[l, i] = VK[sup[i]] * pres.reshape(n, 3)[i]
    return Vc


def vc_full_route(f, Ihat, keep):
    """V^c via the full network Y V = I^c (Algorithm 1 solve step), then the
    voltage copy from each super-node."""
    n = f["n"]
    pres = present(f)
    Y = dense_Y(f)
    Iagg, sup = aggregate(f, Ihat, keep)
    unk = [q for q in range(3, 3 * n) if pres[q]]
    S = Ihat.shape[0]
    Vc = np.zeros((S, n, 3), dtype=np.complex128)
    for l in range(S):
        rhs = Iagg[l].reshape(-1)[unk] - Y[np.ix_(unk, [0, 1, 2])] @ f["V0"]
        Vu = np.linalg.solve(Y[np.ix_(unk, unk)], rhs)
        V = np.zeros(3 * n, dtype=np.complex128)
        V[:3] = f["V0"]
        V[unk] = Vu
        V = V.reshape(n, 3)
        for i in range(n):
            Vc[l, i] = V[sup[i]] * pres.reshape(n, 3)[i]
    return Vc


def v_full_raw(f, Ihat, keep):
    """Physical voltages of every node of the full network carrying the
    aggregated currents (Y V = I^c, Algorithm 1's solve), before any copy from
    super-nodes, and the super-node map."""
    n = f["n"]
    pres = present(f)
    Y = dense_Y(f)
    Iagg, sup = aggregate(f, Ihat, keep)
    unk = [q for q in range(3, 3 * n) if pres[q]]
    S = Ihat.shape[0]
    V = np.zeros((S, 3 * n), dtype=np.complex128)
    for l in range(S):
        rhs = Iagg[l].reshape(-1)[unk] - Y[np.ix_(unk, [0, 1, 2])] @ f["V0"]
        V[l, :3] = f["V0"]
        V[l, unk] = np.linalg.solve(Y[np.ix_(unk, unk)], rhs)
    return V.reshape(S, n, 3), sup


def omega_behavioural(f, Ihat, keep, nodes, tol=1e-12):
    """The nodes a segment's masks can touch, found by experiment rather than
    by a formula: every node whose physical voltage or super-node differs
    from the empty mask's under some single-node mask.  Returns (omega,
    smallest voltage change among the nodes taken in, largest among the nodes
    left out) so callers can check the threshold separates them."""
    base, sup0 = v_full_raw(f, Ihat, keep)
    n = f["n"]
    om = np.zeros(n, dtype=bool)
    dmax = np.zeros(n)
    for v in nodes:
        keep2 = keep.copy()
        keep2[v] = 0
        V, sup = v_full_raw(f, Ihat, keep2)
        d = np.abs(V - base).max(axis=(0, 2))
        om |= (d > tol) | (sup != sup0)
        dmax = np.maximum(dmax, np.where(sup != sup0, np.inf, d))
    inside = dmax[om & np.isfinite(dmax)]
    return om, (inside.min() if inside.size else np.inf), dmax[~om].max(initial=0.0)


def omega(f, keep, g):
    parent = f["parent"]
    seg = f["segment"]
    n = f["n"]
    children = [[] for _ in range(n)]
    for i in range(1, n):
        children[int(parent[i])].append(i)
    om = np.zeros(n, dtype=bool)
    for e in np.nonzero(seg == g)[0]:
        c = int(e)
        while parent[c] >= 0 and (seg[parent[c]] == g or not keep[parent[c]]):
            c = int(parent[c])
        st = [c]
        while st:
            v = st.pop()
            om[v] = True
            st.extend(children[v])
    return om


def score(f, Vhat, Ihat, keep2, om, route=vc_full_route):
    n = f["n"]
    pres = present(f).reshape(n, 3)
    Vc = route(f, Ihat, keep2)
    mag = np.abs(Vc)
    err = np.abs(mag - np.abs(Vhat))
    err[:, ~pres] = 0
    slack = np.minimum(mag - f["v_min"], f["v_max"] - mag)
    slack[:, ~pres] = np.inf
    kept_om = om & keep2.astype(bool)
    # SMICE: per snapshot, the largest error of each cluster (a kept node and
    # the nodes assigned to it, over their phases), summed over clusters
    sup = super_of(f["parent"], keep2)
    node_err = err.max(axis=2)                      # [S, n]
    mice = np.zeros((err.shape[0], n))
    for i in range(n):
        mice[:, sup[i]] = np.maximum(mice[:, sup[i]], node_err[:, i])
    return dict(e_glob=err.max(), e_loc=err[:, om].max(initial=0.0),
                slack_glob=slack.min(), slack_loc=slack[:, kept_om].min(initial=np.inf),
                feasible=bool(err.max() <= f["e_bar"] and slack.min() >= 0),
                smice=float(mice.sum()))


def seg_nodes(f, g):
    from synth_feeders import dfs_preorder
    order = dfs_preorder(f["parent"])
    return [int(v) for v in order if f["segment"][v] == g]


def brute_search(f, Vhat, Ihat, tie_tol=1e-11, secondary="maxerr", smice_tol=1e-9):
    """Exhaustive search over every mask of every segment, in segment order,
    with the lexicographic objective (most reduced, then the smallest key,
    then lowest mask): the key is e_loc (ties within tie_tol) or, with
    secondary="smice", SMICE (ties within smice_tol)."""
    n = f["n"]
    keep = np.ones(n, dtype=np.uint8)
    masks = []
    nseg = int(f["segment"].max()) + 1
    for g in range(nseg):
        nodes = seg_nodes(f, g)
        k = len(nodes)
        om = omega(f, keep, g)
        rows = []
        for m in range(1 << k):
            keep2 = keep.copy()
            for j in range(k):
                if m >> j & 1:
                    keep2[nodes[j]] = 0
            sc = score(f, Vhat, Ihat, keep2, om)
            key = sc["smice"] if secondary == "smice" else sc["e_loc"]
            rows.append((m, bin(m).count("1"), key, sc["feasible"]))
        tol = smice_tol if secondary == "smice" else tie_tol
        feas = [r for r in rows if r[3]]
        best = max(r[1] for r in feas)
        emin = min(r[2] for r in feas if r[1] == best)
        pick = min(r[0] for r in feas if r[1] == best and r[2] <= emin + tol)
        masks.append(pick)
        for j in range(k):
            if pick >> j & 1:
                keep[nodes[j]] = 0
    return keep, masks
