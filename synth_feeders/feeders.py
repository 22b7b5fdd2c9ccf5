"""Seeded synthetic unbalanced three-phase radial feeders.

The paper evaluates on two utility feeders and their 100-1000-node
sub-feeders (Section VI), none of which are available.  These generators
stand in for them with the shapes the build's workloads name: random
recursive trees with a three-phase trunk and one- or two-phase laterals,
per-mile 3x3 line impedances, per-phase constant-PQ loads and per-node
hourly load scales.

Conventions (all values per unit on a per-phase line-to-neutral base):
  * node 0 is the slack (substation), ``parent[0] = -1``;
  * ``phase[i]`` is a bitmask, bit0 = a, bit1 = b, bit2 = c, and a child's
    phases are a subset of its parent's (Section II.A, phase availability);
  * ``Y_off[i]`` is the block Y_{i,parent(i)} = -y_i with
    y_i = (z_i restricted to phase[i])^-1, zero on absent phases, and
    ``Y_diag[i]`` the sum of the incident y blocks (no shunts), so the
    assembled Y is the block nodal admittance matrix of Section II.A;
  * ``S_load[l, i, p]`` is the complex power consumed on phase p of node i
    in snapshot l (P + jQ, lagging);
  * ``eligible[i]`` marks nodes the search may reduce (non-slack, at most
    one child; reducing such nodes never creates a mesh, Section V);
  * ``segment[i]`` is the segment id of an eligible node (-1 otherwise);
    segments are runs of consecutive eligible nodes in DFS preorder.

Only input synthesis lives here: building Y from z needs a 3x3 inverse,
nothing else from the method's arithmetic is used.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional, Tuple

import numpy as np

PHASE_BITS = (1, 2, 4)
PAIRS = (3, 6, 5)  # ab, bc, ca


@dataclasses.dataclass(frozen=True)
class FeederConfig:
    name: str
    n: int
    snapshots: int
    p_single: float = 0.3          # child of a 3-phase node is 1-phase
    p_two: float = 0.3             # child of a 3-phase node is 2-phase
    p_deep: float = 0.0            # attach to the previous node instead of a uniform one
    trunk_frac: float = 0.02       # the first max(1, trunk_frac*n) non-slack nodes are three-phase
    length_mi: Tuple[float, float] = (0.05, 0.5)
    z_self: complex = 0.30 + 1.00j  # ohm / mile
    z_mut: complex = 0.10 + 0.40j   # ohm / mile
    jitter: float = 0.10
    kv_ll: float = 12.47
    s_base_mva: float = 1.0        # three-phase base; per-phase base is a third
    p_kw: Tuple[float, float] = (0.0, 50.0)
    pf: Tuple[float, float] = (0.90, 0.98)
    scale: Tuple[float, float] = (0.3, 1.0)
    kappa: float = 1.0             # global load multiplier (largest power of two keeping every snapshot in band)
    n_eligible: Optional[int] = None   # sample this many eligible nodes (None: all)
    seg_size: Tuple[int, int] = (16, 16)  # inclusive range of segment sizes
    v_min: float = 0.95
    v_max: float = 1.05
    e_bar: float = 0.003


# The five workloads: a 30-bus exact-parity case, the 1000-node headline case,
# and the larger batched / mixed / surrogate cases.  kappa is the largest power
# of two for which the full network's power flow converges and every snapshot
# stays inside the 0.95-1.05 band (checked by tests/test_synth.py with the
# oracle's power flow for the seeds used).
CONFIGS: Dict[str, FeederConfig] = {
    "c1": FeederConfig("c1", n=30, snapshots=1, kappa=1.0, n_eligible=12,
                       seg_size=(12, 12)),
    "c2": FeederConfig("c2", n=1000, snapshots=24, kappa=0.25, seg_size=(16, 16)),
    "c3": FeederConfig("c3", n=6000, snapshots=96, p_single=0.2, p_two=0.4,
                       p_deep=0.5, kappa=1.0 / 32, seg_size=(8, 18)),
    "c4": FeederConfig("c4", n=8400, snapshots=288, p_deep=0.5, kappa=1.0 / 32,
                       seg_size=(8, 20)),
}


def dfs_preorder(parent: np.ndarray) -> np.ndarray:
    """Return the DFS preorder (children visited in increasing node id)."""
    n = len(parent)
    children = [[] for _ in range(n)]
    for i in range(1, n):
        children[int(parent[i])].append(i)
    order = []
    stack = [0]
    while stack:
        v = stack.pop()
        order.append(v)
        stack.extend(reversed(children[v]))
    return np.asarray(order, dtype=np.int64)


def _inv3_restricted(z: np.ndarray, mask: int) -> np.ndarray:
    idx = [p for p in range(3) if mask >> p & 1]
    out = np.zeros((3, 3), dtype=np.complex128)
    sub = z[np.ix_(idx, idx)]
    out[np.ix_(idx, idx)] = np.linalg.inv(sub)
    return out


def make_feeder(cfg, seed: int, **overrides) -> dict:
    """Build one seeded feeder.  ``cfg`` is a FeederConfig or a CONFIGS key;
    keyword overrides replace config fields (e.g. ``n=12`` for tiny cases)."""
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    if overrides:
        cfg = dataclasses.replace(cfg, **overrides)
    rng = np.random.default_rng(np.random.SeedSequence([2510_19608, seed, cfg.n]))
    n, S = cfg.n, cfg.snapshots

    # topology: random recursive tree, optionally biased towards long laterals
    parent = np.full(n, -1, dtype=np.int32)
    n_trunk = max(1, int(cfg.trunk_frac * n))
    phase = np.zeros(n, dtype=np.uint8)
    phase[0] = 7
    for i in range(1, n):
        if cfg.p_deep > 0 and rng.random() < cfg.p_deep:
            p = i - 1
        else:
            p = int(rng.integers(0, i))
        parent[i] = p
        u = rng.random()
        if i <= n_trunk:
            phase[i] = 7
        elif phase[p] == 7:
            if u < cfg.p_single:
                phase[i] = PHASE_BITS[int(rng.integers(0, 3))]
            elif u < cfg.p_single + cfg.p_two:
                phase[i] = PAIRS[int(rng.integers(0, 3))]
            else:
                phase[i] = 7
        else:
            phase[i] = phase[p]

    # lines: per-mile impedance with independent jitter on the 6 unique entries
    zbase = (cfg.kv_ll * 1e3) ** 2 / (cfg.s_base_mva * 1e6)
    Y_off = np.zeros((n, 3, 3), dtype=np.complex128)
    Y_diag = np.zeros((n, 3, 3), dtype=np.complex128)
    for i in range(1, n):
        length = rng.uniform(*cfg.length_mi)
        zpm = np.empty((3, 3), dtype=np.complex128)
        for a in range(3):
            for b in range(a, 3):
                f = rng.uniform(1 - cfg.jitter, 1 + cfg.jitter)
                base = cfg.z_self if a == b else cfg.z_mut
                zpm[a, b] = zpm[b, a] = base * f
        z = zpm * length / zbase
        m = int(phase[i])
        keep = np.array([(m >> p) & 1 for p in range(3)], dtype=bool)
        z[~keep, :] = 0
        z[:, ~keep] = 0
        y = _inv3_restricted(z, m)
        Y_off[i] = -y
        Y_diag[i] += y
        Y_diag[parent[i]] += y

    # loads: P ~ U(kW), lagging pf, per present phase; per-(node, snapshot) scale
    s1 = cfg.s_base_mva * 1e6 / 3.0
    base_load = np.zeros((n, 3), dtype=np.complex128)
    for i in range(1, n):
        for p in range(3):
            if phase[i] >> p & 1:
                P = rng.uniform(*cfg.p_kw) * 1e3
                pf = rng.uniform(*cfg.pf)
                Q = P * math.tan(math.acos(pf))
                base_load[i, p] = cfg.kappa * (P + 1j * Q) / s1
    if S == 1:
        scale = np.ones((1, n))
    else:
        scale = rng.uniform(*cfg.scale, size=(S, n))
    S_load = scale[:, :, None] * base_load[None, :, :]

    # eligibility (non-slack, at most one child) and segments in DFS preorder
    nchild = np.bincount(parent[1:], minlength=n)
    elig_all = np.zeros(n, dtype=bool)
    elig_all[1:] = nchild[1:] <= 1
    order = dfs_preorder(parent)
    cand = [int(v) for v in order if elig_all[v]]
    if cfg.n_eligible is not None and cfg.n_eligible < len(cand):
        pick = set(rng.choice(len(cand), size=cfg.n_eligible, replace=False).tolist())
        cand = [v for j, v in enumerate(cand) if j in pick]
    eligible = np.zeros(n, dtype=np.uint8)
    eligible[cand] = 1
    segment = np.full(n, -1, dtype=np.int32)
    pos, sid = 0, 0
    lo, hi = cfg.seg_size
    while pos < len(cand):
        size = lo if lo == hi else int(rng.integers(lo, hi + 1))
        for v in cand[pos:pos + size]:
            segment[v] = sid
        pos += size
        sid += 1

    V0 = np.exp(-2j * np.pi / 3 * np.arange(3))  # 1/0, 1/-120, 1/+120 degrees
    return dict(
        name=cfg.name, seed=seed, n=n, snapshots=S,
        parent=parent, phase=phase, eligible=eligible, segment=segment,
        Y_diag=Y_diag, Y_off=Y_off, S_load=np.ascontiguousarray(S_load),
        V0=V0.astype(np.complex128),
        e_bar=cfg.e_bar, v_min=cfg.v_min, v_max=cfg.v_max, kappa=cfg.kappa,
        n_segments=sid,
    )


def hourly_feeder(cfg, seed: int, hours: int = 168, **overrides) -> dict:
    """A feeder of ``cfg`` (with overrides) whose scenarios are ``hours``
    hourly load snapshots: every node's base load times a daily profile
    (night trough, daytime peak) times a per-(hour, node) factor
    U(0.85, 1.15).  Stands in for a week of hourly utility load data."""
    f = make_feeder(cfg, seed, **dict(overrides, snapshots=1))
    rng = np.random.default_rng(np.random.SeedSequence([2510_19608, seed, f["n"], hours]))
    h = np.arange(hours) % 24
    daily = 0.45 + 0.55 * np.clip(np.sin(np.pi * (h - 6) / 16.0), 0.0, None)
    scale = daily[:, None] * rng.uniform(0.85, 1.15, size=(hours, f["n"]))
    base = np.asarray(f["S_load"])[0]
    return dict(f, snapshots=hours, S_load=np.ascontiguousarray(scale[:, :, None] * base[None, :, :]))


def extreme_scenarios(f) -> dict:
    """The feeder restricted to its highest- and lowest-loaded scenarios (by
    total apparent power), in that order."""
    tot = np.abs(np.asarray(f["S_load"])).sum(axis=(1, 2))
    pick = [int(np.argmax(tot)), int(np.argmin(tot))]
    return dict(f, snapshots=2, S_load=np.ascontiguousarray(np.asarray(f["S_load"])[pick]), hours_picked=pick)
