"""Writes the oracle's full-size decisions (TEST INFRASTRUCTURE: calls only
oracle/ and the input generator).

For each case: per-segment chosen mask, popcount, e_loc and ambiguity flag,
the final per-snapshot errors and the kept count, as JSON next to this
script.  The oracle runs its descending-popcount search (every mask of a
level scored before the next lower level; the first level holding a feasible
mask decides), which selects the same mask as scoring all 2^k masks.

Cases: the 6000- and 8400-node workloads at e_bar = 3e-3 (where nearly every
segment keeps its top level), the 1000-, 6000- and 8400-node workloads at
an error bound that binds (a quarter or more of the segments choose a mask
below the top level, so the arg-min is decided among many candidates), and
the 1000-node one at that bound with SMICE (Algorithm 1's sum of MICE) as the
key among the most-reducing feasible masks.

    python tests/golden/make_golden.py [case-name ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from synth_feeders import make_feeder  # noqa: E402

CASES = {"c3": ("c3", 0, 3e-3, "oracle_c3_seed0.json"),
         "c4": ("c4", 0, 3e-3, "oracle_c4_seed0.json"),
         "c2_bind": ("c2", 0, 1e-4, "oracle_c2_seed0_ebar1e-4.json"),
         "c3_bind": ("c3", 0, 7e-5, "oracle_c3_seed0_ebar7e-5.json"),
         "c4_bind": ("c4", 0, 7e-5, "oracle_c4_seed0_ebar7e-5.json"),
         "c2_smice": ("c2", 0, 1e-4, "oracle_c2_seed0_ebar1e-4_smice.json", "smice")}


def main():
    names = sys.argv[1:] or list(CASES)
    for key in names:
        cfg, seed, e_bar, fname = CASES[key][:4]
        secondary = CASES[key][4] if len(CASES[key]) > 4 else "maxerr"
        t0 = time.time()
        f = make_feeder(cfg, seed, e_bar=e_bar)
        V, I, st, _ = oracle.powerflow(f)
        assert st == 0, f"load flow status {st}"
        keep, dec, st = oracle.search(f, V, I, secondary=secondary)
        err, _ = oracle.final_errors(f, V, I, keep)
        seg = [dict(mask=int(d["mask"]), popcount=int(d["popcount"]), e_loc=float(d["e_loc"]),
                    ambiguous=int(d["ambiguous"])) for d in dec]
        if secondary == "smice":
            for s, d in zip(seg, dec):
                s["smice_rise"] = float(d["smice_rise"])
                s["key_gap"] = float(d["key_gap"]) if d["key_gap"] < float("inf") else None
        out = dict(workload=cfg, seed=seed, e_bar=e_bar, secondary=secondary, status=int(st),
                   n_kept=int(keep.sum()), err_per_snapshot=[float(x) for x in err], segments=seg)
        name = os.path.join(HERE, fname)
        with open(name, "w") as fh:
            json.dump(out, fh)
        print(f"{name}: {len(dec)} segments, kept {out['n_kept']}, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
