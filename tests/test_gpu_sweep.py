"""Reduction against the error bound (the Fig. 5 sweep) on the GPU: for every
bound of the sweep, the segment search's decisions, kept set and final
error equal the oracle's on a small feeder with two extreme hourly
scenarios."""
import numpy as np
import pytest

import oracle
from synth_feeders import extreme_scenarios, hourly_feeder

pytestmark = pytest.mark.gpu

E_BARS = (1e-4, 2e-4, 5e-4, 1e-3, 2e-3, 5e-3, 1e-2)


@pytest.fixture(scope="module")
def okr():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2510_19608_amd as okr
    okr.lib()
    return okr


@pytest.mark.parametrize("seed", [0, 1])
def test_sweep_points_match_oracle(okr, seed):
    print(f"e_bar sweep seed={seed}", flush=True)
    base = hourly_feeder("c1", seed, n=60, n_eligible=None, seg_size=(4, 8), kappa=1.0)
    f = dict(extreme_scenarios(base), v_min=0.90, v_max=1.10)
    V, I, _, _ = oracle.powerflow(f)
    kept = []
    for eb in E_BARS:
        fe = dict(f, e_bar=eb)
        keep, dec, st = oracle.search(fe, V, I)
        if any(d["ambiguous"] for d in dec):
            continue
        out = okr.reduce_feeder(fe, e_bar=eb, want_vhat=False)
        assert [s["mask"] for s in out["segments"]] == [d["mask"] for d in dec]
        np.testing.assert_array_equal(out["kept"], keep)
        err, _ = oracle.final_errors(fe, V, I, keep)
        np.testing.assert_allclose(out["err_per_snapshot"], err, rtol=0, atol=1e-9)
        assert out["max_err"] <= eb
        kept.append(int(keep.sum()))
    assert len(kept) >= 4
