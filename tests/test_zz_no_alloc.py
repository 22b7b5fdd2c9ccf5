"""The no-allocation entry point (okr_reduce_feeder_noalloc) against
okr_reduce_feeder on the same inputs: two calls in a row on one GPU, the
second with a smaller input (the shared static scratch keeps the first call's
contents).  Decisions must be equal bit for bit, errors and reduced blocks to
the FP64 tolerance (they run the same kernels, so they agree exactly)."""
import sys

import numpy as np
import pytest

from synth_feeders import make_feeder

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


def _both(okr, f, lanes):
    import torch
    R = okr.Reducer(f, device="cuda:0", lanes=lanes)
    try:
        assert R.ws_bytes <= okr.binding.NOALLOC_SCRATCH_BYTES
        R.run(replan=False)
        torch.cuda.synchronize()
        ref = R.result()
        R.run(replan=False, noalloc=True)
        torch.cuda.synchronize()
        got = R.result()
    finally:
        R.close()
    return ref, got


def _compare(ref, got):
    assert [s["mask"] for s in got["segments"]] == [s["mask"] for s in ref["segments"]]
    assert [s["ambiguous"] for s in got["segments"]] == [s["ambiguous"] for s in ref["segments"]]
    assert got["n_kept"] == ref["n_kept"]
    assert np.array_equal(got["super"], ref["super"])
    assert np.array_equal(got["kept_parent"], ref["kept_parent"])
    for a, b in zip(got["segments"], ref["segments"]):
        assert abs(a["e_loc"] - b["e_loc"]) <= TOL
    np.testing.assert_allclose(got["err_per_snapshot"], ref["err_per_snapshot"], rtol=0, atol=TOL)
    np.testing.assert_allclose(got["Yk_diag"], ref["Yk_diag"], rtol=0, atol=1e-9 * max(1.0, np.abs(ref["Yk_diag"]).max()))
    np.testing.assert_allclose(got["Yk_off"], ref["Yk_off"], rtol=0, atol=1e-9 * max(1.0, np.abs(ref["Yk_off"]).max()))


def test_noalloc_matches_workspace_entry_point_twice(okr):
    # first the 1000-node, 24-snapshot workload (one chunk lane, so it fits the
    # static scratch), then the smaller 30-node feeder on the same array
    for cfg, seed, kw, lanes in (("c2", 0, dict(e_bar=1e-4), 1), ("c1", 1, dict(e_bar=3e-4), 1)):
        _say(f"no-alloc entry point: {cfg} seed {seed} {kw}")
        f = make_feeder(cfg, seed, **kw)
        ref, got = _both(okr, f, lanes)
        _compare(ref, got)
        _say(f"  {len(ref['segments'])} segments equal, kept {ref['n_kept']}")
