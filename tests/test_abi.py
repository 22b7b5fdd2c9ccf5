"""The C ABI on the CPU: the library loads, exports every declared symbol, and
its host-side validation reports the documented error codes (no GPU call is
made on these paths)."""
import ctypes
import os
import re

import numpy as np
import pytest

from synth_feeders import make_feeder

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    inc = os.path.join(ROOT, "include")
    src = ""
    for h in sorted(os.listdir(inc)):
        if h.endswith(".h"):
            with open(os.path.join(inc, h)) as fh:
                src += fh.read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\s*\*)\s*(okr_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    import paper_2510_19608_amd as okr
    L = okr.lib()
    names = declared_functions()
    assert {"okr_create", "okr_plan", "okr_reduce_feeder", "okr_destroy", "okr_last_error",
            "okr_dump_scores", "okr_greedy_create", "okr_greedy_plan", "okr_greedy_run", "okr_greedy_evaluate",
            "okr_greedy_destroy", "okr_greedy_last_error"} <= set(names)
    for name in names:
        assert hasattr(L, name), name


def _topo(okr, f, **over):
    arrs = {k: np.ascontiguousarray(over.get(k, f[k]), dtype=dt) for k, dt in
            (("parent", np.int32), ("phase", np.uint8), ("eligible", np.uint8), ("segment", np.int32))}
    T = okr.binding.Topology(len(arrs["parent"]), arrs["parent"].ctypes.data, arrs["phase"].ctypes.data,
                             arrs["eligible"].ctypes.data, arrs["segment"].ctypes.data)
    return T, arrs


def _plan(okr, f, S=1, **over):
    h = okr.okr_create(None)
    try:
        T, keep = _topo(okr, f, **over)
        return okr.okr_plan(h, T, okr.binding.make_margins(f), S)
    finally:
        okr.okr_destroy(h)


def test_plan_sizes():
    import paper_2510_19608_amd as okr
    f = make_feeder("c2", 0)
    ws, sizes = _plan(okr, f, S=24)
    assert sizes.n_segments == f["n_segments"] and sizes.k_max == 16
    assert sizes.n_candidates == sum(1 << int((f["segment"] == g).sum()) for g in range(f["n_segments"]))
    # state arrays alone need 4 x S x n x 3 complex128
    assert ws > 4 * 24 * f["n"] * 3 * 16


@pytest.mark.parametrize("case,code", [
    ("cycle", -2), ("root", -2), ("phase", -3), ("elig_slack", -8), ("elig_branch", -8),
    ("seg_mismatch", -1), ("too_big", -8), ("gap", -1)])
def test_plan_validation_errors(case, code):
    import paper_2510_19608_amd as okr
    f = make_feeder("c1", 0, n_eligible=None, seg_size=(30, 30))
    par, ph, el, sg = f["parent"].copy(), f["phase"].copy(), f["eligible"].copy(), f["segment"].copy()
    nch = np.bincount(par[1:], minlength=f["n"])
    if case == "cycle":
        par[1] = 5 if par[5] != 1 else 6
        par[par[1]] = 1
    elif case == "root":
        par[0] = 3
    elif case == "phase":
        j = int(next(i for i in range(1, f["n"]) if ph[par[i]] != 7))
        ph[j] = 7
    elif case == "elig_slack":
        el[0] = 1
        sg[0] = 0
    elif case == "elig_branch":
        i = int(np.nonzero(nch >= 2)[0][-1])
        el[i] = 1
        sg[i] = 0
    elif case == "seg_mismatch":
        i = int(np.nonzero(el)[0][0])
        sg[i] = -1
    elif case == "too_big":
        big = make_feeder("c2", 0, seg_size=(25, 25))
        par, ph, el, sg = big["parent"], big["phase"], big["eligible"], big["segment"]
    elif case == "gap":
        sg[sg >= 0] = 2
    with pytest.raises(okr.OkrError) as ei:
        _plan(okr, f, parent=par, phase=ph, eligible=el, segment=sg)
    assert ei.value.code == code


def test_reduce_without_plan_is_an_argument_error():
    import paper_2510_19608_amd as okr
    h = okr.okr_create(None)
    try:
        b = okr.binding
        rc = okr.lib().okr_reduce_feeder(h, ctypes.byref(b.YBlocks()), ctypes.byref(b.Topology()),
                                         ctypes.byref(b.Loads()), ctypes.byref(b.Margins()), None, 0,
                                         ctypes.byref(b.Result()))
        assert rc == okr.OKR.E_ARG
        assert "okr_plan" in okr.okr_last_error(h)
    finally:
        okr.okr_destroy(h)


def test_product_path_has_no_cpu_fallback(monkeypatch):
    """Without a GPU the convenience wrapper raises instead of computing."""
    import torch
    import paper_2510_19608_amd as okr
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(okr.OkrError):
        okr.reduce_feeder(make_feeder("c1", 0))


def test_product_sources_do_not_reference_the_oracle():
    for d in ("paper_2510_19608_amd", "include"):
        for root, _, files in os.walk(os.path.join(ROOT, d)):
            for fn in files:
                if fn.endswith((".py", ".hip", ".cpp", ".h")):
                    with open(os.path.join(root, fn)) as fh:
                        src = fh.read()
                    assert "import oracle" not in src and "okr_oracle" not in src and "okro_" not in src, fn


def test_greedy_plan_validation():
    """Host-side checks of okr_greedy_plan: tree, phases, workspace size."""
    import paper_2510_19608_amd as okr
    f = make_feeder("c2", 0, n=100, snapshots=2)
    g = okr.okr_greedy_create(None)
    try:
        ws = okr.okr_greedy_plan(g, f["parent"], f["phase"], 2)
        assert ws > 6 * 2 * 100 * 3 * 16
        bad = f["parent"].copy()
        bad[5] = 7
        bad[7] = 5
        with pytest.raises(okr.OkrError) as e:
            okr.okr_greedy_plan(g, bad, f["phase"], 2)
        assert e.value.code == okr.OKR.E_NOT_TREE
        ph = f["phase"].copy()
        leaf = int(np.flatnonzero(f["parent"] > 0)[0])
        ph[leaf] = 7
        ph[f["parent"][leaf]] = 1
        with pytest.raises(okr.OkrError) as e:
            okr.okr_greedy_plan(g, f["parent"], ph, 2)
        assert e.value.code == okr.OKR.E_PHASE
    finally:
        okr.okr_greedy_destroy(g)


def test_noalloc_entry_point_rejects_before_any_gpu_call():
    """The no-allocation variant refuses the flags that would allocate and a
    plan whose workspace exceeds its static scratch, on the host."""
    import paper_2510_19608_amd as okr
    B = okr.binding
    f = make_feeder("c2", 0)
    h = okr.okr_create(None)
    try:
        T, keep = _topo(okr, f)
        mg = B.make_margins(f)
        mg.lanes = 8
        ws, _ = okr.okr_plan(h, T, mg, 24)
        assert ws > B.NOALLOC_SCRATCH_BYTES
        res = B.Result()
        Y, loads = B.YBlocks(None, None), B.Loads(24, None, None, None)
        rc = B.lib().okr_reduce_feeder_noalloc(h, ctypes.byref(Y), ctypes.byref(T), ctypes.byref(loads),
                                               ctypes.byref(mg), ctypes.byref(res))
        assert rc == B.OKR.E_WORKSPACE and b"static scratch" in B.lib().okr_last_error(h)
        mg.lanes = 1
        ws, _ = okr.okr_plan(h, T, mg, 24)
        assert ws <= B.NOALLOC_SCRATCH_BYTES  # the 1000-node workload fits with one lane
        for flag in (B.OKR.FLAG_TIMING, B.OKR.FLAG_GRAPH, B.OKR.FLAG_AUTOTUNE, B.OKR.FLAG_DUMP_SCORES):
            mg.flags = flag
            rc = B.lib().okr_reduce_feeder_noalloc(h, ctypes.byref(Y), ctypes.byref(T), ctypes.byref(loads),
                                                   ctypes.byref(mg), ctypes.byref(res))
            assert rc == B.OKR.E_ARG
    finally:
        okr.okr_destroy(h)
