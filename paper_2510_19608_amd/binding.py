"""ctypes binding of the C ABI in include/okr.h (argument marshalling only).

torch supplies device memory and the HIP stream; every step of the search
runs in the library's kernels.  The functions named okr_* mirror the C entry
points one to one; ``Reducer`` and ``reduce_feeder`` are conveniences that
plan once, keep inputs resident on the device and call okr_reduce_feeder.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libokr.so")


class OKR:
    OK = 0
    E_ARG = -1
    E_NOT_TREE = -2
    E_PHASE = -3
    E_SINGULAR = -4
    E_PF_DIVERGED = -5
    E_WORKSPACE = -6
    E_HIP = -7
    E_UNSUPPORTED = -8
    W_BASE_OUT_OF_BAND = 1
    PRECISION_FP64 = 0
    PRECISION_MIXED = 1
    PRECISION_FP64_FACTORED = 2
    SECONDARY_MAXERR = 0
    SECONDARY_SMICE = 1
    FLAG_TIMING = 1
    FLAG_VHAT_GIVEN = 2
    FLAG_DUMP_SCORES = 4
    FLAG_GRAPH = 8
    FLAG_AUTOTUNE = 16
    GREEDY_INCREMENTAL = 0x100


class OkrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"okr error {code}: {msg}")
        self.code = code


class Topology(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("parent", ctypes.c_void_p), ("phase", ctypes.c_void_p),
                ("eligible", ctypes.c_void_p), ("segment", ctypes.c_void_p)]


class YBlocks(ctypes.Structure):
    _fields_ = [("Y_diag", ctypes.c_void_p), ("Y_off", ctypes.c_void_p)]


class Loads(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int32), ("S_load", ctypes.c_void_p), ("V0", ctypes.c_void_p),
                ("Vhat", ctypes.c_void_p)]


class Margins(ctypes.Structure):
    _fields_ = [("e_bar", ctypes.c_double), ("v_min", ctypes.c_double), ("v_max", ctypes.c_double),
                ("tie_tol", ctypes.c_double), ("amb_tol", ctypes.c_double), ("pf_tol", ctypes.c_double),
                ("pf_maxit", ctypes.c_int32), ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("top_k", ctypes.c_int32), ("surrogate", ctypes.c_void_p), ("lanes", ctypes.c_int32),
                ("surrogate_margin", ctypes.c_float), ("mixed_delta", ctypes.c_double),
                ("secondary", ctypes.c_int32), ("smice_tol", ctypes.c_double)]


class Sizes(ctypes.Structure):
    _fields_ = [("n_segments", ctypes.c_int32), ("k_max", ctypes.c_int32), ("n_candidates", ctypes.c_int64)]


class SegmentResult(ctypes.Structure):
    _fields_ = [("segment", ctypes.c_int32), ("k", ctypes.c_int32), ("mask", ctypes.c_uint32),
                ("popcount", ctypes.c_int32), ("e_loc", ctypes.c_double), ("e_min", ctypes.c_double),
                ("ambiguous", ctypes.c_int32), ("n_scored", ctypes.c_int32), ("flops", ctypes.c_double),
                ("score_ms", ctypes.c_float), ("n_refined", ctypes.c_int32), ("fp32_dev", ctypes.c_double),
                ("score_groups", ctypes.c_int32), ("score_mpl", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("kernel_flops", ctypes.c_double), ("score_waves", ctypes.c_int32), ("key_gap", ctypes.c_double),
                ("smice_rise", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("super", ctypes.c_void_p), ("kept_parent", ctypes.c_void_p), ("Yk_diag", ctypes.c_void_p),
                ("Yk_off", ctypes.c_void_p), ("err_per_snapshot", ctypes.c_void_p), ("Vhat", ctypes.c_void_p),
                ("seg", ctypes.c_void_p), ("features", ctypes.c_void_p), ("targets", ctypes.c_void_p),
                ("n_kept", ctypes.c_int32), ("warnings", ctypes.c_int32),
                ("max_err", ctypes.c_double), ("t_setup_ms", ctypes.c_double), ("t_pf_ms", ctypes.c_double),
                ("t_search_ms", ctypes.c_double), ("t_final_ms", ctypes.c_double),
                ("score_kernel_ms", ctypes.c_double), ("algorithmic_flops", ctypes.c_double),
                ("pf_iterations", ctypes.c_int32), ("n_score_launches", ctypes.c_int32),
                ("kernel_form_flops", ctypes.c_double)]


class GreedyParams(ctypes.Structure):
    _fields_ = [("e_bar", ctypes.c_double), ("tie_tol", ctypes.c_double), ("amb_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("flags", ctypes.c_uint32), ("pf_tol", ctypes.c_double),
                ("pf_maxit", ctypes.c_int32), ("pad", ctypes.c_int32)]


class GreedyStep(ctypes.Structure):
    _fields_ = [("cand", ctypes.c_int32), ("s", ctypes.c_int32), ("r", ctypes.c_int32),
                ("ambiguous", ctypes.c_int32), ("n_cand", ctypes.c_int32), ("n_feasible", ctypes.c_int32),
                ("smice", ctypes.c_double), ("emax", ctypes.c_double)]


class GreedyResult(ctypes.Structure):
    _fields_ = [("super", ctypes.c_void_p), ("steps", ctypes.c_void_p), ("err_per_snapshot", ctypes.c_void_p),
                ("n_steps", ctypes.c_int32), ("n_kept", ctypes.c_int32), ("max_err", ctypes.c_double),
                ("t_pf_ms", ctypes.c_double), ("t_search_ms", ctypes.c_double),
                ("pf_iterations", ctypes.c_int32), ("n_score_launches", ctypes.c_int32),
                ("t_score_ms", ctypes.c_double), ("n_scored", ctypes.c_int64), ("incremental", ctypes.c_int32),
                ("pad2", ctypes.c_int32)]


_lib = None


def lib():
    """Load libokr.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise OkrError(OKR.E_HIP, f"{_LIB_PATH} is missing: build it (python -m paper_2510_19608_amd.build)")
        L = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        L.okr_create.argtypes = [ctypes.POINTER(vp), vp]
        L.okr_plan.argtypes = [vp, ctypes.POINTER(Topology), ctypes.POINTER(Margins), ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(Sizes)]
        L.okr_reduce_feeder.argtypes = [vp, ctypes.POINTER(YBlocks), ctypes.POINTER(Topology),
                                        ctypes.POINTER(Loads), ctypes.POINTER(Margins), vp, ctypes.c_size_t,
                                        ctypes.POINTER(Result)]
        L.okr_reduce_feeder_noalloc.argtypes = [vp, ctypes.POINTER(YBlocks), ctypes.POINTER(Topology),
                                                ctypes.POINTER(Loads), ctypes.POINTER(Margins),
                                                ctypes.POINTER(Result)]
        L.okr_dump_scores.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.POINTER(ctypes.c_int32)]
        L.okr_destroy.argtypes = [vp]
        L.okr_last_error.argtypes = [vp]
        L.okr_last_error.restype = ctypes.c_char_p
        L.okr_surrogate_workspace.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.okr_train_surrogate.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                          ctypes.c_uint64, vp, vp, ctypes.c_size_t, vp, vp]
        L.okr_surrogate_grad.argtypes = [vp, vp, vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_float), vp,
                                         ctypes.c_size_t, vp]
        L.okr_surrogate_forward.argtypes = [vp, vp, ctypes.c_int64, vp, vp, ctypes.c_size_t, vp]
        L.okr_greedy_create.argtypes = [ctypes.POINTER(vp), vp]
        L.okr_greedy_plan.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.okr_greedy_run.argtypes = [vp, ctypes.POINTER(YBlocks), ctypes.POINTER(Loads),
                                     ctypes.POINTER(GreedyParams), vp, ctypes.POINTER(GreedyResult)]
        L.okr_greedy_evaluate.argtypes = [vp, ctypes.POINTER(YBlocks), ctypes.POINTER(Loads), vp,
                                          ctypes.POINTER(GreedyParams), vp, vp, ctypes.POINTER(ctypes.c_double)]
        L.okr_greedy_radialize.argtypes = [vp, ctypes.POINTER(YBlocks), ctypes.POINTER(Loads), vp,
                                           ctypes.POINTER(GreedyParams), vp, vp, vp, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.okr_greedy_destroy.argtypes = [vp]
        L.okr_greedy_last_error.argtypes = [vp]
        L.okr_greedy_last_error.restype = ctypes.c_char_p
        for fn in ("okr_create", "okr_plan", "okr_reduce_feeder", "okr_reduce_feeder_noalloc", "okr_dump_scores",
                   "okr_destroy",
                   "okr_surrogate_workspace", "okr_train_surrogate", "okr_surrogate_grad",
                   "okr_surrogate_forward", "okr_greedy_create", "okr_greedy_plan", "okr_greedy_run",
                   "okr_greedy_evaluate", "okr_greedy_radialize", "okr_greedy_destroy"):
            getattr(L, fn).restype = ctypes.c_int
        _lib = L
    return _lib


# ---- one-to-one wrappers of the C entry points ---------------------------

def okr_create(stream=None):
    h = ctypes.c_void_p()
    rc = lib().okr_create(ctypes.byref(h), stream)
    if rc != 0:
        raise OkrError(rc, "okr_create failed")
    return h


def okr_last_error(h):
    return lib().okr_last_error(h).decode()


def _check(h, rc):
    if rc < 0:
        raise OkrError(rc, okr_last_error(h))
    return rc


def okr_plan(h, topo: Topology, margins: Margins, S: int):
    ws = ctypes.c_size_t(0)
    sizes = Sizes()
    _check(h, lib().okr_plan(h, ctypes.byref(topo), ctypes.byref(margins), S, ctypes.byref(ws),
                             ctypes.byref(sizes)))
    return ws.value, sizes


def okr_reduce_feeder(h, Y: YBlocks, topo: Topology, loads: Loads, margins: Margins, d_ws, ws_bytes,
                      out: Result):
    return _check(h, lib().okr_reduce_feeder(h, ctypes.byref(Y), ctypes.byref(topo), ctypes.byref(loads),
                                             ctypes.byref(margins), d_ws, ws_bytes, ctypes.byref(out)))


def okr_reduce_feeder_noalloc(h, Y: YBlocks, topo: Topology, loads: Loads, margins: Margins, out):
    """okr_reduce_feeder with the library's static per-GPU scratch as workspace
    (no device allocation; planned workspace at most OKR_NOALLOC_SCRATCH_BYTES)."""
    return _check(h, lib().okr_reduce_feeder_noalloc(h, ctypes.byref(Y), ctypes.byref(topo), ctypes.byref(loads),
                                                     ctypes.byref(margins), ctypes.byref(out)))


NOALLOC_SCRATCH_BYTES = 64 << 20


def okr_dump_scores(h, segment, nmask):
    e = np.zeros(nmask)
    s = np.zeros(nmask)
    k = ctypes.c_int32(0)
    _check(h, lib().okr_dump_scores(h, segment, e.ctypes.data, s.ctypes.data, ctypes.byref(k)))
    return e, s, k.value


def okr_destroy(h):
    return lib().okr_destroy(h)


SURR_FEATURES = 32
SURR_HIDDEN = 256
SURR_PARAMS = 256 * 32 + 256 + 256 * 256 + 256 + 256 + 1


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_of(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _free_check(rc, what):
    if rc != 0:
        raise OkrError(rc, what)


def okr_surrogate_workspace(batch):
    b = ctypes.c_size_t(0)
    _free_check(lib().okr_surrogate_workspace(batch, ctypes.byref(b)), f"bad surrogate batch {batch}")
    return b.value


def okr_train_surrogate(X, t, epochs, batch, lr, seed, params, work):
    """Train ``params`` in place (device tensors: X float [n][32], t float [n],
    params float [SURR_PARAMS], work uint8); returns the per-epoch mean loss."""
    loss = np.zeros(epochs, np.float32)
    rc = lib().okr_train_surrogate(_ptr(X), _ptr(t), X.shape[0], epochs, batch, lr, seed, _ptr(params), _ptr(work),
                                   work.numel(), _stream_of(X), loss.ctypes.data)
    _free_check(rc, "okr_train_surrogate failed")
    return loss


def okr_surrogate_grad(params, X, t, grads, work):
    """Loss gradient of one batch into ``grads``; returns the batch loss."""
    loss = ctypes.c_float(0.0)
    rc = lib().okr_surrogate_grad(_ptr(params), _ptr(X), _ptr(t), X.shape[0], _ptr(grads), ctypes.byref(loss),
                                  _ptr(work), work.numel(), _stream_of(X))
    _free_check(rc, "okr_surrogate_grad failed")
    return loss.value


def okr_surrogate_forward(params, X, y, work):
    rc = lib().okr_surrogate_forward(_ptr(params), _ptr(X), X.shape[0], _ptr(y), _ptr(work), work.numel(),
                                     _stream_of(X))
    _free_check(rc, "okr_surrogate_forward failed")
    return y


# ---- conveniences ----------------------------------------------------------

def make_margins(f=None, *, e_bar=None, v_min=None, v_max=None, tie_tol=1e-11, amb_tol=1e-13,
                 precision="fp64", timing=False, dump=False, vhat_given=False, graph=False, pf_tol=1e-13,
                 pf_maxit=100, top_k=0, surrogate=None, lanes=0, surrogate_margin=0.0, mixed_delta=0.0,
                 secondary="maxerr", smice_tol=0.0):
    f = f or {}
    flags = (OKR.FLAG_TIMING if timing else 0) | (OKR.FLAG_DUMP_SCORES if dump else 0) | \
            (OKR.FLAG_VHAT_GIVEN if vhat_given else 0) | (OKR.FLAG_GRAPH if graph else 0)
    return Margins(e_bar=f.get("e_bar", 0.003) if e_bar is None else e_bar,
                   v_min=f.get("v_min", 0.95) if v_min is None else v_min,
                   v_max=f.get("v_max", 1.05) if v_max is None else v_max,
                   tie_tol=tie_tol, amb_tol=amb_tol, pf_tol=pf_tol, pf_maxit=pf_maxit,
                   precision={"fp64": OKR.PRECISION_FP64, "mixed": OKR.PRECISION_MIXED,
                              "factored": OKR.PRECISION_FP64_FACTORED}[precision],
                   flags=flags, top_k=top_k,
                   surrogate=None if surrogate is None else surrogate.data_ptr(), lanes=lanes,
                   surrogate_margin=surrogate_margin, mixed_delta=mixed_delta,
                   secondary={"maxerr": OKR.SECONDARY_MAXERR, "smice": OKR.SECONDARY_SMICE}[secondary],
                   smice_tol=smice_tol)


class Reducer:
    """Plans once, keeps the feeder's inputs resident on the device and runs
    okr_reduce_feeder on demand (``run``)."""

    def __init__(self, f, device="cuda:0", vhat=None, **margin_kw):
        """margin_kw: make_margins' keywords; ``surrogate`` (a device tensor of
        SURR_PARAMS floats) with ``top_k`` enables learned pruning."""
        import torch
        if not torch.cuda.is_available():
            raise OkrError(OKR.E_HIP, "no GPU visible: the search runs only on the HIP device")
        lib()
        self.torch = torch
        self.device = torch.device(device)
        self.f = f
        n, S = int(f["n"]), int(np.asarray(f["S_load"]).shape[0])
        self.n, self.S = n, S
        self.parent = np.ascontiguousarray(f["parent"], dtype=np.int32)
        self.phase = np.ascontiguousarray(f["phase"], dtype=np.uint8)
        self.eligible = np.ascontiguousarray(f["eligible"], dtype=np.uint8)
        self.segment = np.ascontiguousarray(f["segment"], dtype=np.int32)
        self.topo = Topology(n, self.parent.ctypes.data, self.phase.ctypes.data, self.eligible.ctypes.data,
                             self.segment.ctypes.data)
        self.surrogate = margin_kw.get("surrogate")  # keeps the parameters alive
        self.margins = make_margins(f, vhat_given=vhat is not None, **margin_kw)

        def dev(a):
            t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))
            return torch.view_as_real(t).contiguous().to(self.device)

        with torch.cuda.device(self.device):
            self.Yd = dev(f["Y_diag"])
            self.Yo = dev(f["Y_off"])
            self.Sl = dev(f["S_load"])
            self.Vh = dev(vhat) if vhat is not None else None
            # a stream of the handle's own (default priority): the null stream
            # cannot be captured into a graph
            self.stream = torch.cuda.Stream(device=self.device)
            self.h = okr_create(ctypes.c_void_p(self.stream.cuda_stream))
            self.ws_bytes, self.sizes = okr_plan(self.h, self.topo, self.margins, S)
            self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=self.device)
        self.V0 = np.ascontiguousarray(f["V0"], dtype=np.complex128)
        self.Y = YBlocks(self.Yd.data_ptr(), self.Yo.data_ptr())
        self.loads = Loads(S, self.Sl.data_ptr(), self.V0.ctypes.data,
                           self.Vh.data_ptr() if self.Vh is not None else None)
        nseg = self.sizes.n_segments

        def host(shape, dtype):
            # page-locked host buffers (torch allocates them): the library's
            # device-to-host copies of the outputs then go straight to them
            t = torch.zeros(shape, dtype=dtype, pin_memory=True)
            self._pinned.append(t)
            return t.numpy()
        self._pinned = []
        self.out_super = host((n,), torch.int32)
        self.out_kp = host((n,), torch.int32)
        self.out_Ykd = host((n, 3, 3), torch.complex128)
        self.out_Yko = host((n, 3, 3), torch.complex128)
        self.out_err = host((S,), torch.float64)
        self.out_Vhat = host((S, n, 3), torch.complex128)
        self.out_seg = (SegmentResult * max(nseg, 1))()
        self.res = Result(self.out_super.ctypes.data, self.out_kp.ctypes.data, self.out_Ykd.ctypes.data,
                          self.out_Yko.ctypes.data, self.out_err.ctypes.data, None,
                          ctypes.cast(self.out_seg, ctypes.c_void_p))

    def set_surrogate(self, params, top_k, margin=0.0):
        """Switch learned pruning on (params: device tensor) or off (None);
        top_k must not exceed the value planned with; margin: the ln-error
        slack of the predicted-feasible test."""
        self.surrogate = params
        self.margins.surrogate = None if params is None else params.data_ptr()
        self.margins.top_k = top_k if params is not None else 0
        self.margins.surrogate_margin = margin

    def run(self, replan=True, want_vhat=False, want_features=False, autotune=False, noalloc=False):
        """One pass of the whole search (planning included when replan).  With
        want_features the per-mask surrogate features and FP64 targets of every
        segment are left in ``self.features`` / ``self.targets`` (device).
        With autotune the scoring launch shape is tuned first (kept in the
        handle for later runs)."""
        # inputs written on the caller's stream are complete before the search
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        if replan:
            self.ws_bytes_now, _ = okr_plan(self.h, self.topo, self.margins, self.S)
        self.res.Vhat = self.out_Vhat.ctypes.data if want_vhat else None
        if want_features:
            nc = int(self.sizes.n_candidates)
            if getattr(self, "features", None) is None or self.features.shape[0] != nc:
                self.features = self.torch.zeros((nc, SURR_FEATURES), dtype=self.torch.float32,
                                                 device=self.device)
                self.targets = self.torch.zeros(nc, dtype=self.torch.float32, device=self.device)
            self.res.features = self.features.data_ptr()
            self.res.targets = self.targets.data_ptr()
        else:
            self.res.features = None
            self.res.targets = None
        flags = self.margins.flags
        if autotune:
            self.margins.flags = flags | OKR.FLAG_AUTOTUNE
        try:
            if noalloc:
                rc = okr_reduce_feeder_noalloc(self.h, self.Y, self.topo, self.loads, self.margins, self.res)
            else:
                rc = okr_reduce_feeder(self.h, self.Y, self.topo, self.loads, self.margins,
                                       ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, self.res)
        finally:
            self.margins.flags = flags
        return rc

    def result(self):
        r = self.res
        segs = [dict(segment=s.segment, k=s.k, mask=s.mask, popcount=s.popcount, e_loc=s.e_loc,
                     e_min=s.e_min, ambiguous=bool(s.ambiguous), n_scored=s.n_scored, flops=s.flops,
                     score_ms=s.score_ms, n_refined=s.n_refined, fp32_dev=s.fp32_dev,
                     score_groups=s.score_groups, score_mpl=s.score_mpl, score_waves=s.score_waves, chunk=s.chunk,
                     key_gap=s.key_gap, smice_rise=s.smice_rise,
                     kernel_flops=s.kernel_flops)
                for s in list(self.out_seg)[:self.sizes.n_segments]]
        return dict(super=self.out_super.copy(), kept_parent=self.out_kp.copy(),
                    kept=(self.out_super == np.arange(self.n)).astype(np.uint8),
                    Yk_diag=self.out_Ykd.copy(), Yk_off=self.out_Yko.copy(),
                    err_per_snapshot=self.out_err.copy(), max_err=r.max_err, n_kept=r.n_kept,
                    warnings=r.warnings, segments=segs, t_pf_ms=r.t_pf_ms, t_search_ms=r.t_search_ms,
                    t_final_ms=r.t_final_ms, score_kernel_ms=r.score_kernel_ms,
                    algorithmic_flops=r.algorithmic_flops, kernel_form_flops=r.kernel_form_flops,
                    pf_iterations=r.pf_iterations,
                    n_score_launches=r.n_score_launches, Vhat=self.out_Vhat)

    def dump_scores(self, g):
        k = self.result()["segments"][g]["k"]
        return okr_dump_scores(self.h, g, 1 << k)

    def close(self):
        if getattr(self, "h", None) is not None:
            okr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reduce_feeder(f, device="cuda:0", vhat=None, want_vhat=True, **margin_kw):
    """Run the search once on a feeder dict and return the result dict."""
    R = Reducer(f, device=device, vhat=vhat, **margin_kw)
    try:
        rc = R.run(replan=False, want_vhat=want_vhat)
        R.torch.cuda.synchronize(R.device)
        out = R.result()
        out["status"] = rc
        if margin_kw.get("dump"):
            out["scores"] = {g: R.dump_scores(g) for g in range(R.sizes.n_segments)}
        return out
    finally:
        R.close()


# ---- greedy single-move search (Algorithm 1) and fixed-reduction scoring ----

def okr_greedy_create(stream=None):
    g = ctypes.c_void_p()
    rc = lib().okr_greedy_create(ctypes.byref(g), stream)
    if rc != 0:
        raise OkrError(rc, "okr_greedy_create failed")
    return g


def okr_greedy_last_error(g):
    return lib().okr_greedy_last_error(g).decode()


def _gcheck(g, rc):
    if rc < 0:
        raise OkrError(rc, okr_greedy_last_error(g))
    return rc


def okr_greedy_plan(g, parent, phase, S):
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    ws = ctypes.c_size_t(0)
    _gcheck(g, lib().okr_greedy_plan(g, len(parent), parent.ctypes.data, phase.ctypes.data, S, ctypes.byref(ws)))
    return ws.value


def okr_greedy_run(g, Y: YBlocks, loads: Loads, params: GreedyParams, d_ws, out: GreedyResult):
    return _gcheck(g, lib().okr_greedy_run(g, ctypes.byref(Y), ctypes.byref(loads), ctypes.byref(params), d_ws,
                                           ctypes.byref(out)))


def okr_greedy_evaluate(g, Y: YBlocks, loads: Loads, sup, params: GreedyParams, d_ws, err):
    sup = np.ascontiguousarray(sup, dtype=np.int32)
    mx = ctypes.c_double(0.0)
    _gcheck(g, lib().okr_greedy_evaluate(g, ctypes.byref(Y), ctypes.byref(loads), sup.ctypes.data,
                                         ctypes.byref(params), d_ws, err.ctypes.data, ctypes.byref(mx)))
    return mx.value


def okr_greedy_radialize(g, Y: YBlocks, loads: Loads, sup, params: GreedyParams, d_ws):
    sup = np.ascontiguousarray(sup, dtype=np.int32)
    n = len(sup)
    kept = np.zeros(n, np.uint8)
    kp = np.zeros(n, np.int32)
    nc = ctypes.c_int32(0)
    d1, d2 = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _gcheck(g, lib().okr_greedy_radialize(g, ctypes.byref(Y), ctypes.byref(loads), sup.ctypes.data,
                                          ctypes.byref(params), d_ws, kept.ctypes.data, kp.ctypes.data,
                                          ctypes.byref(nc), ctypes.byref(d1), ctypes.byref(d2)))
    return dict(kept_radial=kept, kept_parent=kp, n_critical=nc.value, dv_radial=d1.value, dv_meshed=d2.value)


def okr_greedy_destroy(g):
    return lib().okr_greedy_destroy(g)


class Greedy:
    """Plans once for a feeder's topology and scenario count, keeps its inputs
    on the device and runs Algorithm 1 (``run``) or scores a fixed
    assignment over the feeder's scenarios (``evaluate``)."""

    def __init__(self, f, device="cuda:0", vhat=None):
        import torch
        if not torch.cuda.is_available():
            raise OkrError(OKR.E_HIP, "no GPU visible: the search runs only on the HIP device")
        lib()
        self.torch = torch
        self.device = torch.device(device)
        n, S = int(f["n"]), int(np.asarray(f["S_load"]).shape[0])
        self.n, self.S = n, S

        def dev(a):
            t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))
            return torch.view_as_real(t).contiguous().to(self.device)

        with torch.cuda.device(self.device):
            self.Yd = dev(f["Y_diag"])
            self.Yo = dev(f["Y_off"])
            self.Sl = dev(f["S_load"])
            self.Vh = dev(vhat) if vhat is not None else None
            self.stream = torch.cuda.Stream(device=self.device)
            self.g = okr_greedy_create(ctypes.c_void_p(self.stream.cuda_stream))
            self.ws_bytes = okr_greedy_plan(self.g, f["parent"], f["phase"], S)
            self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=self.device)
        self.V0 = np.ascontiguousarray(f["V0"], dtype=np.complex128)
        self.Y = YBlocks(self.Yd.data_ptr(), self.Yo.data_ptr())
        self.loads = Loads(S, self.Sl.data_ptr(), self.V0.ctypes.data,
                           self.Vh.data_ptr() if self.Vh is not None else None)
        self.flags = OKR.FLAG_VHAT_GIVEN if vhat is not None else 0
        self.out_super = np.zeros(n, np.int32)
        self.out_steps = (GreedyStep * n)()
        self.out_err = np.zeros(S)
        self.res = GreedyResult(self.out_super.ctypes.data, ctypes.cast(self.out_steps, ctypes.c_void_p),
                                self.out_err.ctypes.data)

    def params(self, e_bar, max_iter=0, tie_tol=1e-11, amb_tol=1e-13, timing=False, incremental=False):
        flags = self.flags | (OKR.FLAG_TIMING if timing else 0) | (OKR.GREEDY_INCREMENTAL if incremental else 0)
        return GreedyParams(e_bar, tie_tol, amb_tol, max_iter, flags, 0.0, 0, 0)

    def run(self, e_bar, max_iter=0, tie_tol=1e-11, amb_tol=1e-13, timing=False, incremental=False):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        okr_greedy_run(self.g, self.Y, self.loads,
                       self.params(e_bar, max_iter, tie_tol, amb_tol, timing, incremental),
                       ctypes.c_void_p(self.ws.data_ptr()), self.res)
        r = self.res
        steps = [dict(cand=s.cand, s=s.s, r=s.r, smice=s.smice, emax=s.emax, ambiguous=bool(s.ambiguous),
                      n_cand=s.n_cand, n_feasible=s.n_feasible) for s in list(self.out_steps)[:r.n_steps]]
        return dict(super=self.out_super.copy(), steps=steps, err_per_snapshot=self.out_err.copy(),
                    n_steps=r.n_steps, n_kept=r.n_kept, max_err=r.max_err, t_pf_ms=r.t_pf_ms,
                    t_search_ms=r.t_search_ms, pf_iterations=r.pf_iterations,
                    n_score_launches=r.n_score_launches, t_score_ms=r.t_score_ms, n_scored=r.n_scored,
                    incremental=bool(r.incremental))

    def evaluate(self, sup):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        err = np.zeros(self.S)
        mx = okr_greedy_evaluate(self.g, self.Y, self.loads, sup, self.params(0.0),
                                 ctypes.c_void_p(self.ws.data_ptr()), err)
        return err, mx

    def radialize(self, sup):
        """Section V radialization of an assignment over this feeder."""
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        return okr_greedy_radialize(self.g, self.Y, self.loads, sup, self.params(0.0),
                                    ctypes.c_void_p(self.ws.data_ptr()))

    def close(self):
        if getattr(self, "g", None) is not None:
            okr_greedy_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def greedy(f, e_bar=None, device="cuda:0", vhat=None, max_iter=0, incremental=False):
    """Run Algorithm 1 once on a feeder dict and return the result dict."""
    G = Greedy(f, device=device, vhat=vhat)
    try:
        return G.run(f["e_bar"] if e_bar is None else e_bar, max_iter=max_iter, incremental=incremental)
    finally:
        G.close()


def evaluate_assignment(f, sup, device="cuda:0", vhat=None):
    """Largest error per scenario of a fixed assignment over f's scenarios."""
    G = Greedy(f, device=device, vhat=vhat)
    try:
        return G.evaluate(sup)
    finally:
        G.close()
