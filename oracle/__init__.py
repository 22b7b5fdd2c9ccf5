"""CPU FP64 oracle of the segment-exhaustive Kron-reduction search.

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg load this; the product path never does.  The C
source (okr_oracle.c) is the reference implementation; this module only
marshals numpy arrays into it.  Every function cites the part of the paper it
follows in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "okr_oracle.c")
_LIB = os.path.join(_HERE, "libokr_oracle.so")

OK = 0
W_BASE_OUT_OF_BAND = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math: plain IEEE FP64)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


class Decision(ctypes.Structure):
    _fields_ = [("segment", ctypes.c_int32), ("k", ctypes.c_int32),
                ("mask", ctypes.c_uint32), ("popcount", ctypes.c_int32),
                ("e_loc", ctypes.c_double), ("e_min", ctypes.c_double),
                ("ambiguous", ctypes.c_int32), ("n_scored", ctypes.c_int32),
                ("key_gap", ctypes.c_double), ("smice_rise", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _net(f):
    parent = np.ascontiguousarray(f["parent"], dtype=np.int32)
    phase = np.ascontiguousarray(f["phase"], dtype=np.uint8)
    segment = np.ascontiguousarray(f["segment"], dtype=np.int32)
    Yd = np.ascontiguousarray(f["Y_diag"], dtype=np.complex128)
    Yo = np.ascontiguousarray(f["Y_off"], dtype=np.complex128)
    return parent, phase, segment, Yd, Yo


def powerflow(f, tol=1e-13, maxit=100):
    """Scenario library (V^, I^) by the backward/forward sweep; returns
    (Vhat[S,n,3], Ihat[S,n,3], status, iterations)."""
    parent, phase, _, Yd, Yo = _net(f)
    S = np.ascontiguousarray(f["S_load"], dtype=np.complex128)
    V0 = np.ascontiguousarray(f["V0"], dtype=np.complex128)
    nS, n = S.shape[0], S.shape[1]
    Vhat = np.zeros((nS, n, 3), dtype=np.complex128)
    Ihat = np.zeros_like(Vhat)
    it = ctypes.c_int(0)
    st = lib().okro_powerflow(ctypes.c_int(n), _p(parent), _p(phase), _p(Yd), _p(Yo),
                              ctypes.c_int(nS), _p(S), _p(V0), ctypes.c_double(tol),
                              ctypes.c_int(maxit), _p(Vhat), _p(Ihat), ctypes.byref(it))
    return Vhat, Ihat, st, it.value


def candidate_voltages(f, Ihat, keep):
    """V^c for a kept set (Kron route with the slack fixed)."""
    parent, phase, _, Yd, Yo = _net(f)
    Ihat = np.ascontiguousarray(Ihat, dtype=np.complex128)
    V0 = np.ascontiguousarray(f["V0"], dtype=np.complex128)
    keep = np.ascontiguousarray(keep, dtype=np.uint8)
    nS, n = Ihat.shape[0], Ihat.shape[1]
    Vc = np.zeros((nS, n, 3), dtype=np.complex128)
    st = lib().okro_candidate_voltages(ctypes.c_int(n), _p(parent), _p(phase), _p(Yd), _p(Yo),
                                       ctypes.c_int(nS), _p(Ihat), _p(V0), _p(keep), _p(Vc))
    if st != OK:
        raise RuntimeError(f"okro_candidate_voltages failed: {st}")
    return Vc


def kron_blocks(f, keep):
    """Radial blocks of Y_Kron for a kept set: (kp, Yk_diag, Yk_off, extra)."""
    parent, phase, _, Yd, Yo = _net(f)
    keep = np.ascontiguousarray(keep, dtype=np.uint8)
    n = len(parent)
    kp = np.zeros(n, dtype=np.int32)
    Ykd = np.zeros((n, 3, 3), dtype=np.complex128)
    Yko = np.zeros((n, 3, 3), dtype=np.complex128)
    extra = ctypes.c_int(0)
    st = lib().okro_kron_blocks(ctypes.c_int(n), _p(parent), _p(phase), _p(Yd), _p(Yo),
                                _p(keep), _p(kp), _p(Ykd), _p(Yko), ctypes.byref(extra))
    if st != OK:
        raise RuntimeError(f"okro_kron_blocks failed: {st}")
    return kp, Ykd, Yko, extra.value


def score_masks(f, Vhat, Ihat, keep_before, g, masks):
    """Score explicit masks of segment g against a kept state."""
    parent, phase, segment, Yd, Yo = _net(f)
    Vhat = np.ascontiguousarray(Vhat, dtype=np.complex128)
    Ihat = np.ascontiguousarray(Ihat, dtype=np.complex128)
    V0 = np.ascontiguousarray(f["V0"], dtype=np.complex128)
    keep = np.ascontiguousarray(keep_before, dtype=np.uint8)
    masks = np.ascontiguousarray(masks, dtype=np.uint32)
    m = len(masks)
    out = {k: np.zeros(m) for k in ("e_glob", "e_loc", "slack_glob", "slack_loc", "smice")}
    feas = np.zeros(m, dtype=np.int32)
    nS, n = Vhat.shape[0], Vhat.shape[1]
    st = lib().okro_score_masks(
        ctypes.c_int(n), _p(parent), _p(phase), _p(segment), _p(Yd), _p(Yo),
        ctypes.c_int(nS), _p(Vhat), _p(Ihat), _p(V0), _p(keep), ctypes.c_int(g),
        _p(masks), ctypes.c_int(m), ctypes.c_double(f["e_bar"]),
        ctypes.c_double(f["v_min"]), ctypes.c_double(f["v_max"]),
        _p(out["e_glob"]), _p(out["e_loc"]), _p(out["slack_glob"]), _p(out["slack_loc"]),
        _p(feas), _p(out["smice"]))
    if st != OK:
        raise RuntimeError(f"okro_score_masks failed: {st}")
    out["feasible"] = feas.astype(bool)
    return out


def omega(f, keep, g):
    """Omega_g of segment g against the kept flags `keep` (bool [n])."""
    parent, phase, segment, Yd, Yo = _net(f)
    keep = np.ascontiguousarray(keep, dtype=np.uint8)
    n = len(parent)
    om = np.zeros(n, dtype=np.uint8)
    st = lib().okro_omega(ctypes.c_int(n), _p(parent), _p(phase), _p(segment), _p(Yd), _p(Yo),
                          _p(keep), ctypes.c_int(g), _p(om))
    if st != OK:
        raise RuntimeError(f"okro_omega failed: {st}")
    return om.astype(bool)


def search(f, Vhat, Ihat, tie_tol=1e-11, amb_tol=1e-13, mode=1, secondary="maxerr", smice_tol=1e-9):
    """Full segment-exhaustive search.  Returns (keep, decisions, status).
    secondary: the key among the most-reducing feasible masks, "maxerr"
    (eq. iter_obj) or "smice" (Algorithm 1's sum of MICE)."""
    sec = {"maxerr": 0, "smice": 1}[secondary]
    parent, phase, segment, Yd, Yo = _net(f)
    Vhat = np.ascontiguousarray(Vhat, dtype=np.complex128)
    Ihat = np.ascontiguousarray(Ihat, dtype=np.complex128)
    V0 = np.ascontiguousarray(f["V0"], dtype=np.complex128)
    nS, n = Vhat.shape[0], Vhat.shape[1]
    nseg_max = int(segment.max()) + 1 if len(segment) else 0
    keep = np.ones(n, dtype=np.uint8)
    dec = (Decision * max(nseg_max, 1))()
    nseg = ctypes.c_int(0)
    st = lib().okro_search(
        ctypes.c_int(n), _p(parent), _p(phase), _p(segment), _p(Yd), _p(Yo),
        ctypes.c_int(nS), _p(Vhat), _p(Ihat), _p(V0), ctypes.c_double(f["e_bar"]),
        ctypes.c_double(f["v_min"]), ctypes.c_double(f["v_max"]),
        ctypes.c_double(tie_tol), ctypes.c_double(amb_tol), ctypes.c_int(mode),
        ctypes.c_int(sec), ctypes.c_double(smice_tol), _p(keep), dec, ctypes.c_int(max(nseg_max, 1)),
        ctypes.byref(nseg))
    if st < 0:
        raise RuntimeError(f"okro_search failed: {st}")
    decs = [dict(segment=d.segment, k=d.k, mask=d.mask, popcount=d.popcount,
                 e_loc=d.e_loc, e_min=d.e_min, ambiguous=bool(d.ambiguous),
                 n_scored=d.n_scored, key_gap=d.key_gap, smice_rise=d.smice_rise)
            for d in list(dec)[:nseg.value]]
    return keep, decs, st


class _RTopology(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("parent", ctypes.c_void_p), ("phase", ctypes.c_void_p),
                ("eligible", ctypes.c_void_p), ("segment", ctypes.c_void_p)]


class _RYBlocks(ctypes.Structure):
    _fields_ = [("Y_diag", ctypes.c_void_p), ("Y_off", ctypes.c_void_p)]


class _RLoads(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int32), ("S_load", ctypes.c_void_p), ("V0", ctypes.c_void_p),
                ("Vhat", ctypes.c_void_p)]


class _RMargins(ctypes.Structure):
    _fields_ = [("e_bar", ctypes.c_double), ("v_min", ctypes.c_double), ("v_max", ctypes.c_double),
                ("tie_tol", ctypes.c_double), ("amb_tol", ctypes.c_double), ("pf_tol", ctypes.c_double),
                ("pf_maxit", ctypes.c_int32), ("secondary", ctypes.c_int32), ("smice_tol", ctypes.c_double)]


class _RResult(ctypes.Structure):
    _fields_ = [("super", ctypes.c_void_p), ("kept_parent", ctypes.c_void_p), ("Yk_diag", ctypes.c_void_p),
                ("Yk_off", ctypes.c_void_p), ("err_per_snapshot", ctypes.c_void_p), ("Vhat", ctypes.c_void_p),
                ("seg", ctypes.c_void_p), ("n_segments", ctypes.c_int32), ("n_kept", ctypes.c_int32),
                ("max_err", ctypes.c_double)]


def reduce_feeder(f, vhat=None, tie_tol=1e-11, amb_tol=1e-13, secondary="maxerr", smice_tol=1e-9,
                  pf_tol=1e-13, pf_maxit=100):
    """The whole reduction in one call (okr_oracle_reduce_feeder): load flow
    (or the given scenario voltages), the segment search, the Kron-reduced
    radial blocks and the final errors, in the result layout of the GPU
    library's reduce_feeder."""
    parent, phase, segment, Yd, Yo = _net(f)
    eligible = np.ascontiguousarray(f.get("eligible", segment >= 0), dtype=np.uint8)
    S_load = np.ascontiguousarray(f["S_load"], dtype=np.complex128)
    V0 = np.ascontiguousarray(f["V0"], dtype=np.complex128)
    nS, n = S_load.shape[0], S_load.shape[1]
    vh_in = None if vhat is None else np.ascontiguousarray(vhat, dtype=np.complex128)
    nseg = int(segment.max()) + 1 if len(segment) and segment.max() >= 0 else 0
    out = dict(super=np.zeros(n, np.int32), kept_parent=np.zeros(n, np.int32),
               Yk_diag=np.zeros((n, 3, 3), np.complex128), Yk_off=np.zeros((n, 3, 3), np.complex128),
               err_per_snapshot=np.zeros(nS), Vhat=np.zeros((nS, n, 3), np.complex128))
    dec = (Decision * max(nseg, 1))()
    T = _RTopology(n, parent.ctypes.data, phase.ctypes.data, eligible.ctypes.data, segment.ctypes.data)
    Y = _RYBlocks(Yd.ctypes.data, Yo.ctypes.data)
    L = _RLoads(nS, S_load.ctypes.data, V0.ctypes.data, None if vh_in is None else vh_in.ctypes.data)
    M = _RMargins(f["e_bar"], f["v_min"], f["v_max"], tie_tol, amb_tol, pf_tol, pf_maxit,
                  {"maxerr": 0, "smice": 1}[secondary], smice_tol)
    R = _RResult(out["super"].ctypes.data, out["kept_parent"].ctypes.data, out["Yk_diag"].ctypes.data,
                 out["Yk_off"].ctypes.data, out["err_per_snapshot"].ctypes.data, out["Vhat"].ctypes.data,
                 ctypes.addressof(dec), 0, 0, 0.0)
    st = lib().okr_oracle_reduce_feeder(ctypes.byref(Y), ctypes.byref(T), ctypes.byref(L), ctypes.byref(M),
                                        ctypes.byref(R))
    if st < 0:
        raise RuntimeError(f"okr_oracle_reduce_feeder failed: {st}")
    out.update(status=st, n_kept=R.n_kept, max_err=R.max_err,
               kept=(out["super"] == np.arange(n)).astype(np.uint8),
               segments=[dict(segment=d.segment, k=d.k, mask=d.mask, popcount=d.popcount, e_loc=d.e_loc,
                              e_min=d.e_min, ambiguous=bool(d.ambiguous), n_scored=d.n_scored,
                              key_gap=d.key_gap, smice_rise=d.smice_rise) for d in list(dec)[:R.n_segments]])
    return out


def final_errors(f, Vhat, Ihat, keep):
    parent, phase, _, Yd, Yo = _net(f)
    Vhat = np.ascontiguousarray(Vhat, dtype=np.complex128)
    Ihat = np.ascontiguousarray(Ihat, dtype=np.complex128)
    V0 = np.ascontiguousarray(f["V0"], dtype=np.complex128)
    keep = np.ascontiguousarray(keep, dtype=np.uint8)
    nS, n = Vhat.shape[0], Vhat.shape[1]
    err = np.zeros(nS)
    Vc = np.zeros((nS, n, 3), dtype=np.complex128)
    st = lib().okro_final_errors(ctypes.c_int(n), _p(parent), _p(phase), _p(Yd), _p(Yo),
                                 ctypes.c_int(nS), _p(Vhat), _p(Ihat), _p(V0), _p(keep),
                                 _p(err), _p(Vc))
    if st != OK:
        raise RuntimeError(f"okro_final_errors failed: {st}")
    return err, Vc


def pinv3(A, mask):
    """Restricted pseudo-inverse of one 3x3 block (present phases in mask)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    out = np.zeros((3, 3), dtype=np.complex128)
    st = lib().okro_pinv3(_p(A), ctypes.c_uint(mask), _p(out))
    if st != OK:
        raise RuntimeError("singular block")
    return out
