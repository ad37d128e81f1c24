"""CPU oracle for the MAP forward-backward decoder (FP64, plain C).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It wraps
``libmapdec_ref.so`` (built from ``mapdec_ref.c`` with gcc) through ctypes
and shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MAPDEC_REF_LIB lets a mutation check load a deliberately broken copy
LIB_PATH = os.environ.get("MAPDEC_REF_LIB", os.path.join(_HERE, "libmapdec_ref.so"))
SOURCES = [os.path.join(_HERE, "mapdec_ref.c")]

REF_OK, REF_EINVAL, REF_EDRIFT, REF_ENOPATH, REF_ENOMEM = 0, 1, 2, 3, 4


def build(path: str = LIB_PATH, opt=("-O2",)) -> str:
    """Compile the oracle with gcc (portable flags by default: the library
    also runs on other hosts)."""
    cmd = ["gcc", *opt, "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", path] + SOURCES + ["-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    return path


def load_build(path: str, opt) -> None:
    """Builds the same sources with other compiler flags (e.g. -O3
    -march=native for timing on the host that runs them) into ``path`` and
    makes every later call use that build."""
    global _lib, LIB_PATH
    build(path, tuple(opt))
    _lib = None
    LIB_PATH = path


class _Code(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("n", ctypes.c_int),
                ("codebook", ctypes.POINTER(ctypes.c_uint8)),
                ("Pi", ctypes.c_double), ("Pd", ctypes.c_double), ("Ps", ctypes.c_double),
                ("I", ctypes.c_int), ("M", ctypes.c_int), ("mn", ctypes.c_int)]


class _GCode(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("n", ctypes.c_int), ("ncb", ctypes.c_int),
                ("codebooks", ctypes.POINTER(ctypes.c_uint8)),
                ("Pi", ctypes.c_double), ("Pd", ctypes.c_double), ("Ps", ctypes.c_double),
                ("I", ctypes.c_int), ("mt_lo", ctypes.c_int), ("mt_hi", ctypes.c_int),
                ("mn_lo", ctypes.c_int), ("mn_hi", ctypes.c_int)]


_dp = ctypes.POINTER(ctypes.c_double)


class _Out(ctypes.Structure):
    _fields_ = [("app", _dp), ("logp", _dp), ("dparams", _dp), ("dprior", _dp),
                ("alpha", _dp), ("beta", _dp), ("logA", _dp), ("logB", _dp), ("logZ", _dp)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.mapdec_ref_run.argtypes = [ctypes.POINTER(_Code), ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_uint8), _dp, ctypes.c_int,
                                     ctypes.POINTER(_Out)]
        L.mapdec_ref_run.restype = ctypes.c_int
        L.mapdec_ref_run_drift.argtypes = [ctypes.POINTER(_Code), ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_uint8), _dp, _dp, _dp,
                                           ctypes.c_int, ctypes.POINTER(_Out)]
        L.mapdec_ref_run_drift.restype = ctypes.c_int
        L.mapdec_ref_lattice.argtypes = [ctypes.POINTER(_Code), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_uint8), ctypes.c_int,
                                         ctypes.c_int, _dp, _dp]
        L.mapdec_ref_lattice.restype = ctypes.c_int
        L.mapdec_ref_check.argtypes = [ctypes.POINTER(_Code)]
        L.mapdec_ref_check.restype = ctypes.c_int
        L.mapdec_ref_gcheck.argtypes = [ctypes.POINTER(_GCode), ctypes.c_int]
        L.mapdec_ref_gcheck.restype = ctypes.c_int
        L.mapdec_ref_run_general.argtypes = [ctypes.POINTER(_GCode), ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_uint8), _dp, _dp, _dp,
                                             ctypes.c_int, ctypes.POINTER(_Out)]
        L.mapdec_ref_run_general.restype = ctypes.c_int
        L.mapdec_ref_glattice.argtypes = [ctypes.POINTER(_GCode), ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_uint8), ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.mapdec_ref_glattice.restype = ctypes.c_int
        L.mapdec_ref_run_pruned.argtypes = [ctypes.POINTER(_GCode), ctypes.c_int, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_uint8), _dp, _dp, _dp,
                                            ctypes.c_double, ctypes.POINTER(_Out)]
        L.mapdec_ref_run_pruned.restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, status: int):
        names = {1: "EINVAL", 2: "EDRIFT", 3: "ENOPATH", 4: "ENOMEM"}
        super().__init__(f"oracle status {names.get(status, status)}")
        self.status = status


def _ptr(a: Optional[np.ndarray], ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _code(codebook, Pi, Pd, Ps, I, M, mn):
    cb = np.ascontiguousarray(codebook, dtype=np.uint8)
    q, n = cb.shape
    c = _Code(q, n, _ptr(cb, ctypes.c_uint8), float(Pi), float(Pd), float(Ps), int(I),
              int(M), int(mn))
    return c, cb


def decode(codebook, y, N, Pi, Pd, Ps, I, M, mn, prior=None, *, start=None, end=None,
           grad=False, trace=False, literal=False, check=True, extrinsic=False):
    """Run the oracle on one frame.  Returns a dict with ``status``, ``logp``,
    ``app`` (N, q) and, on request, ``dparams`` (3,) and ``dprior`` (N, q)
    (grad), ``dprior`` alone (extrinsic: the inner decoder's output for
    iterative decoding, without the gradient's tangents) and
    the trace arrays ``alpha``, ``beta`` ((N+1), 2M+1), ``logA``, ``logB``,
    ``logZ``.  ``start`` / ``end``: priors of the frame's start and end
    drift over [-M, M] (entry m + M), or None for the known boundary."""
    c, cb = _code(codebook, Pi, Pd, Ps, I, M, mn)
    q = c.q
    yb = np.ascontiguousarray(y, dtype=np.uint8)
    pr = None if prior is None else np.ascontiguousarray(prior, dtype=np.float64)
    Mt = 2 * M + 1
    bnd = []
    for v in (start, end):
        if v is not None:
            v = np.ascontiguousarray(v, dtype=np.float64)
            if v.shape != (Mt,):
                raise ValueError(f"drift prior must have 2M+1 = {Mt} entries")
        bnd.append(v)
    res = {"app": np.zeros((N, q)), "logp": np.zeros(1)}
    if grad:
        res["dparams"] = np.zeros(3)
    if grad or extrinsic:
        res["dprior"] = np.zeros((N, q))
    if trace:
        res["alpha"] = np.zeros((N + 1, Mt))
        res["beta"] = np.zeros((N + 1, Mt))
        res["logA"] = np.zeros(N + 1)
        res["logB"] = np.zeros(N + 1)
        res["logZ"] = np.zeros(N)
    out = _Out(*[_ptr(res.get(k), ctypes.c_double) for k in
                 ("app", "logp", "dparams", "dprior", "alpha", "beta", "logA", "logB", "logZ")])
    st = lib().mapdec_ref_run_drift(ctypes.byref(c), int(N), int(yb.shape[0]),
                                    _ptr(yb, ctypes.c_uint8) if yb.size else None,
                                    _ptr(pr, ctypes.c_double), _ptr(bnd[0], ctypes.c_double),
                                    _ptr(bnd[1], ctypes.c_double), int(bool(literal)),
                                    ctypes.byref(out))
    if st and check:
        raise OracleError(st)
    res["status"] = st
    res["logp"] = float(res["logp"][0])
    return res


def _gcode(codebooks, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi):
    cb = np.ascontiguousarray(codebooks, dtype=np.uint8)
    if cb.ndim == 2:
        cb = cb[None]
    ncb, q, n = cb.shape
    c = _GCode(q, n, ncb, _ptr(cb, ctypes.c_uint8), float(Pi), float(Pd), float(Ps), int(I),
               int(mt_lo), int(mt_hi), int(mn_lo), int(mn_hi))
    return c, cb


def decode_general(codebooks, y, N, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi, prior=None, *,
                   start=None, end=None, grad=False, trace=False, literal=False, check=True,
                   theta=0.0):
    """Oracle decode under the general scheme: ``codebooks`` is (q, n) (one
    codebook) or (N, q, n) (C_i per symbol); drift states lie in [mt_lo,
    mt_hi], drift changes in [mn_lo, mn_hi].  Rows and drift priors have
    mt_hi - mt_lo + 1 entries, entry m - mt_lo.  Same outputs as decode().
    ``theta`` > 0: path thresholds (mapdec_ref_run_pruned)."""
    c, cb = _gcode(codebooks, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi)
    q = c.q
    yb = np.ascontiguousarray(y, dtype=np.uint8)
    pr = None if prior is None else np.ascontiguousarray(prior, dtype=np.float64)
    Mt = mt_hi - mt_lo + 1
    bnd = []
    for v in (start, end):
        if v is not None:
            v = np.ascontiguousarray(v, dtype=np.float64)
            if v.shape != (Mt,):
                raise ValueError(f"drift prior must have mt_hi - mt_lo + 1 = {Mt} entries")
        bnd.append(v)
    res = {"app": np.zeros((N, q)), "logp": np.zeros(1)}
    if grad:
        res["dparams"] = np.zeros(3)
        res["dprior"] = np.zeros((N, q))
    if trace:
        res["alpha"] = np.zeros((N + 1, Mt))
        res["beta"] = np.zeros((N + 1, Mt))
        res["logA"] = np.zeros(N + 1)
        res["logB"] = np.zeros(N + 1)
        res["logZ"] = np.zeros(N)
    out = _Out(*[_ptr(res.get(k), ctypes.c_double) for k in
                 ("app", "logp", "dparams", "dprior", "alpha", "beta", "logA", "logB", "logZ")])
    if theta:
        st = lib().mapdec_ref_run_pruned(ctypes.byref(c), int(N), int(yb.shape[0]),
                                         _ptr(yb, ctypes.c_uint8) if yb.size else None,
                                         _ptr(pr, ctypes.c_double),
                                         _ptr(bnd[0], ctypes.c_double),
                                         _ptr(bnd[1], ctypes.c_double), float(theta),
                                         ctypes.byref(out))
    else:
        st = lib().mapdec_ref_run_general(ctypes.byref(c), int(N), int(yb.shape[0]),
                                          _ptr(yb, ctypes.c_uint8) if yb.size else None,
                                          _ptr(pr, ctypes.c_double),
                                          _ptr(bnd[0], ctypes.c_double),
                                          _ptr(bnd[1], ctypes.c_double), int(bool(literal)),
                                          ctypes.byref(out))
    if st and check:
        raise OracleError(st)
    res["status"] = st
    res["logp"] = float(res["logp"][0])
    return res


def glattice(codebooks, y, N, i, s, D, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi,
             tangents=False):
    """R(s, C_i(D), delta) for delta in [mn_lo, mn_hi] under the general
    scheme (and tangents [w][k])."""
    c, cb = _gcode(codebooks, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi)
    yb = np.ascontiguousarray(y, dtype=np.uint8)
    Mn = mn_hi - mn_lo + 1
    R = np.zeros(Mn)
    dR = np.zeros((4, Mn)) if tangents else None
    st = lib().mapdec_ref_glattice(ctypes.byref(c), int(N), int(yb.shape[0]),
                                   _ptr(yb, ctypes.c_uint8) if yb.size else None, int(i), int(s),
                                   int(D), _ptr(R, ctypes.c_double), _ptr(dR, ctypes.c_double))
    if st:
        raise OracleError(st)
    return (R, dR) if tangents else R


def check_general(codebooks, N, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi) -> int:
    c, cb = _gcode(codebooks, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi)
    return lib().mapdec_ref_gcheck(ctypes.byref(c), int(N))


def decode_frame(fr, **kw):
    """Oracle decode of a :class:`paper_1802_08483_amd.workloads.Frame`.
    Frames of the general scheme (``codebooks`` or ``limits`` set) or with
    path thresholds (``theta`` > 0) go through decode_general; their drift
    priors, given over [-M, M], are cut to [mt_lo, mt_hi] (the entries
    outside are ignored by definition)."""
    cbs = getattr(fr, "codebooks", None)
    lim = getattr(fr, "limits", None)
    theta = getattr(fr, "theta", 0.0) or 0.0
    if theta:
        kw.setdefault("theta", theta)
    if cbs is None and lim is None and not theta:
        kw.setdefault("start", getattr(fr, "start_drift", None))
        kw.setdefault("end", getattr(fr, "end_drift", None))
        return decode(fr.codebook, fr.y, fr.N, fr.Pi, fr.Pd, fr.Ps, fr.I, fr.M, fr.mn,
                      prior=fr.prior, **kw)
    lim = lim if lim is not None else (-fr.M, fr.M, -fr.mn, fr.mn)
    for key, attr in (("start", "start_drift"), ("end", "end_drift")):
        v = getattr(fr, attr, None)
        if key not in kw and v is not None:
            kw[key] = np.asarray(v, dtype=np.float64)[lim[0] + fr.M: lim[1] + fr.M + 1]
    res = decode_general(cbs if cbs is not None else fr.codebook, fr.y, fr.N, fr.Pi, fr.Pd,
                         fr.Ps, fr.I, *lim, prior=fr.prior, **kw)
    if "alpha" in res:   # rows over [-M, M] like decode()
        for k in ("alpha", "beta"):
            full = np.zeros((fr.N + 1, 2 * fr.M + 1))
            full[:, lim[0] + fr.M: lim[1] + fr.M + 1] = res[k]
            res[k] = full
    return res


def lattice(codebook, y, s, D, Pi, Pd, Ps, I, M, mn, tangents=False):
    """R(s, D, delta) for delta in [-mn, mn] (and tangents [w][k])."""
    c, cb = _code(codebook, Pi, Pd, Ps, I, M, mn)
    yb = np.ascontiguousarray(y, dtype=np.uint8)
    Mn = 2 * mn + 1
    R = np.zeros(Mn)
    dR = np.zeros((4, Mn)) if tangents else None
    st = lib().mapdec_ref_lattice(ctypes.byref(c), int(yb.shape[0]),
                                  _ptr(yb, ctypes.c_uint8) if yb.size else None, int(s),
                                  int(D), _ptr(R, ctypes.c_double), _ptr(dR, ctypes.c_double))
    if st:
        raise OracleError(st)
    return (R, dR) if tangents else R


def check_code(codebook, Pi, Pd, Ps, I, M, mn) -> int:
    c, cb = _code(codebook, Pi, Pd, Ps, I, M, mn)
    return lib().mapdec_ref_check(ctypes.byref(c))
