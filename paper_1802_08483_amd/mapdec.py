"""ctypes binding of libmapdec (include/mapdec.h).

Argument marshalling only: every step of the decode runs in the HIP
kernels of ``libmapdec.so``.  PyTorch supplies device memory and streams.
There is no CPU fallback: without the built library, or without a GPU,
calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmapdec.so")

OK, EINVAL, EDRIFT, ENOPATH, ENOMEM, ESIZE, EDEVICE, EUNSUPPORTED = range(8)
FP32, FP64 = 0, 1
FLAG_GRAD, FLAG_GRAPH, FLAG_SERIAL, FLAG_TUNE = 1, 2, 4, 8
MAX_N, MAX_MN = 16, 8

# every symbol include/mapdec.h declares
EXPORTS = ["mapdec_create", "mapdec_destroy", "mapdec_workspace_size", "mapdec_decode",
           "mapdec_grad", "mapdec_plan_create", "mapdec_plan_run", "mapdec_plan_destroy",
           "mapdec_plan_profile", "mapdec_plan_launches", "mapdec_phase_name",
           "mapdec_tune_entries",
           "mapdec_tune_reset", "mapdec_last_error",
           "mapdec_strerror", "mapdec_version", "mapdec_decode_noalloc",
           "mapdec_noalloc_limit", "mapdec_create_general", "mapdec_with_threshold",
           "mapdec_outer_create", "mapdec_outer_destroy", "mapdec_outer_workspace_size",
           "mapdec_outer_decode"]


class MapdecError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {strerror(status)}" if what else strerror(status))


class _Frame(ctypes.Structure):
    _fields_ = [("code", ctypes.c_void_p), ("N", ctypes.c_int32), ("rho", ctypes.c_int32),
                ("y", ctypes.c_void_p), ("prior", ctypes.c_void_p), ("app", ctypes.c_void_p),
                ("dprior", ctypes.c_void_p), ("start_drift", ctypes.c_void_p),
                ("end_drift", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "paper_1802_08483_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        fp = ctypes.POINTER(_Frame)
        L.mapdec_create.argtypes = [i32, i32, vp, dbl, dbl, dbl, i32, i32, i32]
        L.mapdec_create.restype = vp
        L.mapdec_create_general.argtypes = [i32, i32, i32, vp, dbl, dbl, dbl, i32, i32, i32,
                                            i32, i32]
        L.mapdec_create_general.restype = vp
        L.mapdec_with_threshold.argtypes = [vp, dbl]
        L.mapdec_with_threshold.restype = vp
        L.mapdec_destroy.argtypes = [vp]
        L.mapdec_destroy.restype = None
        L.mapdec_workspace_size.argtypes = [fp, i32, i32, i32, i32]
        L.mapdec_workspace_size.restype = sz
        L.mapdec_decode.argtypes = [fp, i32, vp, vp, vp, sz, i32, vp]
        L.mapdec_decode.restype = i32
        L.mapdec_grad.argtypes = [fp, i32, vp, vp, vp, vp, sz, i32, i32, vp]
        L.mapdec_grad.restype = i32
        L.mapdec_plan_create.argtypes = [fp, i32, vp, vp, vp, vp, sz, i32, i32, i32, vp]
        L.mapdec_plan_create.restype = vp
        L.mapdec_plan_run.argtypes = [vp, vp]
        L.mapdec_plan_run.restype = i32
        L.mapdec_plan_destroy.argtypes = [vp]
        L.mapdec_plan_destroy.restype = None
        L.mapdec_plan_profile.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_float), i32]
        L.mapdec_plan_profile.restype = i32
        L.mapdec_phase_name.argtypes = [i32]
        L.mapdec_phase_name.restype = ctypes.c_char_p
        L.mapdec_last_error.argtypes = []
        L.mapdec_last_error.restype = i32
        L.mapdec_strerror.argtypes = [i32]
        L.mapdec_strerror.restype = ctypes.c_char_p
        L.mapdec_version.argtypes = []
        L.mapdec_version.restype = i32
        L.mapdec_plan_launches.argtypes = [vp, i32]
        L.mapdec_plan_launches.restype = i32
        L.mapdec_tune_entries.argtypes = []
        L.mapdec_tune_entries.restype = i32
        L.mapdec_tune_reset.argtypes = []
        L.mapdec_tune_reset.restype = None
        L.mapdec_decode_noalloc.argtypes = [fp, i32, vp, vp, i32, vp]
        L.mapdec_decode_noalloc.restype = i32
        L.mapdec_noalloc_limit.argtypes = []
        L.mapdec_noalloc_limit.restype = sz
        L.mapdec_outer_create.argtypes = [i32, i32, i32, vp, vp, vp]
        L.mapdec_outer_create.restype = vp
        L.mapdec_outer_destroy.argtypes = [vp]
        L.mapdec_outer_destroy.restype = None
        L.mapdec_outer_workspace_size.argtypes = [vp, i32, i32]
        L.mapdec_outer_workspace_size.restype = sz
        L.mapdec_outer_decode.argtypes = [vp, i32, vp, vp, vp, i32, vp, sz, i32, vp]
        L.mapdec_outer_decode.restype = i32
        _lib = L
    return _lib


def tune_entries() -> int:
    """Buckets in the process's table of tuned launch choices."""
    return lib().mapdec_tune_entries()


def noalloc_limit() -> int:
    """Bytes of the device array behind mapdec_decode_noalloc."""
    return int(lib().mapdec_noalloc_limit())


def tune_reset() -> None:
    """Empties the process's table of tuned launch choices."""
    lib().mapdec_tune_reset()


def strerror(status: int) -> str:
    return lib().mapdec_strerror(int(status)).decode()


class Code:
    """Owns a ``mapdec_code`` handle (host-only, immutable).

    ``limits`` = (mt_lo, mt_hi, mn_lo, mn_hi) and/or a codebook array of
    shape (N, q, n) (codebook i for symbol i) select the general scheme
    (mapdec_create_general); ``M`` and ``mn`` are then ignored and become
    max(-mt_lo, mt_hi) and max(-mn_lo, mn_hi).  ``theta`` > 0: path
    thresholds (mapdec_with_threshold)."""

    def __init__(self, codebook, Pi: float, Pd: float, Ps: float, I: int, M: int = 0,
                 mn: int = 0, limits=None, theta: float = 0.0):
        import numpy as np
        cb = np.ascontiguousarray(np.asarray(codebook, dtype=np.uint8))
        if cb.ndim not in (2, 3):
            raise ValueError("codebook must be (q, n) or (N, q, n)")
        self.q, self.n = int(cb.shape[-2]), int(cb.shape[-1])
        self.ncb = int(cb.shape[0]) if cb.ndim == 3 else 1
        self.Pi, self.Pd, self.Ps = float(Pi), float(Pd), float(Ps)
        self.I = int(I)
        if limits is None and cb.ndim == 2:
            self.M, self.mn = int(M), int(mn)
            self.limits = (-self.M, self.M, -self.mn, self.mn)
            self._h = lib().mapdec_create(self.q, self.n, cb.ctypes.data, self.Pi, self.Pd,
                                          self.Ps, self.I, self.M, self.mn)
            what = "mapdec_create"
        else:
            lim = tuple(int(v) for v in (limits if limits is not None else (-M, M, -mn, mn)))
            self.limits = lim
            self.M, self.mn = max(-lim[0], lim[1]), max(-lim[2], lim[3])
            self._h = lib().mapdec_create_general(self.q, self.n, self.ncb, cb.ctypes.data,
                                                  self.Pi, self.Pd, self.Ps, self.I, *lim)
            what = "mapdec_create_general"
        if not self._h:
            raise MapdecError(lib().mapdec_last_error(), what)
        self.theta = float(theta)
        if self.theta:
            h = lib().mapdec_with_threshold(self._h, self.theta)
            lib().mapdec_destroy(self._h)
            self._h = h
            if not self._h:
                raise MapdecError(lib().mapdec_last_error(), "mapdec_with_threshold")

    @property
    def handle(self) -> int:
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().mapdec_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Batch:
    """Device buffers and frame table for a batch of frames.

    ``frames``: sequence of (code, y, N, prior) or (code, y, N, prior, start,
    end) with ``y`` a uint8 CUDA tensor of 0/1, ``prior`` an (N, q) CUDA
    tensor of the batch precision or None (uniform), and ``start`` / ``end``
    float64 CUDA tensors of 2M+1 entries, the priors of the frame's start and
    end drift (Sec. II-C), or None for the known boundary.  Allocates the outputs (APP per frame, log P, status,
    gradient buffers) and the workspace, sized for forward checkpoints every
    ``checkpoint_K`` symbols (0: none), which every run of the batch uses.
    """

    def __init__(self, frames: Sequence, precision: int = FP32, grad: bool = False,
                 device=None, checkpoint_K: int = 0, workspace: bool = True,
                 dpriors: Optional[Sequence] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("libmapdec needs a GPU; no device is visible")
        self.device = torch.device(device or "cuda")
        self.precision = precision
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        self.grad = grad
        self.codes = []
        self.ys, self.priors, self.apps, self.dpriors = [], [], [], []
        self.bounds = []
        arr = (_Frame * len(frames))()
        for f, item in enumerate(frames):
            code, y, N, prior = item[:4]
            start, end = (item[4], item[5]) if len(item) > 4 else (None, None)
            for v in (start, end):
                if v is not None and (v.dtype != torch.float64 or not v.is_cuda
                                      or tuple(v.shape) != (2 * code.M + 1,)):
                    raise TypeError("drift priors must be float64 CUDA tensors of 2M+1 entries")
            start = None if start is None else start.contiguous()
            end = None if end is None else end.contiguous()
            self.bounds.append((start, end))
            if y.dtype != torch.uint8 or not y.is_cuda:
                raise TypeError("y must be a uint8 CUDA tensor")
            y = y.contiguous()
            if prior is not None:
                if prior.dtype != self.dtype or tuple(prior.shape) != (N, code.q):
                    raise TypeError("prior must be (N, q) in the batch precision")
                prior = prior.contiguous()
            app = torch.empty((N, code.q), dtype=self.dtype, device=self.device)
            if dpriors is not None:   # the caller's (N, q) output buffers (iterative decoding)
                dpr = dpriors[f]
                if (dpr.dtype != self.dtype or tuple(dpr.shape) != (N, code.q)
                        or not dpr.is_contiguous()):
                    raise TypeError("dprior buffers must be contiguous (N, q) in the batch precision")
            else:
                dpr = torch.empty((N, code.q), dtype=self.dtype, device=self.device) if grad else None
            self.codes.append(code)
            self.ys.append(y)
            self.priors.append(prior)
            self.apps.append(app)
            self.dpriors.append(dpr)
            arr[f] = _Frame(code.handle, int(N), int(y.numel()), _ptr(y), _ptr(prior),
                            _ptr(app), _ptr(dpr), _ptr(start), _ptr(end))
        self.frames = arr
        self.nframes = len(frames)
        self.logp = torch.empty(self.nframes, dtype=torch.float64, device=self.device)
        self.status = torch.empty(self.nframes, dtype=torch.int32, device=self.device)
        self.dparams = (torch.empty((self.nframes, 3), dtype=torch.float64, device=self.device)
                        if grad else None)
        flags = FLAG_GRAD if grad else 0
        self.checkpoint_K = int(checkpoint_K)
        self.ws_bytes = lib().mapdec_workspace_size(self.frames, self.nframes, precision, flags,
                                                    self.checkpoint_K)
        if self.ws_bytes == 0:
            raise MapdecError(EINVAL, "mapdec_workspace_size")
        # workspace=False: the batch is decoded only by decode_noalloc()
        self.ws = (torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
                   if workspace else None)

    def decode(self, stream=None):
        if self.checkpoint_K:
            # mapdec_decode keeps whole frames; checkpointed runs go through a plan
            p = Plan(self, graph=False, stream=stream)
            p.run(stream)
            p.close()
            return self
        st = lib().mapdec_decode(self.frames, self.nframes, _ptr(self.logp), _ptr(self.status),
                                 _ptr(self.ws), self.ws_bytes, self.precision,
                                 _stream_handle(stream))
        if st:
            raise MapdecError(st, "mapdec_decode")
        return self

    def decode_noalloc(self, stream=None):
        """mapdec_decode_noalloc: the decode in the library's fixed device
        array instead of the batch's workspace (at most noalloc_limit()
        bytes)."""
        st = lib().mapdec_decode_noalloc(self.frames, self.nframes, _ptr(self.logp),
                                         _ptr(self.status), self.precision,
                                         _stream_handle(stream))
        if st:
            raise MapdecError(st, "mapdec_decode_noalloc")
        return self

    def run_grad(self, stream=None):
        if not self.grad:
            raise RuntimeError("batch was built without gradient buffers")
        st = lib().mapdec_grad(self.frames, self.nframes, _ptr(self.logp), _ptr(self.dparams),
                               _ptr(self.status), _ptr(self.ws), self.ws_bytes, self.checkpoint_K,
                               self.precision, _stream_handle(stream))
        if st:
            raise MapdecError(st, "mapdec_grad")
        return self

    def plan(self, graph: bool = True, stream=None, serial: bool = False,
             tune: bool = False) -> "Plan":
        return Plan(self, graph=graph, stream=stream, serial=serial, tune=tune)


class Plan:
    """A ``mapdec_plan``: the batch's launches recorded once, replayed by run()."""

    def __init__(self, batch: Batch, graph: bool = True, stream=None, serial: bool = False,
                 tune: bool = False):
        self.batch = batch
        flags = ((FLAG_GRAPH if graph else 0) | (FLAG_GRAD if batch.grad else 0) |
                 (FLAG_SERIAL if serial else 0) | (FLAG_TUNE if tune else 0))
        self._h = lib().mapdec_plan_create(batch.frames, batch.nframes, _ptr(batch.logp),
                                           _ptr(batch.dparams), _ptr(batch.status),
                                           _ptr(batch.ws), batch.ws_bytes, batch.precision,
                                           flags, batch.checkpoint_K, _stream_handle(stream))
        if not self._h:
            raise MapdecError(lib().mapdec_last_error(), "mapdec_plan_create")

    def run(self, stream=None):
        st = lib().mapdec_plan_run(self._h, _stream_handle(stream))
        if st:
            raise MapdecError(st, "mapdec_plan_run")

    def profile(self, stream=None) -> dict:
        """One eager run in the plan's eager schedule with timing events
        around every launch: {phase: sum of its launches' ms}."""
        buf = (ctypes.c_float * 16)()
        n = lib().mapdec_plan_profile(self._h, _stream_handle(stream), buf, 16)
        if n < 0:
            raise MapdecError(-n, "mapdec_plan_profile")
        return {lib().mapdec_phase_name(k).decode(): float(buf[k]) for k in range(n)}

    def launches(self) -> dict:
        """{phase: number of launches in one run}."""
        out, k = {}, 0
        while True:
            name = lib().mapdec_phase_name(k)
            if name is None:
                return out
            out[name.decode()] = lib().mapdec_plan_launches(self._h, k)
            k += 1

    def close(self):
        if getattr(self, "_h", None):
            lib().mapdec_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def code_for(frame, cache: Optional[dict] = None) -> Code:
    """A :class:`Code` for a workloads.Frame (shared when the parameters match)."""
    cbs = getattr(frame, "codebooks", None)
    cb = frame.codebook if cbs is None else cbs
    lim = getattr(frame, "limits", None)
    theta = getattr(frame, "theta", 0.0) or 0.0
    key = (cb.tobytes(), cb.shape, frame.Pi, frame.Pd, frame.Ps, frame.I, frame.M, frame.mn,
           lim, theta)
    if cache is not None and key in cache:
        return cache[key]
    c = Code(cb, frame.Pi, frame.Pd, frame.Ps, frame.I, frame.M, frame.mn, limits=lim,
             theta=theta)
    if cache is not None:
        cache[key] = c
    return c


def batch_from_frames(frames: List, precision: int = FP32, grad: bool = False,
                      device=None, checkpoint_K: int = 0, workspace: bool = True) -> Batch:
    """Uploads workloads.Frame objects and builds a :class:`Batch`."""
    dev = torch.device(device or "cuda")
    dtype = torch.float64 if precision == FP64 else torch.float32
    cache: dict = {}
    items = []
    for fr in frames:
        code = code_for(fr, cache)
        y = torch.from_numpy(fr.y).to(dev)
        prior = None if fr.prior is None else torch.from_numpy(fr.prior).to(dev, dtype)
        bnd = [None if getattr(fr, k, None) is None
               else torch.as_tensor(getattr(fr, k), dtype=torch.float64).contiguous().to(dev)
               for k in ("start_drift", "end_drift")]
        items.append((code, y, fr.N, prior, bnd[0], bnd[1]))
    return Batch(items, precision=precision, grad=grad, device=dev, checkpoint_K=checkpoint_K,
                 workspace=workspace)


class Outer:
    """An outer code over GF(q) for iterative decoding (mapdec_outer_*):
    parity-check matrix in compressed rows (row_ptr, col, coef)."""

    def __init__(self, q: int, N: int, row_ptr, col, coef):
        import numpy as np
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        cf = np.ascontiguousarray(coef, dtype=np.uint8)
        self.q, self.N, self.m = int(q), int(N), int(rp.shape[0] - 1)
        self._keep = (rp, cl, cf)
        h = lib().mapdec_outer_create(self.q, self.N, self.m, rp.ctypes.data, cl.ctypes.data,
                                      cf.ctypes.data)
        if not h:
            raise MapdecError(lib().mapdec_last_error(), "mapdec_outer_create")
        self.handle = h

    @classmethod
    def from_spec(cls, spec) -> "Outer":
        return cls(spec.q, spec.N, spec.row_ptr, spec.col, spec.coef)

    def workspace_size(self, nframes: int, precision: int) -> int:
        return int(lib().mapdec_outer_workspace_size(self.handle, nframes, precision))

    def decode(self, chan: torch.Tensor, extr: torch.Tensor, post: Optional[torch.Tensor],
               iters: int, ws: torch.Tensor, stream=None) -> None:
        """Belief propagation on chan [F, N, q] -> extr (and post)."""
        precision = FP64 if chan.dtype == torch.float64 else FP32
        F = chan.shape[0]
        for t in (chan, extr) + ((post,) if post is not None else ()):
            if (tuple(t.shape) != (F, self.N, self.q) or t.dtype != chan.dtype
                    or not t.is_contiguous() or not t.is_cuda):
                raise TypeError("chan / extr / post must be contiguous (F, N, q) CUDA tensors")
        rc = lib().mapdec_outer_decode(self.handle, F, chan.data_ptr(), extr.data_ptr(),
                                       _ptr(post), int(iters), ws.data_ptr(), ws.numel(),
                                       precision, _stream_handle(stream))
        if rc != OK:
            raise MapdecError(rc, "mapdec_outer_decode")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.mapdec_outer_destroy(h)
            self.handle = None


class Iterative:
    """Iterative decoding of frames that carry codewords of one outer code
    (Sec. II-A): per pass the inner decoder (libmapdec) with the priors in
    ``prior`` (1/q at first), its d log P / d prior into ``chan``, then
    ``bp_iters`` iterations of belief propagation writing the next priors
    (the outer extrinsic output) into ``prior`` and the posteriors into
    ``post``.  Every buffer is one (F, N, q) device tensor; the frames'
    priors and dprior outputs are its rows.

    ``frames``: (code, y, N) or (code, y, N, start, end) as for Batch,
    without priors (they are the iteration's)."""

    def __init__(self, frames: Sequence, outer: Outer, precision: int = FP32,
                 checkpoint_K: int = 0, device=None):
        self.outer = outer
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        dev = torch.device(device or "cuda")
        F = len(frames)
        q, N = outer.q, outer.N
        self.prior = torch.full((F, N, q), 1.0 / q, dtype=self.dtype, device=dev)
        self.chan = torch.zeros((F, N, q), dtype=self.dtype, device=dev)
        self.post = torch.zeros((F, N, q), dtype=self.dtype, device=dev)
        items = []
        for f, fr in enumerate(frames):
            code, y, n_sym = fr[:3]
            if n_sym != N or code.q != q:
                raise ValueError("every frame must have the outer code's N and q")
            items.append((code, y, n_sym, self.prior[f]) + tuple(fr[3:5]))
        self.batch = Batch(items, precision=precision, device=dev, checkpoint_K=checkpoint_K,
                           dpriors=[self.chan[f] for f in range(F)])
        self.ws = torch.empty(outer.workspace_size(F, precision), dtype=torch.uint8, device=dev)
        self.precision = precision

        self.plan = None

    def use_plan(self, graph: bool = True, stream=None) -> "Iterative":
        """Replay the inner decode as a plan (one HIP graph with graph=True):
        its buffers stay fixed, only their contents change between passes."""
        self.plan = Plan(self.batch, graph=graph, stream=stream)
        return self

    def reset(self) -> None:
        """Back to uniform priors (the first pass)."""
        self.prior.fill_(1.0 / self.outer.q)

    def run_pass(self, bp_iters: int, stream=None) -> None:
        if self.plan is not None:
            self.plan.run(stream)
        else:
            self.batch.decode(stream=stream)
        self.outer.decode(self.chan, self.prior, self.post, bp_iters, self.ws, stream=stream)

    def run(self, passes: int, bp_iters: int, stream=None) -> None:
        for _ in range(passes):
            self.run_pass(bp_iters, stream)


def iterative_from_frames(frames: List, spec, precision: int = FP32,
                          checkpoint_K: int = 0, device=None) -> Iterative:
    """Uploads workloads.Frame objects carrying codewords of the outer code
    ``spec`` (workloads.OuterSpec) and builds an :class:`Iterative`."""
    dev = torch.device(device or "cuda")
    cache: dict = {}
    items = []
    for fr in frames:
        code = code_for(fr, cache)
        y = torch.from_numpy(fr.y).to(dev)
        bnd = [None if getattr(fr, k, None) is None
               else torch.as_tensor(getattr(fr, k), dtype=torch.float64).contiguous().to(dev)
               for k in ("start_drift", "end_drift")]
        items.append((code, y, fr.N, bnd[0], bnd[1]))
    return Iterative(items, Outer.from_spec(spec), precision=precision,
                     checkpoint_K=checkpoint_K, device=dev)
