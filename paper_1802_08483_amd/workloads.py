"""Seeded synthetic workloads: codebooks, messages and BSID channel draws.

This module holds input generation only.  It draws codebooks, messages,
prior tables and received sequences; it contains none of the decoder's
arithmetic, so both the GPU path and the CPU oracle can consume its output.

Channel: the binary substitution/insertion/deletion channel of Sec. II-B.
At each channel time step one input bit is considered; an insertion (prob.
Pi) emits a uniform random bit and stays at the same step, a deletion (Pd)
drops the bit, a transmission (Pt = 1 - Pi - Pd) passes it, flipped with
probability Ps.  The simulator caps insertions at ``I`` per time step: once
``I`` insertions have happened at a step, the remaining event is a deletion
with probability Pd / (1 - Pi) or a transmission otherwise.  This matches the
decoder's truncated model, which keeps only paths with at most ``I``
insertions per step.

Encoding: Sec. II-A with one codebook for every symbol position; codewords
are ``q`` distinct integers drawn without replacement from [0, 2^n), written
most-significant bit first.

Seeds: workload ``k`` uses ``numpy.random.SeedSequence([180208483, k])`` and
spawns one child sequence per frame; a frame whose end drift falls outside
[-M, M] is redrawn from the next child of its own sequence.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_ROOT = 180208483


@dataclasses.dataclass
class Frame:
    """One received frame plus the code and channel model used to decode it."""

    q: int
    n: int
    N: int
    codebook: np.ndarray          # (q, n) uint8 of 0/1, row D is C(D)
    message: np.ndarray           # (N,) int64 transmitted symbols
    y: np.ndarray                 # (rho,) uint8 of 0/1 received bits
    Pi: float                     # decoder's channel parameters
    Pd: float
    Ps: float
    I: int                        # insertion cap per channel time step
    M: int                        # frame drift limit, states [-M, M]
    mn: int                       # per-codeword drift limit, [-mn, mn]
    prior: Optional[np.ndarray] = None   # (N, q) float64, None = uniform
    # priors of the frame's start / end drift over [-M, M] (entry m + M),
    # None = known boundary (start drift 0, end drift rho - tau)
    start_drift: Optional[np.ndarray] = None
    end_drift: Optional[np.ndarray] = None
    sim: tuple = ()               # (Pi, Pd, Ps) used to draw y
    redraws: int = 0
    # the general scheme (Sec. II-A / III-B): codebooks (N, q, n), codebook
    # i for symbol i (None: ``codebook`` for every symbol), and the limits
    # (mt_lo, mt_hi, mn_lo, mn_hi) (None: [-M, M] and [-mn, mn]); M and mn
    # are then max(-mt_lo, mt_hi) and max(-mn_lo, mn_hi)
    codebooks: Optional[np.ndarray] = None
    limits: Optional[tuple] = None
    # path thresholds of the decoder (0: none)
    theta: float = 0.0

    @property
    def tau(self) -> int:
        return self.n * self.N

    @property
    def rho(self) -> int:
        return int(self.y.shape[0])


def drift_limit(tau: int, Pd: float) -> int:
    """Frame drift limit of the workloads: ceil(6 sqrt(tau Pd / (1 - Pd)))."""
    return int(math.ceil(6.0 * math.sqrt(tau * Pd / (1.0 - Pd))))


def codeword_drift_limit(n: int, Pd: float, M: int) -> int:
    """Per-codeword drift limit for the uneven batch."""
    return int(min(M, math.ceil(4.0 * math.sqrt(n * Pd / (1.0 - Pd))) + 2))


def random_codebook(rng: np.random.Generator, q: int, n: int) -> np.ndarray:
    if q > (1 << n):
        raise ValueError("q > 2^n")
    words = rng.choice(1 << n, size=q, replace=False)
    shifts = np.arange(n - 1, -1, -1)
    return ((words[:, None] >> shifts[None, :]) & 1).astype(np.uint8)


def bsid_channel(rng: np.random.Generator, x: np.ndarray, Pi: float, Pd: float,
                 Ps: float, I: int) -> np.ndarray:
    """Pass bits ``x`` through the BSID channel with at most ``I`` insertions
    per time step.  Per step: the number of leading insertion outcomes k
    (each with probability Pi, at most I), then a deletion with probability
    Pd / (1 - Pi) or a transmission, flipped with probability Ps."""
    tau = x.shape[0]
    u = rng.random((tau, I)) if I > 0 else np.zeros((tau, 0))
    ins_flags = u < Pi
    if I > 0:
        k = np.argmin(np.concatenate([ins_flags, np.zeros((tau, 1), bool)], axis=1), axis=1)
    else:
        k = np.zeros(tau, dtype=np.int64)
    v = rng.random(tau)
    deleted = v < (Pd / (1.0 - Pi))
    flips = rng.random(tau) < Ps
    ins_bits = rng.integers(0, 2, size=(tau, max(I, 1)), dtype=np.uint8)
    # per time step: k inserted bits followed by 0 or 1 transmitted bit
    width = max(I, 1) + 1
    buf = np.zeros((tau, width), dtype=np.uint8)
    keep = np.zeros((tau, width), dtype=bool)
    if I > 0:
        buf[:, :I] = ins_bits[:, :I]
        keep[:, :I] = np.arange(I)[None, :] < k[:, None]
    tx = (x.astype(np.uint8) ^ flips.astype(np.uint8))
    # place the transmitted bit right after the k insertions
    col = k.astype(np.int64)
    buf[np.arange(tau), col] = np.where(~deleted, tx, buf[np.arange(tau), col])
    keep[np.arange(tau), col] = ~deleted
    return buf[keep].astype(np.uint8)


def encode(codebook: np.ndarray, message: np.ndarray) -> np.ndarray:
    return codebook[message].reshape(-1).astype(np.uint8)


def _draw_frame(ss: np.random.SeedSequence, q, n, N, sim, dec, I, M, mn,
                codebook=None, with_prior=False) -> Frame:
    """Draw one frame: codebook (if not given), message, priors, channel."""
    rng = np.random.Generator(np.random.PCG64(ss))
    if codebook is None:
        codebook = random_codebook(rng, q, n)
    message = rng.integers(0, q, size=N)
    prior = None
    if with_prior:
        logits = rng.standard_normal((N, q))
        e = np.exp(logits - logits.max(axis=1, keepdims=True))
        prior = e / e.sum(axis=1, keepdims=True)
    x = encode(codebook, message)
    tau = n * N
    redraws = 0
    child = ss
    while True:
        y = bsid_channel(rng, x, *sim, I)
        if abs(y.shape[0] - tau) <= M:
            break
        redraws += 1
        child = child.spawn(1)[0]
        rng = np.random.Generator(np.random.PCG64(child))
    return Frame(q=q, n=n, N=N, codebook=codebook, message=message, y=y,
                 Pi=dec[0], Pd=dec[1], Ps=dec[2], I=I, M=M, mn=mn, prior=prior,
                 sim=tuple(sim), redraws=redraws)


# --------------------------------------------------------------------------
# The five workloads.  Sizes follow the decoder's intended operating points:
#   1: one frame, q=8 n=6 N=64, Pi=Pd=0.01 Ps=0, I=2, M=16, mn=4 (FP64)
#   2: 256 frames, q=16 n=10 N=500, Pi=Pd=0.05 Ps=0.01, I=2, M=98, mn=6
#   3: 4096 uneven frames, q in {2,8,16}, n in [max(log2 q,4),10],
#      N in [50,2000], Pi=Pd log-uniform [1e-3,1e-1], Ps=0
#   4: 128 frames, q=16 n=10 N=1000, simulate (.02,.02,.01), decode at
#      (.025,.025,.015), softmax priors of N(0,1) logits, M=97, mn=6
#   5: 16 frames, q=64 n=12 N=10000, Pi=Pd=0.1 Ps=0, M=693, mn=8
# --------------------------------------------------------------------------

WORKLOAD_NAMES = {
    1: "single-frame q8 n6 N64 p0.01 fp64",
    2: "256 frames q16 n10 N500 Pi=Pd=0.05 Ps=0.01 fp32",
    3: "4096 uneven frames q{2,8,16} n[4,10] N[50,2000] fp32",
    4: "128 frames q16 n10 N1000 channel-estimation decode+adjoint",
    5: "16 frames q64 n12 N10000 Pi=Pd=0.1 checkpointed adjoint",
}


def make_workload(k: int, nframes: Optional[int] = None, first: int = 0) -> List[Frame]:
    """Frames ``first .. first+nframes`` of workload ``k`` (deterministic)."""
    root = np.random.SeedSequence([SEED_ROOT, k])
    total = {1: 1, 2: 256, 3: 4096, 4: 128, 5: 16}[k]
    if nframes is None:
        nframes = total - first
    children = root.spawn(total)
    frames = []
    if k in (2, 4, 5):
        # one codebook shared by the whole batch, drawn from its own child
        cb_rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, k, 0])))
        q, n = {2: (16, 10), 4: (16, 10), 5: (64, 12)}[k]
        codebook = random_codebook(cb_rng, q, n)
    for f in range(first, first + nframes):
        ss = children[f]
        if k == 1:
            frames.append(_draw_frame(ss, 8, 6, 64, (0.01, 0.01, 0.0), (0.01, 0.01, 0.0),
                                      2, 16, 4))
        elif k == 2:
            M = drift_limit(5000, 0.05)
            frames.append(_draw_frame(ss, 16, 10, 500, (0.05, 0.05, 0.01), (0.05, 0.05, 0.01),
                                      2, M, 6, codebook=codebook))
        elif k == 3:
            rng = np.random.Generator(np.random.PCG64(ss))
            q = int(rng.choice([2, 8, 16]))
            n = int(rng.integers(max(int(math.log2(q)), 4), 11))
            N = int(rng.integers(50, 2001))
            Pd = float(math.exp(rng.uniform(math.log(1e-3), math.log(1e-1))))
            M = drift_limit(n * N, Pd)
            mn = codeword_drift_limit(n, Pd, M)
            sub = ss.spawn(1)[0]
            frames.append(_draw_frame(sub, q, n, N, (Pd, Pd, 0.0), (Pd, Pd, 0.0), 2, M, mn))
        elif k == 4:
            M = drift_limit(10000, 0.025)
            frames.append(_draw_frame(ss, 16, 10, 1000, (0.02, 0.02, 0.01),
                                      (0.025, 0.025, 0.015), 2, M, 6,
                                      codebook=codebook, with_prior=True))
        elif k == 5:
            M = drift_limit(120000, 0.1)
            frames.append(_draw_frame(ss, 64, 12, 10000, (0.1, 0.1, 0.0), (0.1, 0.1, 0.0),
                                      2, M, 8, codebook=codebook))
        else:
            raise ValueError(f"unknown workload {k}")
    return frames


def general_frame(seed: int, q: int, n: int, N: int, Pi: float, Pd: float, Ps: float, I: int,
                  mt_lo: int, mt_hi: int, mn_lo: int, mn_hi: int, per_symbol: bool = True,
                  with_prior: bool = False, sim: Optional[tuple] = None) -> Frame:
    """A seeded frame of the general scheme: with ``per_symbol`` a random
    codebook C_i for every symbol position (else one for all), drift limits
    [mt_lo, mt_hi] and corridor [mn_lo, mn_hi]; the channel draw is
    repeated (from child seeds) until the end drift rho - tau lies in
    [mt_lo, mt_hi]."""
    ss = np.random.SeedSequence([SEED_ROOT, 2000, seed])
    rng = np.random.Generator(np.random.PCG64(ss))
    if per_symbol:
        codebooks = np.stack([random_codebook(rng, q, n) for _ in range(N)])
    else:
        codebooks = random_codebook(rng, q, n)[None]
    message = rng.integers(0, q, size=N)
    prior = None
    if with_prior:
        logits = rng.standard_normal((N, q))
        e = np.exp(logits - logits.max(axis=1, keepdims=True))
        prior = e / e.sum(axis=1, keepdims=True)
    cbs = codebooks if per_symbol else np.repeat(codebooks, N, axis=0)
    x = cbs[np.arange(N), message].reshape(-1).astype(np.uint8)
    tau = n * N
    sim = sim or (Pi, Pd, Ps)
    redraws = 0
    child = ss
    while True:
        y = bsid_channel(rng, x, *sim, I)
        if mt_lo <= y.shape[0] - tau <= mt_hi:
            break
        redraws += 1
        child = child.spawn(1)[0]
        rng = np.random.Generator(np.random.PCG64(child))
    M, mn = max(-mt_lo, mt_hi), max(-mn_lo, mn_hi)
    return Frame(q=q, n=n, N=N, codebook=codebooks[0], message=message, y=y, Pi=Pi, Pd=Pd,
                 Ps=Ps, I=I, M=M, mn=mn, prior=prior, sim=tuple(sim), redraws=redraws,
                 codebooks=codebooks if per_symbol else None,
                 limits=(mt_lo, mt_hi, mn_lo, mn_hi))


GENERAL_NAME = ("64 frames q16 n10 N500 Pi=Pd=0.05 Ps=0.01, a codebook per symbol, "
                "drift limits [-98, 98], corridor [-5, 6]")


def make_general_workload(nframes: int = 64) -> List[Frame]:
    """The general scheme at the 256-frame batch's operating point: 64 frames
    of q=16, n=10, N=500 at Pi=Pd=0.05, Ps=0.01, I=2, each with a random
    codebook per symbol position, drift limits [-98, 98] and the corridor
    [-5, 6] (one drift change narrower on the deletion side)."""
    return [general_frame(10_000 + f, 16, 10, 500, 0.05, 0.05, 0.01, 2, -98, 98, -5, 6)
            for f in range(nframes)]


def random_frame(seed: int, q: int, n: int, N: int, Pi: float, Pd: float, Ps: float,
                 I: int, M: int, mn: int, with_prior: bool = False,
                 sim: Optional[tuple] = None) -> Frame:
    """A single seeded frame with explicit parameters (tests)."""
    ss = np.random.SeedSequence([SEED_ROOT, 1000, seed])
    return _draw_frame(ss, q, n, N, sim or (Pi, Pd, Ps), (Pi, Pd, Ps), I, M, mn,
                       with_prior=with_prior)


def with_boundary_priors(frames: List[Frame], spread: int = 4) -> List[Frame]:
    """The frames with priors of their start and end drift instead of known
    boundaries: binomial weights over start drifts 0 .. 2 spread and over end
    drifts within spread of rho - tau (clipped to [-M, M]), normalised."""
    from math import comb
    w = np.array([comb(2 * spread, k) for k in range(2 * spread + 1)], dtype=np.float64)
    w /= w.sum()
    out = []
    for fr in frames:
        Mt = 2 * fr.M + 1
        st = np.zeros(Mt)
        en = np.zeros(Mt)
        for k in range(2 * spread + 1):
            m0 = k
            if m0 <= fr.M:
                st[fr.M + m0] += w[k]
            mN = fr.rho - fr.tau + k - spread
            if abs(mN) <= fr.M:
                en[fr.M + mN] += w[k]
        out.append(dataclasses.replace(fr, start_drift=st, end_drift=en))
    return out
