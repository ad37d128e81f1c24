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
                codebook=None, with_prior=False, message=None) -> Frame:
    """Draw one frame: codebook (if not given), message (if not given),
    priors, channel."""
    rng = np.random.Generator(np.random.PCG64(ss))
    if codebook is None:
        codebook = random_codebook(rng, q, n)
    drawn = rng.integers(0, q, size=N)
    message = drawn if message is None else np.asarray(message, dtype=np.int64)
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


# --------------------------------------------------------------------------
# Serial concatenation with an outer code (Sec. II-A): the transmitter.
# The outer code is a linear code over GF(q), q = 2^p (1 <= p <= 6), with a
# sparse parity-check matrix of repeat-accumulate shape: the first K = N - m
# symbols carry the information, each in wc random rows; parity symbol r
# sits in row r and (r < m - 1) row r + 1, so the parity symbols follow one
# by one from the rows (an accumulator).  GF(2^p): integers 0 .. q-1 as
# polynomials over GF(2) (bit k = coefficient of z^k) modulo the primitive
# polynomial _OUTER_PRIM[p]; this module keeps its own exponent and
# logarithm tables for the encoder.
# --------------------------------------------------------------------------

_OUTER_PRIM = {1: 0b11, 2: 0b111, 3: 0b1011, 4: 0b10011, 5: 0b100101, 6: 0b1000011}


@dataclasses.dataclass
class OuterSpec:
    """Parity-check matrix of an outer code over GF(q): row c holds the
    symbols col[row_ptr[c]:row_ptr[c+1]] with coefficients coef[...] in
    1 .. q-1; ``info`` the K information symbols, ``codeword`` the N
    transmitted symbols (H codeword = 0)."""
    q: int
    N: int
    row_ptr: np.ndarray
    col: np.ndarray
    coef: np.ndarray
    info: np.ndarray
    codeword: np.ndarray


def _gf_exp_log(q: int):
    p = q.bit_length() - 1
    if q < 2 or (1 << p) != q or p not in _OUTER_PRIM:
        raise ValueError("outer alphabet must be 2^p, 1 <= p <= 6")
    exp = [0] * (2 * q)
    log = [0] * q
    e = 1
    for k in range(q - 1):
        exp[k] = e
        log[e] = k
        e <<= 1
        if e & q:
            e ^= _OUTER_PRIM[p]
    for k in range(q - 1, 2 * q):
        exp[k] = exp[k - (q - 1)]
    return exp, log


def outer_code(rng: np.random.Generator, q: int, N: int, checks: int, wc: int = 3) -> OuterSpec:
    """A random repeat-accumulate outer code with ``checks`` rows over
    GF(q), and one of its codewords for random information symbols."""
    m, K = int(checks), int(N) - int(checks)
    if m < 1 or K < 0 or (K > 0 and wc > m):
        raise ValueError("need 1 <= checks <= N and wc <= checks")
    exp, log = _gf_exp_log(q)

    def mul(a, b):
        return 0 if a == 0 or b == 0 else exp[log[a] + log[b]]

    def inv(a):
        return exp[(q - 1 - log[a]) % (q - 1)]

    rows = [[] for _ in range(m)]
    for j in range(K):
        for r in rng.choice(m, size=wc, replace=False):
            rows[int(r)].append((j, int(rng.integers(1, q))))
    for r in range(m):
        rows[r].append((K + r, int(rng.integers(1, q))))
        if r > 0:
            rows[r].append((K + r - 1, int(rng.integers(1, q))))
    info = rng.integers(0, q, size=K)
    x = np.zeros(N, dtype=np.int64)
    x[:K] = info
    for r in range(m):   # h_{r,K+r} x_{K+r} = sum of the row's other terms
        acc = 0
        for j, h in rows[r]:
            if j != K + r:
                acc ^= mul(h, int(x[j]))
        h_own = dict(rows[r])[K + r]
        x[K + r] = mul(inv(h_own), acc)
    row_ptr, col, coef = [0], [], []
    for r in range(m):
        for j, h in sorted(rows[r]):
            col.append(j)
            coef.append(h)
        row_ptr.append(len(col))
    for r in range(m):   # every row holds
        acc = 0
        for k in range(row_ptr[r], row_ptr[r + 1]):
            acc ^= mul(coef[k], int(x[col[k]]))
        assert acc == 0
    return OuterSpec(q=q, N=N, row_ptr=np.asarray(row_ptr, dtype=np.int32),
                     col=np.asarray(col, dtype=np.int32), coef=np.asarray(coef, dtype=np.uint8),
                     info=info, codeword=x)


def concatenated_frame(seed: int, q: int, n: int, N: int, Pi: float, Pd: float, Ps: float,
                       I: int, M: int, mn: int, checks: int, wc: int = 3,
                       codebook: Optional[np.ndarray] = None):
    """An outer codeword (``checks`` parity rows) sent through the inner
    code and the channel: returns (OuterSpec, Frame) with the frame's
    message the outer codeword and uniform priors."""
    ss = np.random.SeedSequence([SEED_ROOT, 2000, seed])
    rng = np.random.Generator(np.random.PCG64(ss.spawn(1)[0]))
    spec = outer_code(rng, q, N, checks, wc)
    fr = _draw_frame(ss, q, n, N, (Pi, Pd, Ps), (Pi, Pd, Ps), I, M, mn, codebook=codebook,
                     message=spec.codeword)
    return spec, fr


CONCAT_NAME = "64 frames q16 n10 N500 outer GF(16) code 250 checks, Pi=Pd=0.06 Ps=0.01"


def make_concatenated_workload(nframes: int = 64, first: int = 0):
    """The iterative-decoding workload: frames of the 256-frame batch's
    shape (one codebook) carrying codewords of one outer code over GF(16)
    (rate 1/2, 250 checks, information symbols in 3 checks each), at a
    channel where the inner decoder alone leaves symbol errors."""
    ss = np.random.SeedSequence([SEED_ROOT, 3000])
    cb_rng = np.random.Generator(np.random.PCG64(ss.spawn(1)[0]))
    codebook = random_codebook(cb_rng, 16, 10)
    code_rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 3001])))
    spec = outer_code(code_rng, 16, 500, 250, 3)
    exp, log = _gf_exp_log(16)
    frames = []
    M = drift_limit(5000, 0.06)
    for f in range(first, first + nframes):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 3002, f])))
        # a fresh codeword of the same code: the accumulator again
        info = rng.integers(0, 16, size=250)
        x = _encode_with(spec, info, exp, log)
        frames.append(_draw_frame(np.random.SeedSequence([SEED_ROOT, 3003, f]), 16, 10, 500,
                                  (0.06, 0.06, 0.01), (0.06, 0.06, 0.01), 2, M, 6,
                                  codebook=codebook, message=x))
    return spec, frames


def _encode_with(spec: OuterSpec, info: np.ndarray, exp, log) -> np.ndarray:
    q, N = spec.q, spec.N
    m = spec.row_ptr.shape[0] - 1
    K = N - m

    def mul(a, b):
        return 0 if a == 0 or b == 0 else exp[log[a] + log[b]]

    x = np.zeros(N, dtype=np.int64)
    x[:K] = info
    for r in range(m):
        acc, h_own = 0, None
        for k in range(spec.row_ptr[r], spec.row_ptr[r + 1]):
            j, h = int(spec.col[k]), int(spec.coef[k])
            if j == K + r:
                h_own = h
            else:
                acc ^= mul(h, int(x[j]))
        x[K + r] = mul(exp[(q - 1 - log[h_own]) % (q - 1)], acc)
    return x
