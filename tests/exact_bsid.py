"""Exact brute-force reference for the truncated BSID channel model.

Enumerates every message and, for each, every channel event sequence that
turns the encoded frame into the received sequence, in exact rational
arithmetic (``fractions.Fraction``).  It shares nothing with the oracle's
lattice/forward-backward code: it walks the channel of Sec. II-B event by
event, and applies the decoder's truncation as constraints on the walk:

  (i)   at most I consecutive insertions at one channel time step;
  (ii)  inside codeword c (started at received index s = c n + m'), every
        visited node keeps (p - t) - m' in [mn_lo, mn_hi] ([-mn, mn] for a
        fixed code's symmetric limits), where t counts input bits and p
        received bits;
  (iii) at every codeword boundary the drift p - t lies in [mt_lo, mt_hi]
        ([-M, M]);
  plus start drift 0, all of y consumed, and no insertion after the last
  input bit.

Each path's weight is a monomial in a = Pi/2, d = Pd, t1 = Pt(1 - Ps),
t0 = Pt Ps.  The walk carries exact derivatives of the path sums with
respect to (Pi, Pd, Ps) by propagating first-order terms along each edge.
Only for tiny frames (q^N messages times all event sequences).
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from functools import lru_cache
from typing import Optional, Sequence

F0 = Fraction(0)


def _edge(wv, dw, sub):
    """Extend the path sums ``sub`` = (V, dV/dPi, dV/dPd, dV/dPs) by one edge
    of weight ``wv`` whose derivatives are ``dw``."""
    V = sub[0]
    return (wv * V,
            wv * sub[1] + dw[0] * V,
            wv * sub[2] + dw[1] * V,
            wv * sub[3] + dw[2] * V)


def _add(x, y):
    return tuple(a + b for a, b in zip(x, y))


def channel_sum(X: Sequence[int], y: Sequence[int], n: int, Pi, Pd, Ps, I: int, M: int, mn: int):
    """Sum of the weights of all admissible event sequences X -> y, and its
    derivatives with respect to (Pi, Pd, Ps).  Returns a 4-tuple."""
    return channel_sum_limits(X, y, n, Pi, Pd, Ps, I, -M, M, -mn, mn)


def channel_sum_limits(X: Sequence[int], y: Sequence[int], n: int, Pi, Pd, Ps, I: int,
                       mt_lo: int, mt_hi: int, mn_lo: int, mn_hi: int, allowed=None):
    """channel_sum with drift limits [mt_lo, mt_hi] at codeword boundaries
    and a corridor [mn_lo, mn_hi] inside codewords.  ``allowed``: optional
    per-boundary sets of drifts (allowed[b] for boundary b = 1 .. len(X)/n)
    that a path must also keep to."""
    Pi, Pd, Ps = Fraction(Pi), Fraction(Pd), Fraction(Ps)
    Pt = 1 - Pi - Pd
    a, d, t1, t0 = Pi / 2, Pd, Pt * (1 - Ps), Pt * Ps
    # d(weight)/d(Pi, Pd, Ps) of each event kind
    da = (Fraction(1, 2), F0, F0)
    dd = (F0, Fraction(1), F0)
    dt1 = (-(1 - Ps), -(1 - Ps), -Pt)
    dt0 = (-Ps, -Ps, Pt)
    tau, rho = len(X), len(y)
    zero = (F0, F0, F0, F0)

    @lru_cache(maxsize=None)
    def go(t: int, p: int, k: int, mp: int):
        # state: t input bits done, p received bits consumed, k insertions so
        # far at time t, mp = drift at the start of the current codeword
        if t == tau:
            return (Fraction(1), F0, F0, F0) if p == rho else zero
        total = zero
        # insertion: emit y[p], stay at time t
        if k < I and p < rho and mn_lo <= (p + 1 - t) - mp <= mn_hi:
            total = _add(total, _edge(a, da, go(t, p + 1, k + 1, mp)))

        def advance(np_):
            nt = t + 1
            if not mn_lo <= (np_ - nt) - mp <= mn_hi:
                return None
            if nt % n == 0:
                drift = np_ - nt
                if not mt_lo <= drift <= mt_hi:
                    return None
                if allowed is not None and drift not in allowed[nt // n]:
                    return None
                return go(nt, np_, 0, drift)
            return go(nt, np_, 0, mp)

        sub = advance(p)                          # deletion
        if sub is not None:
            total = _add(total, _edge(d, dd, sub))
        if p < rho:                               # transmission
            sub = advance(p + 1)
            if sub is not None:
                if y[p] == X[t]:
                    total = _add(total, _edge(t1, dt1, sub))
                else:
                    total = _add(total, _edge(t0, dt0, sub))
        return total

    return go(0, 0, 0, 0)


def brute(codebook, y, N: int, Pi, Pd, Ps, I: int, M: int, mn: int,
          prior: Optional[Sequence[Sequence]] = None):
    """Exact P(y), APPs, d log P / d(Pi, Pd, Ps) and d log P / d prior.

    ``codebook``: q rows of n bits; ``prior``: N x q (Fractions or ints/
    floats converted exactly), default 1/q."""
    return brute_general([codebook] * N, y, N, Pi, Pd, Ps, I, -M, M, -mn, mn, prior)


def brute_general(codebooks, y, N: int, Pi, Pd, Ps, I: int, mt_lo: int, mt_hi: int,
                  mn_lo: int, mn_hi: int, prior: Optional[Sequence[Sequence]] = None):
    """brute() under the general scheme: ``codebooks[i]`` (q rows of n bits)
    encodes symbol i (Sec. II-A, C_i), drift limits [mt_lo, mt_hi] and
    corridor [mn_lo, mn_hi]."""
    q = len(codebooks[0])
    n = len(codebooks[0][0])
    if prior is None:
        prior = [[Fraction(1, q)] * q for _ in range(N)]
    else:
        prior = [[Fraction(v) for v in row] for row in prior]
    P = F0
    dP = [F0, F0, F0]
    num = [[F0] * q for _ in range(N)]          # sum over messages with D_i = D
    dpr = [[F0] * q for _ in range(N)]          # d P / d prior_i(D)
    for msg in itertools.product(range(q), repeat=N):
        X = [b for i, D in enumerate(msg) for b in codebooks[i][D]]
        V, dPi, dPd, dPs = channel_sum_limits(X, y, n, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo,
                                              mn_hi)
        if V == 0 and dPi == 0 and dPd == 0 and dPs == 0:
            continue
        pw = Fraction(1)
        for i, D in enumerate(msg):
            pw *= prior[i][D]
        P += pw * V
        dP[0] += pw * dPi
        dP[1] += pw * dPd
        dP[2] += pw * dPs
        for i, D in enumerate(msg):
            num[i][D] += pw * V
            rest = Fraction(1)
            for j, E in enumerate(msg):
                if j != i:
                    rest *= prior[j][E]
            dpr[i][D] += rest * V
    if P == 0:
        return {"P": P}
    return {
        "P": P,
        "app": [[num[i][D] / P for D in range(q)] for i in range(N)],
        "dparams": [g / P for g in dP],
        "dprior": [[dpr[i][D] / P for D in range(q)] for i in range(N)],
    }


def brute_pruned(codebooks, y, N: int, Pi, Pd, Ps, I: int, mt_lo: int, mt_hi: int,
                 mn_lo: int, mn_hi: int, theta, prior: Optional[Sequence[Sequence]] = None):
    """Exact results of the decoder with path thresholds: the drifts kept at
    boundary i are those whose forward mass (the summed weight of all path
    prefixes through the first i codewords, with their priors, that end at
    that drift after consuming exactly the received bits up to it and keep
    to the drifts kept at every earlier boundary) is at least ``theta``
    times the total over drifts; then every result is that of the paths
    that keep to the kept drifts at every boundary.  Returns brute()'s
    dict plus ``kept`` (the kept drift sets, boundaries 1 .. N)."""
    q = len(codebooks[0])
    n = len(codebooks[0][0])
    pr = ([[Fraction(1, q)] * q for _ in range(N)] if prior is None
          else [[Fraction(v) for v in row] for row in prior])
    theta = Fraction(theta)
    kept = [None]   # boundary 0: start drift 0
    for i in range(1, N + 1):
        mass = {}
        for m in range(mt_lo, mt_hi + 1):
            end = n * i + m
            if end < 0 or end > len(y):
                continue
            tot = F0
            for msg in itertools.product(range(q), repeat=i):
                X = [b for j, D in enumerate(msg) for b in codebooks[j][D]]
                allowed = kept + [{m}]
                V = channel_sum_limits(X, y[:end], n, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi,
                                       allowed=allowed)[0]
                if V:
                    w = Fraction(1)
                    for j, D in enumerate(msg):
                        w *= pr[j][D]
                    tot += w * V
            mass[m] = tot
        total = sum(mass.values(), F0)
        kept.append({m for m, v in mass.items() if v > 0 and v >= theta * total})
    P = F0
    dP = [F0, F0, F0]
    num = [[F0] * q for _ in range(N)]
    dpr = [[F0] * q for _ in range(N)]
    for msg in itertools.product(range(q), repeat=N):
        X = [b for i, D in enumerate(msg) for b in codebooks[i][D]]
        V, dPi, dPd, dPs = channel_sum_limits(X, y, n, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo,
                                              mn_hi, allowed=kept)
        if V == 0 and dPi == 0 and dPd == 0 and dPs == 0:
            continue
        pw = Fraction(1)
        for i, D in enumerate(msg):
            pw *= pr[i][D]
        P += pw * V
        for k, g in enumerate((dPi, dPd, dPs)):
            dP[k] += pw * g
        for i, D in enumerate(msg):
            num[i][D] += pw * V
            rest = Fraction(1)
            for j, E in enumerate(msg):
                if j != i:
                    rest *= pr[j][E]
            dpr[i][D] += rest * V
    out = {"P": P, "kept": kept[1:]}
    if P:
        out.update({"app": [[num[i][D] / P for D in range(q)] for i in range(N)],
                    "dparams": [g / P for g in dP],
                    "dprior": [[dpr[i][D] / P for D in range(q)] for i in range(N)]})
    return out
