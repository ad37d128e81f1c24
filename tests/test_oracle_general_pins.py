"""Pins for the oracle's general scheme: a constituent encoding C_i per
symbol position (Sec. II-A) and asymmetric state-space limits m_n^- <= 0 <=
m_n^+, m_tau^- <= m_n^-, m_tau^+ >= m_n^+ (Sec. III-B, flexibility items e
and g).  Every check comes from the channel model, closed forms or exact
enumeration, never from the oracle itself:

  G1  exact brute force over messages x channel event sequences with C_i
      and binding asymmetric limits (P(y), APPs, gradients), Fractions
  G2  total mass of the truncated channel with C_i and wide asymmetric
      limits: sum_y P(y) = (1 - Pi^(I+1))^tau
  G3  memoryless substitution channel with C_i: per-block closed form
  G4  hand-derived n = 1 lattices under one-sided corridors
  G5  P(y) nondecreasing in each of the four limits
  G6  relabelling the symbols of each C_i (and its priors) permutes the APP
      columns and changes nothing else
  G7  validation: the order of the limits, ncb in {1, N}, injective C_i,
      end drift inside [m_tau^-, m_tau^+]
"""
import itertools
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from exact_bsid import brute_general
from paper_1802_08483_amd import workloads as wl


def _rand_general(seed):
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(1, 4))
    q = int(rng.integers(2, min(4, 1 << n) + 1))
    N = int(rng.integers(1, 3 if q > 2 else 4))
    cbs = []
    for _ in range(N):
        words = rng.choice(1 << n, size=q, replace=False)
        cbs.append([[(int(w) >> (n - 1 - r)) & 1 for r in range(n)] for w in words])
    tau = n * N
    mn_lo = -int(rng.integers(0, 3))
    mn_hi = int(rng.integers(0, 3))
    mt_lo = mn_lo - int(rng.integers(0, 3))
    mt_hi = mn_hi + int(rng.integers(0, 3))
    end = int(rng.integers(mt_lo, mt_hi + 1))
    rho = max(0, tau + end)
    y = [int(b) for b in rng.integers(0, 2, size=rho)]
    if not mt_lo <= rho - tau <= mt_hi:
        mt_lo, mt_hi = min(mt_lo, rho - tau), max(mt_hi, rho - tau)
    I = int(rng.integers(0, 3))
    Pi = Fr(int(rng.integers(1, 20)), 100)
    Pd = Fr(int(rng.integers(1, 20)), 100)
    Ps = Fr(int(rng.integers(0, 30)), 100)
    prior = None
    if rng.random() < 0.5:
        prior = [[Fr(int(v), 16) for v in rng.integers(1, 16, size=q)] for _ in range(N)]
    return cbs, y, N, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi, prior


def _dec(cbs, y, N, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi, prior=None, **kw):
    pr = None if prior is None else np.array([[float(v) for v in row] for row in prior])
    return oracle.decode_general(np.array(cbs, dtype=np.uint8), np.array(y, dtype=np.uint8), N,
                                 float(Pi), float(Pd), float(Ps), I, mt_lo, mt_hi, mn_lo, mn_hi,
                                 prior=pr, check=False, **kw)


# ---- G1 --------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_g1_brute_force(seed):
    case = _rand_general(seed)
    cbs, y, N = case[:3]
    b = brute_general(*case)
    r = _dec(*case, grad=True)
    if b["P"] == 0:
        assert r["status"] == oracle.REF_ENOPATH
        return
    assert r["status"] == 0
    lp = math.log(b["P"])
    assert abs(r["logp"] - lp) <= 1e-12 * max(1.0, abs(lp))
    np.testing.assert_allclose(r["app"], np.array(b["app"], dtype=float), rtol=0, atol=1e-13)
    g = np.array(b["dparams"], dtype=float)
    np.testing.assert_allclose(r["dparams"], g, rtol=1e-10, atol=1e-10 * np.abs(g).max())
    dp = np.array(b["dprior"], dtype=float)
    np.testing.assert_allclose(r["dprior"], dp, rtol=1e-11, atol=1e-12 * np.abs(dp).max())


def test_g1_asymmetric_limits_bind():
    # one frame with distinct codebooks per position under a corridor and
    # drift range that lean one way: exact under each, and different
    cbs = [[[0, 1, 1], [1, 0, 0]], [[1, 1, 0], [0, 0, 1]]]
    y = [0, 1, 1, 1, 0, 0, 1]
    Pi, Pd, Ps = Fr(1, 8), Fr(1, 10), Fr(1, 20)
    vals = []
    for lim in [(-1, 2, 0, 1), (-2, 1, -1, 0), (-2, 2, -1, 1), (-3, 3, -2, 2)]:
        b = brute_general(cbs, y, 2, Pi, Pd, Ps, 2, *lim)
        r = _dec(cbs, y, 2, Pi, Pd, Ps, 2, *lim)
        if b["P"] == 0:
            assert r["status"] == oracle.REF_ENOPATH
            vals.append(Fr(0))
            continue
        assert abs(r["logp"] - math.log(b["P"])) < 1e-13 * abs(math.log(b["P"]))
        vals.append(b["P"])
    assert vals[0] != vals[1] and vals[2] < vals[3]


# ---- G2 --------------------------------------------------------------------

@pytest.mark.parametrize("n,N,I,Pi,Pd,Ps", [(2, 2, 2, 0.15, 0.1, 0.05), (1, 3, 1, 0.2, 0.3, 0.0)])
def test_g2_total_mass(n, N, I, Pi, Pd, Ps):
    tau = n * N
    wide = max(I * n, n) + 1
    mn_lo, mn_hi = -wide, wide + 1
    mt_lo, mt_hi = -max(I * tau, wide) - 2, max(I * tau, wide) + 1
    rng = np.random.default_rng(17)
    cbs = np.array([wl.random_codebook(rng, 2, n) for _ in range(N)], dtype=np.uint8)
    prior = rng.dirichlet(np.ones(2), size=N)
    total = 0.0
    for L in range(0, tau * (1 + I) + 1):
        for bits in itertools.product((0, 1), repeat=L):
            r = oracle.decode_general(cbs, np.array(bits, dtype=np.uint8), N, Pi, Pd, Ps, I,
                                      mt_lo, mt_hi, mn_lo, mn_hi, prior=prior, check=False)
            if r["status"] == 0:
                total += math.exp(r["logp"])
            else:
                assert r["status"] in (oracle.REF_ENOPATH, oracle.REF_EDRIFT)
    assert abs(total - (1.0 - Pi ** (I + 1)) ** tau) < 1e-12


# ---- G3 --------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_g3_substitution_channel(seed):
    rng = np.random.default_rng(300 + seed)
    q, n, N = 8, 5, 10
    cbs = np.array([wl.random_codebook(rng, q, n) for _ in range(N)], dtype=np.uint8)
    Ps = float(rng.uniform(0.01, 0.3))
    prior = rng.dirichlet(np.ones(q), size=N)
    y = rng.integers(0, 2, size=n * N).astype(np.uint8)
    r = oracle.decode_general(cbs, y, N, 0.0, 0.0, Ps, 2, -2, 4, -1, 3, prior=prior)
    logp = 0.0
    for i in range(N):
        h = (cbs[i] != y[None, n * i:n * (i + 1)]).sum(axis=1)
        lik = prior[i] * Ps ** h * (1 - Ps) ** (n - h)
        logp += math.log(lik.sum())
        np.testing.assert_allclose(r["app"][i], lik / lik.sum(), rtol=1e-12, atol=1e-15)
    assert abs(r["logp"] - logp) < 1e-12 * abs(logp)


# ---- G4 --------------------------------------------------------------------

@pytest.mark.parametrize("Pi,Pd,Ps", [(0.1, 0.2, 0.05), (0.3, 0.1, 0.0)])
def test_g4_one_sided_corridors(Pi, Pd, Ps):
    cb = np.array([[0], [1]], dtype=np.uint8)
    Pt = 1 - Pi - Pd

    def Q(yb, xb):
        return Pt * (1 - Ps) if yb == xb else Pt * Ps

    def R(y, x, lo, hi, I=2):
        return oracle.glattice(cb, np.array(y, np.uint8), 1, 0, 0, x, Pi, Pd, Ps, I,
                               lo - 1, hi + 1, lo, hi)

    for x in (0, 1):
        # corridor [0, 1] (R[delta], delta = 0, 1): no node left of the
        # diagonal, so no net deletion; one received bit is a transmission
        # or an insertion followed by a deletion; two bits take one
        # insertion then a transmission (a second insertion would leave the
        # corridor, and so would the deletion after it)
        for y1 in (0, 1):
            assert R([y1], x, 0, 1)[0] == pytest.approx(Q(y1, x) + Pi / 2 * Pd, rel=1e-14)
            for y2 in (0, 1):
                assert R([y1, y2], x, 0, 1)[1] == pytest.approx(Pi / 2 * Q(y2, x), rel=1e-14)
        # corridor [-1, 0] (R[delta + 1]): no insertion fits (it steps right
        # of the diagonal); the empty segment is a deletion, one bit a
        # transmission
        assert R([], x, -1, 0)[0] == pytest.approx(Pd, rel=1e-15)
        for y1 in (0, 1):
            assert R([y1], x, -1, 0)[1] == pytest.approx(Q(y1, x), rel=1e-14)


# ---- G5 --------------------------------------------------------------------

def test_g5_monotone_in_each_limit():
    rng = np.random.default_rng(41)
    q, n, N = 4, 5, 16
    cbs = np.array([wl.random_codebook(rng, q, n) for _ in range(N)], dtype=np.uint8)
    fr = wl.random_frame(41, q, n, N, 0.08, 0.08, 0.02, 2, 12, 4)
    y = fr.y
    base = dict(mt_lo=-8, mt_hi=9, mn_lo=-2, mn_hi=3)

    def lp(**kw):
        lim = dict(base, **kw)
        r = oracle.decode_general(cbs, y, N, 0.08, 0.08, 0.02, 2, lim["mt_lo"], lim["mt_hi"],
                                  lim["mn_lo"], lim["mn_hi"], check=False)
        return r["logp"] if r["status"] == 0 else -math.inf

    for key, seq in (("mt_lo", (-4, -6, -8, -12)), ("mt_hi", (5, 7, 9, 13)),
                     ("mn_lo", (0, -1, -2, -4)), ("mn_hi", (1, 2, 3, 5))):
        vals = [lp(**{key: v}) for v in seq]
        assert all(b >= a for a, b in zip(vals, vals[1:])), (key, vals)
        assert vals[-1] > vals[0], key


# ---- G6 --------------------------------------------------------------------

def test_g6_relabelling_per_position():
    rng = np.random.default_rng(77)
    q, n, N = 6, 5, 14
    cbs = np.array([wl.random_codebook(rng, q, n) for _ in range(N)], dtype=np.uint8)
    fr = wl.random_frame(77, q, n, N, 0.05, 0.06, 0.03, 2, 10, 3)
    prior = rng.dirichlet(np.ones(q), size=N)
    perms = [rng.permutation(q) for _ in range(N)]
    cbs2 = np.array([cbs[i][perms[i]] for i in range(N)])
    prior2 = np.array([prior[i][perms[i]] for i in range(N)])
    args = (fr.y, N, 0.05, 0.06, 0.03, 2, -10, 9, -3, 2)
    r = oracle.decode_general(cbs, *args, prior=prior, grad=True)
    r2 = oracle.decode_general(cbs2, *args, prior=prior2, grad=True)
    assert abs(r["logp"] - r2["logp"]) <= 1e-13 * abs(r["logp"])
    for i in range(N):
        np.testing.assert_allclose(r2["app"][i], r["app"][i][perms[i]], atol=1e-14)
    np.testing.assert_allclose(r2["dparams"], r["dparams"], rtol=1e-12)


# ---- G7 --------------------------------------------------------------------

def test_g7_validation():
    rng = np.random.default_rng(3)
    cb = wl.random_codebook(rng, 4, 3)
    ok = (0.05, 0.05, 0.0, 2)
    assert oracle.check_general(cb, 5, *ok, -3, 3, -1, 1) == 0
    assert oracle.check_general(cb, 5, *ok, -3, 3, 1, 2) == oracle.REF_EINVAL    # m_n^- > 0
    assert oracle.check_general(cb, 5, *ok, -3, 3, -2, -1) == oracle.REF_EINVAL  # m_n^+ < 0
    assert oracle.check_general(cb, 5, *ok, 0, 3, -1, 1) == oracle.REF_EINVAL    # m_tau^- > m_n^-
    assert oracle.check_general(cb, 5, *ok, -3, 0, -1, 1) == oracle.REF_EINVAL   # m_tau^+ < m_n^+
    cbs = np.array([wl.random_codebook(rng, 4, 3) for _ in range(5)])
    assert oracle.check_general(cbs, 5, *ok, -3, 3, -1, 1) == 0
    assert oracle.check_general(cbs[:3], 5, *ok, -3, 3, -1, 1) == oracle.REF_EINVAL
    bad = cbs.copy()
    bad[2][1] = bad[2][0]                                                        # C_2 not injective
    assert oracle.check_general(bad, 5, *ok, -3, 3, -1, 1) == oracle.REF_EINVAL
    y = np.zeros(5 * 3 + 3, np.uint8)                                            # end drift +3
    r = oracle.decode_general(cbs, y, 5, *ok, -3, 2, -1, 1, check=False)
    assert r["status"] == oracle.REF_EDRIFT
    r = oracle.decode_general(cbs, y, 5, *ok, -3, 3, -1, 1, check=False)
    assert r["status"] in (0, oracle.REF_ENOPATH)
