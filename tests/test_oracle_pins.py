"""Pins for the FP64 CPU oracle: every check here comes from the channel
model, closed forms or exact enumeration, never from the oracle itself.

  P1  exact brute force over messages x channel event sequences (Fractions)
  P2  total mass of the truncated channel: sum_y P(y) = (1 - Pi^(I+1))^tau
  P3  memoryless substitution channel (Pi = Pd = 0) closed form
  P4  Pi = Pd = 0, Ps = 1/2: output carries no information
  P5  APP rows sum to 1; sum_m alpha_i beta_i gives P(y) at every i, also
      where the product of the two rows lies below the FP64 range
  P6  limits: I >= 2 mn never binds; P(y) nondecreasing in I, M, mn
  P7  hand-derived lattice values for n = 1
  P8  complementing y and every codeword changes nothing
  P9  gradients: central differences of log P in (Pi, Pd, Ps) and in single
      prior entries (independent of the gradient code), and the path-count
      identity linking d/dPi and d/dPd
  P11 priors of the frame boundaries (below)
Consistency checks that are not pins (they compare the oracle with a
restatement of itself; the functions they touch are pinned by P1 and P7):
the softmax-logit form APP - prior of the prior gradient, and per-(i, m')
lattices against the lattices memoised per start index.
      (Sec. II-C): point priors give the known-boundary decode; general
      priors give the prior-weighted sum of exact known-boundary decodes of
      the sub-windows y[m0 : tau + mN]
"""
import itertools
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from exact_bsid import brute
from paper_1802_08483_amd import workloads as wl


def _rand_case(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 4))
    q = int(rng.integers(2, min(4, 1 << n) + 1))
    N = int(rng.integers(1, 3 if q > 2 else 4))
    words = rng.choice(1 << n, size=q, replace=False)
    cb = [[(int(w) >> (n - 1 - r)) & 1 for r in range(n)] for w in words]
    tau = n * N
    rho = int(max(0, tau + rng.integers(-2, 3)))
    y = [int(b) for b in rng.integers(0, 2, size=rho)]
    I = int(rng.integers(0, 3))
    mn = int(rng.integers(0, 3))
    M = int(mn + rng.integers(0, 3))
    M = max(M, abs(rho - tau))
    Pi = Fr(int(rng.integers(1, 20)), 100)
    Pd = Fr(int(rng.integers(1, 20)), 100)
    Ps = Fr(int(rng.integers(0, 30)), 100)
    prior = None
    if rng.random() < 0.5:
        prior = [[Fr(int(v), 16) for v in rng.integers(1, 16, size=q)] for _ in range(N)]
    return cb, y, N, Pi, Pd, Ps, I, M, mn, prior


def _oracle(cb, y, N, Pi, Pd, Ps, I, M, mn, prior=None, **kw):
    pr = None if prior is None else np.array([[float(v) for v in row] for row in prior])
    return oracle.decode(np.array(cb, dtype=np.uint8), np.array(y, dtype=np.uint8), N,
                         float(Pi), float(Pd), float(Ps), I, M, mn, prior=pr, check=False, **kw)


# ---- P1 --------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_p1_brute_force(seed):
    cb, y, N, Pi, Pd, Ps, I, M, mn, prior = _rand_case(seed)
    b = brute(cb, y, N, Pi, Pd, Ps, I, M, mn, prior)
    r = _oracle(cb, y, N, Pi, Pd, Ps, I, M, mn, prior, grad=True)
    if b["P"] == 0:
        assert r["status"] == oracle.REF_ENOPATH
        return
    assert r["status"] == 0
    assert abs(r["logp"] - math.log(b["P"])) <= 1e-12 * max(1.0, abs(math.log(b["P"])))
    app = np.array(b["app"], dtype=float)
    np.testing.assert_allclose(r["app"], app, rtol=0, atol=1e-13)
    g = np.array(b["dparams"], dtype=float)
    np.testing.assert_allclose(r["dparams"], g, rtol=1e-10, atol=1e-10 * np.abs(g).max())
    dp = np.array(b["dprior"], dtype=float)
    np.testing.assert_allclose(r["dprior"], dp, rtol=1e-11, atol=1e-12 * np.abs(dp).max())


def test_p1_binding_limits_change_result():
    # the same frame under tight and loose limits: both exact, and different
    cb = [[0, 1, 1], [1, 0, 0], [1, 1, 0]]
    y = [0, 1, 1, 1, 1, 0, 0]
    res = []
    for (I, M, mn) in [(1, 1, 1), (2, 2, 2), (3, 3, 3)]:
        b = brute(cb, y, 2, Fr(1, 10), Fr(1, 10), Fr(1, 20), I, M, mn)
        r = _oracle(cb, y, 2, Fr(1, 10), Fr(1, 10), Fr(1, 20), I, M, mn)
        assert abs(r["logp"] - math.log(b["P"])) < 1e-13 * abs(math.log(b["P"]))
        res.append(b["P"])
    assert res[0] < res[1] < res[2]


# ---- P2 --------------------------------------------------------------------

@pytest.mark.parametrize("n,N,I,Pi,Pd,Ps", [(2, 2, 2, 0.15, 0.1, 0.05), (1, 3, 1, 0.2, 0.3, 0.0),
                                            (3, 1, 2, 0.1, 0.05, 0.3)])
def test_p2_total_mass(n, N, I, Pi, Pd, Ps):
    tau = n * N
    mn = max(I * n, n) + 1
    M = max(I * tau, mn)
    q = 2
    cb = np.array([[0] * n, [1] * n], dtype=np.uint8)
    rng = np.random.default_rng(7)
    prior = rng.dirichlet(np.ones(q), size=N)
    total = 0.0
    for L in range(0, tau * (1 + I) + 1):
        for bits in itertools.product((0, 1), repeat=L):
            r = oracle.decode(cb, np.array(bits, dtype=np.uint8), N, Pi, Pd, Ps, I, M, mn,
                              prior=prior, check=False)
            if r["status"] == 0:
                total += math.exp(r["logp"])
            else:
                assert r["status"] == oracle.REF_ENOPATH
    assert abs(total - (1.0 - Pi ** (I + 1)) ** tau) < 1e-12


# ---- P3, P4 ----------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_p3_substitution_channel(seed):
    rng = np.random.default_rng(100 + seed)
    q, n, N = 8, 5, 12
    cb = wl.random_codebook(rng, q, n)
    Ps = float(rng.uniform(0.01, 0.3))
    prior = rng.dirichlet(np.ones(q), size=N)
    y = rng.integers(0, 2, size=n * N).astype(np.uint8)
    r = oracle.decode(cb, y, N, 0.0, 0.0, Ps, 2, 3, 2, prior=prior)
    logp = 0.0
    for i in range(N):
        h = (cb != y[None, n * i:n * (i + 1)]).sum(axis=1)
        lik = prior[i] * Ps ** h * (1 - Ps) ** (n - h)
        logp += math.log(lik.sum())
        np.testing.assert_allclose(r["app"][i], lik / lik.sum(), rtol=1e-12, atol=1e-15)
    assert abs(r["logp"] - logp) < 1e-12 * abs(logp)


def test_p4_useless_channel():
    rng = np.random.default_rng(5)
    q, n, N = 4, 3, 10
    cb = wl.random_codebook(rng, q, n)
    prior = rng.uniform(0.1, 1.0, size=(N, q))          # unnormalised on purpose
    y = rng.integers(0, 2, size=n * N).astype(np.uint8)
    r = oracle.decode(cb, y, N, 0.0, 0.0, 0.5, 2, 2, 1, prior=prior)
    np.testing.assert_allclose(r["app"], prior / prior.sum(1, keepdims=True), rtol=1e-13)
    expect = -n * N * math.log(2) + np.log(prior.sum(1)).sum()
    assert abs(r["logp"] - expect) < 1e-12 * abs(expect)


# ---- P5 --------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2])
def test_p5_invariants(k):
    fr = wl.make_workload(k, nframes=1)[0]
    r = oracle.decode_frame(fr, trace=True)
    np.testing.assert_allclose(r["app"].sum(1), 1.0, rtol=0, atol=1e-13)
    lam = np.log((r["alpha"] * r["beta"]).sum(1)) + r["logA"] + r["logB"]
    np.testing.assert_allclose(lam, r["logp"], rtol=1e-12, atol=0)
    assert np.all(r["alpha"] >= 0) and np.all(r["beta"] >= 0)
    np.testing.assert_allclose(r["alpha"][1:].sum(1), 1.0, atol=1e-13)


# ---- P6 --------------------------------------------------------------------

def test_p5_products_below_fp64_range():
    # a long, noisy frame (q=4, n=4, N=5000, Pi=Pd=0.1, M=900): the
    # normalised forward and backward rows peak at opposite ends of the
    # drift range and max_m alpha_i(m) beta_i(m) falls below 1e-308 mid-
    # frame; the invariants must still hold at every i (evaluated in
    # extended precision)
    fr = wl.random_frame(913, 4, 4, 5000, 0.1, 0.1, 0.0, 2, 900, 5)
    r = oracle.decode_frame(fr, trace=True)
    A = r["alpha"].astype(np.longdouble)
    B = r["beta"].astype(np.longdouble)
    ab = (A * B).sum(1)
    assert float(ab.min()) < 1e-308          # the case this pin is for
    lam = np.log(ab).astype(np.float64) + r["logA"] + r["logB"]
    np.testing.assert_allclose(lam, r["logp"], rtol=1e-12, atol=0)
    lz = r["logZ"] + r["logA"][:-1] + r["logB"][1:]
    np.testing.assert_allclose(lz, r["logp"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(r["app"].sum(1), 1.0, rtol=0, atol=1e-12)


def test_p6_insertion_cap_and_monotonicity():
    fr = wl.random_frame(3, 4, 5, 20, 0.08, 0.08, 0.02, 2, 12, 3)
    base = dict(codebook=fr.codebook, y=fr.y, N=fr.N, Pi=fr.Pi, Pd=fr.Pd, Ps=fr.Ps)
    r6 = oracle.decode(I=6, M=12, mn=3, **base)
    r9 = oracle.decode(I=9, M=12, mn=3, **base)
    assert r6["logp"] == r9["logp"]
    assert np.array_equal(r6["app"], r9["app"])
    lp = [oracle.decode(I=I, M=12, mn=3, **base)["logp"] for I in range(0, 7)
          if oracle.decode(I=I, M=12, mn=3, check=False, **base)["status"] == 0]
    assert all(b >= a for a, b in zip(lp, lp[1:]))
    lpM = [oracle.decode(I=2, M=M, mn=3, **base)["logp"] for M in (8, 10, 14, 20)]
    assert all(b >= a for a, b in zip(lpM, lpM[1:]))
    lpm = [oracle.decode(I=2, M=12, mn=mn, **base)["logp"] for mn in (2, 3, 4, 6)]
    assert all(b >= a for a, b in zip(lpm, lpm[1:]))


# ---- P7 --------------------------------------------------------------------

@pytest.mark.parametrize("Pi,Pd,Ps", [(0.1, 0.2, 0.05), (0.3, 0.1, 0.0), (0.05, 0.05, 0.5)])
def test_p7_n1_hand_forms(Pi, Pd, Ps):
    cb = np.array([[0], [1]], dtype=np.uint8)
    Pt = 1 - Pi - Pd

    def Q(yb, xb):
        return Pt * (1 - Ps) if yb == xb else Pt * Ps

    for x in (0, 1):
        R = oracle.lattice(cb, np.zeros(0, np.uint8), 0, x, Pi, Pd, Ps, 2, 2, 2)
        assert R[2 - 1] == pytest.approx(Pd, rel=1e-15)               # ()
        for y1 in (0, 1):
            R = oracle.lattice(cb, np.array([y1], np.uint8), 0, x, Pi, Pd, Ps, 2, 2, 2)
            assert R[2 + 0] == pytest.approx(Q(y1, x) + Pi / 2 * Pd, rel=1e-14)
            for y2 in (0, 1):
                R = oracle.lattice(cb, np.array([y1, y2], np.uint8), 0, x, Pi, Pd, Ps, 2, 2, 2)
                assert R[2 + 1] == pytest.approx(Pi / 2 * Q(y2, x) + (Pi / 2) ** 2 * Pd,
                                                 rel=1e-14)
                # with I = 1 the double insertion is excluded
                R1 = oracle.lattice(cb, np.array([y1, y2], np.uint8), 0, x, Pi, Pd, Ps, 1, 2, 2)
                assert R1[2 + 1] == pytest.approx(Pi / 2 * Q(y2, x), rel=1e-14)


# ---- P8 --------------------------------------------------------------------

def test_p8_complement_symmetry():
    fr = wl.random_frame(11, 8, 6, 30, 0.05, 0.04, 0.03, 2, 14, 4, with_prior=True)
    r = oracle.decode_frame(fr, grad=True)
    r2 = oracle.decode(1 - fr.codebook, 1 - fr.y, fr.N, fr.Pi, fr.Pd, fr.Ps, fr.I, fr.M, fr.mn,
                       prior=fr.prior, grad=True)
    assert r["logp"] == r2["logp"]
    assert np.array_equal(r["app"], r2["app"])
    assert np.array_equal(r["dparams"], r2["dparams"])


# ---- P9 --------------------------------------------------------------------

def test_p9_prior_gradient_central_differences():
    # d log P / d prior[i][D] against central differences of the oracle's
    # log P (pinned by P1) in that one entry, priors used as given
    fr = wl.random_frame(12, 8, 6, 25, 0.04, 0.03, 0.02, 2, 14, 4, with_prior=True)
    r = oracle.decode_frame(fr, grad=True)
    rng = np.random.default_rng(12)
    h = 1e-7
    for _ in range(12):
        i, D = int(rng.integers(0, fr.N)), int(rng.integers(0, fr.q))
        vals = []
        for sgn in (1, -1):
            pr = fr.prior.copy()
            pr[i, D] += sgn * h
            vals.append(oracle.decode(fr.codebook, fr.y, fr.N, fr.Pi, fr.Pd, fr.Ps, fr.I, fr.M,
                                      fr.mn, prior=pr)["logp"])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - r["dprior"][i, D]) <= 1e-6 * max(1.0, abs(fd)), (i, D, fd)


def test_consistency_logit_gradient_form():
    # not a pin: the softmax chain rule restated on the oracle's outputs
    fr = wl.random_frame(12, 8, 6, 25, 0.04, 0.03, 0.02, 2, 14, 4, with_prior=True)
    r = oracle.decode_frame(fr, grad=True)
    pi = fr.prior
    dlogit = pi * r["dprior"] - pi * (pi * r["dprior"]).sum(1, keepdims=True)
    np.testing.assert_allclose(dlogit, r["app"] - pi, atol=1e-13)


@pytest.mark.parametrize("seed,Ps", [(13, 0.02), (14, 0.1)])
def test_p9_central_differences(seed, Ps):
    fr = wl.random_frame(seed, 8, 6, 30, 0.05, 0.04, Ps, 2, 16, 4, with_prior=True)
    r = oracle.decode_frame(fr, grad=True)
    h = 1e-6
    base = [fr.Pi, fr.Pd, fr.Ps]
    for k in range(3):
        up, dn = list(base), list(base)
        up[k] += h
        dn[k] -= h
        lu = oracle.decode(fr.codebook, fr.y, fr.N, *up, fr.I, fr.M, fr.mn, prior=fr.prior)["logp"]
        ld = oracle.decode(fr.codebook, fr.y, fr.N, *dn, fr.I, fr.M, fr.mn, prior=fr.prior)["logp"]
        fd = (lu - ld) / (2 * h)
        assert abs(fd - r["dparams"][k]) <= 1e-6 * max(1.0, abs(r["dparams"][k]))


@pytest.mark.parametrize("seed", [15, 16, 17])
def test_p9_count_identity(seed):
    # every path has ins - del = rho - tau and T = tau - del transmissions,
    # so E[T] recovered from d/dPi and from d/dPd must agree
    fr = wl.random_frame(seed, 16, 8, 40, 0.06, 0.05, 0.02, 2, 20, 5, with_prior=True)
    r = oracle.decode_frame(fr, grad=True)
    A, B = r["dparams"][0], r["dparams"][1]
    Pt = 1 - fr.Pi - fr.Pd
    T1 = (fr.rho / fr.Pi - A) / (1 / fr.Pi + 1 / Pt)
    T2 = (fr.tau / fr.Pd - B) / (1 / fr.Pd + 1 / Pt)
    assert abs(T1 - T2) <= 1e-9 * fr.tau
    assert 0 <= T1 <= min(fr.tau, fr.rho) + 1e-9


# ---- consistency (not a pin) -----------------------------------------------

def test_consistency_literal_equals_memoised():
    fr = wl.random_frame(18, 8, 6, 20, 0.05, 0.05, 0.02, 2, 10, 4, with_prior=True)
    a = oracle.decode_frame(fr, grad=True)
    b = oracle.decode_frame(fr, grad=True, literal=True)
    assert a["logp"] == b["logp"]
    for k in ("app", "dparams", "dprior"):
        assert np.array_equal(a[k], b[k])


# ---- status codes ------------------------------------------------------------

def test_status_codes():
    cb = np.array([[0, 1], [1, 0]], dtype=np.uint8)
    y = np.array([0, 1, 1, 0], dtype=np.uint8)
    assert oracle.check_code(cb, 0.1, 0.1, 0.0, 2, 2, 1) == oracle.REF_OK
    assert oracle.check_code(np.array([[0, 1], [0, 1]], np.uint8), 0.1, 0.1, 0, 2, 2, 1) == 1
    assert oracle.check_code(cb, 0.6, 0.5, 0, 2, 2, 1) == oracle.REF_EINVAL
    assert oracle.check_code(cb, 0.1, 0.1, 0, 2, 1, 2) == oracle.REF_EINVAL
    assert oracle.check_code(cb, 0.1, 0.1, 0, -1, 2, 1) == oracle.REF_EINVAL
    r = oracle.decode(cb, np.zeros(9, np.uint8), 2, 0.1, 0.1, 0.0, 2, 2, 1, check=False)
    assert r["status"] == oracle.REF_EDRIFT
    # no insertion/deletion and no substitution: y must be a codeword string
    r = oracle.decode(cb, np.array([1, 1, 1, 1], np.uint8), 2, 0.0, 0.0, 0.0, 2, 2, 1, check=False)
    assert r["status"] == oracle.REF_ENOPATH
    r = oracle.decode(cb, y, 2, 0.0, 0.0, 0.0, 2, 2, 1)
    np.testing.assert_array_equal(r["app"], [[1, 0], [0, 1]])


# ---- P11 -------------------------------------------------------------------

def test_p11_point_priors_are_the_known_boundaries():
    fr = wl.random_frame(61, 4, 3, 12, 0.05, 0.05, 0.02, 2, 8, 3)
    Mt = 2 * fr.M + 1
    start = np.zeros(Mt)
    start[fr.M] = 1.0
    end = np.zeros(Mt)
    end[fr.M + fr.rho - fr.tau] = 1.0
    a = oracle.decode_frame(fr, grad=True)
    b = oracle.decode_frame(fr, grad=True, start=start, end=end)
    assert b["status"] == 0
    assert a["logp"] == b["logp"]
    np.testing.assert_array_equal(a["app"], b["app"])
    np.testing.assert_array_equal(a["dparams"], b["dparams"])
    np.testing.assert_array_equal(a["dprior"], b["dprior"])


@pytest.mark.parametrize("seed", range(4))
def test_p11_boundary_priors_brute_force(seed):
    # A frame whose first codeword starts at received bit m0 and whose last
    # ends before bit tau + mN, the bits outside it unscored, is the
    # known-boundary frame of the sub-window y[m0 : tau + mN] (end drift
    # mN - m0).  With M above every reachable drift the limits do not bind
    # in either form, so P(y) = sum phi_0(m0) phi_N(mN) P(sub-window), and
    # the APPs and d log P / d(Pi, Pd, Ps) are the same weighted mixtures.
    rng = np.random.default_rng(700 + seed)
    n, N, q = 2, 2, 3
    tau = n * N
    rho = tau + 2
    words = rng.choice(1 << n, size=q, replace=False)
    cb = [[(int(w) >> (n - 1 - r)) & 1 for r in range(n)] for w in words]
    y = [int(b) for b in rng.integers(0, 2, size=rho)]
    Pi, Pd, Ps = Fr(1, 10), Fr(3, 20), Fr(1, 20)
    I, mn = 2, 2
    M = rho + 1
    Mt = 2 * M + 1
    start = [Fr(0)] * Mt
    end = [Fr(0)] * Mt
    for m0 in (0, 1, 2):
        start[M + m0] = Fr(int(rng.integers(1, 9)), 8)
    for mN in (-1, 0, 1, 2):
        end[M + mN] = Fr(int(rng.integers(1, 9)), 8)
    P = Fr(0)
    num = np.zeros((N, q), dtype=object)
    num[:] = Fr(0)
    dP = [Fr(0)] * 3
    for m0 in range(-M, M + 1):
        for mN in range(-M, M + 1):
            w = start[M + m0] * end[M + mN]
            if w == 0:
                continue
            sub = y[m0:tau + mN]
            Msub = max(tau, len(sub)) + 1
            b = brute(cb, sub, N, Pi, Pd, Ps, I, Msub, mn)
            if b["P"] == 0:
                continue
            P += w * b["P"]
            for i in range(N):
                for D in range(q):
                    num[i, D] += w * b["P"] * b["app"][i][D]
            for k in range(3):
                dP[k] += w * b["P"] * b["dparams"][k]
    assert P > 0
    r = _oracle(cb, y, N, Pi, Pd, Ps, I, M, mn, grad=True,
                start=np.array([float(v) for v in start]),
                end=np.array([float(v) for v in end]))
    assert r["status"] == 0
    lp = math.log(P)
    assert abs(r["logp"] - lp) <= 1e-12 * max(1.0, abs(lp))
    app = np.array([[float(num[i, D] / P) for D in range(q)] for i in range(N)])
    np.testing.assert_allclose(r["app"], app, rtol=0, atol=1e-13)
    g = np.array([float(v / P) for v in dP])
    np.testing.assert_allclose(r["dparams"], g, rtol=1e-10, atol=1e-10 * np.abs(g).max())
