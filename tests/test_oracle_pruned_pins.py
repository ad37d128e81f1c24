"""Pins of the oracle's path thresholds (the flexibility list of Sec.
III-B: thresholds so that low-probability trellis paths are not pursued).

  T1  theta = 0 reproduces the plain decode bitwise.
  T2  Exact enumeration in rational arithmetic (tests/exact_bsid.py,
      brute_pruned): the kept drifts at every boundary from the forward
      masses of the kept path prefixes, then P(y), APPs and gradients of
      the kept paths; thresholds that keep different sets on tiny frames.
  T3  Invariants of the pruned trellis: APP rows sum to 1, and
      log sum_m alpha_i beta_i + log A_i + log B_i = log P at every i.
  T4  Monotonicity: the kept paths' P(y) does not increase with theta.
  T5  Invalid thresholds are rejected.
  T6  The start row is pruned like every other row: a start-drift prior
      decodes as the same prior with its entries below theta times its sum
      set to zero (and the others kept as given).
Planted mistakes (backward recursion not restricted to the kept states;
pruning against the row maximum instead of its sum) fail T2; leaving the
start row unpruned fails T6.
"""
import itertools

import numpy as np
import pytest

import oracle
from exact_bsid import brute_pruned

CASES = [
    # (seed, q, n, N, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi, per_symbol, prior)
    (1, 2, 3, 3, 0.2, 0.2, 0.1, 2, -3, 3, -2, 2, False, False),
    (2, 2, 3, 3, 0.15, 0.25, 0.05, 1, -3, 3, -2, 2, True, True),
    (3, 3, 2, 3, 0.2, 0.1, 0.1, 2, -2, 3, -1, 2, True, False),
]


def _frame(seed, q, n, N, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi, per_symbol, prior):
    rng = np.random.default_rng(seed)
    cbs = []
    for _ in range(N if per_symbol else 1):
        words = rng.choice(1 << n, size=q, replace=False)
        cbs.append([[(w >> (n - 1 - r)) & 1 for r in range(n)] for w in words])
    if not per_symbol:
        cbs = cbs * N
    rho = n * N + int(rng.integers(-1, 2))
    y = [int(b) for b in rng.integers(0, 2, rho)]
    pr = None
    if prior:
        p = rng.random((N, q)) + 0.2
        pr = (p / p.sum(1, keepdims=True)).tolist()
    return cbs, y, pr


def _ratios(cbs, y, N, Pi, Pd, Ps, I, lim, pr):
    # the normalised forward metrics of the pruned recursion at theta -> 0+
    # (every nonzero state kept): candidate thresholds between them
    r = oracle.decode_general(np.array(cbs, np.uint8), np.array(y, np.uint8), N, Pi, Pd, Ps,
                              I, *lim, prior=None if pr is None else np.array(pr),
                              trace=True, theta=1e-300)
    a = r["alpha"][1:]
    return sorted({float(v) for v in a.ravel() if v > 0})


@pytest.mark.parametrize("case", CASES)
def test_t1_theta_zero_is_plain(case):
    seed, q, n, N, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi, per_sym, prior = case
    cbs, y, pr = _frame(*case)
    args = (np.array(cbs, np.uint8), np.array(y, np.uint8), N, Pi, Pd, Ps, I, mt_lo, mt_hi,
            mn_lo, mn_hi)
    prr = None if pr is None else np.array(pr)
    a = oracle.decode_general(*args, prior=prr, grad=True)
    b = oracle.decode_general(*args, prior=prr, grad=True, theta=0.0)
    assert a["logp"] == b["logp"]
    assert np.array_equal(a["app"], b["app"]) and np.array_equal(a["dparams"], b["dparams"])


@pytest.mark.parametrize("case", CASES)
def test_t2_brute_force(case):
    seed, q, n, N, Pi, Pd, Ps, I, mt_lo, mt_hi, mn_lo, mn_hi, per_sym, prior = case
    cbs, y, pr = _frame(*case)
    lim = (mt_lo, mt_hi, mn_lo, mn_hi)
    vals = _ratios(cbs, y, N, Pi, Pd, Ps, I, lim, pr)
    # thresholds midway between neighbouring metric values (no decision
    # near a tie), a few of them, smallest to largest
    mids = [(u + v) / 2 for u, v in zip(vals, vals[1:]) if v > u * (1 + 1e-6)]
    picks = [m for m in mids if m < 0.5][:: max(1, len(mids) // 4)][:4]
    assert picks, "no threshold prunes anything"
    pruned_any = False
    for theta in picks:
        ex = brute_pruned(cbs, y, N, Pi, Pd, Ps, I, *lim, theta=theta, prior=pr)
        r = oracle.decode_general(np.array(cbs, np.uint8), np.array(y, np.uint8), N, Pi, Pd,
                                  Ps, I, *lim, prior=None if pr is None else np.array(pr),
                                  grad=True, theta=theta, check=False)
        if ex["P"] == 0:
            assert r["status"] == oracle.REF_ENOPATH
            continue
        assert r["status"] == 0
        full = sum(len(range(mt_lo, mt_hi + 1)) for _ in range(N))
        pruned_any |= sum(len(k) for k in ex["kept"]) < full
        assert abs(r["logp"] - float(np.log(float(ex["P"])))) <= 1e-12 * abs(r["logp"]) + 1e-13
        app = np.array([[float(v) for v in row] for row in ex["app"]])
        assert np.abs(r["app"] - app).max() <= 1e-13
        dp = np.array([float(v) for v in ex["dparams"]])
        assert np.abs(r["dparams"] - dp).max() <= 1e-12 * max(1.0, np.abs(dp).max())
        dpr = np.array([[float(v) for v in row] for row in ex["dprior"]])
        assert np.abs(r["dprior"] - dpr).max() <= 1e-12 * max(1.0, np.abs(dpr).max())
    assert pruned_any


@pytest.mark.parametrize("theta", [1e-9, 1e-6, 1e-3])
def test_t3_invariants(theta):
    from paper_1802_08483_amd import workloads as wl
    fr = wl.general_frame(41, 8, 6, 60, 0.05, 0.05, 0.01, 2, -12, 12, -3, 3)
    r = oracle.decode_general(fr.codebooks, fr.y, fr.N, fr.Pi, fr.Pd, fr.Ps, fr.I, *fr.limits,
                              trace=True, theta=theta)
    assert np.abs(r["app"].sum(1) - 1).max() <= 1e-12
    for i in range(fr.N + 1):
        s = float((r["alpha"][i] * r["beta"][i]).sum())
        assert abs(np.log(s) + r["logA"][i] + r["logB"][i] - r["logp"]) <= 1e-9 * abs(r["logp"])
    kept = (r["alpha"] > 0).sum()
    assert kept < (r["alpha"].shape[0] * r["alpha"].shape[1])   # something was pruned


def test_t4_monotone_in_theta():
    from paper_1802_08483_amd import workloads as wl
    fr = wl.general_frame(42, 8, 6, 80, 0.05, 0.05, 0.01, 2, -14, 14, -3, 3)
    lps = [oracle.decode_general(fr.codebooks, fr.y, fr.N, fr.Pi, fr.Pd, fr.Ps, fr.I,
                                 *fr.limits, theta=t)["logp"]
           for t in (0.0, 1e-12, 1e-6, 1e-4, 1e-3)]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(lps, lps[1:]))
    assert lps[-1] < lps[0]


def test_t5_invalid_theta():
    cbs, y, pr = _frame(*CASES[0])
    for theta in (-0.1, 1.0, float("nan")):
        r = oracle.decode_general(np.array(cbs, np.uint8), np.array(y, np.uint8), 3, 0.2, 0.2,
                                  0.1, 2, -3, 3, -2, 2, theta=theta, check=False)
        assert r["status"] == oracle.REF_EINVAL


def test_t6_start_row_pruned():
    from paper_1802_08483_amd import workloads as wl
    fr = wl.general_frame(43, 4, 6, 40, 0.05, 0.05, 0.01, 2, -10, 10, -3, 3)
    Mt = 21
    start = np.zeros(Mt)
    start[10:15] = [0.5, 0.3, 0.15, 1e-5, 2e-4]   # drifts 0 .. 4
    theta = 1e-3
    cut = np.where(start < theta * start.sum(), 0.0, start)
    args = (fr.codebooks, fr.y, fr.N, fr.Pi, fr.Pd, fr.Ps, fr.I, *fr.limits)
    a = oracle.decode_general(*args, start=start, theta=theta, grad=True)
    b = oracle.decode_general(*args, start=cut, theta=theta, grad=True)
    assert abs(a["logp"] - b["logp"]) <= 1e-13 * abs(a["logp"])
    assert np.abs(a["app"] - b["app"]).max() <= 1e-13
    c = oracle.decode_general(*args, start=start, theta=0.0)
    assert abs(c["logp"] - a["logp"]) > 1e-9   # the two small entries mattered
