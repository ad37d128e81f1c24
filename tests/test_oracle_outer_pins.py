"""Pins of the outer-code oracle (oracle/outer.py) against what the
mathematics fixes, independent of its own formulas.

  O1  GF(2^p), p = 1..6: the table is a field (commutative, associative,
      distributive over XOR, unit 1, every nonzero element invertible).
  O2  the polynomial is primitive: the powers of z (element 2) run through
      all q - 1 nonzero elements (p >= 2).
  O3  on codes whose factor graph is a tree, sum-product decoding gives the
      exact marginals: posterior and extrinsic against brute-force
      enumeration of every codeword (q = 2, 4, 8, 16; coefficients drawn so
      that h and 1/h differ).
  O4  the inner decoder's extrinsic output on a tiny frame against exact
      rational enumeration of the channel (tests/exact_bsid.py): the APP
      with the prior divided out, at non-uniform priors.
  O5  one pass of iterate() chains the pieces: the second pass's priors are
      the first pass's outer extrinsic, and its inner APP is the oracle
      decode at those priors.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import outer
from paper_1802_08483_amd import workloads as wl
from exact_bsid import brute


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_o1_field_axioms(p):
    q = 1 << p
    t = outer.gf_table(q)
    a = np.arange(q)
    assert (t == t.T).all()
    assert (t[1] == a).all() and (t[0] == 0).all()
    rng = np.random.default_rng(p)
    trip = (itertools.product(range(q), repeat=3) if q <= 16
            else (tuple(rng.integers(0, q, 3)) for _ in range(20000)))
    for x, y, z in trip:
        assert t[t[x, y], z] == t[x, t[y, z]]
        assert t[x, y ^ z] == t[x, y] ^ t[x, z]
    inv = outer.gf_inverse(q)
    for x in range(1, q):
        assert t[x, inv[x]] == 1
        assert (t[x, 1:] != 0).all()          # no zero divisors


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_o2_primitive(p):
    q = 1 << p
    t = outer.gf_table(q)
    seen, e = set(), 1
    for _ in range(q - 1):
        seen.add(e)
        e = int(t[e, 2])
    assert e == 1 and seen == set(range(1, q))


def _tree_code(q, rows, N, seed):
    rng = np.random.default_rng(seed)
    inv = outer.gf_inverse(q)
    row_ptr, col, coef = [0], [], []
    for r in rows:
        for j in r:
            # prefer coefficients with h != 1/h so a swapped inverse shows
            choices = [h for h in range(1, q) if inv[h] != h] or [1]
            col.append(j)
            coef.append(int(rng.choice(choices)))
        row_ptr.append(len(col))
    return outer.OuterCode(q, N, row_ptr, col, coef)


TREES = [
    (2, 7, [[0, 1, 2], [2, 3, 4], [4, 5, 6]]),
    (4, 7, [[0, 1, 2, 3], [3, 4], [1, 5, 6]]),
    (8, 5, [[0, 1, 2], [2, 3, 4]]),
    (16, 4, [[0, 1, 2], [2, 3]]),
]


@pytest.mark.parametrize("q,N,rows", TREES)
def test_o3_tree_codes_exact(q, N, rows):
    code = _tree_code(q, rows, N, seed=q)
    rng = np.random.default_rng(100 + q)
    L = rng.random((N, q)) + 0.05
    L /= L.sum(1, keepdims=True)
    post, ext = outer.brute_marginals(code, L)
    r = outer.bp_decode(code, L, iters=6)
    np.testing.assert_allclose(r["Q"], post, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["E"], ext, rtol=0, atol=1e-12)


def test_o3_single_check_closed_form():
    # one check x0 + h1 x1 + h2 x2 = 0 over GF(4): the message to x0 is the
    # distribution of h1 x1 + h2 x2, enumerated pair by pair
    q = 4
    t = outer.gf_table(q)
    code = outer.OuterCode(q, 3, [0, 3], [0, 1, 2], [1, 2, 3])
    rng = np.random.default_rng(5)
    L = rng.random((3, q))
    L /= L.sum(1, keepdims=True)
    want = np.zeros(q)
    for x1 in range(q):
        for x2 in range(q):
            want[t[2, x1] ^ t[3, x2]] += L[1, x1] * L[2, x2]
    want /= want.sum()
    r = outer.bp_decode(code, L, iters=1)
    np.testing.assert_allclose(r["E"][0], want, rtol=0, atol=1e-14)


def test_o4_inner_extrinsic_exact():
    fr = wl.random_frame(7, 4, 3, 4, 0.08, 0.06, 0.05, 2, 6, 3, with_prior=True)
    ex = brute(fr.codebook.tolist(), fr.y.tolist(), fr.N, Fraction(fr.Pi), Fraction(fr.Pd),
               Fraction(fr.Ps), fr.I, fr.M, fr.mn,
               prior=[[Fraction(float(v)) for v in row] for row in fr.prior])
    # extrinsic: APP_i(D) / prior_i(D), normalised over D
    want = np.array([[float(ex["app"][i][D] / Fraction(float(fr.prior[i][D])))
                      for D in range(fr.q)] for i in range(fr.N)])
    want /= want.sum(1, keepdims=True)
    r = oracle.decode(fr.codebook, fr.y, fr.N, fr.Pi, fr.Pd, fr.Ps, fr.I, fr.M, fr.mn,
                      prior=fr.prior, extrinsic=True)
    np.testing.assert_allclose(outer.inner_extrinsic(r["dprior"]), want, rtol=0, atol=1e-13)


def test_o5_passes_chain():
    spec, fr = wl.concatenated_frame(11, q=8, n=6, N=24, Pi=0.05, Pd=0.05, Ps=0.01, I=2,
                                     M=12, mn=4, checks=12)
    code = outer.OuterCode(spec.q, spec.N, spec.row_ptr, spec.col, spec.coef)
    assert not code.syndrome(fr.message).any()     # the generator sent a codeword
    out = outer.iterate(fr, code, outer_iters=2, bp_iters=4)
    assert np.allclose(out[0]["prior"], 1.0 / 8)
    np.testing.assert_array_equal(out[1]["prior"], out[0]["E"])
    r = oracle.decode(fr.codebook, fr.y, fr.N, fr.Pi, fr.Pd, fr.Ps, fr.I, fr.M, fr.mn,
                      prior=out[0]["E"])
    np.testing.assert_array_equal(out[1]["app"], r["app"])
    for rec in out:
        for k in ("L", "E", "Q"):
            np.testing.assert_allclose(rec[k].sum(1), 1.0, atol=1e-12)
