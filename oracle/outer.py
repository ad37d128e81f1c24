"""Iterative decoding with an outer code: FP64 CPU oracle (numpy).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code
with the GPU library.

Sec. II-A: the inner code is normally serially concatenated with an outer
code; the MAP decoder's posteriors start the outer decoder, and iterative
decoding sets the inner decoder's symbol priors P(D_i = D) (Sec. II-C) from
the outer decoder's extrinsic information of the previous pass.

The outer code is a linear code over GF(q), q = 2^p, 1 <= p <= 6, given by
a sparse parity-check matrix H over GF(q): x is a codeword when
sum_j H[c, j] x_j = 0 in GF(q) for every row c.  GF(2^p): the elements are
the integers 0 .. q-1 read as polynomials over GF(2) (bit k the coefficient
of z^k), addition is bitwise XOR, multiplication is the product of the
polynomials reduced modulo the primitive polynomial PRIMITIVE[p].

It is decoded by belief propagation (sum-product) on its factor graph,
written out from its definition, flooding schedule:
  - v(j->c)(a) proportional to L_j(a) prod_{c' != c} u(c'->j)(a), at first
    L_j(a) (L: the channel, here the inner decoder's extrinsic output);
  - u(c->j)(a): the probability that row c holds when x_j = a and the other
    symbols x_k of the row are independent with distributions v(k->c): the
    distribution of sum_{k != j} H[c, k] x_k (a convolution under XOR of
    the distributions of the products H[c, k] x_k) at H[c, j] a (in
    characteristic 2, -y = y);
  - after the last iteration: posterior Q_j(a) proportional to
    L_j(a) prod_c u(c->j)(a), extrinsic E_j(a) proportional to
    prod_c u(c->j)(a).
Every message is normalised to sum 1; a vector that sums to 0 becomes
uniform.  One iteration = every check update, then every variable update.

The inner decoder's extrinsic output is the APP with the symbol's own prior
divided out: APP_i(D) = prior_i(D) U_i(D) / Z_i (eqs. 1-3), so the
extrinsic is U_i(D) / sum_D U_i(D), i.e. d log P / d prior_i(D) normalised.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

# primitive polynomials of GF(2^p) over GF(2), bit k = coefficient of z^k
PRIMITIVE = {1: 0b11, 2: 0b111, 3: 0b1011, 4: 0b10011, 5: 0b100101, 6: 0b1000011}


def field_bits(q: int) -> int:
    p = int(q).bit_length() - 1
    if q < 2 or (1 << p) != q or p not in PRIMITIVE:
        raise ValueError("outer code alphabet must be 2^p, 1 <= p <= 6")
    return p


def gf_mul(a: int, b: int, p: int) -> int:
    """Product in GF(2^p): carry-less multiplication, then reduction."""
    r = 0
    for k in range(p):
        if (b >> k) & 1:
            r ^= a << k
    for k in range(2 * p - 2, p - 1, -1):
        if (r >> k) & 1:
            r ^= PRIMITIVE[p] << (k - p)
    return r


def gf_table(q: int) -> np.ndarray:
    """q x q multiplication table of GF(q)."""
    p = field_bits(q)
    return np.array([[gf_mul(a, b, p) for b in range(q)] for a in range(q)], dtype=np.int64)


def gf_inverse(q: int) -> np.ndarray:
    """inv[a] with a inv[a] = 1 (inv[0] = 0), by search over the table."""
    t = gf_table(q)
    inv = np.zeros(q, dtype=np.int64)
    for a in range(1, q):
        inv[a] = int(np.nonzero(t[a] == 1)[0][0])
    return inv


def _normalise(v: np.ndarray) -> np.ndarray:
    s = v.sum()
    return v / s if s > 0 else np.full_like(v, 1.0 / v.shape[0])


def _xor_conv(f: np.ndarray, g: np.ndarray, xidx: np.ndarray) -> np.ndarray:
    """(f * g)(a) = sum_b f(b) g(a XOR b); xidx[b, a] = a XOR b."""
    return (f[:, None] * g[xidx]).sum(axis=0)


class OuterCode:
    """Parity-check matrix in row-compressed form: row c holds the symbols
    col[row_ptr[c] : row_ptr[c+1]] with coefficients coef[...] (1 .. q-1)."""

    def __init__(self, q: int, N: int, row_ptr: Sequence[int], col: Sequence[int],
                 coef: Sequence[int]):
        self.q, self.N = int(q), int(N)
        self.p = field_bits(q)
        self.row_ptr = np.asarray(row_ptr, dtype=np.int64)
        self.col = np.asarray(col, dtype=np.int64)
        self.coef = np.asarray(coef, dtype=np.int64)
        self.m = self.row_ptr.shape[0] - 1
        if (self.coef < 1).any() or (self.coef >= q).any():
            raise ValueError("coefficients must be nonzero field elements")
        if (self.col < 0).any() or (self.col >= N).any():
            raise ValueError("column index out of range")
        self.mul = gf_table(q)

    def rows(self):
        for c in range(self.m):
            a, b = self.row_ptr[c], self.row_ptr[c + 1]
            yield c, self.col[a:b], self.coef[a:b]

    def syndrome(self, x: Sequence[int]) -> np.ndarray:
        x = np.asarray(x, dtype=np.int64)
        out = np.zeros(self.m, dtype=np.int64)
        for c, js, hs in self.rows():
            s = 0
            for j, h in zip(js, hs):
                s ^= int(self.mul[h, x[j]])
            out[c] = s
        return out


def bp_decode(code: OuterCode, L: np.ndarray, iters: int) -> Dict[str, np.ndarray]:
    """Sum-product decoding of ``code`` with channel distributions L (N x q).
    Returns the extrinsic ``E`` and posterior ``Q`` (N x q) after ``iters``
    iterations (iters >= 1), and the last check-to-variable messages."""
    if iters < 1:
        raise ValueError("iters >= 1")
    q, N = code.q, code.N
    L = np.asarray(L, dtype=np.float64)
    if L.shape != (N, q):
        raise ValueError("L must be N x q")
    Ln = np.array([_normalise(L[j]) for j in range(N)])
    xidx = np.bitwise_xor.outer(np.arange(q), np.arange(q))   # [b, a] = a ^ b
    E_edges = code.col.shape[0]
    v = np.array([Ln[code.col[e]] for e in range(E_edges)])   # v(j->c) per edge
    u = np.zeros_like(v)
    for _ in range(iters):
        # check updates
        for c, js, hs in code.rows():
            base = code.row_ptr[c]
            d = js.shape[0]
            # distribution of the product h x for each edge: w[h x] = v[x]
            w = np.zeros((d, q))
            for k in range(d):
                w[k, code.mul[hs[k], np.arange(q)]] = v[base + k]
            for t in range(d):
                s = np.zeros(q)
                s[0] = 1.0
                for k in range(d):
                    if k != t:
                        s = _xor_conv(s, w[k], xidx)
                u[base + t] = _normalise(s[code.mul[hs[t], np.arange(q)]])
        # variable updates
        edges_of = [[] for _ in range(N)]
        for e in range(E_edges):
            edges_of[code.col[e]].append(e)
        for j in range(N):
            for e in edges_of[j]:
                prod = Ln[j].copy()
                for e2 in edges_of[j]:
                    if e2 != e:
                        prod = prod * u[e2]
                v[e] = _normalise(prod)
    E = np.zeros((N, q))
    Q = np.zeros((N, q))
    edges_of = [[] for _ in range(N)]
    for e in range(E_edges):
        edges_of[code.col[e]].append(e)
    for j in range(N):
        ext = np.ones(q)
        for e in edges_of[j]:
            ext = ext * u[e]
        E[j] = _normalise(ext)
        Q[j] = _normalise(Ln[j] * ext)
    return {"E": E, "Q": Q, "u": u}


def inner_extrinsic(dprior: np.ndarray) -> np.ndarray:
    """U_i(D) / sum_D U_i(D) from d log P / d prior_i(D) = U_i(D) / Z_i."""
    return np.array([_normalise(r) for r in np.asarray(dprior, dtype=np.float64)])


def iterate(frame, code: OuterCode, outer_iters: int, bp_iters: int) -> List[Dict]:
    """Iterative decoding of one frame (workloads.Frame whose message is a
    codeword of ``code``): per pass the inner MAP decoder (the plain oracle)
    with the current priors (uniform at first), its extrinsic output as the
    outer decoder's channel, ``bp_iters`` iterations of belief propagation,
    and the outer extrinsic output as the next pass's priors.  Returns per
    pass: inner ``app`` and ``logp``, ``L`` (inner extrinsic), ``E`` and
    ``Q`` (outer extrinsic and posterior), ``prior`` (the pass's priors)."""
    from . import decode   # the plain inner oracle

    if frame.q != code.q or frame.N != code.N:
        raise ValueError("frame and outer code disagree on q or N")
    prior = None
    out = []
    for _ in range(outer_iters):
        r = decode(frame.codebook, frame.y, frame.N, frame.Pi, frame.Pd, frame.Ps, frame.I,
                   frame.M, frame.mn, prior=prior, extrinsic=True)
        L = inner_extrinsic(r["dprior"])
        b = bp_decode(code, L, bp_iters)
        out.append({"app": r["app"], "logp": r["logp"], "L": L, "E": b["E"], "Q": b["Q"],
                    "prior": (np.full((frame.N, frame.q), 1.0 / frame.q) if prior is None
                              else prior)})
        prior = b["E"]
    return out


def brute_marginals(code: OuterCode, L: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Exact posterior marginals of every symbol over all codewords of a
    tiny code, P(x_j = a) proportional to sum over codewords with x_j = a of
    prod_k L_k(x_k), and the extrinsic (the same sum with L_j left out)."""
    q, N = code.q, code.N
    import itertools
    post = np.zeros((N, q))
    ext = np.zeros((N, q))
    for x in itertools.product(range(q), repeat=N):
        if code.syndrome(x).any():
            continue
        w = np.array([L[k, x[k]] for k in range(N)])
        tot = w.prod()
        for j in range(N):
            post[j, x[j]] += tot
            ext[j, x[j]] += np.prod(np.delete(w, j))
    return (np.array([_normalise(r) for r in post]), np.array([_normalise(r) for r in ext]))
