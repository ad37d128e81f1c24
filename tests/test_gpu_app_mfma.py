"""GPU parity of the APP on the matrix units (FP32 batches, one codebook,
16 < q <= 64) against the FP64 CPU oracle.

Bars as for every FP32 decode: APP max abs error <= 1e-5, relative log P(y)
error <= 1e-6; gradients (d log P / d prior, d log P / d(Pi, Pd, Ps))
relative error <= 1e-4.  The cases span one and two D tiles (q from 17 to
64), blocks of 64 symbols with ragged last blocks, a block's span split
into parts (a batch of few blocks) and not split (a batch of many), general
priors, and rows whose products lie far below the FP32 range.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1802_08483_amd import mapdec
from paper_1802_08483_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _check(b, f, ref, label, grad=False):
    assert int(b.status[f]) == 0, label
    app = b.apps[f].double().cpu().numpy()
    err = float(np.abs(app - ref["app"]).max())
    assert err <= 1e-5, f"{label}: APP err {err:.3e}"
    lp = float(b.logp[f])
    assert abs(lp - ref["logp"]) <= 1e-6 * max(1.0, abs(ref["logp"])), f"{label}: logP"
    if grad:
        def rel(a, r):
            a, r = np.asarray(a, float), np.asarray(r, float)
            return float(np.abs(a - r).max() / max(np.abs(r).max(), 1e-300))
        assert rel(b.dparams[f].cpu().numpy(), ref["dparams"]) <= 1e-4, f"{label}: dparams"
        assert rel(b.dpriors[f].double().cpu().numpy(), ref["dprior"]) <= 1e-4, f"{label}: dprior"


def _few_block_frames():
    specs = [
        # seed, q, n, N, Pi, Pd, Ps, I, M, mn, prior
        (61, 17, 5, 64, 0.05, 0.05, 0.01, 2, 60, 4, False),    # one full block
        (62, 32, 8, 137, 0.05, 0.04, 0.02, 2, 150, 5, True),   # 2 blocks + 9 symbols
        (63, 48, 6, 200, 0.04, 0.05, 0.01, 2, 90, 6, False),   # two D tiles, 16 idle
        (64, 64, 12, 100, 0.06, 0.06, 0.00, 2, 120, 8, True),  # mn = 8, two full D tiles
        (65, 24, 5, 30, 0.03, 0.03, 0.01, 2, 40, 3, False),    # a block of 30 rows
    ]
    return [wl.random_frame(s, q, n, N, Pi, Pd, Ps, I, M, mn, with_prior=pr)
            for (s, q, n, N, Pi, Pd, Ps, I, M, mn, pr) in specs]


def test_decode_few_blocks_split_spans():
    # 13 blocks in the batch: each block's span is split into parts
    frames = _few_block_frames()
    refs = [oracle.decode_frame(fr) for fr in frames]
    b = mapdec.batch_from_frames(frames, precision=mapdec.FP32)
    b.decode()
    torch.cuda.synchronize()
    for f, (fr, ref) in enumerate(zip(frames, refs)):
        _check(b, f, ref, f"frame {f} q={fr.q} N={fr.N}")


def test_gradients_few_blocks():
    frames = _few_block_frames()
    refs = [oracle.decode_frame(fr, grad=True) for fr in frames]
    b = mapdec.batch_from_frames(frames, precision=mapdec.FP32, grad=True)
    b.run_grad()
    torch.cuda.synchronize()
    for f, (fr, ref) in enumerate(zip(frames, refs)):
        _check(b, f, ref, f"grad frame {f} q={fr.q}", grad=True)


def test_many_blocks_sampled():
    # 600 blocks: one part per block; frames checked at three positions
    frames = [wl.random_frame(700 + k, 32, 8, 320, 0.04, 0.04, 0.01, 2, 60, 5,
                              with_prior=(k % 3 == 0)) for k in range(120)]
    b = mapdec.batch_from_frames(frames, precision=mapdec.FP32)
    b.decode()
    torch.cuda.synchronize()
    assert (b.status.cpu().numpy() == 0).all()
    for f in range(len(frames)):
        s = b.apps[f].double().sum(1).cpu().numpy()
        assert np.abs(s - 1).max() < 1e-5
    for f in (0, 59, 119):
        _check(b, f, oracle.decode_frame(frames[f]), f"batch frame {f}")


def test_row_products_below_fp32_range():
    # q=32, N=1500, Pi=Pd=0.1, M=450: mid-frame the forward and backward
    # rows peak at opposite ends of the drift range and the largest product
    # alpha_i(m) beta_i(m) of a row lies far below the FP32 range, so the
    # matrix operands are formed from mantissas and exponent sums
    fr = wl.random_frame(914, 32, 5, 1500, 0.1, 0.1, 0.0, 2, 450, 5)
    tr = oracle.decode_frame(fr, trace=True)
    ab = (tr["alpha"].astype(np.longdouble) * tr["beta"].astype(np.longdouble)).sum(1)
    assert float(ab.min()) < 1e-100          # the case this test is for
    ref = oracle.decode_frame(fr, grad=True)
    b = mapdec.batch_from_frames([fr], precision=mapdec.FP32, grad=True)
    b.run_grad()
    torch.cuda.synchronize()
    _check(b, 0, ref, "underflow case q=32", grad=True)
