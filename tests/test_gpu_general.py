"""The general scheme on the GPU against the oracle (Sec. II-A: a codebook
C_i per symbol position; Sec. III-B: asymmetric limits m_n^-, m_n^+,
m_tau^-, m_tau^+), through the C ABI.

Cases: per-symbol codebooks with symmetric limits; one codebook with
binding asymmetric limits (the tiled APP path); per-symbol codebooks with
asymmetric limits and general priors; one-sided corridors (m_n^- = 0 and
m_n^+ = 0); a drift range wider than one wave per symbol; checkpointed
gradients; a mixed batch with fixed-code frames; boundary drift priors.
Bars: FP64 APP and log P <= 1e-12, gradient <= 1e-9; FP32 APP <= 1e-5, log
P <= 1e-6 relative, gradient <= 1e-4 (norm-wise per block).
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_1802_08483_amd import mapdec
from paper_1802_08483_amd import workloads as wl

pytestmark = pytest.mark.gpu

BARS = {mapdec.FP64: (1e-12, 1e-12, 1e-9), mapdec.FP32: (1e-5, 1e-6, 1e-4)}


def _frames():
    g = wl.general_frame
    return [
        # per-symbol codebooks, symmetric limits
        g(1, 4, 6, 40, 0.05, 0.05, 0.01, 2, -8, 8, -3, 3),
        # one codebook, asymmetric limits that bind (insertions dominate)
        g(2, 8, 6, 50, 0.08, 0.02, 0.0, 2, -3, 12, -2, 4, per_symbol=False),
        # per-symbol codebooks, asymmetric limits, general priors
        g(3, 16, 8, 30, 0.04, 0.06, 0.02, 2, -9, 5, -3, 1, with_prior=True),
        # one-sided corridors
        g(4, 4, 5, 35, 0.05, 0.03, 0.01, 2, -6, 8, 0, 2),
        g(5, 4, 5, 35, 0.03, 0.05, 0.01, 3, -8, 6, -2, 0),
        # drift range wider than a wave per symbol
        g(6, 8, 7, 60, 0.1, 0.1, 0.0, 2, -40, 40, -5, 5),
    ]


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _check(frames, prec, grad, K=0):
    t_app, t_lp, t_g = BARS[prec]
    b = mapdec.batch_from_frames(frames, precision=prec, grad=grad, checkpoint_K=K)
    if grad:
        b.run_grad()
    else:
        b.decode()
    torch.cuda.synchronize()
    assert (b.status.cpu().numpy() == 0).all()
    for f, fr in enumerate(frames):
        ref = oracle.decode_frame(fr, grad=grad)
        app = b.apps[f].double().cpu().numpy()
        e_app = float(np.abs(app - ref["app"]).max())
        e_lp = abs(float(b.logp[f]) - ref["logp"]) / abs(ref["logp"])
        print(f"frame {f} (q={fr.q} n={fr.n} N={fr.N} limits={fr.limits} "
              f"per-symbol={fr.codebooks is not None}): APP {e_app:.2e} logP {e_lp:.2e}",
              flush=True)
        assert e_app <= t_app, f"frame {f}: APP err {e_app}"
        assert e_lp <= t_lp, f"frame {f}: log P err {e_lp}"
        if grad:
            e_p = _rel(b.dparams[f].cpu().numpy(), ref["dparams"])
            e_pr = _rel(b.dpriors[f].double().cpu().numpy(), ref["dprior"])
            assert e_p <= t_g, f"frame {f}: dparams {b.dparams[f].cpu().numpy()} vs {ref['dparams']}"
            assert e_pr <= t_g, f"frame {f}: dprior err {e_pr}"


def test_limits_bind():
    # the asymmetric limits change the result: the oracle under the
    # symmetric limits that contain them differs
    fr = _frames()[1]
    a = oracle.decode_frame(fr)
    b = oracle.decode(fr.codebook, fr.y, fr.N, fr.Pi, fr.Pd, fr.Ps, fr.I, fr.M, fr.mn)
    assert abs(a["logp"] - b["logp"]) > 1e-6


@pytest.mark.parametrize("prec", [mapdec.FP64, mapdec.FP32])
def test_general_decode(prec):
    _check(_frames(), prec, grad=False)


@pytest.mark.parametrize("prec", [mapdec.FP64, mapdec.FP32])
def test_general_grad(prec):
    _check(_frames(), prec, grad=True)


@pytest.mark.parametrize("prec", [mapdec.FP64, mapdec.FP32])
def test_general_checkpointed(prec):
    _check(_frames()[:3], prec, grad=True, K=7)


def test_general_mixed_with_fixed_code():
    frames = _frames()[:3] + [wl.random_frame(7, 8, 6, 40, 0.05, 0.05, 0.01, 2, 14, 4)]
    _check(frames, mapdec.FP32, grad=True)


def test_general_boundary_priors():
    rng = np.random.default_rng(11)
    frames = []
    for fr in _frames()[:3]:
        Mt = 2 * fr.M + 1
        st = np.zeros(Mt)
        en = np.zeros(Mt)
        lo, hi = fr.limits[0], fr.limits[1]
        for m in range(0, 4):        # start drifts 0..3 (inside the limits)
            if lo <= m <= hi:
                st[fr.M + m] = rng.random()
        d = fr.rho - fr.tau
        for m in range(d - 3, d + 4):
            if -fr.M <= m <= fr.M:
                en[fr.M + m] = rng.random()   # some outside [lo, hi]: ignored
        frames.append(dataclasses.replace(fr, start_drift=st, end_drift=en))
    for prec in (mapdec.FP64, mapdec.FP32):
        _check(frames, prec, grad=True)
