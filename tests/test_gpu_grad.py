"""GPU adjoint against the FP64 oracle's forward-mode gradient and against
central differences.

Bars (norm-wise per block, ||g - g_ref||_inf / ||g_ref||_inf): FP64 adjoint
<= 1e-9; FP32 adjoint <= 1e-4 (the stated target), for d log P / d(Pi, Pd,
Ps) and for d log P / d prior.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1802_08483_amd import mapdec
from paper_1802_08483_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {mapdec.FP64: 1e-9, mapdec.FP32: 1e-4}


def _grad(frames, prec):
    b = mapdec.batch_from_frames(frames, precision=prec, grad=True)
    b.run_grad()
    torch.cuda.synchronize()
    return b


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _check(b, f, fr, ref, prec, label):
    assert int(b.status[f]) == 0, label
    gp = b.dparams[f].cpu().numpy()
    assert _rel(gp, ref["dparams"]) <= TOL[prec], f"{label}: dparams {gp} vs {ref['dparams']}"
    dpr = b.dpriors[f].double().cpu().numpy()
    assert _rel(dpr, ref["dprior"]) <= TOL[prec], f"{label}: dprior"
    assert abs(float(b.logp[f]) - ref["logp"]) <= 1e-6 * abs(ref["logp"]), label


def _frames():
    specs = [
        # seed, q, n, N, Pi, Pd, Ps, I, M, mn, prior
        (41, 4, 3, 40, 0.06, 0.05, 0.03, 2, 10, 3, True),
        (42, 8, 6, 50, 0.04, 0.04, 0.01, 2, 14, 4, False),
        (43, 16, 10, 30, 0.05, 0.05, 0.02, 2, 18, 6, True),
        (44, 2, 4, 80, 0.03, 0.02, 0.00, 1, 12, 2, False),    # Ps = 0: d/dPs still defined
        (45, 8, 5, 40, 0.05, 0.06, 0.05, 3, 14, 4, True),     # general insertion cap
        (46, 32, 8, 25, 0.04, 0.03, 0.50, 2, 16, 5, False),   # Ps = 1/2: t1 = t0
        (47, 64, 12, 15, 0.05, 0.05, 0.01, 2, 20, 8, False),
    ]
    return [wl.random_frame(s, q, n, N, Pi, Pd, Ps, I, M, mn, with_prior=pr)
            for (s, q, n, N, Pi, Pd, Ps, I, M, mn, pr) in specs]


@pytest.mark.parametrize("prec", [mapdec.FP64, mapdec.FP32])
def test_adjoint_matches_oracle(prec):
    frames = _frames()
    refs = [oracle.decode_frame(fr, grad=True) for fr in frames]
    b = _grad(frames, prec)
    for f, (fr, ref) in enumerate(zip(frames, refs)):
        _check(b, f, fr, ref, prec, f"frame {f} q={fr.q} n={fr.n} Ps={fr.Ps}")


def test_adjoint_large_drift_range():
    frames = [wl.random_frame(48, 4, 5, 40, 0.10, 0.10, 0.01, 2, 400, 6)]
    ref = oracle.decode_frame(frames[0], grad=True)
    for prec in (mapdec.FP64, mapdec.FP32):
        b = _grad(frames, prec)
        _check(b, 0, frames[0], ref, prec, f"M=400 prec={prec}")


def test_channel_estimation_workload_sampled():
    # 128 frames, q=16 n=10 N=1000, priors from softmax logits, decoded at
    # (0.025, 0.025, 0.015); oracle gradient on sampled frames
    frames = wl.make_workload(4)
    b = _grad(frames, mapdec.FP32)
    assert (b.status.cpu().numpy() == 0).all()
    assert np.isfinite(b.dparams.cpu().numpy()).all()
    for f in (0, 77):
        ref = oracle.decode_frame(frames[f], grad=True)
        _check(b, f, frames[f], ref, mapdec.FP32, f"workload4 frame {f}")


def test_central_differences_of_gpu_decode():
    # FP64 central differences (step 1e-6) of the GPU's own FP64 log P(y)
    fr = wl.make_workload(4, nframes=1)[0]
    g32 = _grad([fr], mapdec.FP32).dparams[0].cpu().numpy()
    h = 1e-6
    fd = []
    for k in range(3):
        vals = []
        for sgn in (1, -1):
            p = [fr.Pi, fr.Pd, fr.Ps]
            p[k] += sgn * h
            code = mapdec.Code(fr.codebook, *p, fr.I, fr.M, fr.mn)
            y = torch.from_numpy(fr.y).cuda()
            prior = torch.from_numpy(fr.prior).cuda()
            bb = mapdec.Batch([(code, y, fr.N, prior)], precision=mapdec.FP64).decode()
            torch.cuda.synchronize()
            vals.append(float(bb.logp[0]))
        fd.append((vals[0] - vals[1]) / (2 * h))
    assert _rel(g32, fd) <= 1e-4, f"{g32} vs {fd}"


def test_autograd_function_logits_and_params():
    # autograd through softmax logits and (Pi, Pd, Ps) against the closed
    # form APP - prior for the logits and the oracle for the parameters
    from paper_1802_08483_amd.autograd import MapDecFn
    frames = wl.make_workload(4, nframes=3)
    fr0 = frames[0]
    logits = torch.from_numpy(np.log(np.stack([f.prior for f in frames]))).cuda()
    logits = logits.float().requires_grad_(True)
    params = torch.tensor([fr0.Pi, fr0.Pd, fr0.Ps], dtype=torch.float64, requires_grad=True)
    ys = [torch.from_numpy(f.y).cuda() for f in frames]
    prior = torch.softmax(logits, dim=-1)
    logp, app = MapDecFn.apply(prior, params, ys, fr0.codebook, fr0.I, fr0.M, fr0.mn)
    logp.sum().backward()
    gl = logits.grad.double().cpu().numpy()
    closed = app.double().cpu().numpy() - prior.detach().double().cpu().numpy()
    assert _rel(gl, closed) <= 1e-4
    refs = [oracle.decode_frame(f, grad=True) for f in frames]
    gp_ref = np.sum([r["dparams"] for r in refs], axis=0)
    assert _rel(params.grad.numpy(), gp_ref) <= 1e-4


def test_row_products_below_fp64_range():
    # q=4, n=4, N=5000, Pi=Pd=0.1, M=900: mid-frame the forward and
    # backward rows peak at opposite ends of the drift range and their
    # product at the posterior's drifts lies below 1e-308 (the oracle pins
    # this case); APP, log P and the gradient must still match the oracle
    fr = wl.random_frame(913, 4, 4, 5000, 0.1, 0.1, 0.0, 2, 900, 5)
    ref = oracle.decode_frame(fr, grad=True)
    for prec in (mapdec.FP64, mapdec.FP32):
        b = _grad([fr], prec)
        _check(b, 0, fr, ref, prec, f"underflow case prec={prec}")
        app = b.apps[0].double().cpu().numpy()
        assert np.abs(app - ref["app"]).max() <= (1e-12 if prec == mapdec.FP64 else 1e-5)
