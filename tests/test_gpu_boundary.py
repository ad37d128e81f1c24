"""GPU parity for priors of the frame boundaries (Sec. II-C: the forward
and backward metrics start from the priors of the frame's start and end
drift), through the C ABI, against the FP64 oracle.

Bars as for the known-boundary decode and gradient: FP64 APP max abs error
<= 1e-12, relative log P <= 1e-12, gradients <= 1e-9 (norm-wise); FP32 APP
<= 1e-5, relative log P <= 1e-6, gradients <= 1e-4.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_1802_08483_amd import mapdec
from paper_1802_08483_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL_DEC = {mapdec.FP64: (1e-12, 1e-12), mapdec.FP32: (1e-5, 1e-6)}
TOL_GRAD = {mapdec.FP64: 1e-9, mapdec.FP32: 1e-4}


def _bounded(fr, seed, start=True, end=True):
    """The frame with random (unnormalised) priors on start drifts -1..3 and
    on end drifts within 2 of rho - tau."""
    rng = np.random.default_rng(seed)
    Mt = 2 * fr.M + 1
    st = en = None
    if start:
        st = np.zeros(Mt)
        for m in range(-1, 4):
            st[fr.M + m] = rng.uniform(0.1, 1.0)
    if end:
        en = np.zeros(Mt)
        e0 = fr.rho - fr.tau
        for m in range(e0 - 2, e0 + 3):
            if abs(m) <= fr.M:
                en[fr.M + m] = rng.uniform(0.1, 1.0)
    return dataclasses.replace(fr, start_drift=st, end_drift=en)


def _frames():
    specs = [
        # seed, q, n, N, Pi, Pd, Ps, I, M, mn, prior, start, end
        (81, 4, 3, 40, 0.06, 0.05, 0.03, 2, 10, 3, True, True, True),
        (82, 8, 6, 50, 0.04, 0.04, 0.01, 2, 14, 4, False, True, False),
        (83, 16, 10, 30, 0.05, 0.05, 0.02, 2, 18, 6, True, False, True),
        (84, 2, 4, 80, 0.03, 0.02, 0.00, 1, 12, 2, False, True, True),
        (85, 8, 5, 40, 0.05, 0.06, 0.05, 3, 14, 4, True, True, True),
        (86, 8, 6, 40, 0.05, 0.05, 0.01, 2, 12, 4, False, False, False),
    ]
    out = []
    for (s, q, n, N, Pi, Pd, Ps, I, M, mn, pr, st, en) in specs:
        fr = wl.random_frame(s, q, n, N, Pi, Pd, Ps, I, M, mn, with_prior=pr)
        out.append(_bounded(fr, s, st, en))
    return out


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _check(b, f, ref, prec, grad, label):
    assert int(b.status[f]) == 0, label
    tol_app, tol_lp = TOL_DEC[prec]
    app = b.apps[f].double().cpu().numpy()
    assert float(np.abs(app - ref["app"]).max()) <= tol_app, f"{label}: APP"
    lp = float(b.logp[f])
    assert abs(lp - ref["logp"]) / max(1.0, abs(ref["logp"])) <= tol_lp, f"{label}: log P"
    if grad:
        assert _rel(b.dparams[f].cpu().numpy(), ref["dparams"]) <= TOL_GRAD[prec], \
            f"{label}: dparams {b.dparams[f].cpu().numpy()} vs {ref['dparams']}"
        assert _rel(b.dpriors[f].double().cpu().numpy(), ref["dprior"]) <= TOL_GRAD[prec], \
            f"{label}: dprior"


@pytest.mark.parametrize("prec", [mapdec.FP64, mapdec.FP32])
def test_boundary_priors_decode_and_grad(prec):
    frames = _frames()
    refs = [oracle.decode_frame(fr, grad=True) for fr in frames]
    b = mapdec.batch_from_frames(frames, precision=prec)
    b.decode()
    torch.cuda.synchronize()
    for f, ref in enumerate(refs):
        _check(b, f, ref, prec, False, f"decode frame {f}")
    g = mapdec.batch_from_frames(frames, precision=prec, grad=True)
    g.run_grad()
    torch.cuda.synchronize()
    for f, ref in enumerate(refs):
        _check(g, f, ref, prec, True, f"grad frame {f}")


@pytest.mark.parametrize("prec", [mapdec.FP64, mapdec.FP32])
def test_boundary_priors_checkpointed(prec):
    # segments of 7 symbols: the start prior enters the first segment, the
    # end prior the last one's backward chain and log P
    fr = _bounded(wl.random_frame(91, 8, 5, 60, 0.05, 0.05, 0.01, 2, 16, 4, with_prior=True), 91)
    plain = wl.random_frame(92, 4, 4, 45, 0.04, 0.04, 0.02, 2, 12, 3)
    frames = [fr, plain]
    refs = [oracle.decode_frame(x, grad=True) for x in frames]
    g = mapdec.batch_from_frames(frames, precision=prec, grad=True, checkpoint_K=7)
    g.run_grad()
    torch.cuda.synchronize()
    for f, ref in enumerate(refs):
        _check(g, f, ref, prec, True, f"checkpointed frame {f}")


def test_point_priors_equal_known_boundary():
    fr = wl.random_frame(93, 8, 6, 50, 0.05, 0.05, 0.01, 2, 14, 4)
    Mt = 2 * fr.M + 1
    st = np.zeros(Mt)
    st[fr.M] = 1.0
    en = np.zeros(Mt)
    en[fr.M + fr.rho - fr.tau] = 1.0
    pt = dataclasses.replace(fr, start_drift=st, end_drift=en)
    for prec in (mapdec.FP64, mapdec.FP32):
        a = mapdec.batch_from_frames([fr], precision=prec, grad=True)
        b = mapdec.batch_from_frames([pt], precision=prec, grad=True)
        a.run_grad()
        b.run_grad()
        torch.cuda.synchronize()
        assert torch.equal(a.logp, b.logp)
        assert torch.equal(a.apps[0], b.apps[0])
        assert torch.equal(a.dpriors[0], b.dpriors[0])
        # d/dPi: a g_a - d g_d is rho - tau without priors and the posterior
        # mean of mN - m0 (computed from the rows) with them: equal up to
        # rounding
        assert _rel(b.dparams[0].cpu().numpy(), a.dparams[0].cpu().numpy()) <= TOL_GRAD[prec]


def test_drift_prior_shape_is_checked():
    fr = wl.random_frame(94, 4, 3, 10, 0.05, 0.05, 0.01, 2, 6, 2)
    bad = dataclasses.replace(fr, start_drift=np.ones(2 * fr.M))
    with pytest.raises(TypeError):
        mapdec.batch_from_frames([bad], precision=mapdec.FP64)


def test_boundary_priors_full_batch_sampled():
    # the 256-frame batch (q = 16, n = 10, N = 500) with the boundary priors
    # the benchmark uses, FP32 decode + adjoint as one HIP graph; sampled
    # frames against the oracle, APP row sums on all
    frames = wl.with_boundary_priors(wl.make_workload(2))
    b = mapdec.batch_from_frames(frames, precision=mapdec.FP32, grad=True)
    p = b.plan(graph=True)
    p.run()
    torch.cuda.synchronize()
    assert (b.status.cpu().numpy() == 0).all()
    for f in range(len(frames)):
        s = b.apps[f].double().sum(1).cpu().numpy()
        assert np.abs(s - 1).max() < 1e-5
    for f in (0, 255):
        ref = oracle.decode_frame(frames[f], grad=True)
        _check(b, f, ref, mapdec.FP32, True, f"full batch frame {f}")
    p.close()


def test_autograd_with_boundary_priors():
    # the autograd binding with boundary priors: d log P / d(Pi, Pd, Ps)
    # summed over the batch against the oracle
    from paper_1802_08483_amd.autograd import MapDecFn
    base = [wl.random_frame(95 + k, 8, 5, 40, 0.05, 0.05, 0.02, 2, 14, 4, with_prior=True)
            for k in range(3)]
    frames = [_bounded(fr, 95 + k) for k, fr in enumerate(base)]
    fr0 = frames[0]
    assert all(f.N == fr0.N for f in frames)
    # one shared codebook: draw the received bits of every frame with frame 0's
    frames = [dataclasses.replace(f, codebook=fr0.codebook) for f in frames]
    prior = torch.from_numpy(np.stack([f.prior for f in frames])).cuda()
    params = torch.tensor([fr0.Pi, fr0.Pd, fr0.Ps], dtype=torch.float64, requires_grad=True)
    ys = [torch.from_numpy(f.y).cuda() for f in frames]
    start = torch.from_numpy(np.stack([f.start_drift for f in frames])).cuda()
    end = torch.from_numpy(np.stack([f.end_drift for f in frames])).cuda()
    logp, app = MapDecFn.apply(prior, params, ys, fr0.codebook, fr0.I, fr0.M, fr0.mn,
                               mapdec.FP64, start, end)
    logp.sum().backward()
    refs = [oracle.decode_frame(f, grad=True) for f in frames]
    np.testing.assert_allclose(logp.detach().cpu().numpy(), [r["logp"] for r in refs],
                               rtol=1e-12)
    gp_ref = np.sum([r["dparams"] for r in refs], axis=0)
    assert _rel(params.grad.numpy(), gp_ref) <= 1e-9


def _random_bounded(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 7))
    q = int(rng.integers(2, min(16, 1 << n) + 1))
    N = int(rng.integers(3, 30))
    M = int(rng.integers(6, 20))
    mn = int(rng.integers(1, min(M, 5) + 1))
    fr = wl.random_frame(500 + seed, q, n, N, 0.05, 0.05, 0.02, 2, M, mn,
                         with_prior=bool(rng.integers(0, 2)))
    Mt = 2 * M + 1
    st = en = None
    if rng.random() < 0.8:   # random support, some entries before the received bits
        st = np.where(rng.random(Mt) < 0.3, rng.random(Mt), 0.0)
        st[M] = rng.random() + 0.1
    if rng.random() < 0.8:   # random support around rho - tau, some past the end
        en = np.where(rng.random(Mt) < 0.3, rng.random(Mt), 0.0)
        en[M + fr.rho - fr.tau] = rng.random() + 0.1
    return dataclasses.replace(fr, start_drift=st, end_drift=en)


@pytest.mark.parametrize("prec", [mapdec.FP64, mapdec.FP32])
def test_boundary_priors_random(prec):
    # seeded random frames and supports, plus a frame whose end prior lies
    # wholly past the received bits (no path on either side)
    frames = [_random_bounded(k) for k in range(12)]
    nop = wl.random_frame(530, 4, 3, 10, 0.05, 0.05, 0.02, 2, 8, 3)
    en = np.zeros(2 * nop.M + 1)
    for m in range(-nop.M, nop.M + 1):
        if nop.tau + m > nop.rho:
            en[nop.M + m] = 1.0
    frames.append(dataclasses.replace(nop, end_drift=en))
    refs = [oracle.decode_frame(fr, grad=True, check=False) for fr in frames]
    assert refs[-1]["status"] == oracle.REF_ENOPATH
    g = mapdec.batch_from_frames(frames, precision=prec, grad=True)
    g.run_grad()
    torch.cuda.synchronize()
    for f, ref in enumerate(refs):
        if ref["status"] != 0:
            assert int(g.status[f]) == mapdec.ENOPATH, f"frame {f}"
            continue
        _check(g, f, ref, prec, True, f"random frame {f}")
