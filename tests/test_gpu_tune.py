"""Tuned launch choices (MAPDEC_FLAG_TUNE): the tiled APP's D tile and
waves, and the ring chain's workgroup shape, timed per bucket at plan
creation and kept in a process-wide table.

A tuned plan computes the same quantities with a different grouping of the
same arithmetic (only the order of some sums changes), so its results agree
with the default plan's to rounding: FP32 APP <= 1e-5 absolute, log P <=
1e-6 relative, gradient <= 1e-4 relative; FP64 to 1e-11.  The workspace
size does not depend on the choices, and buckets already tuned are not
timed again.
"""
import numpy as np
import pytest
import torch

from paper_1802_08483_amd import mapdec
from paper_1802_08483_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {mapdec.FP32: (1e-5, 1e-6, 1e-4), mapdec.FP64: (1e-11, 1e-11, 1e-9)}


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _run(frames, prec, tune, graph, grad=True, K=0):
    b = mapdec.batch_from_frames(frames, precision=prec, grad=grad, checkpoint_K=K)
    p = b.plan(graph=graph, tune=tune)
    p.run()
    p.run()
    torch.cuda.synchronize()
    p.close()
    return b


@pytest.mark.parametrize("prec", [mapdec.FP32, mapdec.FP64])
def test_tuned_plan_matches_default(prec):
    mapdec.tune_reset()
    frames = wl.make_workload(3, nframes=160)
    ref = _run(frames, prec, tune=False, graph=True)
    assert mapdec.tune_entries() == 0
    for graph, K in ((True, 0), (False, 0), (True, 29)):
        b = _run(frames, prec, tune=True, graph=graph, K=K)
        assert b.ws_bytes == mapdec.batch_from_frames(frames, precision=prec, grad=True,
                                                      checkpoint_K=K).ws_bytes
        assert (b.status.cpu().numpy() == 0).all()
        t_app, t_lp, t_g = TOL[prec]
        for f in range(len(frames)):
            app = b.apps[f].double().cpu().numpy()
            assert float(np.abs(app - ref.apps[f].double().cpu().numpy()).max()) <= t_app, f
            lp, lr = float(b.logp[f]), float(ref.logp[f])
            assert abs(lp - lr) <= t_lp * max(1.0, abs(lr)), f
            assert _rel(b.dparams[f].cpu().numpy(), ref.dparams[f].cpu().numpy()) <= t_g, f
            assert _rel(b.dpriors[f].double().cpu().numpy(),
                        ref.dpriors[f].double().cpu().numpy()) <= t_g, f
    n = mapdec.tune_entries()
    assert n > 0
    # the same buckets again: nothing new is timed
    _run(frames[:40], prec, tune=True, graph=True)
    assert mapdec.tune_entries() == n
    mapdec.tune_reset()
    assert mapdec.tune_entries() == 0
