"""Plans read no workspace byte before writing it: every kind of plan (one
codebook, general priors, the MFMA APP, a codebook per symbol, path
thresholds, priors of the frame boundaries; FP32 and FP64; whole frames and
checkpoints; eager, graph and serial schedules) gives the same bits on a
workspace filled with zeros and on one filled with 0xFF bytes (NaN in
either precision).  The eager checkpointed schedule once depended on this:
its sweep parts run beside the rounds of the Gamma pre-pass."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_1802_08483_amd import mapdec
from paper_1802_08483_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _sets():
    g = wl.general_frame
    r = dataclasses.replace
    Mt = lambda fr: 2 * fr.M + 1
    bfr = wl.random_frame(81, 4, 3, 40, 0.06, 0.05, 0.03, 2, 10, 3, with_prior=True)
    st = np.zeros(Mt(bfr))
    for m in range(-1, 4):
        st[bfr.M + m] = 0.2 + 0.1 * (m + 1)
    return {
        "one codebook": [wl.random_frame(5 + f, 16, 10, 300, 0.05, 0.05, 0.01, 2, 40, 6)
                         for f in range(4)],
        "general priors": [wl.random_frame(31 + f, 8, 6, 120, 0.04, 0.05, 0.02, 2, 20, 4,
                                           with_prior=True) for f in range(3)],
        "matrix-unit APP": [wl.random_frame(70 + f, 64, 12, 150, 0.1, 0.1, 0.0, 2, 85, 8)
                            for f in range(2)],
        "codebook per symbol": [g(1, 4, 6, 40, 0.05, 0.05, 0.01, 2, -8, 8, -3, 3),
                                g(6, 8, 7, 60, 0.1, 0.1, 0.0, 2, -40, 40, -5, 5)],
        "path thresholds": [r(wl.random_frame(21, 8, 6, 80, 0.05, 0.05, 0.01, 2, 20, 4),
                              theta=1e-8)],
        "boundary priors": [r(bfr, start_drift=st)],
    }


def _outputs(frames, prec, K, fill, **kw):
    b = mapdec.batch_from_frames(frames, precision=prec, grad=True, checkpoint_K=K)
    b.ws.fill_(fill)
    p = b.plan(**kw)
    p.run()
    torch.cuda.synchronize()
    out = [b.status.cpu().clone(), b.logp.cpu().clone(), b.dparams.cpu().clone()]
    out += [a.cpu().clone() for a in b.apps] + [d.cpu().clone() for d in b.dpriors]
    p.close()
    return out


@pytest.mark.parametrize("prec", [mapdec.FP32, mapdec.FP64])
def test_plans_on_a_stale_workspace(prec):
    for name, frames in _sets().items():
        for K in (0, 9):
            for kw in (dict(graph=False), dict(graph=True), dict(graph=False, serial=True)):
                clean = _outputs(frames, prec, K, 0, **kw)
                stale = _outputs(frames, prec, K, 255, **kw)
                assert (clean[0] == 0).all(), (name, K, kw)
                for k, (a, s) in enumerate(zip(clean, stale)):
                    assert torch.equal(a, s), f"{name} K={K} {kw}: output {k}"
