"""torch.autograd binding of the decoder's adjoint (mapdec_grad).

``MapDecFn.apply(prior, params, y, codebook, I, M, mn, precision, start,
end)`` returns (log P(y) per frame, APP per frame) for a batch of frames
that share one codebook and equal N, and back-propagates d log P / d prior
and d log P / d (Pi, Pd, Ps) computed by the GPU adjoint.  ``start`` /
``end``: optional (B, 2M+1) float64 CUDA tensors, the priors of each
frame's start and end drift (Sec. II-C), inputs only.  The APP output is
not differentiable here.  All arithmetic runs in libmapdec.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import mapdec


class MapDecFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, prior: torch.Tensor, params: torch.Tensor, ys: Sequence[torch.Tensor],
                codebook, I: int, M: int, mn: int, precision: int = mapdec.FP32,
                start=None, end=None):
        """prior: (B, N, q) CUDA tensor (float32 for FP32, float64 for FP64);
        params: (3,) tensor (Pi, Pd, Ps); ys: B uint8 CUDA tensors of 0/1."""
        if prior.dim() != 3:
            raise ValueError("prior must be (B, N, q)")
        B, N, q = prior.shape
        Pi, Pd, Ps = (float(v) for v in params.detach().cpu().tolist())
        code = mapdec.Code(codebook, Pi, Pd, Ps, I, M, mn)
        pr = prior.detach().contiguous()
        batch = mapdec.Batch([(code, ys[b], N, pr[b],
                               None if start is None else start[b],
                               None if end is None else end[b]) for b in range(B)],
                             precision=precision, grad=True, device=prior.device)
        batch.run_grad()
        status = batch.status
        if bool((status != 0).any()):
            raise mapdec.MapdecError(int(status[status != 0][0]), "decode")
        app = torch.stack(batch.apps)
        dprior = torch.stack(batch.dpriors)
        ctx.save_for_backward(dprior, batch.dparams)
        ctx.params_dtype = params.dtype
        ctx.params_device = params.device
        ctx.mark_non_differentiable(app)
        return batch.logp.clone(), app

    @staticmethod
    def backward(ctx, g_logp, g_app):
        dprior, dparams = ctx.saved_tensors
        g = g_logp.to(torch.float64)
        gprior = (g[:, None, None] * dprior.to(torch.float64)).to(dprior.dtype)
        gparams = (g[:, None] * dparams).sum(0).to(ctx.params_device, ctx.params_dtype)
        return gprior, gparams, None, None, None, None, None, None, None, None


def decode_with_grad(prior, params, ys, codebook, I, M, mn, precision=mapdec.FP32,
                     start=None, end=None):
    """Convenience wrapper: (logp, app) with autograd through prior and params."""
    return MapDecFn.apply(prior, params, ys, codebook, I, M, mn, precision, start, end)
