"""GPU parity of iterative decoding with an outer code (Sec. II-A) against
the FP64 CPU oracle (oracle/outer.py), through the C ABI.

Bars.  Belief propagation alone from the same channel: FP64 max abs error
<= 1e-12, FP32 <= 2e-5 (Walsh-Hadamard transforms of log2 q stages and
products over up to 31 messages in FP32, against direct convolutions in
FP64).  Whole passes (inner decoder, then belief propagation, the outer
extrinsic output fed back as priors): FP64 <= 1e-9 on every pass's inner
APP, extrinsic and posterior; FP32 <= 1e-4 (the inner FP32 APP's 1e-5
carried through the outer iterations).
"""
import numpy as np
import pytest
import torch

from oracle import outer as ref
from paper_1802_08483_amd import mapdec
from paper_1802_08483_amd import workloads as wl

pytestmark = pytest.mark.gpu

BP_TOL = {mapdec.FP64: 1e-12, mapdec.FP32: 2e-5}
PASS_TOL = {mapdec.FP64: 1e-9, mapdec.FP32: 1e-4}


def _ref_code(spec):
    return ref.OuterCode(spec.q, spec.N, spec.row_ptr, spec.col, spec.coef)


def _bp_gpu(spec, chan, iters, prec):
    dt = torch.float64 if prec == mapdec.FP64 else torch.float32
    oc = mapdec.Outer.from_spec(spec)
    ch = torch.as_tensor(chan, dtype=dt).cuda().contiguous()
    extr = torch.zeros_like(ch)
    post = torch.zeros_like(ch)
    ws = torch.empty(oc.workspace_size(ch.shape[0], prec), dtype=torch.uint8, device="cuda")
    oc.decode(ch, extr, post, iters, ws)
    torch.cuda.synchronize()
    return extr.double().cpu().numpy(), post.double().cpu().numpy()


def _random_channel(rng, F, N, q):
    L = rng.random((F, N, q)) ** 3 + 1e-3
    return L / L.sum(2, keepdims=True)


@pytest.mark.parametrize("prec", [mapdec.FP64, mapdec.FP32])
@pytest.mark.parametrize("q,N,checks", [(2, 40, 20), (4, 60, 30), (16, 120, 60), (64, 48, 24)])
def test_belief_propagation_against_oracle(prec, q, N, checks):
    rng = np.random.default_rng(q * 1000 + N)
    spec = wl.outer_code(rng, q, N, checks, 3)
    chan = _random_channel(rng, 3, N, q)
    code = _ref_code(spec)
    for iters in (1, 4):
        extr, post = _bp_gpu(spec, chan, iters, prec)
        for f in range(chan.shape[0]):
            r = ref.bp_decode(code, chan[f], iters)
            assert np.abs(extr[f] - r["E"]).max() <= BP_TOL[prec], f"q={q} it={iters} E"
            assert np.abs(post[f] - r["Q"]).max() <= BP_TOL[prec], f"q={q} it={iters} Q"


def test_unnormalised_and_zero_channel_rows():
    # rows are divided by their sum; a row summing to zero counts as uniform
    rng = np.random.default_rng(9)
    spec = wl.outer_code(rng, 8, 32, 16, 3)
    chan = _random_channel(rng, 1, 32, 8) * 7.5
    chan[0, 3] = 0.0
    extr, post = _bp_gpu(spec, chan, 3, mapdec.FP64)
    fixed = chan[0].copy()
    fixed[3] = 1.0 / 8
    r = ref.bp_decode(_ref_code(spec), fixed, 3)
    assert np.abs(extr[0] - r["E"]).max() <= 1e-12
    assert np.abs(post[0] - r["Q"]).max() <= 1e-12


@pytest.mark.parametrize("prec", [mapdec.FP64, mapdec.FP32])
def test_iterative_passes_against_oracle(prec):
    frames, specs = [], []
    for seed, (q, n, N, checks) in enumerate([(8, 6, 48, 24), (16, 8, 40, 16), (4, 5, 64, 32)]):
        spec, fr = wl.concatenated_frame(seed + 20, q=q, n=n, N=N, Pi=0.06, Pd=0.06, Ps=0.02,
                                         I=2, M=14, mn=4, checks=checks)
        frames.append(fr)
        specs.append(spec)
    passes, bp_iters = 3, 5
    for fr, spec in zip(frames, specs):
        refs = ref.iterate(fr, _ref_code(spec), passes, bp_iters)
        it = mapdec.iterative_from_frames([fr], spec, precision=prec)
        for p in range(passes):
            it.run_pass(bp_iters)
            torch.cuda.synchronize()
            app = it.batch.apps[0].double().cpu().numpy()
            tol = PASS_TOL[prec]
            assert np.abs(app - refs[p]["app"]).max() <= tol, f"q={fr.q} pass {p} APP"
            E = it.prior[0].double().cpu().numpy()
            Q = it.post[0].double().cpu().numpy()
            assert np.abs(E - refs[p]["E"]).max() <= tol, f"q={fr.q} pass {p} E"
            assert np.abs(Q - refs[p]["Q"]).max() <= tol, f"q={fr.q} pass {p} Q"


def test_concatenated_workload_sampled():
    # 64 frames of the 256-frame batch's shape carrying codewords of one
    # GF(16) code: three passes of (inner decode, 8 BP iterations); frames
    # 0 and 63 against the oracle, every frame's outputs normalised, and the
    # passes lowering the symbol errors of the hard decisions
    spec, frames = wl.make_concatenated_workload(64)
    it = mapdec.iterative_from_frames(frames, spec, precision=mapdec.FP32)
    errs = []
    for p in range(3):
        it.run_pass(8)
        torch.cuda.synchronize()
        Q = it.post.double().cpu().numpy()
        np.testing.assert_allclose(Q.sum(2), 1.0, atol=1e-5)
        dec = Q.argmax(2)
        errs.append(int(sum((dec[f] != frames[f].message).sum() for f in range(len(frames)))))
    assert errs[-1] <= errs[0]
    code = _ref_code(spec)
    for f in (0, 63):
        refs = ref.iterate(frames[f], code, 3, 8)
        Q = it.post[f].double().cpu().numpy()
        assert np.abs(Q - refs[-1]["Q"]).max() <= PASS_TOL[mapdec.FP32], f"frame {f}"


def test_plan_replays_match_calls():
    # the inner decode replayed as one HIP graph per pass gives the same
    # bits as direct decode calls; a reset starts again from uniform priors
    spec, frames = wl.make_concatenated_workload(8)
    a = mapdec.iterative_from_frames(frames, spec, precision=mapdec.FP32)
    b = mapdec.iterative_from_frames(frames, spec, precision=mapdec.FP32).use_plan()
    a.run(2, 6)
    for rep in range(2):
        b.reset()
        b.run(2, 6)
        torch.cuda.synchronize()
        assert torch.equal(a.post, b.post), f"replay {rep}"
        assert torch.equal(a.prior, b.prior), f"replay {rep}"
    b.plan.close()
