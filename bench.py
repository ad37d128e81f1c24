#!/usr/bin/env python3
"""Throughput of the MAP forward-backward decoder on one MI355X.

Workload: 256 frames, q=16 codewords of n=10 bits, N=500 symbols per frame
(tau = 5000 bits), BSID channel Pi=Pd=0.05, Ps=0.01, insertion cap I=2,
drift limits M=98 and mn=6, uniform priors, seeded synthetic frames.  A
step is one FP32 batched decode plus adjoint of the whole batch
(receiver-metric lattice, forward/backward chains, APPs, log P(y), then
d log P(y) / d(Pi, Pd, Ps) and d log P(y) / d prior), with every input
already in HBM, run as an eager plan: 4 slices of 64 frames on 4 HIP
streams, the compute-bound launches staggered slice by slice so that each
slice's forward/backward chains run beside the next slice's lattice and the
previous slice's APP.  The same step replayed as one single-stream HIP
graph is reported beside it.

Prints one JSON line: symbols per second, the roofline of the dominant
kernel (live HIP-event timing per phase), the FP32 decode alone and the
FP64 plain GPU decode of the same frames, the FP32 errors against the FP64
CPU oracle, and the oracle's own throughput (decode plus gradient) on a
bounded sample (host cores).  Beside it, the FP32 decode of the uneven
4096-frame batch (tuned choices, launch groups on forked streams).
"""
import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (packed); unpacked issue is half of it
PEAK_FP64_TFLOPS = 78.6
WORKLOAD = 2


def corridor_nodes(n, mn):
    """Lattice nodes (r, j), 0 <= r <= n, max(0, r - mn) <= j <= r + mn."""
    return sum(r + mn - max(0, r - mn) + 1 for r in range(n + 1))


def phase_flops(frames):
    """Algorithmic flops of each phase for a batch (FMA = 2 flops).
    lattice: rho q C(n, mn) (3 + 2I); chain: 4 N M_tau M_n (alpha and beta);
    app: 2 N M_tau M_n (q + 1); wgrad: 3 N M_tau M_n (uniform priors) or
    4 N M_tau M_n q; adjoint: three lattice passes (forward recompute,
    adjoint propagation, parameter products)."""
    out = {"lattice": 0.0, "chain": 0.0, "app": 0.0, "wgrad": 0.0, "adjoint": 0.0}
    for fr in frames:
        Mt, Mn = 2 * fr.M + 1, 2 * fr.mn + 1
        lat = fr.rho * fr.q * corridor_nodes(fr.n, fr.mn) * (3 + 2 * fr.I)
        out["lattice"] += lat
        out["chain"] += 4.0 * fr.N * Mt * Mn
        out["app"] += 2.0 * fr.N * Mt * Mn * (fr.q + 1)
        out["wgrad"] += (3.0 if fr.prior is None else 4.0 * fr.q) * fr.N * Mt * Mn
        out["adjoint"] += 3.0 * lat
    return out


PHASE_KERNEL = {"lattice": "k_lattice", "chain": "k_chain_ring", "app": "k_app_tile",
                "wgrad": "k_wadj", "adjoint": "k_adjoint"}


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE counters (scaled by a 1 GiB copy's readings), or
    None when the kernel's sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    k = rec["kernels"].get(kernel)
    if not k:
        return None
    h = hashlib.sha256()
    for f in k["sources"] + ["paper_1802_08483_amd/csrc/device_common.h",
                             "paper_1802_08483_amd/csrc/kernels.h",
                             "paper_1802_08483_amd/csrc/mapdec_internal.h"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != k["sha256"]:
        return None
    return round((k["fetch_kib"] * rec["copy_factor_fetch"] +
                  k["write_kib"] * rec["copy_factor_write"]) * 1024)


def time_plan(plan, steps, warmup, torch):
    for _ in range(warmup):
        plan.run()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        plan.run()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cpu_baseline(frames, budget_s=15.0):
    """The FP64 oracle (decode and gradient) on a bounded sample of the
    batch, one frame per host thread.  Returns (baseline dict, {frame index:
    oracle result})."""
    import oracle
    nthreads = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    first = oracle.decode_frame(frames[0], grad=True)
    t1 = time.perf_counter() - t0
    nsample = int(min(len(frames), max(nthreads, round(budget_s / max(t1, 1e-3)))))
    # whole rounds of one frame per thread (rounded up, so the sample holds
    # about budget_s of CPU work or more)
    if nsample >= nthreads:
        nsample = min(len(frames), -(-nsample // nthreads) * nthreads)
    idx = list(range(nsample))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=nthreads) as ex:
        res = list(ex.map(lambda f: oracle.decode_frame(frames[f], grad=True), idx))
    wall = time.perf_counter() - t0
    syms = sum(frames[f].N for f in idx)
    refs = dict(zip(idx, res))
    refs.setdefault(0, first)
    return ({"value": syms / wall, "unit": "symbols/s", "cores": nthreads, "kind": "oracle",
             "sample": f"{nsample} of {len(frames)} frames (oracle FP64 decode and gradient, one frame per "
                       f"thread, {wall:.2f} s wall, ~{t1 * nsample:.1f} s CPU)"}, refs)


def uneven_batch(mapdec, workloads, torch, steps):
    """FP32 decode of the uneven batch (4096 frames, q in {2, 8, 16}, n in
    [4, 10], N in [50, 2000], Pi = Pd log-uniform in [1e-3, 1e-1]): first
    every launch in order as one HIP graph with the default choices, then
    an eager plan with tuned choices and launch groups forked over four
    streams."""
    frames = workloads.make_workload(3)
    syms = sum(fr.N for fr in frames)
    b = mapdec.batch_from_frames(frames, precision=mapdec.FP32)
    mapdec.tune_reset()
    p = b.plan(graph=True)
    ms_graph = time_plan(p, steps, 1, torch)
    p.close()
    t0 = time.perf_counter()
    p = b.plan(graph=False, tune=True)
    tune_s = time.perf_counter() - t0
    ms = time_plan(p, steps, 1, torch)
    p.close()
    ok = bool((b.status == 0).all())
    worst = max(float((a.double().sum(1) - 1).abs().max()) for a in b.apps)
    out = {"workload": workloads.WORKLOAD_NAMES[3], "step": "decode",
           "value": round(syms / (ms * 1e-3), 1), "unit": "symbols/s",
           "ms_per_step": round(ms, 4), "schedule": "eager, tuned, launch groups on 4 streams",
           "tune_s": round(tune_s, 2), "tuned_buckets": mapdec.tune_entries(),
           "graph_one_stream_default": {"value": round(syms / (ms_graph * 1e-3), 1),
                                        "ms_per_step": round(ms_graph, 4)},
           "all_frames_ok": ok, "app_row_sum_max_err": worst}
    mapdec.tune_reset()
    del b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--graph-only", action="store_true",
                    help="time only the single-stream graph replay (every launch a full-batch "
                         "launch running alone, as in the roofline measurement)")
    ap.add_argument("--no-boundary", action="store_true",
                    help="skip the same step with priors of the frame boundaries")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven 4096-frame batch (reported beside the main line)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES bytes device-to-device a few times (a plain copy "
                         "kernel of known size, to calibrate HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the decoder's frames "
              "are independent and would shard by frame across GPUs, but only the "
              "single-GPU run is implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "dispatches": 3}))
        return
    from paper_1802_08483_amd import build as libbuild
    from paper_1802_08483_amd import mapdec, workloads

    if not os.path.exists(libbuild.LIB):
        libbuild.build()
    frames = workloads.make_workload(WORKLOAD)
    total_syms = sum(fr.N for fr in frames)

    b32 = mapdec.batch_from_frames(frames, precision=mapdec.FP32, grad=True)
    if not args.graph_only:
        # frame slices on the run's stream and 3 forked ones; timed and closed
        # before any other plan creates a stream (the device gives a process 4
        # hardware queues, and streams beyond them share one)
        plan = b32.plan(graph=False)
        ms = time_plan(plan, args.steps, args.warmup, torch)
        if not (b32.status == 0).all():
            raise RuntimeError("a frame reported no path")
        plan.close()
        schedule = "eager, 4 frame slices on 4 streams"
    pg = b32.plan(graph=True)       # one stream, full-batch launches
    msg = time_plan(pg, args.steps, args.warmup, torch)
    graph_line = {"value": round(total_syms / (msg * 1e-3), 1), "ms_per_step": round(msg, 4),
                  "schedule": "one HIP graph, every launch in order on one stream"}
    if args.graph_only:
        ms, schedule = msg, graph_line["schedule"]
    if not (b32.status == 0).all():
        raise RuntimeError("a frame reported no path")

    bdec = mapdec.batch_from_frames(frames, precision=mapdec.FP32)
    pdec = bdec.plan(graph=True)
    msdec = time_plan(pdec, args.steps, 1, torch)
    decode_only = {"value": round(total_syms / (msdec * 1e-3), 1), "ms_per_step": round(msdec, 4)}
    pdec.close()
    del bdec

    # Per-phase kernel time of the graph replay's launches (each a full-batch
    # launch running alone on one stream), from HIP events recorded just
    # before and after every launch on that stream, averaged over the steps.
    # The sliced schedule overlaps kernels on purpose, so its launch times
    # mix several kernels' work and are not a per-kernel roofline measure.
    acc = {}
    for _ in range(args.steps):
        for k, v in pg.profile().items():
            acc[k] = acc.get(k, 0.0) + v
    phases = {k: v / args.steps for k, v in acc.items()}
    nlaunch = pg.launches()
    pg.close()   # before the uneven batch's plan creates its streams
    flops = phase_flops(frames)
    dom = max((k for k in flops), key=lambda k: phases.get(k, 0.0))
    nl = max(1, nlaunch.get(dom, 1))
    achieved = flops[dom] / (phases[dom] * 1e-3) / 1e12   # = per-launch flops / launch time
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": measured_traffic(PHASE_KERNEL[dom]), "kernel": PHASE_KERNEL[dom],
                "launches_per_step": nl, "flops_per_launch": flops[dom] / nl,
                "launch_ms": round(phases[dom] / nl, 4),
                "measured_in": "single-stream graph replay (full-batch launches, each alone)"}

    fp64 = None
    if not args.no_fp64:
        b64 = mapdec.batch_from_frames(frames, precision=mapdec.FP64)
        p64 = b64.plan(graph=True)
        ms64 = time_plan(p64, max(3, args.steps // 2), 1, torch)
        fp64 = {"value": round(total_syms / (ms64 * 1e-3), 1), "ms_per_step": round(ms64, 4)}
        p64.close()
        del b64

    boundary = None
    if not args.no_boundary and not args.graph_only:
        # the same decode+adjoint step with priors of every frame's start and
        # end drift (Sec. II-C), as one HIP graph
        bframes = workloads.with_boundary_priors(frames)
        bb = mapdec.batch_from_frames(bframes, precision=mapdec.FP32, grad=True)
        pbd = bb.plan(graph=True)
        msb = time_plan(pbd, max(3, args.steps // 2), 1, torch)
        if not (bb.status == 0).all():
            raise RuntimeError("a frame with boundary priors reported no path")
        boundary = {"value": round(total_syms / (msb * 1e-3), 1), "ms_per_step": round(msb, 4),
                    "schedule": "one HIP graph, every launch in order on one stream",
                    "priors": "start drift 0..8, end drift rho-tau-4..rho-tau+4, binomial"}
        pbd.close()
        del bb

    uneven = None
    if not args.no_uneven:
        uneven = uneven_batch(mapdec, workloads, torch, max(3, args.steps // 4))

    # the single small frame (q = 8, n = 6, N = 64, FP64 decode): a launch-
    # and latency-bound case, one HIP graph
    small = None
    if not args.graph_only:
        sf = workloads.make_workload(1)
        bs = mapdec.batch_from_frames(sf, precision=mapdec.FP64)
        ps = bs.plan(graph=True)
        mss = time_plan(ps, max(10, args.steps), 3, torch)
        small = {"workload": workloads.WORKLOAD_NAMES[1], "gpu_graph_ms": round(mss, 4)}
        ps.close()
        del bs

    cpu, refs = (None, {})
    if not args.no_cpu_baseline:
        cpu, refs = cpu_baseline(frames)
        if small is not None:
            import oracle
            t0 = time.perf_counter()
            for _ in range(5):
                oracle.decode_frame(sf[0])
            small["oracle_1core_ms"] = round((time.perf_counter() - t0) / 5 * 1e3, 3)
    else:
        import oracle
        refs = {0: oracle.decode_frame(frames[0], grad=True)}
    app_err, lp_err, g_err = 0.0, 0.0, 0.0
    for f, ref in refs.items():
        app = b32.apps[f].double().cpu().numpy()
        app_err = max(app_err, float(np.abs(app - ref["app"]).max()))
        lp_err = max(lp_err, abs(float(b32.logp[f]) - ref["logp"]) / abs(ref["logp"]))
        gp = b32.dparams[f].cpu().numpy()
        g_err = max(g_err, float(np.abs(gp - ref["dparams"]).max() /
                                 np.abs(ref["dparams"]).max()))
        dpr = b32.dpriors[f].double().cpu().numpy()
        g_err = max(g_err, float(np.abs(dpr - ref["dprior"]).max() /
                                 np.abs(ref["dprior"]).max()))

    line = {
        "metric": "symbols decoded/sec, FP32 batched+adjoint vs FP64 plain, APP err <=1e-5",
        "value": round(total_syms / (ms * 1e-3), 1),
        "unit": "symbols/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": workloads.WORKLOAD_NAMES[WORKLOAD], "frames": len(frames),
                   "q": 16, "n": 10, "N": 500, "Pi": 0.05, "Pd": 0.05, "Ps": 0.01, "I": 2,
                   "M": frames[0].M, "mn": frames[0].mn, "priors": "uniform",
                   "schedule": schedule,
                   "step": "decode+adjoint"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "graph_replay": graph_line,
        "decode_only": decode_only,
        "fp64_plain": fp64,
        "accuracy": {"frames_checked": len(refs), "app_max_abs_err": app_err,
                     "logp_max_rel_err": lp_err, "grad_max_rel_err": g_err},
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        # the chain phase is a sequence of N dependent banded steps (forward
        # and backward chains of every frame run side by side): its latency
        # per step
        "chain_step_us": round(phases.get("chain", 0.0) * 1e3 / max(fr.N for fr in frames), 4),
        "boundary_priors": boundary,
        "small_frame": small,
        "uneven": uneven,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
