#!/usr/bin/env python3
"""Throughput of the MAP forward-backward decoder on one MI355X.

Headline workload: 16 frames, q=64 codewords of n=12 bits, N=10000 symbols
per frame (tau = 120000 bits), BSID channel Pi=Pd=0.1, Ps=0, insertion cap
I=2, drift limits M=693 and mn=8, uniform priors, seeded synthetic frames.
A step is one FP32 batched decode plus adjoint of the whole batch
(receiver-metric lattice, forward/backward chains, APPs, log P(y), then
d log P(y) / d(Pi, Pd, Ps) and d log P(y) / d prior) with forward (and
backward) metric checkpoints every K = ceil(sqrt(N)) = 100 symbols and the
receiver metric recomputed for the APP and adjoint passes, every input
already in HBM, replayed as one HIP graph.

Beside it, each with its own roofline figure: the channel-estimation batch
(128 frames, q=16, n=10, N=1000, softmax priors, decode+adjoint), the
256-frame batch (q=16, n=10, N=500, decode+adjoint, decode alone and the
FP64 plain decode), the general scheme (64 frames of that batch's shape with
a codebook per symbol position and a narrower corridor, decode+adjoint),
the uneven 4096-frame batch (decode, tuned choices) and
the single small frame (FP64 decode).

Prints one JSON line.  The roofline of a line is that of its dominant
kernel: algorithmic flops per launch (the method's work, recomputation
excluded; FMA = 2 flops) over the kernel's average launch time, measured
live with HIP events recorded on the launch's own stream around every launch
(one eager pass of the same plan).  The CPU baseline is the FP64 oracle
(decode and gradient), built -O3 -march=native on this host, on a bounded
sample of the headline workload, one frame per host thread.
"""
import argparse
import json
import math
import os
import platform
import subprocess
import sys
import tempfile
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (packed); unpacked issue is half of it
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
HEADLINE = 5
# host threads a GPU's share of the machine holds (one MI355X: 16)
HOST_THREADS_CAP = 16


def corridor_nodes(n, mn, lo=None):
    """Lattice nodes (r, j), 0 <= r <= n, max(0, r + lo) <= j <= r + mn
    (lo = -mn unless given: the corridor [lo, mn])."""
    lo = -mn if lo is None else lo
    return sum(r + mn - max(0, r + lo) + 1 for r in range(n + 1))


GROUP_SPAN = 4   # groups of checkpoint segments reach at most 1/4 more start indices


def group_symbols(fr, K):
    """Symbols per main pass of a checkpointed frame: whole segments of K,
    enough that the group's n K_G received bits are at least 4 x 2M."""
    nck = -(-fr.N // K)
    per = max(1, -(-(GROUP_SPAN * 2 * fr.M) // (fr.n * K)))
    return min(fr.N, min(nck, per) * K)


def covered_starts(fr, K):
    """Start indices the lattice and adjoint launches of one run cover.
    Without checkpoints: the whole received range once each.  With
    checkpoints every K symbols: the lattice once over the whole frame for
    Gamma (uniform priors; per group with general priors) and once per
    group in the main passes, each group reaching [n i0 - M, n (i1 - 1) + M]
    clipped to [0, rho]; the adjoint once per group."""
    if not K or K >= fr.N:
        return fr.rho + 1, fr.rho + 1
    KG = group_symbols(fr, K)
    tot = 0
    for i0 in range(0, fr.N, KG):
        i1 = min(fr.N, i0 + KG)
        s0 = max(0, fr.n * i0 - fr.M)
        s1 = min(fr.rho, fr.n * (i1 - 1) + fr.M)
        tot += s1 - s0 + 1
    pre = fr.rho + 1 if fr.prior is None else tot
    return pre + tot, tot


def phase_flops(frames, K=0):
    """Algorithmic flops of each phase for a batch (FMA = 2 flops), and the
    flops the phases execute on top of them (recomputation).
    lattice: W_R = rho q C(n, mn) (3 + 2I); gamma (general priors):
    2 N Mt Mn q; chain: 4 N Mt Mn (alpha and beta); app: 2 N Mt Mn (q + 1);
    wgrad: 3 N Mt Mn (uniform priors) or 4 N Mt Mn q; adjoint: 2 W_R (the
    reverse sweep's adjoint propagation and parameter products).  Executed
    on top: the lattice and adjoint over every pass's covered start indices
    (checkpointed groups overlap by 2M), the forward and backward
    recursions recomputed from the checkpoints, and the adjoint's recompute
    of the forward lattice (one more W_R over what it covers)."""
    alg = {"lattice": 0.0, "gamma": 0.0, "chain": 0.0, "app": 0.0, "wgrad": 0.0,
           "adjoint": 0.0}
    extra = {"lattice": 0.0, "adjoint": 0.0, "rechain": 0.0}
    for fr in frames:
        lim = getattr(fr, "limits", None) or (-fr.M, fr.M, -fr.mn, fr.mn)
        Mt, Mn = lim[1] - lim[0] + 1, lim[3] - lim[2] + 1
        # the method's lattice work: nodes of the corridor [lo, hi]; the
        # kernels run the symmetric corridor that contains it
        per_s = fr.q * corridor_nodes(fr.n, lim[3], lim[2]) * (3 + 2 * fr.I)
        per_x = fr.q * corridor_nodes(fr.n, fr.mn) * (3 + 2 * fr.I)
        if getattr(fr, "codebooks", None) is not None:
            # a codebook per symbol: one lattice per (symbol, drift state, D)
            lat = fr.N * Mt * per_s
            lat_cov = adj_cov = fr.N * (2 * fr.M + 1)
        else:
            lat = (fr.rho + 1) * per_s
            lat_cov, adj_cov = covered_starts(fr, K)
        per_s = per_x
        alg["lattice"] += lat
        extra["lattice"] += lat_cov * per_x - lat
        if fr.prior is not None:
            alg["gamma"] += 2.0 * fr.N * Mt * Mn * fr.q
        alg["chain"] += 4.0 * fr.N * Mt * Mn
        if K and K < fr.N:   # both recursions again from the checkpoints
            extra["rechain"] += 4.0 * fr.N * Mt * Mn
        alg["app"] += 2.0 * fr.N * Mt * Mn * (fr.q + 1)
        alg["wgrad"] += (3.0 if fr.prior is None else 4.0 * fr.q) * fr.N * Mt * Mn
        alg["adjoint"] += 2.0 * lat
        extra["adjoint"] += 3.0 * adj_cov * per_s - 2.0 * lat
    return alg, extra


PHASE_KERNEL = {"lattice": "k_lattice", "gamma": "k_gamma", "chain": "k_chain_ring",
                "app": "k_app_tile", "wgrad": "k_wadj", "adjoint": "k_adjoint"}
# FP32 frames with one codebook, 16 < q <= 64 and 2M+1 <= 2048 take the APP
# on the matrix units: per pass k_app_scale, k_app_mfma and k_app_fin, one
# launch each per configuration.
APP_MFMA_KERNELS = "k_app_scale+k_app_mfma+k_app_fin"


def gamma_bytes(frames, tsize):
    """Algorithmic bytes of Gamma for general priors: R read once (q Mn
    values per received start index), the priors (N q), Gamma written (N Mt
    Mn)."""
    tot = 0.0
    for fr in frames:
        if fr.prior is None:
            continue
        lim = getattr(fr, "limits", None) or (-fr.M, fr.M, -fr.mn, fr.mn)
        Mt, Mn = lim[1] - lim[0] + 1, lim[3] - lim[2] + 1
        tot += tsize * (fr.q * Mn * (fr.rho + 1) + fr.N * fr.q + fr.N * Mt * Mn)
    return tot


def app_on_mfma(frames, fp64):
    return not fp64 and all(16 < fr.q <= 64 and getattr(fr, "codebooks", None) is None
                            and 2 * fr.M + 1 <= 2048 for fr in frames)


def measured_traffic(kernel, workload):
    """HBM bytes per launch of ``kernel`` on ``workload`` from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE counters (scaled by a plain copy's
    readings), or None when there are none or the kernel's sources changed
    since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    k = rec.get("workloads", {}).get(str(workload), {}).get(kernel)
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
    """Average ms per run over ``steps`` runs after ``warmup`` untimed ones,
    bracketed by device synchronisation."""
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


def roofline_of(plan, frames, K, steps, workload, precision_peak, fp64=False):
    """Per-phase launch times (HIP events on each launch's stream, summed
    per phase, averaged over ``steps`` eager passes of the plan) and the
    roofline of the phase that takes longest.  An APP on the matrix units
    is priced against the FP32 matrix peak, its three kernels' launches
    counted as one."""
    acc = {}
    reps = max(1, steps)
    for _ in range(reps):
        for k, v in plan.profile().items():
            acc[k] = acc.get(k, 0.0) + v
    phases = {k: v / reps for k, v in acc.items()}
    nlaunch = plan.launches()
    alg, extra = phase_flops(frames, K)
    # the chains are bound by the latency of their N dependent steps, not by
    # an ALU or HBM roofline: they are reported as time per step instead
    dom = max((k for k in alg if alg[k] > 0 and k != "chain"),
              key=lambda k: phases.get(k, 0.0))
    nl = max(1, nlaunch.get(dom, 1))
    kernel, bound = PHASE_KERNEL[dom], "alu"
    if dom == "app" and app_on_mfma(frames, fp64):
        kernel, bound, nl = APP_MFMA_KERNELS, "mfma", max(1, nl // 3)
    ms = phases[dom]
    if dom == "gamma":
        # Gamma of general priors streams R and the priors in and Gamma out:
        # priced against HBM with its algorithmic bytes
        nbytes = gamma_bytes(frames, 8 if fp64 else 4)
        achieved = nbytes / (ms * 1e-3) / 1e9
        return ({"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                 "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                 "traffic": measured_traffic(kernel, workload), "kernel": kernel,
                 "launches_per_step": nl, "bytes_per_launch": nbytes / nl,
                 "launch_ms": round(ms / nl, 5),
                 "measured_in": "HIP events around every launch on its stream, one "
                                "one-stream pass of the plan per repeat"}, phases, nlaunch)
    achieved = alg[dom] / (ms * 1e-3) / 1e12
    roof = {"bound": bound, "achieved": round(achieved, 3), "peak": precision_peak,
            "unit": "TFLOP/s", "frac": round(achieved / precision_peak, 4),
            "traffic": measured_traffic(kernel, workload),
            "kernel": kernel, "launches_per_step": nl,
            "flops_per_launch": alg[dom] / nl, "launch_ms": round(ms / nl, 5),
            "recompute_flops_per_launch": extra.get(dom, 0.0) / nl,
            "measured_in": "HIP events around every launch on its stream, one "
                           "one-stream pass of the plan per repeat"}
    return roof, phases, nlaunch


def host_info(nthreads):
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": aff,
            "threads_used": nthreads}


def oracle_native():
    """The oracle built -O3 -march=native for this host (the committed
    build is portable -O2); returns (module, flags)."""
    import oracle
    d = tempfile.mkdtemp(prefix="mapdec_ref_native_")
    path = os.path.join(d, "libmapdec_ref.so")
    flags = ["-O3", "-march=native"]
    try:
        oracle.load_build(path, flags)
        return oracle, " ".join(flags)
    except (subprocess.CalledProcessError, OSError):
        return oracle, "-O2 (committed portable build; native build failed)"


def run_oracle_pool(fn, items, nthreads):
    with ThreadPoolExecutor(max_workers=nthreads) as ex:
        return list(ex.map(fn, items))


def cpu_baseline(nthreads, sample_N=150):
    """The FP64 oracle (decode and gradient) on a bounded sample of the
    headline workload: nthreads frames of sample_N symbols with the
    workload's code and channel (q=64, n=12, Pi=Pd=0.1, Ps=0, I=2, M=693,
    mn=8), one frame per host thread."""
    from paper_1802_08483_amd import workloads as wl
    orc, flags = oracle_native()
    full = wl.make_workload(HEADLINE, nframes=1)[0]
    frames = [wl.random_frame(9000 + k, full.q, full.n, sample_N, full.Pi, full.Pd, full.Ps,
                              full.I, full.M, full.mn) for k in range(nthreads)]
    t0 = time.perf_counter()
    run_oracle_pool(lambda fr: orc.decode_frame(fr, grad=True), frames, nthreads)
    wall = time.perf_counter() - t0
    syms = sum(fr.N for fr in frames)
    info = host_info(nthreads)
    return {"value": round(syms / wall, 2), "unit": "symbols/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"{len(frames)} frames of {sample_N} symbols with the workload's code, "
                      f"channel and drift limits (q=64 n=12 Pi=Pd=0.1 Ps=0 I=2 M={full.M} "
                      f"mn={full.mn}), FP64 decode and gradient, one frame per thread, "
                      f"{wall:.2f} s wall; oracle built {flags}",
            "host": info}


def accuracy_vs(batch, f, ref, grad):
    import numpy as np
    out = {}
    app = batch.apps[f].double().cpu().numpy()
    out["app"] = float(np.abs(app - ref["app"]).max())
    out["logp"] = abs(float(batch.logp[f]) - ref["logp"]) / abs(ref["logp"])
    if grad:
        gp = batch.dparams[f].cpu().numpy()
        g = float(np.abs(gp - ref["dparams"]).max() / np.abs(ref["dparams"]).max())
        dpr = batch.dpriors[f].double().cpu().numpy()
        g = max(g, float(np.abs(dpr - ref["dprior"]).max() / np.abs(ref["dprior"]).max()))
        out["grad"] = g
    return out


def merge_acc(items):
    res = {"frames_checked": len(items)}
    for key, name in (("app", "app_max_abs_err"), ("logp", "logp_max_rel_err"),
                      ("grad", "grad_max_rel_err")):
        vals = [a[key] for a in items if key in a]
        if vals:
            res[name] = max(vals)
    return res


def golden_accuracy(batch):
    """The long-frame batch against the oracle's stored values (frames 0 and
    15: log P, d/d(Pi, Pd, Ps), every 50th row of APP and d/d prior)."""
    import numpy as np
    items = []
    for f in (0, 15):
        path = os.path.join(ROOT, "tests", "golden", f"long_frame_w5_f{f}.json")
        if not os.path.exists(path):
            continue
        g = json.load(open(path))
        rows = g["rows"]
        app = batch.apps[f].double().cpu().numpy()[rows]
        dpr = batch.dpriors[f].double().cpu().numpy()[rows]
        ref_dp = np.array([float(v) for v in g["dparams"]])
        ref_pr = np.array(g["dprior"])
        gp = batch.dparams[f].cpu().numpy()
        lp = float(g["logp"])
        items.append({"app": float(np.abs(app - np.array(g["app"])).max()),
                      "logp": abs(float(batch.logp[f]) - lp) / abs(lp),
                      "grad": max(float(np.abs(gp - ref_dp).max() / np.abs(ref_dp).max()),
                                  float(np.abs(dpr - ref_pr).max() / np.abs(ref_pr).max()))})
    out = merge_acc(items)
    out["against"] = "stored oracle values (tests/golden), frames 0 and 15, every 50th row"
    return out


def line_grad(mapdec, workloads, torch, k, K, steps, warmup, graph=True):
    """FP32 decode + adjoint of workload k as one plan: throughput, phases,
    roofline."""
    frames = workloads.make_workload(k)
    syms = sum(fr.N for fr in frames)
    b = mapdec.batch_from_frames(frames, precision=mapdec.FP32, grad=True, checkpoint_K=K)
    plan = b.plan(graph=graph)
    ms = time_plan(plan, steps, warmup, torch)
    if not (b.status == 0).all():
        raise RuntimeError(f"workload {k}: a frame reported no path")
    # kernel times for the roofline from the one-stream order, where every
    # launch runs alone (the eager schedule overlaps launches on purpose)
    rplan = plan if graph else b.plan(graph=True)
    roof, phases, nl = roofline_of(rplan, frames, K, max(1, min(steps, 5)), k, PEAK_FP32_TFLOPS)
    if rplan is not plan:
        rplan.close()
    plan.close()
    return b, frames, {"workload": workloads.WORKLOAD_NAMES[k],
                       "value": round(syms / (ms * 1e-3), 1), "unit": "symbols/s",
                       "ms_per_step": round(ms, 4), "frames": len(frames),
                       "checkpoint_K": K, "workspace_bytes": b.ws_bytes,
                       "schedule": "one HIP graph" if graph else
                       "eager plan (launch groups and sweep parts forked over streams)",
                       "roofline": roof,
                       "phases_ms": {p: round(v, 4) for p, v in phases.items()},
                       "launches": nl,
                       # time per step of the whole frame's recursions (the
                       # sweep when checkpointed): one launch over N steps
                       # (both directions), or, with the sweep in parts, a
                       # forward and a backward launch per part over N /
                       # parts steps each
                       "chain_step_us": round(phases.get("chain", 0.0) * 1e3 /
                                              max(1, nl.get("chain", 1)) /
                                              (max(fr.N for fr in frames) /
                                               max(1, nl.get("chain", 1) // 2)
                                               if K and nl.get("chain", 1) > 1
                                               else max(fr.N for fr in frames)), 4)}


def line_general(mapdec, workloads, torch, steps, warmup):
    """The general scheme (a codebook per symbol position, a narrower
    corridor): FP32 decode + adjoint as one HIP graph, with its roofline."""
    frames = workloads.make_general_workload()
    syms = sum(fr.N for fr in frames)
    b = mapdec.batch_from_frames(frames, precision=mapdec.FP32, grad=True)
    plan = b.plan(graph=True)
    ms = time_plan(plan, steps, warmup, torch)
    if not (b.status == 0).all():
        raise RuntimeError("general scheme: a frame reported no path")
    roof, phases, nl = roofline_of(plan, frames, 0, max(1, min(steps, 5)), "general",
                                   PEAK_FP32_TFLOPS)
    plan.close()
    return b, frames, {"workload": workloads.GENERAL_NAME,
                       "value": round(syms / (ms * 1e-3), 1), "unit": "symbols/s",
                       "ms_per_step": round(ms, 4), "frames": len(frames),
                       "step": "decode+adjoint", "schedule": "one HIP graph",
                       "workspace_bytes": b.ws_bytes, "roofline": roof,
                       "phases_ms": {p: round(v, 4) for p, v in phases.items()},
                       "launches": nl}


def line_iterative(mapdec, workloads, torch, steps, warmup, passes=3, bp_iters=8):
    """Iterative decoding with the outer code (Sec. II-A): a step is the
    whole decoding of the batch, ``passes`` times (the inner FP32 decode as
    one HIP graph, then ``bp_iters`` iterations of belief propagation),
    from uniform priors."""
    import numpy as np
    spec, frames = workloads.make_concatenated_workload()
    syms = sum(fr.N for fr in frames)
    it = mapdec.iterative_from_frames(frames, spec, precision=mapdec.FP32).use_plan()

    class Step:
        def run(self):
            it.reset()
            it.run(passes, bp_iters)

    ms = time_plan(Step(), steps, warmup, torch)
    # time of the parts: one inner pass (graph), one outer decode
    ms_inner = time_plan(it.plan, steps, 1, torch)

    class Outer:
        def run(self):
            it.outer.decode(it.chan, it.prior, it.post, bp_iters, it.ws)

    ms_outer = time_plan(Outer(), steps, 1, torch)
    Step().run()
    torch.cuda.synchronize()
    Q = it.post.double().cpu().numpy()
    msg = np.stack([fr.message for fr in frames])
    errs = int((Q.argmax(2) != msg).sum())
    it.reset()
    it.run_pass(bp_iters)
    torch.cuda.synchronize()
    inner_errs = int((np.stack([a.double().cpu().numpy() for a in it.batch.apps]).argmax(2)
                      != msg).sum())
    out = {"workload": workloads.CONCAT_NAME, "step": f"{passes} passes x (inner decode, "
           f"{bp_iters} BP iterations)", "value": round(syms / (ms * 1e-3), 1),
           "unit": "symbols/s", "ms_per_step": round(ms, 4), "frames": len(frames),
           "inner_pass_ms": round(ms_inner, 4), "outer_decode_ms": round(ms_outer, 4),
           "symbol_errors_inner_alone": inner_errs, "symbol_errors_after": errs,
           "symbols": syms}
    it.plan.close()
    del it
    torch.cuda.empty_cache()
    return out


def uneven_batch(mapdec, workloads, torch, steps):
    """FP32 decode of the uneven batch (4096 frames, q in {2, 8, 16}, n in
    [4, 10], N in [50, 2000], Pi = Pd log-uniform in [1e-3, 1e-1]): the eager
    plan with tuned choices and launch groups forked over four streams (the
    line's value), beside one HIP graph launch per step (every launch in
    order on one stream) with the default and with the tuned choices."""
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
    ms_eager = time_plan(p, steps, 1, torch)
    p.close()
    p = b.plan(graph=True)   # tuned choices (the table is filled)
    ms_graph_tuned = time_plan(p, steps, 1, torch)
    p.close()
    ms = ms_eager
    ok = bool((b.status == 0).all())
    worst = max(float((a.double().sum(1) - 1).abs().max()) for a in b.apps)
    out = {"workload": workloads.WORKLOAD_NAMES[3], "step": "decode",
           "value": round(syms / (ms * 1e-3), 1), "unit": "symbols/s",
           "ms_per_step": round(ms, 4),
           "schedule": "eager, tuned, launch groups on 4 streams",
           "tune_s": round(tune_s, 2), "tuned_buckets": mapdec.tune_entries(),
           "graph_default_choices": {"value": round(syms / (ms_graph * 1e-3), 1),
                                     "ms_per_step": round(ms_graph, 4)},
           "graph_tuned_choices": {"value": round(syms / (ms_graph_tuned * 1e-3), 1),
                                   "ms_per_step": round(ms_graph_tuned, 4)},
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
    ap.add_argument("--workloads", default="5,4,2,6,7,3,1",
                    help="comma-separated workloads to run (5 = the headline line; 6 = the "
                         "general scheme: a codebook per symbol, a narrower corridor; 7 = "
                         "iterative decoding with the outer code)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip every oracle comparison (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES bytes device-to-device a few times (a plain copy "
                         "kernel of known size, to calibrate HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the decoder's frames "
              "are independent and would shard by frame across GPUs, but only the "
              "single-GPU run is implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
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
    wanted = [int(w) for w in args.workloads.split(",") if w]
    nthreads = max(1, min(HOST_THREADS_CAP, len(os.sched_getaffinity(0))))
    lines = {}

    # headline: the long-frame batch, decode + adjoint, checkpoints every 100
    head = None
    if HEADLINE in wanted:
        fr0 = workloads.make_workload(HEADLINE, nframes=1)[0]
        K = int(math.ceil(math.sqrt(fr0.N)))
        b5, frames5, head = line_grad(mapdec, workloads, torch, HEADLINE, K, args.steps,
                                      args.warmup, graph=False)
        # the one-stream HIP graph of the same step (the sweep in one launch,
        # no main pass beside it)
        pg = b5.plan(graph=True)
        msg = time_plan(pg, max(2, args.steps // 2), 1, torch)
        pg.close()
        head["graph_replay"] = {"value": round(sum(f.N for f in frames5) / (msg * 1e-3), 1),
                                "ms_per_step": round(msg, 4), "schedule": "one HIP graph"}
        if not args.no_oracle:
            head["accuracy"] = golden_accuracy(b5)
        # the FP64 plain decode of the same frames (same checkpoints)
        b64 = mapdec.batch_from_frames(frames5, precision=mapdec.FP64, checkpoint_K=K)
        p64 = b64.plan(graph=True)
        ms64 = time_plan(p64, max(2, args.steps // 4), 1, torch)
        head["fp64_plain"] = {"value": round(sum(f.N for f in frames5) / (ms64 * 1e-3), 1),
                              "ms_per_step": round(ms64, 4), "step": "decode"}
        p64.close()
        del b64, b5
        torch.cuda.empty_cache()

    if 4 in wanted:
        b4, frames4, line = line_grad(mapdec, workloads, torch, 4, 0, args.steps, args.warmup)
        if not args.no_oracle:
            import oracle
            idx = list(range(0, len(frames4), max(1, len(frames4) // nthreads)))[:nthreads]
            t0 = time.perf_counter()
            refs = run_oracle_pool(lambda f: oracle.decode_frame(frames4[f], grad=True), idx,
                                   nthreads)
            wall = time.perf_counter() - t0
            line["accuracy"] = merge_acc([accuracy_vs(b4, f, r, True) for f, r in zip(idx, refs)])
            line["oracle_sample_symbols_per_s"] = round(sum(frames4[f].N for f in idx) / wall, 1)
        lines["channel_estimation"] = line
        del b4
        torch.cuda.empty_cache()

    if 2 in wanted:
        b2, frames2, line = line_grad(mapdec, workloads, torch, 2, 0, args.steps, args.warmup)
        # the same step as the eager sliced plan (4 frame slices on 4 streams)
        ps = b2.plan(graph=False)
        mss = time_plan(ps, args.steps, args.warmup, torch)
        ps.close()
        syms2 = sum(fr.N for fr in frames2)
        line["sliced_eager"] = {"value": round(syms2 / (mss * 1e-3), 1),
                                "ms_per_step": round(mss, 4),
                                "schedule": "eager, 4 frame slices on 4 streams"}
        bdec = mapdec.batch_from_frames(frames2, precision=mapdec.FP32)
        pdec = bdec.plan(graph=True)
        msdec = time_plan(pdec, args.steps, 1, torch)
        line["decode_only"] = {"value": round(syms2 / (msdec * 1e-3), 1),
                               "ms_per_step": round(msdec, 4)}
        pdec.close()
        del bdec
        b64 = mapdec.batch_from_frames(frames2, precision=mapdec.FP64)
        p64 = b64.plan(graph=True)
        ms64 = time_plan(p64, max(3, args.steps // 2), 1, torch)
        line["fp64_plain"] = {"value": round(syms2 / (ms64 * 1e-3), 1),
                              "ms_per_step": round(ms64, 4), "step": "decode"}
        p64.close()
        del b64
        if not args.no_oracle:
            import oracle
            idx = list(range(0, len(frames2), max(1, len(frames2) // nthreads)))[:nthreads]
            refs = run_oracle_pool(lambda f: oracle.decode_frame(frames2[f], grad=True), idx,
                                   nthreads)
            line["accuracy"] = merge_acc([accuracy_vs(b2, f, r, True) for f, r in zip(idx, refs)])
        lines["batch256"] = line
        del b2
        torch.cuda.empty_cache()

    if 6 in wanted:
        bg, framesg, line = line_general(mapdec, workloads, torch, args.steps, args.warmup)
        if not args.no_oracle:
            import oracle
            idx = list(range(0, len(framesg), max(1, len(framesg) // nthreads)))[:nthreads]
            refs = run_oracle_pool(lambda f: oracle.decode_frame(framesg[f], grad=True), idx,
                                   nthreads)
            line["accuracy"] = merge_acc([accuracy_vs(bg, f, r, True) for f, r in zip(idx, refs)])
        lines["general"] = line
        del bg
        torch.cuda.empty_cache()

    if 7 in wanted:
        lines["iterative"] = line_iterative(mapdec, workloads, torch, max(3, args.steps // 4),
                                            1)

    if 3 in wanted:
        lines["uneven"] = uneven_batch(mapdec, workloads, torch, max(3, args.steps // 4))

    if 1 in wanted:
        sf = workloads.make_workload(1)
        bs = mapdec.batch_from_frames(sf, precision=mapdec.FP64)
        ps = bs.plan(graph=True)
        mss = time_plan(ps, max(10, args.steps), 3, torch)
        small = {"workload": workloads.WORKLOAD_NAMES[1], "gpu_graph_ms": round(mss, 4)}
        ps.close()
        if not args.no_oracle:
            import oracle
            t0 = time.perf_counter()
            for _ in range(5):
                oracle.decode_frame(sf[0])
            small["oracle_1core_ms"] = round((time.perf_counter() - t0) / 5 * 1e3, 3)
        lines["small_frame"] = small

    cpu = None
    if head is not None and not args.no_cpu_baseline:
        cpu = cpu_baseline(nthreads)

    if head is None:
        # no headline requested (profiling runs): print the lines only
        print(json.dumps({"lines": lines}))
        return
    line = {
        "metric": "symbols decoded/sec, FP32 batched+adjoint vs FP64 plain, APP err <=1e-5",
        "value": head["value"],
        "unit": "symbols/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": workloads.WORKLOAD_NAMES[HEADLINE], "frames": 16,
                   "q": 64, "n": 12, "N": 10000, "Pi": 0.1, "Pd": 0.1, "Ps": 0.0, "I": 2,
                   "M": 693, "mn": 8, "priors": "uniform", "checkpoint_K": head["checkpoint_K"],
                   "schedule": head["schedule"], "step": "decode+adjoint"},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "accuracy": head.get("accuracy"),
        "fp64_plain": head["fp64_plain"],
        "workspace_bytes": head["workspace_bytes"],
        "phases_ms": head["phases_ms"],
        "launches": head["launches"],
        "chain_step_us": head["chain_step_us"],
        "graph_replay": head.get("graph_replay"),
        "other_workloads": lines,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
