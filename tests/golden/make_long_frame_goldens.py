#!/usr/bin/env python3
"""Writes the oracle's expected values for the long-frame workload.

The long-frame batch (16 frames, q = 64, n = 12, N = 10 000 symbols, Pi =
Pd = 0.1, Ps = 0, I = 2, M = 693, mn = 8, uniform priors) is too large for
the FP64 oracle to decode inside a GPU test (several minutes per frame), so
this script decodes frames 0 and 15 once, on a CPU, and stores for each:
log P(y), d log P / d(Pi, Pd, Ps), and every 50th row (plus the last) of
the APP table and of d log P / d prior.  It calls only the oracle and the
seeded input generator; no value comes from the GPU library.

Usage: python tests/golden/make_long_frame_goldens.py [frame ...]
(default: 0 15).  Each frame takes several minutes and ~6 GB of memory.
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1802_08483_amd import workloads as wl  # noqa: E402

ROW_STEP = 50


def golden_path(f):
    return os.path.join(HERE, f"long_frame_w5_f{f}.json")


def make(f):
    fr = wl.make_workload(5, nframes=1, first=f)[0]
    t0 = time.time()
    ref = oracle.decode_frame(fr, grad=True)
    rows = list(range(0, fr.N, ROW_STEP))
    if rows[-1] != fr.N - 1:
        rows.append(fr.N - 1)
    rec = {
        "what": "FP64 oracle decode and gradient of one frame of the long-frame workload "
                "(16 frames q=64 n=12 N=10000 Pi=Pd=0.1 Ps=0 I=2 M=693 mn=8, uniform priors)",
        "script": "tests/golden/make_long_frame_goldens.py",
        "frame": f, "N": fr.N, "rho": fr.rho, "q": fr.q, "n": fr.n, "M": fr.M, "mn": fr.mn,
        "logp": repr(ref["logp"]),
        "dparams": [repr(float(v)) for v in ref["dparams"]],
        "rows": rows,
        "app": [[float(f"{v:.10e}") for v in ref["app"][i]] for i in rows],
        "dprior": [[float(f"{v:.10e}") for v in ref["dprior"][i]] for i in rows],
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(golden_path(f), "w") as fh:
        json.dump(rec, fh, separators=(",", ":"))
        fh.write("\n")
    return f, rec["oracle_seconds"]


def main():
    frames = [int(a) for a in sys.argv[1:]] or [0, 15]
    oracle.build()
    with ThreadPoolExecutor(max_workers=len(frames)) as ex:
        for f, s in ex.map(make, frames):
            print(f"frame {f}: {s} s -> {golden_path(f)}", flush=True)


if __name__ == "__main__":
    main()
