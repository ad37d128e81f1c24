"""libmapdec's host code (layout, work tables, launch ops, stream forking,
tuning, graph capture bookkeeping) on a CPU: mapdec.cpp is compiled with
g++ against a stub of the HIP runtime calls and kernel launchers
(tests/host/plan_stub.cpp), under AddressSanitizer and UBSan.  The stub
reads every launch's work table and checks, with vector clocks over
streams and events, that each launch is ordered after the previous launch
of every frame it touches and that the caller's stream is joined with
every forked stream; it aborts otherwise.  Sweep parts of checkpointed
frames must also follow the writers of the Gamma blocks their rows read
(the pre-pass runs in rounds beside them), and segment recomputations,
which touch only the group's rows, must follow the Gamma blocks they read.  Eager plans of many frames run
in frame slices (one stream each, compute-bound launches staggered slice
by slice).  No kernel runs.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1802_08483_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")

GRAD, GRAPH, SERIAL, TUNE = 1, 2, 4, 8


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++") or not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(HOST, "plan_driver.cpp"), os.path.join(HOST, "plan_stub.cpp"),
           os.path.join(CSRC, "mapdec.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


@pytest.mark.parametrize("nframes,K,flags,uniform", [
    (240, 0, GRAD, 0),                 # eager, forked launch groups
    (240, 0, 0, 0),                    # decode only, forked
    (240, 0, GRAD | GRAPH, 0),         # graph capture: one stream
    (240, 0, GRAD | SERIAL, 0),        # eager, one stream
    (120, 23, GRAD, 0),                # checkpointed passes, forked
    (120, 23, GRAPH, 0),
    (160, 0, GRAD | TUNE, 0),          # tuning plan, then the tuned plan
    (32, 0, GRAD | GRAPH, 1),          # uniform batch: one group per phase
    (32, 40, GRAD, 1),
    (2, 13, 0, 1),                     # sweep in parts whose first forward part is empty
    (2, 13, GRAD, 1),
    (8, 13, 0, 0),                     # decode only, sweep in parts
    (4, 7, GRAD, 1),                   # Gamma pre-pass in rounds beside the sweep parts
    (4, 7, 0, 1),
    (16, 100, GRAD, 1),                # one segment per group: its recomputation waits for Gamma
    (2, 13, GRAD, 3),                  # the MFMA APP: its scale pass follows the recomputation
    (2, 13, 0, 3),
    (128, 0, GRAD, 1),                 # eager uniform batch in frame slices
    (128, 0, GRAD | SERIAL, 1),
    (60, 0, GRAD, 2),                  # with general-scheme frames
    (60, 11, GRAD, 2),
    (60, 0, GRAPH, 2),
])
def test_plan_host_logic(driver, nframes, K, flags, uniform):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
    r = subprocess.run([driver, str(nframes), str(K), str(flags), str(uniform)],
                       capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert r.stdout.startswith("ok"), r.stdout
