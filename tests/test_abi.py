"""Host-side checks of libmapdec: symbols and argument validation.

No kernel runs here: every call below returns before any HIP work is
enqueued (validation happens first), so these run without a GPU.  Device
pointers passed to the library in these tests are never dereferenced.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1802_08483_amd import build as libbuild
from paper_1802_08483_amd import mapdec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(libbuild.LIB):
        libbuild.build()
    return mapdec.lib()


def _declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(mapdec_[a-z_]+)\s*\(", txt)
    return sorted(set(names))


def test_exports_every_declared_symbol(L):
    declared = _declared_functions()
    assert set(declared) == set(mapdec.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name
    assert L.mapdec_version() == 107
    for st in range(8):
        assert L.mapdec_strerror(st)


def _code(q=4, n=3, Pi=0.1, Pd=0.1, Ps=0.01, I=2, M=6, mn=2, cb=None):
    if cb is None:
        cb = np.array([[(w >> (n - 1 - r)) & 1 for r in range(n)] for w in range(q)], np.uint8)
    return mapdec.Code(cb, Pi, Pd, Ps, I, M, mn)


@pytest.mark.parametrize("kw", [dict(Pi=0.6, Pd=0.5), dict(Pi=-0.1), dict(Ps=1.5), dict(I=-1),
                                dict(M=1, mn=2), dict(q=9, n=3), dict(q=1)])
def test_create_rejects_invalid(L, kw):
    with pytest.raises(mapdec.MapdecError) as e:
        _code(**kw)
    assert e.value.status == mapdec.EINVAL


def test_create_rejects_duplicate_and_nonbinary_codewords(L):
    with pytest.raises(mapdec.MapdecError):
        _code(q=2, n=2, cb=np.array([[0, 1], [0, 1]], np.uint8))
    with pytest.raises(mapdec.MapdecError):
        _code(q=2, n=2, cb=np.array([[0, 2], [1, 1]], np.uint8))


def _frames(specs):
    arr = (mapdec._Frame * len(specs))()
    for i, (code, N, rho) in enumerate(specs):
        arr[i] = mapdec._Frame(code.handle, N, rho, 0x1000 if rho else None, None, None, None)
    return arr


def test_workspace_size_and_validation(L):
    c = _code()
    fr = _frames([(c, 10, 30), (c, 5, 17)])
    ws32 = L.mapdec_workspace_size(fr, 2, mapdec.FP32, 0, 0)
    ws64 = L.mapdec_workspace_size(fr, 2, mapdec.FP64, 0, 0)
    assert 0 < ws32 < ws64
    assert L.mapdec_workspace_size(fr, 2, mapdec.FP32, 0, -1) == 0
    # end drift outside [-M, M]
    bad = _frames([(c, 10, 30 + 7)])
    assert L.mapdec_workspace_size(bad, 1, mapdec.FP32, 0, 0) == 0
    dummy = ctypes.c_void_p(0x1000)
    st = L.mapdec_decode(bad, 1, dummy, dummy, dummy, 1 << 30, mapdec.FP32, None)
    assert st == mapdec.EDRIFT
    # workspace too small
    st = L.mapdec_decode(fr, 2, dummy, dummy, dummy, ws32 - 1, mapdec.FP32, None)
    assert st == mapdec.ESIZE
    # bad precision, no frames, y missing
    assert L.mapdec_decode(fr, 2, dummy, dummy, dummy, ws32, 7, None) == mapdec.EINVAL
    assert L.mapdec_decode(fr, 0, dummy, dummy, dummy, ws32, mapdec.FP32, None) == mapdec.EINVAL
    noy = (mapdec._Frame * 1)()
    noy[0] = mapdec._Frame(c.handle, 10, 30, None, None, None, None)
    assert L.mapdec_decode(noy, 1, dummy, dummy, dummy, ws32, mapdec.FP32, None) == mapdec.EINVAL


def test_general_code_validation(L):
    cb = np.array([[[(w >> (3 - r)) & 1 for r in range(4)] for w in range(4)]] * 5, np.uint8)
    # limits must satisfy m_n^- <= 0 <= m_n^+, m_tau^- <= m_n^-, m_tau^+ >= m_n^+
    for lim in [(-4, 4, 1, 2), (-4, 4, -2, -1), (-1, 4, -2, 2), (-4, 1, -2, 2)]:
        with pytest.raises(mapdec.MapdecError) as e:
            mapdec.Code(cb, 0.05, 0.05, 0.0, 2, limits=lim)
        assert e.value.status == mapdec.EINVAL
    bad = cb.copy()
    bad[2, 1] = bad[2, 0]   # codebook 2 not injective
    with pytest.raises(mapdec.MapdecError):
        mapdec.Code(bad, 0.05, 0.05, 0.0, 2, limits=(-4, 4, -2, 2))
    c = mapdec.Code(cb, 0.05, 0.05, 0.0, 2, limits=(-3, 6, -1, 2))
    assert (c.M, c.mn) == (6, 2)
    dummy = ctypes.c_void_p(0x1000)
    # N must equal the number of codebooks
    fr = _frames([(c, 4, 16)])
    assert L.mapdec_decode(fr, 1, dummy, dummy, dummy, 1 << 30, mapdec.FP32, None) \
        == mapdec.EINVAL
    # end drift inside [-M, M] but outside [mt_lo, mt_hi]
    fr = _frames([(c, 5, 20 - 5)])
    assert L.mapdec_decode(fr, 1, dummy, dummy, dummy, 1 << 30, mapdec.FP32, None) \
        == mapdec.EDRIFT
    fr = _frames([(c, 5, 20 + 6)])
    assert L.mapdec_workspace_size(fr, 1, mapdec.FP32, 0, 0) > 0


def test_noalloc_limit_and_size_check(L):
    # the allocation-free decode validates like mapdec_decode and rejects a
    # layout beyond its fixed array before any device call
    assert L.mapdec_noalloc_limit() == 64 << 20
    c = _code(q=16, n=10, M=98, mn=6, cb=np.array(
        [[(w >> (9 - r)) & 1 for r in range(10)] for w in range(16)], np.uint8))
    big = _frames([(c, 500, 5000)] * 32)
    need = L.mapdec_workspace_size(big, 32, mapdec.FP32, 0, 0)
    assert need > L.mapdec_noalloc_limit()
    dummy = ctypes.c_void_p(0x1000)
    assert L.mapdec_decode_noalloc(big, 32, dummy, dummy, mapdec.FP32, None) == mapdec.ESIZE
    bad = _frames([(c, 500, 5000 + 99)])
    assert L.mapdec_decode_noalloc(bad, 1, dummy, dummy, mapdec.FP32, None) == mapdec.EDRIFT
    assert L.mapdec_decode_noalloc(big, 0, dummy, dummy, mapdec.FP32, None) == mapdec.EINVAL


def test_checkpointed_workspace_is_smaller(L):
    # a long frame: groups of checkpoint segments keep O(K) metric rows and
    # one group's receiver metric instead of the whole frame's; what stays
    # O(N) is Gamma (2mn+1 values per received bit, the chains' input), the
    # checkpoints and the per-symbol logs
    c = _code()
    fr = _frames([(c, 2000, 6000)])
    full = L.mapdec_workspace_size(fr, 1, mapdec.FP32, mapdec.FLAG_GRAD, 0)
    ck = L.mapdec_workspace_size(fr, 1, mapdec.FP32, mapdec.FLAG_GRAD, 45)
    assert 0 < ck < full / 3
    # K >= N is a single segment: the same layout as K = 0
    assert L.mapdec_workspace_size(fr, 1, mapdec.FP32, mapdec.FLAG_GRAD, 2000) == full


def test_unsupported_sizes(L):
    big_n = np.zeros((2, 17), np.uint8)
    big_n[1, 0] = 1
    c = mapdec.Code(big_n, 0.01, 0.01, 0, 2, 10, 2)
    fr = _frames([(c, 3, 51)])
    dummy = ctypes.c_void_p(0x1000)
    assert L.mapdec_decode(fr, 1, dummy, dummy, dummy, 1 << 30, mapdec.FP32, None) \
        == mapdec.EUNSUPPORTED
    c2 = _code(M=20, mn=9)
    fr2 = _frames([(c2, 10, 30)])
    assert L.mapdec_decode(fr2, 1, dummy, dummy, dummy, 1 << 30, mapdec.FP32, None) \
        == mapdec.EUNSUPPORTED


def test_frame_struct_layout_matches_header(tmp_path):
    # the binding's ctypes mirror of mapdec_frame has the size and field
    # offsets that a C compiler gives the header's struct
    fields = [f[0] for f in mapdec._Frame._fields_]
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "mapdec.h"\n'
        "int main(void) {\n"
        '    printf("%zu", sizeof(mapdec_frame));\n'
        + "".join(f'    printf(" %zu", offsetof(mapdec_frame, {f}));\n' for f in fields)
        + "    return 0;\n}\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True)
    vals = [int(v) for v in out.stdout.split()]
    assert vals[0] == ctypes.sizeof(mapdec._Frame)
    assert vals[1:] == [getattr(mapdec._Frame, f).offset for f in fields]


def test_outer_code_validation(L):
    # host-side checks before any device call: every case returns NULL
    import numpy as np
    rp = np.array([0, 3], np.int32)
    cl = np.array([0, 1, 2], np.int32)
    cf = np.array([1, 2, 3], np.uint8)
    def create(q, N, m, rp, cl, cf):
        return L.mapdec_outer_create(q, N, m, rp.ctypes.data, cl.ctypes.data, cf.ctypes.data)
    for args, st in [((6, 3, 1, rp, cl, cf), mapdec.EINVAL),            # q not a power of 2
                     ((128, 3, 1, rp, cl, cf), mapdec.EINVAL),          # q above 64
                     ((4, 3, 1, rp, cl, np.array([1, 0, 3], np.uint8)), mapdec.EINVAL),  # zero
                     ((4, 3, 1, rp, cl, np.array([1, 2, 4], np.uint8)), mapdec.EINVAL),  # >= q
                     ((4, 3, 1, rp, np.array([0, 1, 1], np.int32), cf), mapdec.EINVAL),  # repeat
                     ((4, 2, 1, rp, cl, cf), mapdec.EINVAL),            # column >= N
                     ((4, 3, 1, np.array([1, 3], np.int32), cl, cf), mapdec.EINVAL),
                     ((4, 40, 1, np.array([0, 33], np.int32), np.arange(33, dtype=np.int32),
                       np.ones(33, np.uint8)), mapdec.EUNSUPPORTED)]:   # row degree 33
        assert not create(*args)
        assert L.mapdec_last_error() == st
    assert L.mapdec_outer_workspace_size(None, 1, mapdec.FP32) == 0
    assert L.mapdec_outer_decode(None, 1, None, None, None, 1, None, 0, mapdec.FP32,
                                 None) == mapdec.EINVAL
