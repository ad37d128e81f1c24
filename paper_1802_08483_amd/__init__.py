"""MI355X-native MAP forward-backward decoder for synchronization-error
correction (inner code on the BSID channel).

The compute path is ``libmapdec.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/mapdec.h``); :mod:`.mapdec` is its ctypes binding and
:mod:`.workloads` generates seeded synthetic frames.  Importing the package
loads nothing; the library is opened on first use.
"""

__all__ = ["mapdec", "workloads", "build"]
