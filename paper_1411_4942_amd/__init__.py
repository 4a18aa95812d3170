"""MI355X-native 3-path sampling for 4-vertex induced subgraph counts.

The compute path lives in the HIP library ``libpathsamp.so`` (sources under
``csrc/``, C ABI declared in ``include/pathsamp.h``); :mod:`.pathsamp` is its
thin ctypes binding and :mod:`.synth` makes seeded synthetic graphs.
Importing the package loads nothing; the library is opened on first use.
"""
__all__ = ["pathsamp", "synth"]
