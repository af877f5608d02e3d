"""Build and load the C helper of the input generators (workloads/_wendland.c).

python -m workloads.native     (gcc, in-tree: workloads/_lib/libwendland.so)

The helper only speeds up building large Wendland covariances; without it
the NumPy path builds the same matrices.
"""
from __future__ import annotations

import ctypes as C
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "_wendland.c")
LIB = os.path.join(HERE, "_lib", "libwendland.so")
_lib = None


def build() -> str:
    gcc = shutil.which("gcc") or shutil.which("cc")
    if gcc is None:
        raise RuntimeError("gcc not found")
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp"
    # no contraction into fused multiply-adds: the per-pair arithmetic must
    # round as NumPy's separate operations do
    subprocess.run([gcc, "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                    SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def lib():
    """The loaded helper, or None when it has not been built."""
    global _lib
    if _lib is None and os.path.exists(LIB):
        h = C.CDLL(LIB)
        i64, dp, i64p, i32p = C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int64), \
            C.POINTER(C.c_int32)
        h.wendland_count.argtypes = [i64, i64, dp, i64p, i64p, i64, C.c_double, i64p]
        h.wendland_count.restype = None
        h.wendland_fill.argtypes = [i64, i64, dp, i64p, i64p, i64, C.c_double, C.c_double,
                                    C.c_double, i64p, i32p, dp]
        h.wendland_fill.restype = None
        _lib = h
    return _lib


if __name__ == "__main__":
    print(build())
