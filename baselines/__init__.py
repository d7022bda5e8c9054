"""CPU baselines timed beside the GPU path (never used by the library).

`local_max` is a multicore (OpenMP) run of the same local-max rounds, the
shared-memory CPU form of the method that the paper also evaluates
(Section 6).  It is a performance comparison: results are checked against the
oracle in the tests like any other implementation.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_local_max.c")
LIB = os.path.join(HERE, "_cpu_local_max.so")
_lib = None


def build() -> str:
    subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", LIB, SRC],
                   check=True)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        lib.cpu_local_max.restype = ctypes.c_int
        lib.cpu_local_max.argtypes = [ctypes.c_int32, ctypes.c_int32, p, p, p, ctypes.c_uint32,
                                      ctypes.c_int, ctypes.c_int, p, p, p]
        _lib = lib
    return _lib


def local_max(n, m, e_off, e_pins, w, seed, reseed=False, threads=0):
    """Returns (bits uint32[ceil(m/32)], rounds, sum of live pins over rounds)."""
    e_off = np.ascontiguousarray(e_off, dtype=np.int32)
    e_pins = np.ascontiguousarray(e_pins, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    bits = np.zeros(max((m + 31) // 32, 1), dtype=np.uint32)
    rounds = ctypes.c_int32(0)
    pins = ctypes.c_int64(0)
    rc = _load().cpu_local_max(n, m, e_off.ctypes.data, e_pins.ctypes.data, w.ctypes.data,
                               seed & 0xFFFFFFFF, 1 if reseed else 0, threads, bits.ctypes.data,
                               ctypes.byref(rounds), ctypes.byref(pins))
    if rc != 0:
        raise RuntimeError(f"cpu_local_max failed ({rc})")
    return bits[:(m + 31) // 32], rounds.value, pins.value
