"""Build and load the reference C loops (TEST INFRASTRUCTURE ONLY).

Compiled with gcc, -O2 -fno-fast-math -ffp-contract=off, so the FP64
arithmetic is evaluated exactly in the order written in the C sources.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["stencil.c", "z4c.c"]
OUT = os.path.join(HERE, "_build", "liboracle.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall"]

_lib = None


def build(force: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    if not force and os.path.exists(OUT):
        t = os.path.getmtime(OUT)
        if all(os.path.getmtime(s) <= t for s in srcs):
            return OUT
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    tmp = OUT + f".tmp{os.getpid()}"
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, *srcs, "-lm"], check=True)
    os.replace(tmp, OUT)
    return OUT


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        i64p = ctypes.c_void_p
        d = ctypes.c_double
        i = ctypes.c_int
        L = ctypes.c_int64
        _lib.orc_wave_rhs.argtypes = [i, i64p, i, L, i64p, i64p, d, d]
        _lib.orc_wave_rhs8.argtypes = [i, i64p, i, L, i64p, i64p, d, d]
        _lib.orc_wave_rhs8.restype = None
        _lib.orc_wave_rhs8_ko9.argtypes = [i, i64p, i, L, i64p, i64p, d, d]
        _lib.orc_wave_rhs8_ko9.restype = None
        _lib.orc_stage.argtypes = [i, i64p, i, L, i, i64p, i64p, i64p, d]
        _lib.orc_final.argtypes = [i, i64p, i, L, i, i64p, i64p, i64p, i64p, i64p, i64p, d]
        _lib.orc_copy_points.argtypes = [L, i64p, i64p, i, L, i64p]
        _lib.orc_prolong.argtypes = [L, i64p, i64p, i64p, i, L, i64p, i64p]
        _lib.orc_prolong.restype = None
        for f in (_lib.orc_wave_rhs, _lib.orc_stage, _lib.orc_final, _lib.orc_copy_points):
            f.restype = None
        if hasattr(_lib, "orc_z4c_rhs"):
            for f in (_lib.orc_z4c_rhs, _lib.orc_z4c_rhs8, _lib.orc_z4c_rhs8_ko9):
                f.argtypes = [i, i64p, i, L, i64p, i64p, d, i64p, i64p, i64p, i64p]
                f.restype = None
    return _lib


def ptr(a):
    return ctypes.c_void_p(a.ctypes.data)
