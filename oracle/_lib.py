"""Loader for the C part of the oracle (``lc_oracle.c``).

Test infrastructure only: the product library never imports this package.
The shared object is built in-tree with the host C compiler (``gcc -O3
-fopenmp``); :func:`build` always recompiles, :func:`load` compiles only
when no built library is present.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lc_oracle.c")
LIB = os.path.join(HERE, "liblc_oracle.so")

_lib = None


def build() -> str:
    """Compile ``lc_oracle.c`` into ``liblc_oracle.so`` (always rebuilds)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    vp, lg = ctypes.c_void_p, ctypes.c_long
    lib.oracle_gauss_legendre.argtypes = [lg, vp, vp]
    lib.oracle_gauss_legendre.restype = ctypes.c_int
    lib.oracle_legendre_coeffs.argtypes = [lg, vp, vp, vp, lg, vp]
    lib.oracle_legendre_coeffs.restype = ctypes.c_int
    lib.oracle_fourier_coeffs.argtypes = [lg, vp, vp, lg, vp, vp]
    lib.oracle_fourier_coeffs.restype = ctypes.c_int
    lib.oracle_fourier_coeffs_idx.argtypes = [lg, vp, vp, lg, vp, vp, vp]
    lib.oracle_fourier_coeffs_idx.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def threads() -> int:
    """Number of OpenMP threads the oracle's parallel loops use."""
    return int(load().oracle_max_threads())
