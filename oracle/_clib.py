"""Loader for the plain C part of the oracle (``dd_oracle.c``).

Test infrastructure only.  The shared library is compiled with gcc (OpenMP,
-O2, no fast-math) into ``oracle/liboracle.so``; ``build()`` recompiles it,
and ``lib()`` compiles it on first use when it is missing or older than its
source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dd_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc; returns the path of the shared library."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


def lib() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = ctypes.CDLL(_SO)
            P = ctypes.c_void_p
            I = ctypes.c_int
            D = ctypes.c_double
            L.or_gamma.argtypes = [I, P]
            L.or_gamma.restype = None
            L.or_hop_full.argtypes = [P, I, P, P, P]
            L.or_hop_full.restype = None
            L.or_dirac_full.argtypes = [P, I, D, P, P, P]
            L.or_dirac_full.restype = None
            L.or_hop_box.argtypes = [P, I, P, P, P, P, P]
            L.or_hop_box.restype = None
            L.or_dirac_box.argtypes = [P, I, D, P, P, P, P, P]
            L.or_dirac_box.restype = None
            L.or_box_parity.argtypes = [P, P, P, P]
            L.or_box_parity.restype = None
            L.or_solve_box.argtypes = [P, I, D, P, P, P, P, P, D, I, P]
            L.or_solve_box.restype = I
            L.or_solve_many.argtypes = [P, I, D, P, I, P, I, P, P, D, I, P, P, I]
            L.or_solve_many.restype = I
            L.or_num_threads.argtypes = []
            L.or_num_threads.restype = I
            _lib = L
    return _lib
