"""Builds and loads the oracle's plain-C loops (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "das.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_OUT_DIR, "liboracle_das.so")
_lock = threading.Lock()
_handle = None


class Probe(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int), ("pitch", ctypes.c_double), ("c", ctypes.c_double),
                ("f0", ctypes.c_double), ("fs", ctypes.c_double), ("t_start", ctypes.c_double),
                ("n_samp", ctypes.c_int)]


def compile_c(src: str, out: str) -> str:
    """Compile one C file of FP64 loops into a shared library (gcc, OpenMP)."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                    "-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile das.c (FP64, OpenMP) unless an up-to-date library exists."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_c(_SRC, _LIB)
    return _LIB


def load(path: str):
    """Load a library built from das.c (or a copy of it) and declare its entry points."""
    h = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    c_int, c_double = ctypes.c_int, ctypes.c_double
    h.oracle_das_stage1.argtypes = [
        dp, c_int, c_int, c_int, dp, ctypes.POINTER(Probe), c_int, c_int, c_double,
        c_double, c_double, c_double, c_double, dp]
    h.oracle_das_stage1.restype = None
    h.oracle_das_3d_slab.argtypes = [
        dp, c_int, c_int, c_int, dp, ctypes.POINTER(Probe), c_int, c_int, c_double,
        c_double, c_double, c_double, c_double, c_double, c_int, c_int, dp]
    h.oracle_das_3d_slab.restype = None
    return h


def lib():
    global _handle
    with _lock:
        if _handle is None:
            _handle = load(build())
    return _handle


def dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
