"""ctypes loader of the plain serial C fitness (serial.c): test
infrastructure and the single-thread CPU baseline of the benchmark.  Built
by ``build()`` (gcc, no GPU code)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "serial.c")
LIB = os.path.join(HERE, "liboracle_serial.so")
_lib = None


def build() -> str:
    """Compiles serial.c into oracle/liboracle_serial.so."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", SRC, "-o", LIB, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.oracle_fitness_serial.restype = ctypes.c_int
        L.oracle_fitness_serial.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
            ctypes.c_void_p]
        _lib = L
    return _lib


def fitness(X, t, genes, basis: int, degree: int, error_fn: int = 0, R: float = 0.0):
    """Fitness [n] float64 of genes [n x K] over X [NP x N], t [NP] (float32
    inputs, as the GPU path takes them)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    genes = np.ascontiguousarray(np.atleast_2d(genes), dtype=np.float32)
    out = np.empty(genes.shape[0], dtype=np.float64)
    rc = lib().oracle_fitness_serial(X.ctypes.data, t.ctypes.data, X.shape[0], X.shape[1],
                                     genes.ctypes.data, genes.shape[0], basis, degree, error_fn,
                                     R, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_fitness_serial: bad argument")
    return out
