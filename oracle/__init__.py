"""FP64 CPU oracle for iterated stencils with a fixed zero halo.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the GPU path.

`apply` calls the plain C implementation in ``stencil_oracle.c`` (the stencil
definition of SPIDER Sec. 2.2 written out in fp64, zero halo, Jacobi steps);
see that file's header for the exact summation order.  `build` compiles it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stencil_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")            # -march=x86-64-v3 (AVX2, FMA unit unused)
_LIB_GENERIC = os.path.join(_HERE, "liboracle_generic.so")  # baseline x86-64
_V3_FLAGS = ("avx2", "bmi1", "bmi2", "fma", "f16c", "abm", "movbe", "xsave")
_lib = None


def build():
    """Compile the oracle with gcc (fp64, no FMA contraction, no fast-math, OpenMP), once
    for x86-64-v3 hosts and once for baseline x86-64.  The flags change only the
    instructions chosen: with contraction and fast-math off every product and sum is
    the same IEEE operation in the same order, so both give identical results."""
    for lib, march in ((_LIB, ["-march=x86-64-v3"]), (_LIB_GENERIC, [])):
        cmd = ["gcc", "-O3"] + march + ["-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                                        "-fno-fast-math", "-std=c11", "-Wall", "-Wextra", "-o", lib + ".tmp", _SRC]
        subprocess.check_call(cmd)
        os.replace(lib + ".tmp", lib)


def ensure_built():
    """Build the oracle if its libraries are missing (tests, smoke check, benchmark)."""
    if not (os.path.exists(_LIB) and os.path.exists(_LIB_GENERIC)):
        build()


def _host_is_v3():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("flags"):
                    flags = set(line.split(":", 1)[1].split())
                    return all(fl in flags for fl in _V3_FLAGS)
    except OSError:
        pass
    return False


def _load():
    global _lib
    if _lib is None:
        path = _LIB if _host_is_v3() else _LIB_GENERIC
        if not os.path.exists(path):
            raise RuntimeError("oracle library not built: run __graft_entry__.build() or oracle.build()")
        lib = ctypes.CDLL(path)
        lib.oracle_stencil.restype = ctypes.c_int
        lib.oracle_stencil.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int, ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads():
    """Number of OpenMP threads the oracle uses by default."""
    return _load().oracle_max_threads()


def apply(coeffs, x, steps, nthreads=0):
    """Return S^steps(x) in fp64.

    coeffs: (2r+1,)*ndim array, w[dz][dy][dx] multiplies x[p + (dz, dy, dx) - r].
    x: 1-D, 2-D or 3-D array (any real dtype; converted exactly to fp64).
    """
    w = np.ascontiguousarray(coeffs, dtype=np.float64)
    xin = np.ascontiguousarray(x, dtype=np.float64)
    ndim = xin.ndim
    if w.ndim != ndim or len(set(w.shape)) != 1 or w.shape[0] % 2 != 1:
        raise ValueError("coeffs must be (2r+1,)*ndim")
    r = (w.shape[0] - 1) // 2
    out = np.empty_like(xin)
    shape = (ctypes.c_int64 * ndim)(*xin.shape)
    rc = _load().oracle_stencil(ndim, shape, r, w.ctypes.data, xin.ctypes.data, out.ctypes.data,
                                int(steps), int(nthreads))
    if rc != 0:
        raise RuntimeError("oracle_stencil failed with code %d" % rc)
    return out


def rel_errors(y, ref):
    """Normwise relative errors of y against the fp64 reference: (rel-RMS, rel-max).

    rel-RMS = ||y - ref||_2 / ||ref||_2,  rel-max = ||y - ref||_inf / ||ref||_inf.
    """
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = y - ref
    nr = np.sqrt(np.sum(ref * ref))
    mr = np.max(np.abs(ref))
    return float(np.sqrt(np.sum(d * d)) / nr), float(np.max(np.abs(d)) / mr)
