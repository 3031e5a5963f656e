"""Build and load the oracle's C loops (``srj_oracle.c``) -- test infrastructure.

The library is compiled with gcc, ``-O2 -ffp-contract=off`` (no fused multiply-add, so
every floating-point operation is the one written in the source) and OpenMP over
rows.  ``build()`` always recompiles; ``lib()`` compiles only when no library exists.
"""
import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "srj_oracle.c")
SO = os.path.join(_HERE, "liboracle.so")

_lib = None


def build():
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-o", SO + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(SRC):
        build()
    L = ctypes.CDLL(SO)
    i64, dbl, flt, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_float, ctypes.c_void_p
    # every sweep and residual routine takes the axis weights wt = {wy, wz, dg} (binary64, or
    # their binary32 roundings for the binary32 / bfloat16 routines) before its coefficient
    sig = {
        "or_sweep2d": [i64, i64, vp, vp, vp, dbl, vp],
        "or_sweep3d": [i64, i64, i64, vp, vp, vp, dbl, vp],
        "or_jacobi2d": [i64, i64, vp, vp, vp],
        "or_jacobi3d": [i64, i64, i64, vp, vp, vp],
        "or_srj2d": [i64, i64, vp, vp, vp, vp, i64, i64, i64, vp],
        "or_srj3d": [i64, i64, i64, vp, vp, vp, vp, i64, i64, i64, vp],
        "or_residual2d": [i64, i64, vp, vp, vp, vp, vp, vp],
        "or_residual3d": [i64, i64, i64, vp, vp, vp, vp, vp, vp],
        "or_residual_field2d": [i64, i64, vp, vp, vp, vp],
        "or_residual_field3d": [i64, i64, i64, vp, vp, vp, vp],
        "or_sweep2d_f32": [i64, i64, vp, vp, vp, flt, vp],
        "or_sweep3d_f32": [i64, i64, i64, vp, vp, vp, flt, vp],
        "or_sweep2d_bf16": [i64, i64, vp, vp, vp, flt, vp],
        "or_sweep3d_bf16": [i64, i64, i64, vp, vp, vp, flt, vp],
        "or_sweep2d_neu": [i64, i64, vp, vp, vp, dbl, vp],
        "or_sweep3d_neu": [i64, i64, i64, vp, vp, vp, dbl, vp],
        "or_residual_neu": [i64, i64, i64, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp],
        "or_op_scale": [i64, ctypes.c_int, vp, vp, vp, vp],
        "or_op_sweep": [i64, i64, i64, ctypes.c_int, vp, vp, vp, vp, dbl, vp],
        "or_op_residual": [i64, i64, i64, ctypes.c_int, vp, vp, vp, vp, ctypes.c_int, vp, vp, vp, vp, vp],
        "or_f32_to_bf16": [i64, vp, vp],
        "or_bf16_to_f32": [i64, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = None
    _lib = L
    return L


def set_threads(n):
    """Set the OpenMP thread count used by the C loops (returns the previous value)."""
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_get_max_threads.restype = ctypes.c_int
    prev = gomp.omp_get_max_threads()
    gomp.omp_set_num_threads(ctypes.c_int(int(n)))
    return prev


def max_threads():
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_get_max_threads.restype = ctypes.c_int
    return int(gomp.omp_get_max_threads())
