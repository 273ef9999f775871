"""ctypes loader for ring_oracle.c (test infrastructure only).

Builds the shared object with gcc on first use if it is missing.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ring_oracle.c")
_LIB = os.path.join(_HERE, "libring_oracle.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = False) -> str:
    """Compile ring_oracle.c with gcc (plain C11, OpenMP over limbs)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.or_powmod.argtypes = [u64, u64, u64]
        L.or_powmod.restype = u64
        L.or_invmod.argtypes = [u64, u64]
        L.or_invmod.restype = u64
        L.or_ntt_definition.argtypes = [_u64p, _u64p, u32, u64, u64]
        L.or_ntt_fast.argtypes = [_u64p, _u64p, u32, u64, u64]
        L.or_intt_fast.argtypes = [_u64p, _u64p, u32, u64, u64]
        L.or_set_mul_mode.argtypes = [i32]
        L.or_get_mul_mode.restype = i32
        L.or_mul_limb.argtypes = [_u64p, _u64p, _u64p, u32, u64, u64, i32]
        L.or_poly_mul.argtypes = [_u64p, _u64p, _u64p, u32, _u64p, _u64p, u32]
        L.or_pointwise_mul.argtypes = [_u64p, _u64p, _u64p, u64, u64]
        L.or_scalar_mul.argtypes = [_u64p, u64, _u64p, u64, u64]
        L.or_automorphism.argtypes = [_u64p, _u64p, u32, u64, u64]
        L.or_base_convert.argtypes = [_u64p, _u64p, u32, _u64p, u32, _u64p, u32]
        L.or_mul_coeff.argtypes = [_u64p, _u64p, u32, u64, u32]
        L.or_mul_coeff.restype = u64
        _lib = L
    return _lib


def ptr(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(_u64p)


def u64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint64)
