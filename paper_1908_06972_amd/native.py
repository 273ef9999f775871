"""ctypes binding of libpft (include/pft.h): argument marshalling only.

Every function here forwards to the C ABI of the same name and raises
PftError on a non-zero status.  Device memory for ciphertexts and plaintexts
comes from torch tensors (int64 storage holding uint64 residues); the HIP
stream is torch's current stream.  There is no fallback: if libpft.so is
missing or was built for another target, loading fails loudly.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpft.so")

PFT_OK, PFT_EINVAL, PFT_EPARAM, PFT_ELEVEL, PFT_ESCALE, PFT_ENOKEY, PFT_ENOMEM, PFT_EHIP = 0, -1, -2, -3, -4, -5, -6, -7

_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_dblp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class PftError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libpft error %d: %s" % (code, msg))
        self.code = code


class ParamSpec(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32), ("q0_bits", ctypes.c_uint32),
                ("q_bits", ctypes.c_uint32), ("n_p", ctypes.c_uint32), ("p_bits", ctypes.c_uint32),
                ("dnum", ctypes.c_uint32), ("rescale_mode", ctypes.c_uint32), ("scale", ctypes.c_double)]


class ParamPrimes(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32), ("q", _u64p), ("p", _u64p),
                ("n_p", ctypes.c_uint32), ("dnum", ctypes.c_uint32), ("rescale_mode", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("scale", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p), ("budget_bytes", ctypes.c_uint64)]


class CtDesc(ctypes.Structure):
    _fields_ = [("data", _vp), ("level", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("scale", ctypes.c_double)]


PtDesc = CtDesc  # same layout: pft_pt


class OpDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("a", ctypes.c_uint32), ("b", ctypes.c_uint32), ("out", ctypes.c_uint32),
                ("step", ctypes.c_int32), ("mode", ctypes.c_uint32)]


PFT_OP_NTT, PFT_OP_INTT, PFT_OP_ADD, PFT_OP_MUL_RELIN, PFT_OP_RESCALE, PFT_OP_ROTATE = 1, 2, 3, 4, 5, 6
PFT_OP_MUL_PLAIN = 7
PFT_RESCALE_DEFAULT = 2

# (name, argtypes, restype) of every exported symbol declared in include/pft.h
SIGNATURES = [
    ("pft_params_create", [ctypes.POINTER(ParamSpec), ctypes.POINTER(_vp)], ctypes.c_int),
    ("pft_params_destroy", [_vp], None),
    ("pft_params_moduli", [_vp, _u64p, _u64p], ctypes.c_int),
    ("pft_params_dims", [_vp, _u32p], ctypes.c_int),
    ("pft_last_error", [], ctypes.c_char_p),
    ("pft_params_create_primes", [ctypes.POINTER(ParamPrimes), ctypes.POINTER(_vp)], ctypes.c_int),
    ("pft_params_rescale_mode", [_vp, _u32p], ctypes.c_int),
    ("pft_ctx_create", [_vp, ctypes.c_int, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    ("pft_ctx_create_alloc", [_vp, ctypes.c_int, _vp, ctypes.POINTER(Allocator), ctypes.POINTER(_vp)], ctypes.c_int),
    ("pft_ctx_set_budget", [_vp, ctypes.c_uint64], ctypes.c_int),
    ("pft_ctx_memory", [_vp, _u64p], ctypes.c_int),
    ("pft_ptmat_plan", [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(OpDesc), ctypes.c_uint32,
                        _u32p], ctypes.c_int),
    ("pft_ptmat_plan_export", [_vp, ctypes.POINTER(OpDesc), ctypes.c_uint32, _u32p, _i64p], ctypes.c_int),
    ("pft_ctx_destroy", [_vp], None),
    ("pft_ctx_synchronize", [_vp], ctypes.c_int),
    ("pft_set_secret", [_vp, _i64p], ctypes.c_int),
    ("pft_gen_public_key", [_vp, _u64p, _i64p], ctypes.c_int),
    ("pft_gen_relin_key", [_vp, _u64p, _i64p], ctypes.c_int),
    ("pft_gen_rotation_key", [_vp, ctypes.c_int32, _u64p, _i64p], ctypes.c_int),
    ("pft_ctx_device_bytes", [_vp, _u64p], ctypes.c_int),
    ("pft_encrypt", [_vp, _i64p, ctypes.c_uint32, ctypes.c_double, _i64p, _i64p, _i64p, ctypes.POINTER(CtDesc)],
     ctypes.c_int),
    ("pft_decrypt", [_vp, ctypes.POINTER(CtDesc), _u64p], ctypes.c_int),
    ("pft_ct_export", [_vp, ctypes.POINTER(CtDesc), _u64p], ctypes.c_int),
    ("pft_ct_import", [_vp, _u64p, ctypes.c_uint32, ctypes.c_double, ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_pt_from_coeffs", [_vp, _i64p, ctypes.c_uint32, ctypes.c_double, ctypes.POINTER(PtDesc)], ctypes.c_int),
    ("pft_add", [_vp, ctypes.POINTER(CtDesc), ctypes.POINTER(CtDesc), ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_add_plain", [_vp, ctypes.POINTER(CtDesc), ctypes.POINTER(PtDesc), ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_mul_plain", [_vp, ctypes.POINTER(CtDesc), ctypes.POINTER(PtDesc), ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_mul_relin", [_vp, ctypes.POINTER(CtDesc), ctypes.POINTER(CtDesc), ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_mul_relin_batch", [_vp, ctypes.c_uint32, ctypes.POINTER(CtDesc), ctypes.POINTER(CtDesc),
                             ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_rescale", [_vp, ctypes.POINTER(CtDesc), ctypes.c_uint32, ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_rescale_batch", [_vp, ctypes.c_uint32, ctypes.POINTER(CtDesc), ctypes.c_uint32, ctypes.POINTER(CtDesc)],
     ctypes.c_int),
    ("pft_mod_drop", [_vp, ctypes.POINTER(CtDesc), ctypes.c_uint32, ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_rotate", [_vp, ctypes.POINTER(CtDesc), ctypes.c_int32, ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_rotate_batch", [_vp, ctypes.c_uint32, ctypes.POINTER(CtDesc), ctypes.c_int32, ctypes.POINTER(CtDesc)],
     ctypes.c_int),
    ("pft_rotate_pow2", [_vp, ctypes.POINTER(CtDesc), ctypes.c_int32, ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_rotate_pow2_batch", [_vp, ctypes.c_uint32, ctypes.POINTER(CtDesc), ctypes.c_int32, ctypes.POINTER(CtDesc)],
     ctypes.c_int),
    ("pft_total_sum", [_vp, ctypes.POINTER(CtDesc), ctypes.c_uint32, ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_total_sum_batch", [_vp, ctypes.c_uint32, ctypes.POINTER(CtDesc), ctypes.c_uint32, ctypes.POINTER(CtDesc)],
     ctypes.c_int),
    ("pft_mul_const", [_vp, ctypes.POINTER(CtDesc), ctypes.c_double, ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_mul_const_batch", [_vp, ctypes.c_uint32, ctypes.POINTER(CtDesc), _dblp, ctypes.POINTER(CtDesc)],
     ctypes.c_int),
    ("pft_ptmat_create", [_vp, _dblp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                          ctypes.POINTER(_vp)], ctypes.c_int),
    ("pft_ptmat_create_from_coeffs", [_vp, _i64p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_double, ctypes.POINTER(_vp)], ctypes.c_int),
    ("pft_ptmat_info", [_vp, _u32p], ctypes.c_int),
    ("pft_ptmat_destroy", [_vp], None),
    ("pft_ptmatvec", [_vp, _vp, ctypes.c_uint32, ctypes.POINTER(CtDesc), ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_set_key_cache", [_vp, ctypes.c_uint32], ctypes.c_int),
    ("pft_keygen", [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), ctypes.c_uint32], ctypes.c_int),
    ("pft_gaussian_cdt", [_u64p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
    ("pft_encrypt_seeded", [_vp, _i64p, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(CtDesc)],
     ctypes.c_int),
    ("pft_key_cache_stats", [_vp, _u64p], ctypes.c_int),
    ("pft_key_cache_plan", [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_uint32], ctypes.c_int),
    ("pft_mul_relin_batch_noalloc", [_vp, ctypes.c_uint32, ctypes.POINTER(CtDesc), ctypes.POINTER(CtDesc),
                                     ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_ptdot_create", [_vp, _dblp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _vp], ctypes.c_int),
    ("pft_ptdot_create_from_coeffs", [_vp, _i64p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double,
                                      _vp], ctypes.c_int),
    ("pft_ptdot_destroy", [_vp], None),
    ("pft_ptdot_apply", [_vp, _vp, ctypes.c_uint32, ctypes.POINTER(CtDesc), ctypes.c_uint32, ctypes.POINTER(CtDesc)],
     ctypes.c_int),
    ("pft_diagonals_encode", [_vp, _dblp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, _i64p],
     ctypes.c_int),
    ("pft_add_const", [_vp, ctypes.POINTER(CtDesc), ctypes.c_double, ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_add_const_batch", [_vp, ctypes.c_uint32, ctypes.POINTER(CtDesc), _dblp, ctypes.POINTER(CtDesc)],
     ctypes.c_int),
    ("pft_ctmatvec", [_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(CtDesc), ctypes.c_uint32,
                      ctypes.POINTER(CtDesc), ctypes.POINTER(CtDesc)], ctypes.c_int),
    ("pft_ntt_forward", [_vp, _vp, ctypes.c_uint32, ctypes.c_uint32], ctypes.c_int),
    ("pft_ntt_inverse", [_vp, _vp, ctypes.c_uint32, ctypes.c_uint32], ctypes.c_int),
    ("pft_bconv_mode", [_vp, ctypes.c_int], ctypes.c_int),
    ("pft_ntt_candidates", [_vp, _u32p, ctypes.c_uint32], ctypes.c_int),
    ("pft_ntt_autotune", [_vp, ctypes.c_int], ctypes.c_int),
    ("pft_ntt_set_schedule", [_vp, ctypes.c_int, _u32p], ctypes.c_int),
    ("pft_ntt_get_schedule", [_vp, ctypes.c_int, ctypes.c_uint64, _u32p], ctypes.c_int),
    ("pft_ntt_tuning_export", [_vp, _u32p, ctypes.c_uint32], ctypes.c_int),
    ("pft_ntt_tuning_import", [_vp, _u32p, ctypes.c_uint32], ctypes.c_int),
    ("pft_exec_batch", [_vp, ctypes.POINTER(CtDesc), ctypes.c_uint32, ctypes.POINTER(OpDesc), ctypes.c_uint32],
     ctypes.c_int),
    ("pft_exec_plan", [ctypes.POINTER(OpDesc), ctypes.c_uint32, _u32p, ctypes.c_uint32, _u32p, _u32p], ctypes.c_int),
    ("pft_ctx_reserve", [_vp, ctypes.c_uint64, ctypes.c_uint64], ctypes.c_int),
    ("pft_graph_begin", [_vp], ctypes.c_int),
    ("pft_graph_end", [_vp, ctypes.POINTER(_vp)], ctypes.c_int),
    ("pft_graph_launch", [_vp, _vp], ctypes.c_int),
    ("pft_graph_destroy", [_vp], None),
    ("pft_prof_enable", [_vp, ctypes.c_uint32], ctypes.c_int),
    ("pft_prof_read", [_vp, ctypes.c_uint32, _dblp, _u64p, _dblp, _dblp], ctypes.c_int),
    ("pft_prof_read_variants", [_vp, ctypes.c_uint32, ctypes.c_uint32, _u32p, _dblp, _u64p, _dblp, _dblp],
     ctypes.c_int),
    ("pft_encode", [_vp, _dblp, _dblp, ctypes.c_uint32, ctypes.c_double, _i64p], ctypes.c_int),
    ("pft_decode", [_vp, _u64p, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint32, _dblp, _dblp], ctypes.c_int),
]

_lib = None


def load():
    """Load libpft.so (built in-tree by paper_1908_06972_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpft.so is not built: run `python -m paper_1908_06972_amd.build` "
                               "(or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, argt, rest in SIGNATURES:
            f = getattr(lib, name)
            f.argtypes = argt
            f.restype = rest
        _lib = lib
    return _lib


def check(status):
    if status != PFT_OK:
        raise PftError(status, load().pft_last_error().decode())
    return status


def u64p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_u64p)


def i64p(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_i64p)


def dblp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dblp)
