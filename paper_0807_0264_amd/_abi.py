"""ctypes declaration of the C ABI in include/mcg.h (libmcg.so).

Loading fails loudly when the gfx950 library is not built: there is no CPU
fallback anywhere in this package.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmcg.so")

MCG_OK, MCG_WNOTCONV, MCG_EINVAL, MCG_ENOMEM, MCG_EHIP, MCG_EINPUT = 0, 1, -1, -2, -3, -4
MCG_F64, MCG_F32 = 0, 1
MCG_NUM_VARIANTS = 6
MCG_OPT_TWO_ROW = 1
MCG_OPT_SLABS = 2
MCG_OPT_HITS = 3
MCG_OPT_STOP_EVERY = 4
MCG_OPT_CHECK = 5
MCG_OPT_SCRATCH_LIMIT_MIB = 6
MCG_OPT_EXACT = 7
MCG_OPT_ORDER = 8
MCG_OPT_DEFER_G = 9
MCG_OPT_PAIRED = 10
MCG_VORTEX_ONLY, MCG_VORTEX_REMOVED = 0, 1


class Dims(C.Structure):
    _fields_ = [("L", C.c_int32 * 4)]


class Field(C.Structure):
    _fields_ = [("d", Dims), ("prec", C.c_int32), ("pad_", C.c_int32), ("ptr", C.c_void_p)]


class Gauge(C.Structure):
    _fields_ = [("d", Dims), ("ptr", C.c_void_p)]


class TuneChoice(C.Structure):
    _fields_ = [("variant", C.c_int32), ("order", C.c_int32), ("paired", C.c_int32), ("slabs", C.c_int32),
                ("ms_per_sweep", C.c_double), ("ms_default", C.c_double)]


class FixOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("omega", C.c_double), ("max_sweeps", C.c_int32),
                ("reunit_every", C.c_int32), ("start_sweep", C.c_int32),
                ("check_every", C.c_int32), ("traj", C.POINTER(C.c_double))]


class FixResult(C.Structure):
    _fields_ = [("R", C.c_double), ("dR", C.c_double), ("theta", C.c_double),
                ("sweeps", C.c_int32), ("blocks50", C.c_int32), ("status", C.c_int32),
                ("pad_", C.c_int32)]


class PrecondResult(C.Structure):
    _fields_ = [("smeared", FixResult), ("fixed", FixResult), ("min_margin", C.c_double),
                ("vortices", C.c_int64), ("per_plane", C.c_int64 * 6), ("per_charge", C.c_int64 * 2)]


_P = C.c_void_p
_S = C.c_int32  # mcg_status
_CTX = C.c_void_p

# name: (restype, argtypes)
SIGNATURES = {
    "mcg_create": (_S, [C.POINTER(_CTX), C.c_int32]),
    "mcg_destroy": (_S, [_CTX]),
    "mcg_status_string": (C.c_char_p, [_S]),
    "mcg_last_error": (C.c_char_p, [_CTX]),
    "mcg_field_bytes": (C.c_size_t, [Dims, C.c_int32]),
    "mcg_gauge_bytes": (C.c_size_t, [Dims]),
    "mcg_pack_links": (_S, [_CTX, _P, C.c_int32, C.POINTER(Field), _P]),
    "mcg_unpack_links": (_S, [_CTX, C.POINTER(Field), _P, C.c_int32, _P]),
    "mcg_pack_gauge": (_S, [_CTX, _P, C.POINTER(Gauge), _P]),
    "mcg_unpack_gauge": (_S, [_CTX, C.POINTER(Gauge), _P, _P]),
    "mcg_gauge_identity": (_S, [_CTX, C.POINTER(Gauge), _P]),
    "mcg_gauge_reunit": (_S, [_CTX, C.POINTER(Gauge), _P]),
    "mcg_smear": (_S, [_CTX, C.POINTER(Field), C.POINTER(Field), C.c_double, C.c_double,
                       C.c_int32, _P]),
    "mcg_apply_gauge": (_S, [_CTX, C.POINTER(Field), C.POINTER(Gauge), C.POINTER(Field), _P]),
    "mcg_functional": (_S, [_CTX, C.POINTER(Field), C.POINTER(C.c_double), _P]),
    "mcg_plaquette": (_S, [_CTX, C.POINTER(Field), C.POINTER(C.c_double), _P]),
    "mcg_theta": (_S, [_CTX, C.POINTER(Field), C.POINTER(C.c_double), _P]),
    "mcg_halfsweep": (_S, [_CTX, C.POINTER(Field), C.POINTER(Gauge), C.c_int32, C.c_double, _P]),
    "mcg_sweeps": (_S, [_CTX, C.POINTER(Field), C.POINTER(Gauge), C.c_int32, C.c_double, _P]),
    "mcg_sweeps_timed": (_S, [_CTX, C.POINTER(Field), C.POINTER(Gauge), C.c_int32, C.c_double,
                              C.POINTER(C.c_double), _P]),
    "mcg_fix": (_S, [_CTX, C.POINTER(Field), C.POINTER(Gauge), C.POINTER(FixOpts),
                     C.POINTER(FixResult), _P]),
    "mcg_fix_batch": (_S, [_CTX, C.c_int32, C.POINTER(Field), C.POINTER(Gauge),
                           C.POINTER(FixOpts), C.POINTER(FixResult), _P]),
    "mcg_precondition_batch": (_S, [_CTX, C.c_int32, C.POINTER(Field), C.c_double, C.c_double, C.c_int32,
                                    C.POINTER(FixOpts), C.POINTER(Gauge), C.POINTER(C.c_void_p),
                                    C.POINTER(PrecondResult), _P]),
    "mcg_center_project": (_S, [_CTX, C.POINTER(Field), C.POINTER(Gauge), _P,
                                C.POINTER(C.c_double), _P]),
    "mcg_center_project_noalloc": (_S, [_CTX, C.POINTER(Field), C.POINTER(Gauge), _P,
                                        C.POINTER(C.c_double), _P]),
    "mcg_count_vortices": (_S, [_CTX, _P, Dims, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int64), _P]),
    "mcg_unitarity": (_S, [_CTX, C.POINTER(Field), C.POINTER(Gauge), C.POINTER(C.c_double),
                           C.POINTER(C.c_double), _P]),
    "mcg_vortex_field": (_S, [_CTX, C.POINTER(Field), C.POINTER(Gauge), _P, C.c_int32, C.POINTER(Field), _P]),
    "mcg_wilson_loops": (_S, [_CTX, C.POINTER(Field), C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.c_int32,
                              C.POINTER(C.c_double), _P]),
    "mcg_smear_mcg_backward": (_S, [_CTX, C.POINTER(Field), C.c_double, C.c_double, C.c_int32,
                                    C.POINTER(Gauge), C.c_int32, C.POINTER(Field),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), _P]),
    "mcg_autotune": (_S, [_CTX, C.POINTER(Field), C.POINTER(C.c_int32), C.POINTER(C.c_double), _P]),
    "mcg_autotune_batch": (_S, [_CTX, C.c_int32, C.POINTER(Field), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                _P]),
    "mcg_tune_batch": (_S, [_CTX, C.c_int32, C.POINTER(Field), C.POINTER(TuneChoice), _P]),
    "mcg_clear_tuning": (_S, [_CTX]),
    "mcg_set_variant": (_S, [_CTX, C.c_int32, C.c_int32]),
    "mcg_get_variant": (_S, [_CTX, C.c_int32, C.POINTER(C.c_int32)]),
    "mcg_set_option": (_S, [_CTX, C.c_int32, C.c_int32]),
    "mcg_get_option": (_S, [_CTX, C.c_int32, C.POINTER(C.c_int32)]),
}

_lib = None


def load(path=LIBPATH):
    """Load libmcg.so and declare every entry point; raises if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(
                f"{path} is not built: the MCG library runs only as gfx950 HIP code "
                "(build it with `python -m paper_0807_0264_amd.build`)")
        lib = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib
