"""ctypes binding of libcmmlfma.so (include/cmmlfma.h).  Argument marshalling
only: every step of the method runs inside the library."""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcmmlfma.so")

CM_OK, CM_E_BADARG, CM_E_MESH, CM_E_OOM, CM_E_HIP, CM_E_NOT_BUILT, CM_E_NUMERIC, CM_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
CM_E_NOT_CONVERGED = -8
OPS = {"Z": 0, "R": 1, "X": 2, "ZH": 3, "DZDK": 4}
CM_C64, CM_C128 = 0, 1
CM_FLAG_HOST_ONLY, CM_FLAG_DERIV, CM_FLAG_CHECK, CM_FLAG_NO_MATRIX_CORES, CM_FLAG_NEAR_FP32 = 1, 2, 4, 8, 16
CM_FLAG_WIDE_NEAR, CM_FLAG_AUTOTUNE, CM_FLAG_R_STANDARD, CM_FLAG_VERBOSE, CM_FLAG_M2L_TILE16 = 32, 64, 128, 256, 512
CM_FLAG_M2L_SINGLE_TILES, CM_FLAG_SWEEP_SHARED = 1024, 2048

EXPORTS = ["cm_default_opts", "cm_create", "cm_destroy", "cm_num_unknowns", "cm_rwg_table", "cm_apply",
           "cm_apply_noalloc",
           "cm_sai_build", "cm_sai_apply", "cm_vdot", "cm_real_currents", "cm_modal_correlation", "cm_dlambda_dk",
           "cm_gmres", "cm_eigs", "cm_eigs_xinv", "cm_cmp_build", "cm_cmp_apply", "cm_cmp_export", "cm_jd", "cm_export_near", "cm_stats", "cm_set_translation_kernel",
           "cm_stage_timing",
           "cm_stage_times", "cm_last_error"]


class cm_opts(C.Structure):
    _fields_ = [("nlv", C.c_int32), ("d0", C.c_double), ("interp_p", C.c_int32), ("eta", C.c_double),
                ("flags", C.c_uint32), ("max_cols", C.c_int32), ("k_sampling", C.c_double)]


class CmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cmmlfma error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load the library; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1412_1756_amd/build.py "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    L.cm_default_opts.argtypes = [C.POINTER(cm_opts)]
    L.cm_default_opts.restype = None
    L.cm_create.argtypes = [vp, i64, vp, i64, vp, i32, C.POINTER(cm_opts), vp, C.POINTER(vp)]
    L.cm_create.restype = C.c_int
    L.cm_destroy.argtypes = [vp]
    L.cm_destroy.restype = None
    L.cm_num_unknowns.argtypes = [vp, C.POINTER(i64)]
    L.cm_num_unknowns.restype = C.c_int
    L.cm_rwg_table.argtypes = [vp, vp, vp]
    L.cm_rwg_table.restype = C.c_int
    L.cm_apply.argtypes = [vp, C.c_int, vp, vp, i64, i32, vp, C.c_int, vp]
    L.cm_apply.restype = C.c_int
    L.cm_apply_noalloc.argtypes = [vp, C.c_int, vp, vp, i64, i32, C.c_int, vp]
    L.cm_apply_noalloc.restype = C.c_int
    L.cm_sai_build.argtypes = [vp, dbl, dbl, dbl, i32, dbl]
    L.cm_sai_build.restype = C.c_int
    L.cm_sai_apply.argtypes = [vp, vp, vp, i64, i32, vp, dbl, C.c_int, vp]
    L.cm_sai_apply.restype = C.c_int
    L.cm_vdot.argtypes = [vp, vp, vp, i64, i32, C.c_int, vp, vp]
    L.cm_vdot.restype = C.c_int
    L.cm_real_currents.argtypes = [vp, vp, i64, i32, vp, vp, i64, vp]
    L.cm_real_currents.restype = C.c_int
    L.cm_modal_correlation.argtypes = [vp, vp, i64, i32, vp, i64, i32, vp, vp]
    L.cm_modal_correlation.restype = C.c_int
    L.cm_dlambda_dk.argtypes = [vp, dbl, vp, i64, i32, vp, vp]
    L.cm_dlambda_dk.restype = C.c_int
    L.cm_export_near.argtypes = [vp, i32, C.POINTER(i64), vp, vp, vp]
    L.cm_export_near.restype = C.c_int
    L.cm_stats.argtypes = [vp, C.c_char_p, i64, C.POINTER(i64)]
    L.cm_stats.restype = C.c_int
    L.cm_gmres.argtypes = [vp, vp, vp, i32, i32, dbl, i32, C.c_int, C.POINTER(i32), C.POINTER(dbl), vp]
    L.cm_gmres.restype = C.c_int
    L.cm_eigs.argtypes = [vp, i32, i32, i32, dbl, vp, i32, i32, dbl, i32, dbl, C.c_int, vp, vp, vp, C.POINTER(i32), vp,
                          vp]
    L.cm_eigs.restype = C.c_int
    L.cm_eigs_xinv.argtypes = [vp, i32, i32, i32, dbl, vp, i32, i32, dbl, i32, C.c_int, vp, vp, vp, C.POINTER(i32), vp,
                               vp]
    L.cm_eigs_xinv.restype = C.c_int
    L.cm_jd.argtypes = [vp, i32, dbl, i32, i32, i32, dbl, i32, i32, i32, vp, C.c_int, vp, vp, vp, C.POINTER(i32), vp,
                        vp]
    L.cm_jd.restype = C.c_int
    L.cm_cmp_build.argtypes = [vp, i32, i32, dbl, vp, vp]
    L.cm_cmp_build.restype = C.c_int
    L.cm_cmp_apply.argtypes = [vp, i32, vp, vp, C.c_int, vp]
    L.cm_cmp_apply.restype = C.c_int
    L.cm_cmp_export.argtypes = [vp, i32, C.POINTER(i64), C.POINTER(i64), vp, vp, vp]
    L.cm_cmp_export.restype = C.c_int
    L.cm_set_translation_kernel.argtypes = [vp, i32]
    L.cm_set_translation_kernel.restype = C.c_int
    L.cm_stage_timing.argtypes = [vp, i32]
    L.cm_stage_timing.restype = C.c_int
    L.cm_stage_times.argtypes = [vp, C.c_char_p, i64, C.POINTER(i64)]
    L.cm_stage_times.restype = C.c_int
    L.cm_last_error.argtypes = []
    L.cm_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(status):
    if status != CM_OK:
        msg = lib().cm_last_error().decode(errors="replace")
        raise CmError(status, msg)
