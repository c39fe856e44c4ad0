"""ctypes declarations mirroring include/apr.h, and the library loader."""
import ctypes as C
import os

APR_ERR_RANGE = 6
APR_OK, APR_ERR_INVALID, APR_ERR_CAPACITY, APR_ERR_NOCONVERGE, APR_ERR_HIP, APR_ERR_OVERFLOW = (
    0, 1, 2, 3, 4, 5)
APR_FP64, APR_FP32 = 0, 1
APR_EOS_ISOTHERMAL, APR_EOS_LOCALLY_ISOTHERMAL, APR_EOS_ADIABATIC = 0, 1, 2
APR_SPLIT_TANGENTIAL, APR_SPLIT_RANDOM = 0, 1
APR_KERNEL_M4, APR_KERNEL_WC2 = 0, 1
APR_ZONE_SPHERE, APR_ZONE_CYLINDER = 0, 1
(APR_PROF_DENSITY, APR_PROF_FORCES, APR_PROF_CELLS, APR_PROF_SPLITMERGE, APR_PROF_VJP,
 APR_PROF_CAND, APR_PROF_N) = (0, 1, 2, 3, 4, 5, 6)

_HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path():
    return os.path.join(_HERE, "libapr.so")


class AprError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("apr error %d: %s" % (code, msg))
        self.code = code


class Params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("eos", C.c_int32), ("hfact", C.c_double),
                ("tol_h", C.c_double), ("max_iter", C.c_int32), ("kernel", C.c_int32),
                ("cs0", C.c_double),
                ("q_cs", C.c_double), ("r_ref", C.c_double), ("gamma", C.c_double),
                ("av_alpha", C.c_double), ("av_beta", C.c_double), ("periodic", C.c_int32),
                ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3), ("m0", C.c_double),
                ("r_sep_factor", C.c_double), ("nn_cap", C.c_double), ("split_mode", C.c_int32),
                ("ell_background", C.c_int32), ("derefine", C.c_int32), ("seed", C.c_uint64),
                ("G", C.c_double)]


class CState(C.Structure):
    _fields_ = [("n", C.c_int64), ("capacity", C.c_int64), ("next_id", C.c_int64)] + [
        (k, C.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "ax", "ay", "az",
                                  "dudt", "level", "id")]


class Zone(C.Structure):
    _fields_ = [("c", C.c_double * 3), ("n", C.c_int32), ("ell", C.c_int32 * 8),
                ("shape", C.c_int32), ("r", C.c_double * 8)]


class Sink(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("m", C.c_double), ("eps", C.c_double)]


_LIB = None
_vp = C.c_void_p
_i64p = C.POINTER(C.c_int64)


def lib():
    """Load libapr.so (after torch, whose HIP runtime it shares).  Fails loudly
    if the library has not been built: there is no fallback path."""
    global _LIB
    if _LIB is not None:
        return _LIB
    import torch  # noqa: F401  (loads the HIP runtime libapr.so links against)
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError("libapr.so not built: run __graft_entry__.build() "
                          "(or python paper_2409_11470_amd/build.py)")
    L = C.CDLL(path)
    L.apr_default_params.restype = None
    L.apr_default_params.argtypes = [C.POINTER(Params)]
    L.apr_ctx_create.argtypes = [C.POINTER(_vp), C.POINTER(Params), _vp]
    L.apr_ctx_destroy.argtypes = [_vp]
    L.apr_ctx_set_stream.argtypes = [_vp, _vp]
    L.apr_set_cell_grid.argtypes = [_vp, C.c_int64]
    L.apr_last_error.restype = C.c_char_p
    L.apr_last_error.argtypes = [_vp]
    L.apr_build_cells.argtypes = [_vp, C.POINTER(CState), _vp]
    L.apr_density.argtypes = [_vp, C.POINTER(CState), _vp, _vp, _vp, _vp]
    L.apr_forces.argtypes = [_vp, C.POINTER(CState), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.apr_timestep_noalloc.argtypes = [_vp, C.POINTER(CState), C.c_double, _vp]
    L.apr_vjp.argtypes = [_vp, C.POINTER(CState)] + [_vp] * 12
    L.apr_bins_init.argtypes = [_vp, C.POINTER(CState), _vp, C.POINTER(Sink), C.c_int32,
                                C.c_double, C.c_double, C.c_int32]
    L.apr_step_bins.argtypes = [_vp, C.POINTER(CState), _vp, C.POINTER(Zone), C.c_int32,
                                C.POINTER(Sink), C.c_int32, C.c_double, C.c_double, C.c_int32,
                                C.c_int64, C.POINTER(C.c_int32)]
    L.apr_relax.argtypes = [_vp, C.POINTER(CState), _vp, C.POINTER(CState), _vp, _vp, _vp, _vp,
                            C.c_int32, C.c_double, C.POINTER(C.c_int32),
                            C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.apr_neighbours.argtypes = [_vp, C.POINTER(CState), _vp, C.c_int32, _vp, _vp, _vp,
                                 C.c_int64, _i64p]
    L.apr_split_merge.argtypes = [_vp, C.POINTER(CState), C.POINTER(Zone), C.c_int32, C.c_int64,
                                  C.c_int32, _i64p, _i64p, _i64p]
    L.apr_step.argtypes = [_vp, C.POINTER(CState), C.POINTER(Zone), C.c_int32,
                           C.POINTER(Sink), C.c_int32, C.c_double, C.c_int64]
    L.apr_accel.argtypes = [_vp, C.POINTER(CState), C.POINTER(Sink), C.c_int32]
    L.apr_timestep.argtypes = [_vp, C.POINTER(CState), C.c_double, C.POINTER(C.c_double)]
    L.apr_sync_status.argtypes = [_vp, _i64p]
    L.apr_profile_enable.argtypes = [_vp, C.c_int]
    L.apr_profile_select.argtypes = [_vp, C.c_uint32]
    L.apr_counters.argtypes = [_vp, _i64p, C.c_int]
    L.apr_profile_read.argtypes = [_vp, C.POINTER(C.c_double), _i64p, C.c_int]
    for f in ("apr_ctx_create", "apr_ctx_destroy", "apr_ctx_set_stream", "apr_set_cell_grid",
              "apr_build_cells",
              "apr_density", "apr_forces", "apr_vjp", "apr_relax", "apr_bins_init",
              "apr_step_bins", "apr_neighbours",
              "apr_split_merge", "apr_step",
              "apr_accel", "apr_timestep", "apr_timestep_noalloc", "apr_sync_status",
              "apr_profile_enable", "apr_profile_select",
              "apr_profile_read", "apr_counters"):
        getattr(L, f).restype = C.c_int
    _LIB = L
    return L


def apr_default_params():
    p = Params()
    lib().apr_default_params(C.byref(p))
    return p
