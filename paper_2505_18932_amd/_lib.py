"""ctypes loader of libggeom.so, the gfx950 geometry-stage library.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/ggeom.h.  There is no fallback:
if the library is missing, loading fails loudly.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libggeom.so")

GG_OK = 0
GG_ERR_INVALID = -1
GG_ERR_WORKSPACE = -2
GG_ERR_HIP = -3
GG_ERR_UNSUPPORTED = -4
GG_MAX_VIEWS = 16

GG_OP_SPLAT = 1
GG_OP_SPLAT_BACKWARD = 2
GG_OP_TSDF_INTEGRATE = 3
GG_OP_TSDF_INTEGRATE_BACKWARD = 4
GG_OP_DIFFERENCE_MASKS = 5
GG_OP_SPLAT_EWA = 6


class GGCamera(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("width", C.c_int32), ("height", C.c_int32)]


class GGSplatParams(C.Structure):
    _fields_ = [("sigma_px", C.c_float), ("band_rel", C.c_float), ("z_min", C.c_float),
                ("r_max_px", C.c_float)]


class GGTsdfParams(C.Structure):
    _fields_ = [("z_near", C.c_float), ("z_far", C.c_float), ("num_bins", C.c_int32),
                ("trunc", C.c_float), ("trunc_in_bins", C.c_int32),
                ("conf_tau", C.c_float), ("conf_scale", C.c_float), ("conf_window", C.c_int32),
                ("decay", C.c_float), ("weight_cap", C.c_float)]


class GGMaskParams(C.Structure):
    _fields_ = [("beta", C.c_float), ("lambda_t", C.c_float), ("factor", C.c_int32)]


class GGVolumeTuning(C.Structure):
    _fields_ = [("pixels_per_block", C.c_int32), ("pixels_per_row", C.c_int32),
                ("bins_per_thread", C.c_int32), ("band_width", C.c_int32)]


class GGBatchItem(C.Structure):
    _fields_ = [("src", C.POINTER(GGCamera)), ("K", C.c_int32), ("depth", C.c_void_p),
                ("rgb", C.c_void_p), ("tgt", GGCamera), ("splat", GGSplatParams),
                ("tsdf", GGTsdfParams), ("temporal_mask", C.c_void_p), ("F_prev", C.c_void_p),
                ("W_prev", C.c_void_p), ("F", C.c_void_p), ("W", C.c_void_p),
                ("out_depth", C.c_void_p), ("out_bin", C.c_void_p), ("win_idx", C.c_void_p),
                ("sp_depth", C.c_void_p), ("sp_rgb", C.c_void_p), ("sp_alpha", C.c_void_p),
                ("sp_tape", C.c_void_p), ("volume", GGVolumeTuning)]


class GGBatchTuning(C.Structure):
    _fields_ = [("pixels_per_block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("bins_per_thread", C.c_int32), ("branches", C.c_int32)]


P = C.c_void_p
CAM = C.POINTER(GGCamera)
SPP = C.POINTER(GGSplatParams)
TSP = C.POINTER(GGTsdfParams)
VTP = C.POINTER(GGVolumeTuning)
I32 = C.c_int32
SZ = C.c_size_t

# name -> (restype, argtypes); every entry point of include/ggeom.h
SIGNATURES = {
    "gg_workspace_size": (SZ, [C.c_int, I32, I32, I32, I32, I32, I32, SPP]),
    "splat_views": (C.c_int, [CAM, I32, P, P, CAM, SPP, P, P, P, P, P, P, SZ, P]),
    "splat_views_masked": (C.c_int, [CAM, I32, P, P, CAM, SPP, P, P, P, P, P, P, P, P, P, SZ,
                                     P]),
    "splat_views_ewa": (C.c_int, [CAM, I32, P, P, CAM, SPP, C.c_float, I32, P, P, P, P, SZ, P]),
    "splat_views_backward": (C.c_int, [CAM, I32, P, P, CAM, SPP, P, P, P, P, P, P, P, P, P, P,
                                       SZ, P]),
    "difference_masks": (C.c_int, [I32, I32, I32, P, P, C.POINTER(GGMaskParams), P, P, P, P, P,
                                   SZ, P]),
    "tsdf_integrate": (C.c_int, [CAM, I32, P, CAM, TSP, P, P, P, P, P, P, P, VTP, P, SZ, P]),
    "tsdf_view_table": (C.c_int, [CAM, I32, P, TSP, P, SZ, P]),
    "tsdf_integrate_noalloc": (C.c_int, [CAM, I32, P, CAM, TSP, P, P, P, P, P, P, P, VTP, P]),
    "tsdf_integrate_tabled": (C.c_int, [CAM, I32, CAM, TSP, P, P, P, P, P, P, P, VTP, P, SZ,
                                        P]),
    "tsdf_raymarch": (C.c_int, [CAM, I32, P, CAM, TSP, P, P, P, P, P, P, P, SZ, P]),
    "network_inputs": (C.c_int, [CAM, I32, CAM, P, P, P, P, P, P]),
    "blend_views": (C.c_int, [I32, I32, I32, P, P, P, P, P, P, P, P, P]),
    "tsdf_extract_depth": (C.c_int, [CAM, TSP, P, P, P, P, VTP, P]),
    "tsdf_extract_depth_backward": (C.c_int, [CAM, TSP, P, P, P, P, P, P]),
    "tsdf_integrate_backward": (C.c_int, [CAM, I32, P, CAM, TSP, P, P, P, P, P, P, SZ, P]),
    "gg_last_error": (C.c_char_p, []),
    "gg_relative_projection": (C.c_int, [CAM, CAM, P, P]),
    "gg_timing_enable": (C.c_int, [C.c_int]),
    "gg_timing_filter": (C.c_int, [C.c_char_p]),
    "gg_timing_reset": (C.c_int, []),
    "gg_timing_read": (C.c_int, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "gg_selftest_reciprocal": (C.c_int, [I32, I32, P, P]),
    "gg_batch_plan": (C.c_int, [C.POINTER(GGBatchItem), I32, C.POINTER(GGBatchTuning),
                                C.POINTER(C.c_void_p)]),
    "gg_batch_launch": (C.c_int, [P, P]),
    "gg_batch_device_bytes": (SZ, [P]),
    "gg_batch_free": (C.c_int, [P]),
    "gg_fast_reciprocal": (C.c_int, [P, P, C.c_int64, P]),
    "gg_fusion_stream_probe": (C.c_int, [CAM, TSP, P, P, P, P, P, P, VTP, P, SZ, P]),
}

_lib = None


class GGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_2505_18932_amd.build` "
                "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != GG_OK:
        raise GGError(rc, lib().gg_last_error().decode())
    return rc
