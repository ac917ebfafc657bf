"""ctypes declarations of libjde's C ABI (include/jde.h).

Loading fails loudly when the library is missing: there is no fallback path.
"""

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libjde.so")

JDE_OK, JDE_EINVAL, JDE_ENOMEM, JDE_EDEVICE, JDE_ECAPACITY, JDE_EUNSUPPORTED, JDE_ESTATE, JDE_EBUDGET = \
    0, -1, -2, -3, -4, -5, -6, -7
JDE_FP32, JDE_BF16, JDE_FP16, JDE_FP8, JDE_FP6, JDE_FP4 = 0, 1, 2, 3, 4, 5

c_float_p = ctypes.POINTER(ctypes.c_float)
c_double_p = ctypes.POINTER(ctypes.c_double)
c_int_p = ctypes.POINTER(ctypes.c_int)
c_size_p = ctypes.POINTER(ctypes.c_size_t)


class JdeConfig(ctypes.Structure):
    _fields_ = [("base_ch", ctypes.c_int), ("blocks", ctypes.c_int * 5), ("emb_dim", ctypes.c_int),
                ("num_anchors", ctypes.c_int), ("anchors", ((ctypes.c_float * 2) * 4) * 3),
                ("precision", ctypes.c_int), ("max_frames", ctypes.c_int), ("max_h", ctypes.c_int),
                ("max_w", ctypes.c_int), ("max_candidates", ctypes.c_int), ("max_pixels", ctypes.c_size_t)]


class JdeFrameDesc(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int), ("w", ctypes.c_int)]


class JdeHeadOut(ctypes.Structure):
    _fields_ = [("det", ctypes.c_void_p * 3), ("emb", ctypes.c_void_p * 3)]


class JdeDets(ctypes.Structure):
    _fields_ = [("boxes", ctypes.c_void_p), ("scores", ctypes.c_void_p), ("margins", ctypes.c_void_p),
                ("emb", ctypes.c_void_p), ("anchor_idx", ctypes.c_void_p), ("count", ctypes.c_void_p),
                ("n_cand", ctypes.c_void_p), ("overflow", ctypes.c_void_p), ("cap", ctypes.c_int)]


# name -> (restype, argtypes); every symbol include/jde.h declares.
SIGNATURES = {
    "jde_create": (ctypes.c_int, [ctypes.POINTER(JdeConfig), ctypes.POINTER(ctypes.c_void_p)]),
    "jde_destroy": (None, [ctypes.c_void_p]),
    "jde_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "jde_last_error": (ctypes.c_char_p, []),
    "jde_num_layers": (ctypes.c_int, [ctypes.c_void_p]),
    "jde_layer_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, c_int_p, c_int_p, c_int_p, c_int_p]),
    "jde_blob_floats": (ctypes.c_size_t, [ctypes.c_void_p]),
    "jde_weights_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "jde_load_weights": (ctypes.c_int, [ctypes.c_void_p, c_float_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.c_void_p]),
    "jde_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "jde_head_sizes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(JdeFrameDesc), ctypes.c_int, c_size_p,
                                      c_size_p]),
    "jde_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(JdeFrameDesc), ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(JdeHeadOut), ctypes.c_void_p]),
    "jde_decode": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(JdeHeadOut), ctypes.POINTER(JdeFrameDesc),
                                  ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_size_t, ctypes.POINTER(JdeDets), ctypes.c_void_p]),
    "jde_frame_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "jde_ingest": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(JdeFrameDesc), ctypes.c_void_p, ctypes.c_void_p]),
    "jde_admit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(JdeFrameDesc), ctypes.c_int, ctypes.c_size_t,
                                 ctypes.c_size_t, c_int_p]),
    "jde_box_to_z": (None, [ctypes.c_int, c_float_p, c_double_p]),
    "jde_nms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                               ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p]),
    "jde_nms_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "jde_cost_matrix": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "jde_cost_matrix_dets": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.POINTER(JdeDets), ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "jde_cost_matrix_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, c_int_p,
                                             ctypes.POINTER(JdeDets), ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "jde_cost_matrix_batch_fused": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, c_int_p,
                                                   ctypes.POINTER(JdeDets), ctypes.c_int, ctypes.c_int,
                                                   ctypes.c_double, ctypes.c_float, ctypes.c_void_p,
                                                   ctypes.c_void_p]),
    "jde_iou_cost_batch": (ctypes.c_int, [ctypes.c_void_p, c_int_p, ctypes.POINTER(JdeDets), ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "jde_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(JdeFrameDesc), ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(JdeHeadOut), ctypes.c_int,
                                    ctypes.c_void_p]),
    "jde_tiles": (ctypes.c_int, [ctypes.c_void_p, c_int_p, ctypes.c_int, ctypes.c_int]),
    "jde_graph_capture": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(JdeFrameDesc),
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(JdeHeadOut),
                                         ctypes.c_float, ctypes.c_float, ctypes.c_void_p, ctypes.POINTER(JdeDets),
                                         ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, c_int_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "jde_graph_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "jde_graph_capture_any": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                             ctypes.POINTER(JdeHeadOut), ctypes.c_float, ctypes.c_float,
                                             ctypes.c_void_p, ctypes.POINTER(JdeDets), ctypes.c_void_p,
                                             ctypes.POINTER(ctypes.c_void_p)]),
    "jde_graph_launch_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(JdeFrameDesc), ctypes.c_int,
                                              ctypes.c_void_p]),
    "jde_graph_destroy": (None, [ctypes.c_void_p]),
    "jde_calibrate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(JdeFrameDesc), ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(JdeHeadOut), ctypes.c_void_p]),
    "jde_fp8_scales": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int]),
    "jde_fuse_stem": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "jde_fp8_block_scales": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "jde_fuse_blocks": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "jde_window_convs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "jde_fold_det": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "jde_window_down": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "jde_sparse_emb": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "jde_fp8_encode": (None, [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_uint8), ctypes.c_size_t]),
    "jde_mx_encode": (None, [ctypes.c_int, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_uint8),
                             ctypes.c_size_t]),
    "jde_profile_begin": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "jde_profile_collect": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, c_double_p, c_double_p, c_int_p, c_int_p,
                                           c_int_p]),
    "jde_track_emb_update": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                            ctypes.c_void_p]),
    "jde_kf_predict_dev": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "jde_kf_update_dev": (ctypes.c_int, [c_int_p, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(JdeDets),
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "jde_assign_dev": (ctypes.c_int, [ctypes.c_void_p, c_int_p, ctypes.c_int, ctypes.POINTER(JdeDets),
                                      ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "jde_kf_initiate": (None, [c_double_p, c_double_p, c_double_p]),
    "jde_kf_predict": (None, [ctypes.c_int, c_double_p, c_double_p]),
    "jde_kf_initiate_n": (None, [ctypes.c_int, c_double_p, c_double_p, c_double_p]),
    "jde_kf_update": (ctypes.c_int, [c_double_p, c_double_p, c_double_p]),
    "jde_kf_update_n": (ctypes.c_int, [ctypes.c_int, c_int_p, c_int_p, c_double_p, c_double_p, c_double_p]),
    "jde_assign": (ctypes.c_int, [c_float_p, ctypes.c_int, ctypes.c_int, ctypes.c_float, c_int_p, c_int_p,
                                  c_double_p]),
}

_lib = None


def load():
    """The loaded library (raises if libjde.so has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2011_03910_amd.build` "
                           "(the JDE path has no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


_host = None
HOST_CALLS = ("jde_kf_initiate", "jde_kf_initiate_n", "jde_kf_predict", "jde_kf_update", "jde_kf_update_n",
              "jde_assign", "jde_fp8_encode", "jde_mx_encode", "jde_box_to_z")


def load_host():
    """The same library, for its short host-only calls (Kalman filter,
    assignment, FP8 encoding): these keep the interpreter lock for their few
    microseconds instead of releasing and re-acquiring it around each call, which
    under a busy second thread (the serving loop) costs far more than the call."""
    global _host
    if _host is not None:
        return _host
    load()
    lib = ctypes.PyDLL(LIB_PATH)
    for name in HOST_CALLS:
        res, args = SIGNATURES[name]
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _host = lib
    return lib


class JdeError(RuntimeError):
    def __init__(self, status, where):
        lib = load()
        msg = lib.jde_last_error().decode()
        super().__init__(f"{where}: {lib.jde_status_str(status).decode()} ({status}): {msg}")
        self.status = status


def check(status, where):
    if status != JDE_OK:
        raise JdeError(status, where)
    return status
