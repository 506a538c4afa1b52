"""ctypes view of libqtt's C ABI (include/qtt.h).  Argument marshalling only.

The shared library is built in-tree (``python -m paper_2510_23089_amd.build``);
loading fails loudly if it is missing -- there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqtt.so")

QTT_C64, QTT_C128, QTT_F32, QTT_F64 = 1, 2, 3, 4
PREC_FP32, PREC_BF16, PREC_FP64, PREC_BF16X3 = 0, 1, 2, 3
OP_ENCODE, OP_APPLY, OP_TRUNCATE, OP_TO_DENSE, OP_APPLY_BACKWARD = 1, 2, 3, 4, 5
OP_TO_DENSE_BACKWARD, OP_LOSS = 6, 7

STATUS = {
    0: "QTT_OK", -1: "QTT_ERR_ARG", -2: "QTT_ERR_SHAPE", -3: "QTT_ERR_DTYPE",
    -4: "QTT_ERR_WORKSPACE", -5: "QTT_ERR_CAPACITY", -6: "QTT_ERR_HIP",
    -7: "QTT_ERR_NONFINITE", -8: "QTT_ERR_NOCONVERGE",
}

# every symbol include/qtt.h declares
EXPORTS = [
    "tt_workspace_size", "tt_encode", "mpo_apply", "tt_truncate", "tt_to_dense",
    "tt_saved_size", "mpo_apply_backward", "tt_to_dense_backward",
    "tt_check_status", "tt_last_error", "tt_version",
    "tt_cgemm", "tt_heev_workspace_size", "tt_heev", "tt_prof_begin", "tt_prof_end",
    "tt_prof_begin_flops", "tt_prof_times",
    "tt_workspace_size_batched", "tt_encode_batched", "mpo_apply_batched", "tt_to_dense_batched",
    "tt_saved_size_batched", "mpo_apply_backward_batched", "tt_to_dense_backward_batched", "tt_intensity_loss",
    "tt_autotune_record", "tt_autotune_workspace_size", "tt_autotune_run", "tt_autotune_export",
    "tt_autotune_import", "tt_autotune_clear",
    "tt_encode_separable_workspace_size", "tt_encode_separable", "tt_eval_points_workspace_size", "tt_eval_points",
    "tt_encode_low_rank_workspace_size", "tt_encode_low_rank", "tt_sample_workspace_size", "tt_sample",
    "tt_to_dense_block_workspace_size", "tt_to_dense_block", "mpo_apply_noalloc",
    "tt_to_dense_window_workspace_size", "tt_to_dense_window", "tt_hadamard_workspace_size", "tt_hadamard",
]


class QttMps(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("chi_cap", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("cores", ctypes.c_void_p), ("bonds", ctypes.c_void_p), ("norm", ctypes.c_void_p)]


class QttMpo(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("d_cap", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("cores", ctypes.c_void_p), ("d_bonds", ctypes.c_void_p), ("site_kind", ctypes.c_void_p)]


class QttMpsBatch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("n_sites", ctypes.c_int32), ("chi_cap", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("cores", ctypes.c_void_p), ("bonds", ctypes.c_void_p),
                ("norms", ctypes.c_void_p)]


class QttMpoBatch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("n_sites", ctypes.c_int32), ("d_cap", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("cores", ctypes.c_void_p), ("d_bonds", ctypes.c_void_p),
                ("site_kind", ctypes.c_void_p)]


class QttOpts(ctypes.Structure):
    _fields_ = [("chi_max", ctypes.c_int32), ("chi_zip", ctypes.c_int32), ("cutoff", ctypes.c_double),
                ("tau", ctypes.c_double), ("prec", ctypes.c_int32), ("refine", ctypes.c_int32)]


class QttError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__("%s failed with %s (%d): %s" % (where, STATUS.get(code, "?"), code, msg))
        self.code = code


_lib = None


def load(path=LIB_PATH):
    """Load libqtt.so and declare the signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libqtt.so not built at %s; run `python -m paper_2510_23089_amd.build`" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, sz, i32, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    lib.tt_workspace_size.argtypes = [i32, i32, i32, i32, i32]
    lib.tt_workspace_size.restype = sz
    lib.tt_saved_size.argtypes = [i32, i32, i32, i32]
    lib.tt_saved_size.restype = sz
    lib.tt_encode.argtypes = [vp, i32, i32, P(QttOpts), P(QttMps), vp, sz, vp]
    lib.tt_encode.restype = i32
    lib.mpo_apply.argtypes = [P(QttMps), P(QttMpo), P(QttOpts), P(QttMps), vp, sz, vp, sz, vp]
    lib.mpo_apply.restype = i32
    lib.tt_truncate.argtypes = [P(QttMps), P(QttOpts), vp, sz, vp]
    lib.tt_truncate.restype = i32
    lib.tt_to_dense.argtypes = [P(QttMps), vp, i32, vp, sz, vp]
    lib.tt_to_dense.restype = i32
    lib.mpo_apply_backward.argtypes = [P(QttMps), P(QttMpo), P(QttOpts), vp, sz, P(QttMps), P(QttMps),
                                       P(QttMps), vp, sz, vp]
    lib.mpo_apply_backward.restype = i32
    lib.tt_to_dense_backward.argtypes = [P(QttMps), vp, P(QttMps), vp, sz, vp]
    lib.tt_to_dense_backward.restype = i32
    lib.tt_cgemm.argtypes = [i32, i32, i32, vp, i32, i32, vp, i32, i32, vp, i32, i32, vp]
    lib.tt_cgemm.restype = i32
    lib.tt_heev_workspace_size.argtypes = [i32, i32, i32]
    lib.tt_heev_workspace_size.restype = sz
    lib.tt_heev.argtypes = [vp, i32, i32, i32, dbl, dbl, vp, vp, vp, vp, sz, vp]
    lib.tt_heev.restype = i32
    lib.tt_prof_begin.argtypes = [i32, vp, i32, i32]
    lib.tt_prof_begin.restype = i32
    lib.tt_prof_end.argtypes = [P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_double)]
    lib.tt_prof_end.restype = i32
    lib.tt_prof_begin_flops.argtypes = [vp, i32]
    lib.tt_prof_begin_flops.restype = i32
    lib.tt_prof_times.argtypes = [P(ctypes.c_float), i32]
    lib.tt_prof_times.restype = i32
    lib.tt_workspace_size_batched.argtypes = [i32, i32, i32, i32, i32, i32]
    lib.tt_workspace_size_batched.restype = sz
    lib.tt_encode_batched.argtypes = [vp, i32, i32, P(QttOpts), vp, P(QttMpsBatch), vp, sz, vp]
    lib.tt_encode_batched.restype = i32
    lib.mpo_apply_batched.argtypes = [P(QttMpsBatch), P(QttMpoBatch), P(QttOpts), vp, P(QttMpsBatch), vp, sz, vp, sz,
                                      vp]
    lib.mpo_apply_batched.restype = i32
    lib.tt_saved_size_batched.argtypes = [i32, i32, i32, i32, i32]
    lib.tt_saved_size_batched.restype = sz
    lib.mpo_apply_backward_batched.argtypes = [P(QttMpsBatch), P(QttMpoBatch), P(QttOpts), vp, sz, P(QttMpsBatch),
                                               P(QttMpsBatch), P(QttMpsBatch), vp, sz, vp]
    lib.mpo_apply_backward_batched.restype = i32
    lib.tt_to_dense_backward_batched.argtypes = [P(QttMpsBatch), vp, P(QttMpsBatch), vp, sz, vp]
    lib.tt_to_dense_backward_batched.restype = i32
    lib.tt_intensity_loss.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, sz, vp]
    lib.tt_intensity_loss.restype = i32
    lib.tt_to_dense_batched.argtypes = [P(QttMpsBatch), vp, i32, vp, sz, vp]
    lib.tt_to_dense_batched.restype = i32
    lib.tt_autotune_record.argtypes = [i32]
    lib.tt_autotune_record.restype = i32
    lib.tt_autotune_workspace_size.argtypes = []
    lib.tt_autotune_workspace_size.restype = sz
    lib.tt_autotune_run.argtypes = [vp, sz, vp, P(ctypes.c_int)]
    lib.tt_autotune_run.restype = i32
    lib.tt_autotune_export.argtypes = [vp, i32]
    lib.tt_autotune_export.restype = i32
    lib.tt_autotune_import.argtypes = [vp, i32]
    lib.tt_autotune_import.restype = i32
    lib.tt_autotune_clear.argtypes = []
    lib.tt_autotune_clear.restype = i32
    lib.tt_encode_separable_workspace_size.argtypes = [i32, i32, i32]
    lib.tt_encode_separable_workspace_size.restype = sz
    lib.tt_encode_separable.argtypes = [vp, vp, i32, i32, P(QttMps), vp, sz, vp]
    lib.tt_encode_separable.restype = i32
    lib.tt_encode_low_rank_workspace_size.argtypes = [i32, i32, i32, i32, i32]
    lib.tt_encode_low_rank_workspace_size.restype = sz
    lib.tt_encode_low_rank.argtypes = [vp, vp, i32, i32, i32, i32, P(QttMps), P(QttOpts), vp, sz, vp]
    lib.tt_encode_low_rank.restype = i32
    lib.tt_sample_workspace_size.argtypes = [i32, i32, i32, i32]
    lib.tt_sample_workspace_size.restype = sz
    lib.tt_sample.argtypes = [P(QttMps), vp, i32, vp, vp, vp, sz, vp]
    lib.tt_sample.restype = i32
    lib.tt_eval_points_workspace_size.argtypes = [i32, i32, i32, i32]
    lib.tt_eval_points_workspace_size.restype = sz
    lib.tt_eval_points.argtypes = [P(QttMps), vp, vp, i32, vp, vp, sz, vp]
    lib.tt_eval_points.restype = i32
    lib.tt_to_dense_block_workspace_size.argtypes = [i32, i32, i32, i32]
    lib.tt_to_dense_block_workspace_size.restype = sz
    lib.tt_to_dense_block.argtypes = [P(QttMps), i32, i32, i32, vp, i32, vp, sz, vp]
    lib.tt_to_dense_block.restype = i32
    lib.tt_to_dense_window_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32]
    lib.tt_to_dense_window_workspace_size.restype = sz
    lib.tt_to_dense_window.argtypes = [P(QttMps), i32, i32, i32, i32, i32, vp, i32, vp, sz, vp]
    lib.tt_to_dense_window.restype = i32
    lib.tt_hadamard_workspace_size.argtypes = [i32, i32, i32, i32]
    lib.tt_hadamard_workspace_size.restype = sz
    lib.tt_hadamard.argtypes = [P(QttMps), i32, P(QttMps), P(QttOpts), P(QttMps), vp, sz, vp]
    lib.tt_hadamard.restype = i32
    lib.mpo_apply_noalloc.argtypes = [P(QttMps), P(QttMpo), P(QttOpts), P(QttMps), vp, vp]
    lib.mpo_apply_noalloc.restype = i32
    lib.tt_check_status.argtypes = [vp, vp]
    lib.tt_check_status.restype = i32
    lib.tt_last_error.argtypes = []
    lib.tt_last_error.restype = ctypes.c_char_p
    lib.tt_version.argtypes = []
    lib.tt_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(code, where):
    if code != 0:
        msg = _lib.tt_last_error().decode() if _lib is not None else ""
        raise QttError(code, where, msg)
