"""ctypes view of the C ABI declared in include/mmstencil.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

from ._build import LIB

MMS_OK, MMS_EINVAL, MMS_EUNSUPPORTED, MMS_EHIP, MMS_ENOMEM, MMS_EUNSTABLE = 0, -1, -2, -3, -4, -5
MMS_REDUCE_WORK = 2048
MMS_STAR, MMS_BOX, MMS_STAR2D, MMS_BOX2D = 0, 1, 2, 3
MMS_FP32, MMS_BF16X3, MMS_FP16X3S, MMS_BF16X1 = 0, 1, 2, 3

EXPORTS = ("mms_stencil_apply", "mms_wave_step", "mms_wave_record", "mms_wave_forward",
           "mms_wave_adjoint_step", "mms_wave_adjoint", "mms_wave_adjoint_mu", "mms_wave_scale_mu",
           "mms_wave_energy", "mms_dot_f64",
           "mms_flat_dot_f64", "mms_flat_misfit_f64", "mms_dense_to_grid", "mms_grid_aligned",
           "mms_strerror", "mms_last_error", "mms_abi_version", "mms_vti_step", "mms_tti_step",
           "mms_wave_energy_work", "mms_flat_scale_f32", "mms_check_reduction",
           "mms_wave_energy_noalloc")


class MmsGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("halo", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("sy", ctypes.c_int64), ("sz", ctypes.c_int64)]


class MmsWave(ctypes.Structure):
    _fields_ = [("g", MmsGrid), ("radius", ctypes.c_int32), ("lap", ctypes.c_float * 5),
                ("c2", ctypes.c_void_p), ("c2_scale", ctypes.c_float),
                ("sponge_width", ctypes.c_int32), ("sponge_alpha", ctypes.c_float),
                ("sponge_faces", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("src_z", ctypes.c_int64), ("src_y", ctypes.c_int64), ("src_x", ctypes.c_int64),
                ("src_dt2f", ctypes.c_void_p), ("traces", ctypes.c_void_p),
                ("image", ctypes.c_void_p), ("acc_part", ctypes.c_void_p),
                ("acc_block", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class MmsTti(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_void_p), ("delta", ctypes.c_void_p), ("theta", ctypes.c_void_p),
                ("phi", ctypes.c_void_p), ("sigma", ctypes.c_float), ("alpha", ctypes.c_float),
                ("d1", ctypes.c_float * 4), ("work", ctypes.c_void_p)]


class MmsError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code}) {detail}".strip())


_lib = None


def lib():
    """Load libmmstencil.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is missing: build it with __graft_entry__.build() "
                              "(the HIP library has no CPU fallback)")
        L = ctypes.CDLL(LIB)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        gp, wp = ctypes.POINTER(MmsGrid), ctypes.POINTER(MmsWave)
        L.mms_stencil_apply.argtypes = [vp, vp, gp, i32, i32, ctypes.POINTER(ctypes.c_float),
                                        i32, i32, vp]
        L.mms_wave_step.argtypes = [wp, i32, vp, vp, vp, vp]
        L.mms_wave_record.argtypes = [wp, i32, vp, vp]
        L.mms_wave_forward.argtypes = [wp, i32, i32, ctypes.POINTER(vp), vp]
        L.mms_wave_adjoint_step.argtypes = [wp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.mms_wave_adjoint.argtypes = [wp, i32, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), vp,
                                       vp, vp]
        L.mms_wave_adjoint_mu.argtypes = [wp, i32, i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                          vp, vp, vp]
        L.mms_wave_scale_mu.argtypes = [wp, vp, vp, i32, vp]
        L.mms_grid_aligned.argtypes = [i64, i64, i64, ctypes.c_int32, gp, ctypes.POINTER(i64)]
        L.mms_wave_energy_work.argtypes = [wp, ctypes.POINTER(i64)]
        L.mms_wave_energy.argtypes = [wp, vp, vp, vp, vp, i64, vp]
        L.mms_wave_energy_noalloc.argtypes = [wp, vp, vp, vp, vp]
        L.mms_vti_step.argtypes = [wp, i32] + [vp] * 8 + [vp]
        L.mms_tti_step.argtypes = [wp, ctypes.POINTER(MmsTti), i32] + [vp] * 6 + [vp]
        L.mms_dot_f64.argtypes = [vp, vp, gp, vp, vp, vp]
        L.mms_flat_dot_f64.argtypes = [vp, vp, i64, vp, vp, vp]
        L.mms_flat_misfit_f64.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.mms_flat_scale_f32.argtypes = [vp, vp, vp, i64, vp]
        L.mms_check_reduction.argtypes = [ctypes.POINTER(ctypes.c_double)]
        L.mms_dense_to_grid.argtypes = [vp, vp, gp, ctypes.c_double, vp]
        L.mms_strerror.argtypes = [i32]
        L.mms_strerror.restype = ctypes.c_char_p
        L.mms_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("mms_strerror", "mms_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().mms_strerror(code).decode()


def check(rc: int, where: str) -> None:
    if rc != MMS_OK:
        detail = lib().mms_last_error().decode() if rc == MMS_EHIP else ""
        raise MmsError(rc, where, detail)
