"""ctypes view of the C ABI in include/krylov_phi.h (argument marshalling only).

The shared library is built in-tree (paper_2410_14917_amd/libkrylov_phi.so) by
paper_2410_14917_amd.build.build().  Loading fails loudly if it is absent:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkrylov_phi.so")
TIMELINE_LIB_PATH = os.path.join(HERE, "libkrylov_phi_timeline.so")   # profiling build

# ---- constants (mirror include/krylov_phi.h) --------------------------------
KP_OK, KP_EINVAL, KP_ENOMEM, KP_EHIP, KP_EUNSUPPORTED, KP_ESTATE, KP_ETOOLARGE = \
    0, -1, -2, -3, -4, -5, -6
KP_NOALLOC_BYTES = 64 << 20
KP_STATUS_OK, KP_STATUS_NOT_CONVERGED, KP_STATUS_NONFINITE, KP_STATUS_ABORTED = 0, 1, 2, 3
KP_ORTH_H_GSMGS, KP_ORTH_H_CWY, KP_ORTH_H_NCWY, KP_ORTH_MGS, KP_ORTH_IOCGS = 0, 1, 2, 3, 4
KP_CTRL_POWER, KP_CTRL_PI = 0, 1
KP_OP_ADR, KP_OP_ALLEN_CAHN, KP_OP_BRUSSELATOR = 0, 1, 2
KP_BASIS_F64, KP_BASIS_F32 = 0, 1
KP_RHS_ALLEN_CAHN, KP_RHS_ADR = 0, 1
KP_EPI4, KP_EPI5, KP_SRERK3 = 0, 1, 2
METHODS = {"epi4": KP_EPI4, "epi5": KP_EPI5, "srerk3": KP_SRERK3}
KP_MMAX, KP_PMAX = 64, 8

ORTH = {"h-gsmgs": KP_ORTH_H_GSMGS, "h-cwy": KP_ORTH_H_CWY, "h-ncwy": KP_ORTH_H_NCWY,
        "mgs": KP_ORTH_MGS, "iocgs": KP_ORTH_IOCGS}
CTRL = {"power": KP_CTRL_POWER, "pi": KP_CTRL_PI}
BASIS = {"f64": KP_BASIS_F64, "f32": KP_BASIS_F32}

# Exported symbols (every function declared in the header).
SYMBOLS = ("kp_create", "kp_destroy", "kp_set_config", "kp_phi_combo", "kp_phi_combo_noalloc",
           "kp_phi_combo_tangent",
           "kp_phi_combo_backward", "kp_phi_combo_batched", "kp_get_batch_schedule", "kp_batch_plan", "kp_get_schedule",
           "kp_arnoldi_begin", "kp_arnoldi_step", "kp_arnoldi_read", "kp_expm_hbar",
           "kp_integrate", "kp_calibrate",
           "kp_strerror", "kp_last_error", "kp_version", "kp_runtime_version",
           "kp_set_timeline", "kp_timeline_layout", "kp_read_bandwidth")


class KpOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("transpose", ctypes.c_int32), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("nu", ctypes.c_double), ("nu2", ctypes.c_double), ("ax", ctypes.c_double),
                ("ay", ctypes.c_double), ("react", ctypes.c_double),
                ("brus_a", ctypes.c_double), ("brus_b", ctypes.c_double),
                ("field0", ctypes.c_void_p), ("field1", ctypes.c_void_p)]


class KpConfig(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("orth", ctypes.c_int32),
                ("basis_dtype", ctypes.c_int32), ("m_init", ctypes.c_int32),
                ("max_substeps", ctypes.c_int32), ("fixed_m", ctypes.c_int32),
                ("fixed_substeps", ctypes.c_int32), ("fallback_delta", ctypes.c_double),
                ("breakdown_eps", ctypes.c_double), ("tau_init", ctypes.c_double),
                ("controller", ctypes.c_int32), ("rows_per_wg", ctypes.c_int32)]


class KpRhs(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("nu", ctypes.c_double), ("ax", ctypes.c_double), ("ay", ctypes.c_double),
                ("gamma", ctypes.c_double)]


class KpInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("substeps", ctypes.c_int32),
                ("rejected", ctypes.c_int32), ("arnoldi_steps", ctypes.c_int32),
                ("expm_evals", ctypes.c_int32), ("m_last", ctypes.c_int32),
                ("n_fallback", ctypes.c_int32), ("breakdowns", ctypes.c_int32),
                ("schedule_len", ctypes.c_int32), ("onchip_passes", ctypes.c_int32),
                ("err_max", ctypes.c_double), ("mu", ctypes.c_double),
                ("t_end", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libkrylov_phi.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with paper_2410_14917_amd.build.build() "
            "(there is no CPU fallback)")
    # The library links the system HIP runtime; PyTorch carries its own copy.
    # With both in one process, torch's has to be loaded first: loaded the
    # other way round, the library's first device query reports no device
    # once torch has initialised its runtime (measured on MI355X, ROCm 7.2).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.kp_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(KpConfig)]
    lib.kp_destroy.argtypes = [P]
    lib.kp_set_config.argtypes = [P, ctypes.POINTER(KpConfig)]
    lib.kp_phi_combo.argtypes = [P, ctypes.POINTER(KpOp), P, I32, I64, D, D, I32, P,
                                 ctypes.POINTER(KpInfo)]
    lib.kp_phi_combo_noalloc.argtypes = [P, ctypes.POINTER(KpOp), P, I32, I64, D, D, I32, P,
                                         ctypes.POINTER(KpInfo)]
    lib.kp_phi_combo_tangent.argtypes = [P, ctypes.POINTER(KpOp), ctypes.POINTER(KpOp), P, I32,
                                         I64, D, D, I32, P, P, ctypes.POINTER(KpInfo)]
    PI32, PD = ctypes.POINTER(I32), ctypes.POINTER(D)
    lib.kp_phi_combo_backward.argtypes = [P, ctypes.POINTER(KpOp), P, I32, I64, D, D, I32, P, P, I64,
                                          I32, P, ctypes.POINTER(KpInfo)]
    lib.kp_phi_combo_batched.argtypes = [P, I32, ctypes.POINTER(KpOp), ctypes.POINTER(P), PI32,
                                         ctypes.POINTER(I64), PD, D, I32, ctypes.POINTER(P),
                                         ctypes.POINTER(KpInfo)]
    lib.kp_batch_plan.argtypes = [I32, ctypes.POINTER(KpOp), PI32, PD, I32, I32, PI32, PI32, PI32,
                                  PI32, PD, PD]
    lib.kp_get_batch_schedule.argtypes = [P, I32, P, P, I32]
    lib.kp_get_schedule.argtypes = [P, P, P, I32]
    lib.kp_arnoldi_begin.argtypes = [P, ctypes.POINTER(KpOp), P, I32, I64, I32]
    lib.kp_arnoldi_step.argtypes = [P, I32]
    lib.kp_arnoldi_read.argtypes = [P, P, P, P, P, P]
    lib.kp_expm_hbar.argtypes = [P, P, I32, I32, D, P]
    lib.kp_calibrate.argtypes = [P, I32, P]
    lib.kp_integrate.argtypes = [P, ctypes.POINTER(KpRhs), I32, D, I32, I32, P, D, I32,
                                 ctypes.POINTER(KpInfo)]
    lib.kp_strerror.argtypes = [ctypes.c_int]
    lib.kp_strerror.restype = ctypes.c_char_p
    lib.kp_last_error.argtypes = [P]
    lib.kp_last_error.restype = ctypes.c_char_p
    lib.kp_version.argtypes = []
    lib.kp_runtime_version.argtypes = [P, P]
    lib.kp_set_timeline.argtypes = [P, P, I32]
    lib.kp_timeline_layout.argtypes = [P, P]
    lib.kp_read_bandwidth.argtypes = [P, I64, I32, P]
    for name in SYMBOLS:
        fn = getattr(lib, name)
        if fn.restype is None and name not in ("kp_strerror", "kp_last_error"):
            fn.restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc: int, ctx=None) -> int:
    if rc < 0:
        lib = load()
        msg = lib.kp_strerror(rc).decode()
        if ctx is not None:
            extra = lib.kp_last_error(ctx).decode()
            if extra:
                msg += f" ({extra})"
        raise RuntimeError(f"libkrylov_phi: {msg} [{rc}]")
    return rc
