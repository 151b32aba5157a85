"""ctypes binding of libabacus_nf.so (the C ABI declared in include/abacus_nf.h).

Argument marshalling only: every step of the near-field path runs in the HIP
kernels of the library.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libabacus_nf.so")

OK = 0
EINVAL = -1
ERANGE = -2
EWORKSPACE = -3
EHIP = -4
ESCRATCH = -5

STATUS_BADPOS = 0x1
STATUS_CELLFULL = 0x2

SINGLE_ACC = 0x1
CHUNKED = 0x2
COMPENSATED = 0x4
COUNT_PAIRS = 0x10
PLUMMER = 0x20
REDUCED = 0x40

TIMER_FORWARD = 0
TIMER_ADJOINT = 1
TIMER_BIN = 2
TIMER_PLAN = 3
TIMER_MULTIPOLES = 4
TIMER_KICK_DRIFT = 5


class Box(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("box", ctypes.c_double), ("cpd", ctypes.c_int32),
                ("radius", ctypes.c_int32), ("eps_plummer", ctypes.c_double),
                ("density_radius", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("unroll", ctypes.c_int32), ("pipeline", ctypes.c_int32),
                ("span", ctypes.c_int32), ("grid_mult", ctypes.c_int32),
                ("split", ctypes.c_int32)]

    def asdict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


KERNEL_FORWARD = 0
KERNEL_ADJOINT = 1


class Binned(ctypes.Structure):
    _fields_ = [("cell_offsets", ctypes.c_void_p), ("perm", ctypes.c_void_p),
                ("rel", ctypes.c_void_p), ("status", ctypes.c_void_p)]


EXPORTS = ("abacus_nf_layout", "abacus_nf_workspace_bytes", "abacus_nf_bin", "abacus_nf_forces",
           "abacus_nf_forces_vjp", "abacus_nf_strerror", "abacus_nf_autotune",
           "abacus_nf_get_tuning", "abacus_nf_set_tuning", "abacus_nf_timing_enable",
           "abacus_nf_timing_read", "abacus_nf_timing_reset", "abacus_nf_multipole_terms",
           "abacus_nf_multipoles_workspace_bytes", "abacus_nf_multipoles",
           "abacus_nf_kick_drift_workspace_bytes", "abacus_nf_kick_drift", "abacus_nf_timestep",
           "abacus_nf_forces_f64", "abacus_nf_forces_vjp_f64", "abacus_nf_forces_noalloc",
           "abacus_nf_forces_slab", "abacus_nf_forces_vjp_slab")

_lib = None


class NearFieldError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} (code {code})")


def load() -> ctypes.CDLL:
    """Load the HIP library; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2110_11392_amd.build.build() "
                          "(there is no CPU fallback for the near-field path)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                             ctypes.c_size_t)
    BoxP = ctypes.POINTER(Box)
    BinnedP = ctypes.POINTER(Binned)
    lib.abacus_nf_layout.argtypes = [BoxP, ctypes.c_int, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.abacus_nf_workspace_bytes.argtypes = [BoxP, ctypes.c_int, ctypes.POINTER(sz)]
    lib.abacus_nf_bin.argtypes = [BoxP, ctypes.c_int, vp, BinnedP, vp, sz, vp]
    lib.abacus_nf_forces.argtypes = [BoxP, ctypes.c_int, BinnedP, vp, vp, vp, vp, u32, vp, sz, vp]
    lib.abacus_nf_forces_vjp.argtypes = [BoxP, ctypes.c_int, BinnedP, vp, vp, u32, vp, sz, vp]
    lib.abacus_nf_forces_f64.argtypes = [BoxP, ctypes.c_int, BinnedP, vp, u32, vp, sz, vp]
    lib.abacus_nf_forces_vjp_f64.argtypes = [BoxP, ctypes.c_int, BinnedP, vp, vp, u32, vp, sz,
                                             vp]
    lib.abacus_nf_forces_noalloc.argtypes = [BoxP, ctypes.c_int, BinnedP, vp, vp, vp, vp, u32, vp]
    lib.abacus_nf_forces_slab.argtypes = [BoxP, ctypes.c_int, BinnedP, i32, i32, vp, u32, vp, sz,
                                          vp]
    lib.abacus_nf_forces_vjp_slab.argtypes = [BoxP, ctypes.c_int, BinnedP, i32, i32, vp, vp, u32,
                                              vp, sz, vp]
    TuneP = ctypes.POINTER(Tuning)
    lib.abacus_nf_autotune.argtypes = [BoxP, ctypes.c_int, BinnedP, vp, u32, vp, sz, vp, TuneP,
                                       TuneP]
    lib.abacus_nf_get_tuning.argtypes = [BoxP, ctypes.c_int, u32, ctypes.c_int, TuneP]
    lib.abacus_nf_set_tuning.argtypes = [BoxP, ctypes.c_int, u32, ctypes.c_int, TuneP]
    lib.abacus_nf_strerror.argtypes = [ctypes.c_int]
    lib.abacus_nf_strerror.restype = ctypes.c_char_p
    lib.abacus_nf_timing_enable.argtypes = [ctypes.c_int]
    lib.abacus_nf_timing_read.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(i64)]
    lib.abacus_nf_timing_reset.argtypes = []
    lib.abacus_nf_multipole_terms.argtypes = [ctypes.c_int, u32, ctypes.POINTER(i64)]
    lib.abacus_nf_multipoles_workspace_bytes.argtypes = [BoxP, ctypes.c_int, ctypes.c_int, u32,
                                                         ctypes.POINTER(sz)]
    lib.abacus_nf_multipoles.argtypes = [BoxP, ctypes.c_int, BinnedP, ctypes.c_int, u32, vp, vp,
                                         sz, vp]
    lib.abacus_nf_kick_drift_workspace_bytes.argtypes = [BoxP, ctypes.c_int, ctypes.POINTER(sz)]
    lib.abacus_nf_kick_drift.argtypes = [BoxP, ctypes.c_int, BinnedP, vp, vp, vp, vp, vp, vp, vp,
                                         vp, sz, vp]
    lib.abacus_nf_timestep.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double]
    for name in EXPORTS:
        if name not in ("abacus_nf_strerror", "abacus_nf_timestep"):
            getattr(lib, name).restype = ctypes.c_int
    lib.abacus_nf_timestep.restype = ctypes.c_double
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().abacus_nf_strerror(int(code)).decode()


def check(code: int, what: str) -> None:
    if code != OK:
        raise NearFieldError(code, what)


def box_array(boxes):
    """ctypes array of Box from a sequence of (n, box, cpd, radius, eps_plummer[,
    density_radius])."""
    arr = (Box * len(boxes))()
    for k, b in enumerate(boxes):
        dens = float(b[5]) if len(b) > 5 else 0.0
        arr[k] = Box(int(b[0]), float(b[1]), int(b[2]), int(b[3]), float(b[4]), dens)
    return arr
