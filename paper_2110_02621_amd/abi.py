"""ctypes mirror of ``include/sph.h``: structs, constants and prototypes.

Argument marshalling only.  ``load()`` raises if the compiled library is
missing; there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

SPH_OK, SPH_ERR_ARG, SPH_ERR_CONFIG, SPH_ERR_LAUNCH, SPH_ERR_CAPACITY = 0, 1, 2, 3, 4
SPH_F32, SPH_F64 = 0, 1
SPH_CONTINUITY, SPH_MOMENTUM, SPH_NO_KICK = 1, 2, 4
SPH_STATUS_OUT_OF_GRID, SPH_STATUS_FAST, SPH_STATUS_NONFINITE, SPH_STATUS_LIST_OVERFLOW = 0, 1, 2, 3
SPH_STATUS_LEN = 4
SPH_DIAG_MASS, SPH_DIAG_MOM, SPH_DIAG_EKIN, SPH_DIAG_EPOT = 0, 1, 4, 5
SPH_DIAG_VMAX, SPH_DIAG_PROBE, SPH_DIAG_STEPS, SPH_DIAG_LEN = 6, 7, 8, 16
SPH_DIAG_NOALLOC_BYTES, SPH_DIAG_NOALLOC_MAX_FLUID = 4 << 20, 1 << 24

EXPORTED = ["sph_configure", "sph_scratch_bytes", "sph_init", "sph_build_cells", "sph_density",
            "sph_wall_bc", "sph_forces", "sph_step", "sph_diag", "sph_diag_noalloc", "sph_export",
            "sph_export_walls",
            "sph_neighbours", "sph_strerror",
            "sph_adjoint_work_bytes", "sph_adjoint_zero", "sph_forces_bwd", "sph_wall_bc_bwd",
            "sph_density_bwd", "sph_step_bwd", "sph_init_bwd", "sph_step_frame"]


class Desc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("precision", C.c_int32), ("penalty_all", C.c_int32),
        ("two_phase", C.c_int32),
        ("dx", C.c_double), ("h", C.c_double), ("rho0", C.c_double), ("c0", C.c_double),
        ("mu", C.c_double), ("gamma_p", C.c_double), ("dt", C.c_double),
        ("g", C.c_double * 3), ("a_wall", C.c_double * 3), ("lo", C.c_double * 3),
        ("hi", C.c_double * 3), ("n_heavy", C.c_int64), ("rho0_light", C.c_double),
        ("motion_amp", C.c_double * 3), ("motion_freq", C.c_double),
        ("cross_phase", C.c_int32), ("reserved1", C.c_int32),
        ("cell", C.c_double), ("sigma0", C.c_double), ("grid", C.c_int32 * 3),
        ("reserved2", C.c_int32), ("n_cells", C.c_int64),
    ]


class Buffers(C.Structure):
    _fields_ = [
        ("n_fluid", C.c_int64), ("n_wall", C.c_int64),
        ("key", C.c_void_p * 2), ("pid", C.c_void_p * 2), ("off", C.c_void_p * 2),
        ("vel", C.c_void_p * 2), ("rho", C.c_void_p * 2), ("acc", C.c_void_p),
        ("sel_vel", C.c_int32), ("sel_rho", C.c_int32),
        ("wkey", C.c_void_p), ("wpid", C.c_void_p), ("woff", C.c_void_p), ("pw", C.c_void_p),
        ("nrm", C.c_void_p), ("fstart", C.c_void_p), ("wstart", C.c_void_p),
        ("scratch", C.c_void_p), ("scratch_bytes", C.c_size_t),
        ("status", C.c_void_p), ("diag", C.c_void_p), ("sigma_out", C.c_void_p),
        ("probe", C.c_void_p), ("n_probe", C.c_int32), ("sigma_ready", C.c_int32),
        ("nbr_ff", C.c_void_p), ("nbr_fw", C.c_void_p), ("nbr_wf", C.c_void_p),
        ("cnt_ff", C.c_void_p), ("cnt_fw", C.c_void_p), ("cnt_wf", C.c_void_p),
        ("nstep", C.c_int64),
    ]


_lib = None


def load():
    """Load libsph.so and declare its prototypes.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2110_02621_amd.build` "
                           "(hipcc, gfx950); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.POINTER(Desc)
    bp = C.POINTER(Buffers)
    L.sph_configure.argtypes = [dp]
    L.sph_scratch_bytes.argtypes = [dp, C.c_int64, C.c_int64]
    L.sph_scratch_bytes.restype = C.c_size_t
    L.sph_init.argtypes = [dp, bp, vp, vp, vp, vp, vp]
    for name in ("sph_build_cells", "sph_density", "sph_wall_bc", "sph_diag", "sph_diag_noalloc"):
        getattr(L, name).argtypes = [dp, bp, vp]
    L.sph_forces.argtypes = [dp, bp, C.c_uint, vp]
    L.sph_step.argtypes = [dp, bp, C.c_int, vp]
    L.sph_export.argtypes = [dp, bp, vp, vp, vp, vp, vp]
    L.sph_export_walls.argtypes = [dp, bp, vp, vp, vp]
    L.sph_neighbours.argtypes = [dp, bp, C.c_int, vp, vp, vp, C.c_int64, vp]
    L.sph_strerror.argtypes = [C.c_int]
    L.sph_strerror.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("sph_scratch_bytes", "sph_strerror"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class SPHError(RuntimeError):
    pass


def check(rc: int, what: str):
    if rc != SPH_OK:
        msg = load().sph_strerror(rc).decode()
        raise SPHError(f"{what}: {msg} (code {rc})")
