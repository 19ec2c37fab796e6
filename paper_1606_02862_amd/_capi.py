"""ctypes declarations of the C ABI in include/pic.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_MAX_SPECIES = 4
PIC_MAX_ZSTATES = 8
PIC_LOTZ_SHELLS = 3

STATUS = {0: "PIC_OK", -1: "PIC_ERR_ARG", -2: "PIC_ERR_OOM", -3: "PIC_ERR_HIP", -4: "PIC_ERR_CAPACITY",
          -5: "PIC_ERR_CFL", -6: "PIC_ERR_NONFINITE", -7: "PIC_ERR_STATE"}
PIC_OK, PIC_ERR_ARG, PIC_ERR_OOM, PIC_ERR_HIP, PIC_ERR_CAPACITY, PIC_ERR_CFL, PIC_ERR_NONFINITE, PIC_ERR_STATE = (
    0, -1, -2, -3, -4, -5, -6, -7)


class GridT(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("precision", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("dt", C.c_double),
                ("b0", C.c_double * 3), ("rho_bg", C.c_double), ("seed", C.c_uint64), ("n_ref_cm3", C.c_double),
                ("gather", C.c_int32), ("options", C.c_int32)]


class LotzShellT(C.Structure):
    _fields_ = [("p_ev", C.c_double), ("a", C.c_double), ("b", C.c_double), ("c", C.c_double),
                ("q", C.c_int32), ("reserved", C.c_int32)]


class SpeciesT(C.Structure):
    _fields_ = [("charge", C.c_double), ("mass", C.c_double), ("density", C.c_double), ("u_th", C.c_double),
                ("drift_beta", C.c_double * 3), ("ppc", C.c_int32), ("layout", C.c_int32), ("mobile", C.c_int32),
                ("coincident_with", C.c_int32), ("z_init", C.c_int32), ("z_max", C.c_int32),
                ("cap_ppc", C.c_int32), ("ionize_into", C.c_int32),
                ("ionization_ev", C.c_double * PIC_MAX_ZSTATES),
                ("lotz", (LotzShellT * PIC_LOTZ_SHELLS) * PIC_MAX_ZSTATES),
                ("max_events", C.c_int32), ("energy_loss", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class AllocT(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class MomentsT(C.Structure):
    _fields_ = [("w_e", C.c_double), ("w_b", C.c_double), ("kinetic", C.c_double * PIC_MAX_SPECIES),
                ("kinetic_total", C.c_double), ("charge_total", C.c_double), ("rho_max", C.c_double),
                ("gauss_max", C.c_double), ("divb_max", C.c_double), ("count", C.c_int64 * PIC_MAX_SPECIES),
                ("step", C.c_int64), ("nonfinite", C.c_int32), ("reserved", C.c_int32),
                ("continuity_max", C.c_double), ("j_max", C.c_double)]


class RunStateT(C.Structure):
    _fields_ = [("step", C.c_int64), ("seed", C.c_uint64), ("weight_bound", C.c_double * PIC_MAX_SPECIES)]


class ParticlesView64T(C.Structure):
    _fields_ = [("count", C.c_int64), ("capacity", C.c_int64),
                ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)), ("z", C.POINTER(C.c_double)),
                ("ux", C.POINTER(C.c_double)), ("uy", C.POINTER(C.c_double)), ("uz", C.POINTER(C.c_double)),
                ("w", C.POINTER(C.c_double)), ("id", C.POINTER(C.c_int64)), ("zstate", C.POINTER(C.c_int32))]


class ParticlesViewT(C.Structure):
    _fields_ = [("count", C.c_int64), ("capacity", C.c_int64),
                ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)), ("z", C.POINTER(C.c_double)),
                ("ux", C.POINTER(C.c_float)), ("uy", C.POINTER(C.c_float)), ("uz", C.POINTER(C.c_float)),
                ("w", C.POINTER(C.c_float)), ("id", C.POINTER(C.c_int64)), ("zstate", C.POINTER(C.c_int32))]


class TimingT(C.Structure):
    _fields_ = [("push_ms", C.c_double), ("migrate_ms", C.c_double), ("field_ms", C.c_double),
                ("push_launches", C.c_int64), ("push_particles", C.c_int64)]


class IonizeStatsT(C.Structure):
    _fields_ = [("ions_active", C.c_int64), ("ionized", C.c_int64), ("fallback", C.c_int64),
                ("electrons", C.c_int64), ("rate_ms", C.c_double), ("total_ms", C.c_double)]


class MlpTrainCfgT(C.Structure):
    _fields_ = [("n_train", C.c_int64), ("batch", C.c_int32), ("steps", C.c_int32), ("lr", C.c_double),
                ("lr_final", C.c_double), ("seed", C.c_uint64), ("t_min_ev", C.c_double), ("t_max_ev", C.c_double),
                ("n_min_cm3", C.c_double), ("n_max_cm3", C.c_double), ("activation", C.c_int32),
                ("reserved", C.c_int32)]


class MlpReportT(C.Structure):
    _fields_ = [("loss_first", C.c_double), ("loss_last", C.c_double), ("mu", C.c_double), ("s", C.c_double),
                ("train_ms", C.c_double), ("steps", C.c_int64)]


PIC_MLP_NPARAM = 4801
PIC_MLP_SILU, PIC_MLP_RELU = 0, 1
PIC_RATE_EXACT, PIC_RATE_MLP = 0, 1
PIC_OPT_DETERMINISTIC_J, PIC_OPT_CONTINUITY = 1, 2
PIC_RATE_EVAL_NOALLOC_MAX = 65536

_DP = C.POINTER(C.c_double)
_FP = C.POINTER(C.c_float)
_IP = C.POINTER(C.c_int32)

# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "pic_abi_version": (C.c_int, []),
    "pic_init": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(GridT), C.POINTER(SpeciesT), C.c_int, C.c_int,
                           C.POINTER(AllocT), C.c_void_p]),
    "pic_step": (C.c_int, [C.c_void_p, C.c_int]),
    "pic_moments": (C.c_int, [C.c_void_p, C.POINTER(MomentsT)]),
    "pic_get_run_state": (C.c_int, [C.c_void_p, C.POINTER(RunStateT)]),
    "pic_set_run_state": (C.c_int, [C.c_void_p, C.POINTER(RunStateT)]),
    "pic_particle_count": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int64)]),
    "pic_get_particles": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(ParticlesViewT)]),
    "pic_set_particles": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(ParticlesViewT)]),
    "pic_get_fields": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pic_set_fields": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pic_get_particles64": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(ParticlesView64T)]),
    "pic_set_particles64": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(ParticlesView64T)]),
    "pic_get_fields64": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pic_set_fields64": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pic_mark_reference": (C.c_int, [C.c_void_p]),
    "pic_timing": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(TimingT)]),
    "pic_ionize": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(IonizeStatsT)]),
    "pic_ionize_staged": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(IonizeStatsT)]),
    "pic_cell_moments_device": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    "pic_cell_moments": (C.c_int, [C.c_void_p, C.c_int, _DP, _DP]),
    "pic_rate_eval": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int64, _DP, _DP, _IP, _DP]),
    "pic_rate_eval_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int64, _DP, _DP, _IP, _DP]),
    "pic_gauss_laguerre64": (C.c_int, [_DP, _DP]),
    "pic_mlp_train": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(MlpTrainCfgT), C.POINTER(MlpReportT)]),
    "pic_mlp_get_params": (C.c_int, [C.c_void_p, C.c_int, _FP, _DP, _DP, C.POINTER(C.c_int32)]),
    "pic_mlp_set_params": (C.c_int, [C.c_void_p, C.c_int, _FP, _DP, _DP, C.c_int32]),
    "pic_mlp_loss_grad": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, _FP, _FP, _DP, _FP]),
    "pic_destroy": (C.c_int, [C.c_void_p]),
    "pic_last_error": (C.c_char_p, [C.c_void_p]),
}

_lib = None


class PicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def load() -> C.CDLL:
    """Load the built HIP library; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1606_02862_amd.build.build()")
        # torch ships its own HIP runtime under the same soname as the system
        # one; whichever is loaded first serves the whole process.  Load torch
        # first so the library binds the runtime torch's streams and allocator
        # live in (the other order leaves pinned host allocations failing).
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc: int, ctx=None):
    if rc != PIC_OK:
        msg = load().pic_last_error(ctx)
        raise PicError(rc, msg.decode() if msg else "")
    return rc
