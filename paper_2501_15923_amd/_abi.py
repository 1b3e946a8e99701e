"""ctypes declarations of the C-ABI in include/icarus_hip.h (argument
marshalling only).  Loading fails loudly if libicarus_hip.so is missing."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libicarus_hip.so")

ICR_OK, ICR_ERR_ARG, ICR_ERR_STATE, ICR_ERR_NONPHYSICAL, ICR_ERR_HIP, ICR_ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5
FLUX_TVDLF, FLUX_HLL, FLUX_HLLD = 0, 1, 2
LIM_MINMOD, LIM_MC, LIM_WENO5 = 0, 1, 2
PREC_F64, PREC_F32 = 64, 32
BCT_MAP, BCT_ASYMM = 0, 1
STATE_PRIM_SI, STATE_CONS_CODE = 0, 1


class IcrGrid(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int), ("n_theta", ctypes.c_int), ("n_phi", ctypes.c_int),
                ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
                ("th_min", ctypes.c_double), ("th_max", ctypes.c_double),
                ("max_maps", ctypes.c_int), ("max_cmes", ctypes.c_int),
                ("max_probes", ctypes.c_int), ("max_traj_pts", ctypes.c_int),
                ("probe_log_rows", ctypes.c_int)]


class IcrPhys(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("omega", ctypes.c_double), ("cfl", ctypes.c_double),
                ("flux", ctypes.c_int), ("limiter", ctypes.c_int), ("precision", ctypes.c_int),
                ("gravity", ctypes.c_int), ("corotation", ctypes.c_int), ("tracer", ctypes.c_int),
                ("bc_transverse", ctypes.c_int)]


class IcrAmrParams(ctypes.Structure):
    _fields_ = [("block_r", ctypes.c_int), ("block_theta", ctypes.c_int),
                ("block_phi", ctypes.c_int), ("max_level", ctypes.c_int),
                ("criterion", ctypes.c_int), ("tau_threshold", ctypes.c_double),
                ("shock_threshold", ctypes.c_double), ("regrid_every", ctypes.c_int),
                ("max_blocks", ctypes.c_int)]


class IcrClock(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("step", ctypes.c_longlong),
                ("last_dt", ctypes.c_double), ("next_dt", ctypes.c_double),
                ("residual", ctypes.c_double), ("t_code", ctypes.c_double)]


class IcrStepInfo(ctypes.Structure):
    _fields_ = [("steps_taken", ctypes.c_int), ("status", ctypes.c_int),
                ("bad_cell", ctypes.c_longlong), ("t", ctypes.c_double),
                ("last_dt", ctypes.c_double), ("residual", ctypes.c_double)]


class NnShape(ctypes.Structure):
    _fields_ = [("n_theta", ctypes.c_int), ("n_phi", ctypes.c_int), ("n_r", ctypes.c_int),
                ("c1", ctypes.c_int), ("c2", ctypes.c_int), ("hidden", ctypes.c_int),
                ("batch_max", ctypes.c_int), ("phi_lo", ctypes.c_int), ("phi_hi", ctypes.c_int),
                ("coord", ctypes.c_int)]


class IcarusError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"icarus error {code}: {msg}")
        self.code = code


_lib = None

P = ctypes.c_void_p
D = ctypes.POINTER(ctypes.c_double)
I = ctypes.c_int

SIGNATURES = {
    "icr_last_error": (ctypes.c_char_p, []),
    "icr_units": (I, [D]),
    "icr_workspace_bytes": (I, [ctypes.POINTER(IcrGrid), ctypes.POINTER(IcrPhys),
                                ctypes.POINTER(ctypes.c_size_t)]),
    "icr_create": (I, [ctypes.POINTER(IcrGrid), ctypes.POINTER(IcrPhys), P, ctypes.c_size_t, P,
                       ctypes.POINTER(P)]),
    "icr_destroy": (None, [P]),
    "icr_grid_edges": (I, [P, D, D, D]),
    "icr_set_boundary_maps": (I, [P, I, D, D, I]),
    "icr_set_cmes": (I, [P, I, D]),
    "icr_init_radial": (I, [P]),
    "icr_set_state": (I, [P, D, I, I]),
    "icr_get_state": (I, [P, D, I, I]),
    "icr_get_clock": (I, [P, ctypes.POINTER(IcrClock)]),
    "icr_set_clock": (I, [P, ctypes.c_double, ctypes.c_longlong]),
    "icr_set_clock_code": (I, [P, ctypes.c_double, ctypes.c_longlong]),
    "icr_step": (I, [P, I, ctypes.c_double, ctypes.POINTER(IcrStepInfo)]),
    "icr_step_noalloc": (I, [P, I, ctypes.c_double, ctypes.POINTER(IcrStepInfo)]),
    "icr_set_probes": (I, [P, I, I, D, ctypes.c_double]),
    "icr_sample_probes": (I, [P, D]),
    "icr_read_probe_log": (I, [P, D, I, ctypes.POINTER(ctypes.c_int)]),
    "icr_boundary_at": (I, [P, ctypes.c_double, D]),
    "icr_set_launch": (I, [P, I, I, I, I]),
    "icr_profile_steps": (I, [P, I, D]),
    "icr_fast_math": (I, [D, ctypes.c_longlong, D, D, P]),
    "icr_ens_workspace_bytes": (I, [I, ctypes.POINTER(IcrGrid), ctypes.POINTER(IcrPhys),
                                    ctypes.POINTER(ctypes.c_size_t)]),
    "icr_ens_create": (I, [I, ctypes.POINTER(IcrGrid), ctypes.POINTER(IcrPhys), P,
                           ctypes.c_size_t, P, ctypes.POINTER(P)]),
    "icr_ens_destroy": (None, [P]),
    "icr_ens_run": (I, [P, I, ctypes.POINTER(P)]),
    "icr_ens_set_planes": (I, [P, I, I]),
    "icr_ens_set_mode": (I, [P, I, I, I]),
    "icr_ens_step": (I, [P, I, ctypes.c_double, ctypes.POINTER(IcrStepInfo)]),
    "icr_append_boundary_maps": (I, [P, I, D, D, I, ctypes.POINTER(ctypes.c_int)]),
    "icr_set_tracer": (I, [P, D, I]),
    "icr_get_tracer": (I, [P, D, I]),
    "icr_divv": (I, [P, D, I]),
    "icr_sample_shell": (I, [P, ctypes.c_double, D]),
    "icr_amr_workspace_bytes": (I, [ctypes.POINTER(IcrGrid), ctypes.POINTER(IcrPhys),
                                    ctypes.POINTER(IcrAmrParams), ctypes.POINTER(ctypes.c_size_t)]),
    "icr_amr_create": (I, [ctypes.POINTER(IcrGrid), ctypes.POINTER(IcrPhys),
                           ctypes.POINTER(IcrAmrParams), P, ctypes.c_size_t, P,
                           ctypes.POINTER(P)]),
    "icr_amr_destroy": (None, [P]),
    "icr_amr_set_boundary_maps": (I, [P, I, D, D]),
    "icr_amr_set_cmes": (I, [P, I, D]),
    "icr_amr_init_radial": (I, [P]),
    "icr_amr_step": (I, [P, I, ctypes.c_double, ctypes.POINTER(IcrStepInfo)]),
    "icr_amr_force_refine": (I, [P, I, ctypes.POINTER(ctypes.c_int)]),
    "icr_amr_leaves": (I, [P, I, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "icr_amr_get_block": (I, [P, ctypes.POINTER(ctypes.c_int), D]),
    "icr_amr_get_clock": (I, [P, ctypes.POINTER(IcrClock)]),
    # warm-start network (include/icarus_nn.h)
    "icr_nn_last_error": (ctypes.c_char_p, []),
    "icr_nn_param_count": (I, [ctypes.POINTER(NnShape), ctypes.POINTER(ctypes.c_longlong)]),
    "icr_nn_workspace_bytes": (I, [ctypes.POINTER(NnShape), ctypes.POINTER(ctypes.c_size_t)]),
    "icr_nn_create": (I, [ctypes.POINTER(NnShape), P, ctypes.c_size_t, P, ctypes.POINTER(P)]),
    "icr_nn_destroy": (None, [P]),
    "icr_nn_set_params": (I, [P, ctypes.POINTER(ctypes.c_float)]),
    "icr_nn_get_params": (I, [P, ctypes.POINTER(ctypes.c_float)]),
    "icr_nn_forward": (I, [P, I, P, P]),
    "icr_nn_loss_grad": (I, [P, I, P, P, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_float)]),
    "icr_nn_adam_step": (I, [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    "icr_nn_encode_map": (I, [P, I, D, D, ctypes.c_double, ctypes.c_double, P]),
    "icr_nn_encode_target": (I, [P, D, D, D, D, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, P]),
    "icr_nn_decode_state": (I, [P, D, P, D, D, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, D]),
    "icr_nn_gemm_bf16": (I, [I, I, I, I, I, P, I, P, I, P, I, P, P]),
}


def lib():
    """Load libicarus_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() or "
                "python -m paper_2501_15923_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int):
    if rc != ICR_OK:
        raise IcarusError(rc, lib().icr_last_error().decode())
    return rc


def dptr(a):
    return ctypes.cast(a, D)
