"""ctypes declarations of libchfsi (include/chfsi.h).  Loads the in-tree
library and fails loudly when it is missing: there is no fallback path."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchfsi.so")

OK, NOTCONV, EINVAL, ENOMEM, EHIP, ECHOL, EDIVERGE = 0, 1, -1, -2, -3, -4, -5
F64, F32, BF16, C128, C64 = 0, 1, 2, 3, 4
RHO_NODES, RHO_GAUSS = 0, 1

# every symbol include/chfsi.h declares
EXPORTS = [
    "chfsi_ctx_create", "chfsi_ctx_destroy", "chfsi_last_error", "chfsi_sync", "chfsi_version", "chfsi_abi_sizes",
    "chfsi_op_build", "chfsi_op_destroy", "chfsi_op_info", "chfsi_op_tables",
    "chfsi_apply", "chfsi_apply_noalloc", "chfsi_bounds", "chfsi_filter", "chfsi_orthonormalize",
    "chfsi_rayleigh_ritz", "chfsi_solve", "chfsi_pass", "chfsi_set_timing", "chfsi_set_deterministic", "chfsi_kernel_time",
    "chfsi_filter_batched", "chfsi_solve_batched", "chfsi_autotune", "chfsi_load_tuning", "chfsi_get_tuning",
    "chfsi_features", "chfsi_mlp_create", "chfsi_mlp_destroy", "chfsi_mlp_info", "chfsi_mlp_params",
    "chfsi_mlp_set_norm", "chfsi_mlp_forward", "chfsi_mlp_loss_grad", "chfsi_mlp_train_step",
    "chfsi_initial_block", "chfsi_next_prec", "chfsi_fermi_level", "chfsi_density",
    "chfsi_rayleigh_ritz_split", "chfsi_op_build_quadrature", "chfsi_op_set_potential", "chfsi_hartree",
    "chfsi_scf", "chfsi_scf_kpoints",
]


class System(C.Structure):
    _fields_ = [
        ("L", C.c_double), ("ncell", C.c_int32), ("p", C.c_int32), ("natoms", C.c_int32),
        ("has_proj", C.c_int32),
        ("pos", C.POINTER(C.c_double)), ("Z", C.POINTER(C.c_double)), ("s", C.POINTER(C.c_double)),
        ("w", C.POINTER(C.c_double)), ("h_s", C.POINTER(C.c_double)), ("h_p", C.POINTER(C.c_double)),
        ("k", C.c_double * 3),
    ]


class Params(C.Structure):
    _fields_ = [
        ("nwanted", C.c_int32), ("n_buf", C.c_int32), ("m", C.c_int32), ("block", C.c_int32),
        ("fixed_passes", C.c_int32), ("max_passes", C.c_int32), ("tol", C.c_double),
        ("filter_prec", C.c_int32), ("lanczos_steps", C.c_int32), ("b_upper", C.c_double),
        ("lanczos_v0", C.POINTER(C.c_double)), ("seed", C.c_uint64),
        ("prec_switch", C.c_int32), ("hist_len", C.c_int32),
        ("hist_time_ms", C.POINTER(C.c_double)), ("hist_max_resid", C.POINTER(C.c_double)),
        ("hist_prec", C.POINTER(C.c_int32)), ("hist_theta", C.POINTER(C.c_double)),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("t_bounds", C.c_double), ("t_filter", C.c_double), ("t_cholgs", C.c_double),
        ("t_rr", C.c_double), ("t_total", C.c_double), ("passes", C.c_int32),
        ("hx_columns", C.c_int64), ("hx_flops", C.c_double), ("b_upper", C.c_double),
        ("a_last", C.c_double), ("aL_last", C.c_double), ("max_resid", C.c_double),
        ("final_prec", C.c_int32), ("prec_changes", C.c_int32), ("redrawn_columns", C.c_int32),
    ]


_lib = None


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2203_07820_amd.build` "
            "(hipcc, gfx950). There is no CPU fallback.")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64
    pd = C.POINTER(C.c_double)
    sig = {
        "chfsi_ctx_create": (C.c_int, [C.POINTER(vp), C.c_int, vp]),
        "chfsi_ctx_destroy": (C.c_int, [vp]),
        "chfsi_last_error": (C.c_char_p, [vp]),
        "chfsi_sync": (C.c_int, [vp]),
        "chfsi_version": (C.c_char_p, []),
        "chfsi_abi_sizes": (C.c_int, [C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]),
        "chfsi_op_build": (C.c_int, [vp, C.POINTER(System), C.POINTER(vp)]),
        "chfsi_op_destroy": (C.c_int, [vp]),
        "chfsi_op_build_quadrature": (C.c_int, [vp, C.POINTER(System), C.POINTER(vp)]),
        "chfsi_op_info": (C.c_int, [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32), C.POINTER(i32),
                                    C.POINTER(i64), C.POINTER(i32)]),
        "chfsi_op_tables": (C.c_int, [vp, pd, pd, pd, pd, pd]),
        "chfsi_apply": (C.c_int, [vp, vp, vp, i64, i64, i32]),
        "chfsi_apply_noalloc": (C.c_int, [vp, vp, vp, i64, i64, i32]),
        "chfsi_bounds": (C.c_int, [vp, i32, vp, u64, pd, pd]),
        "chfsi_filter": (C.c_int, [vp, vp, i64, i64, i32, dbl, dbl, dbl, i32, i32]),
        "chfsi_orthonormalize": (C.c_int, [vp, vp, i64, i64, pd]),
        "chfsi_rayleigh_ritz": (C.c_int, [vp, vp, i64, i64, pd, pd]),
        "chfsi_solve": (C.c_int, [vp, C.POINTER(Params), vp, i64, pd, pd, C.POINTER(Stats)]),
        "chfsi_pass": (C.c_int, [vp, C.POINTER(Params), vp, i64, dbl, dbl, dbl, pd, pd]),
        "chfsi_set_timing": (C.c_int, [vp, i32]),
        "chfsi_set_deterministic": (C.c_int, [vp, i32]),
        "chfsi_kernel_time": (C.c_int, [vp, pd, C.POINTER(i64), pd, i32]),
        "chfsi_filter_batched": (C.c_int, [vp, i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(i64), C.POINTER(i64),
                                           i32, pd, pd, pd, i32, i32, i32]),
        "chfsi_solve_batched": (C.c_int, [vp, i32, C.POINTER(vp), C.POINTER(Params), C.POINTER(vp),
                                          C.POINTER(i64), C.POINTER(pd), C.POINTER(pd), C.POINTER(Stats), i32]),
        "chfsi_autotune": (C.c_int, [vp, C.c_char_p, i32, i32, i32]),
        "chfsi_load_tuning": (C.c_int, [vp, C.c_char_p]),
        "chfsi_get_tuning": (C.c_int, [vp, i32, i32, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), pd]),
        "chfsi_features": (C.c_int, [vp, vp]),
        "chfsi_mlp_create": (C.c_int, [vp, i32, i32, i32, u64, C.POINTER(vp)]),
        "chfsi_mlp_destroy": (C.c_int, [vp]),
        "chfsi_mlp_info": (C.c_int, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i64)]),
        "chfsi_mlp_params": (C.c_int, [vp, C.POINTER(C.c_float), i32]),
        "chfsi_mlp_set_norm": (C.c_int, [vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
        "chfsi_mlp_forward": (C.c_int, [vp, vp, i64, vp]),
        "chfsi_mlp_loss_grad": (C.c_int, [vp, vp, i64, vp, i32, pd, C.POINTER(C.c_float)]),
        "chfsi_mlp_train_step": (C.c_int, [vp, vp, i64, vp, i32, C.c_float, pd]),
        "chfsi_initial_block": (C.c_int, [vp, vp, u64, vp, i64, i64, C.POINTER(i32)]),
        "chfsi_next_prec": (i32, [i32, pd, i32, dbl]),
        "chfsi_fermi_level": (C.c_int, [pd, i32, pd, dbl, dbl, pd, pd]),
        "chfsi_density": (C.c_int, [vp, vp, i64, i64, pd, i32, i32, vp]),
        "chfsi_rayleigh_ritz_split": (C.c_int, [vp, vp, i64, i64, i32, i32, pd, vp, i64]),
        "chfsi_op_set_potential": (C.c_int, [vp, vp]),
        "chfsi_hartree": (C.c_int, [vp, vp, vp, dbl, i32, C.POINTER(i32), pd]),
        "chfsi_scf": (C.c_int, [vp, vp, i64, i32, i32, i32, i32, i32, dbl, dbl, dbl, i32, dbl, i32, vp, pd, pd, pd,
                                C.POINTER(i32)]),
        "chfsi_scf_kpoints": (C.c_int, [vp, i32, vp, vp, vp, vp, i32, i32, i32, i32, i32, dbl, dbl, dbl, i32, dbl,
                                        i32, vp, vp, pd, pd, C.POINTER(C.c_int32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
