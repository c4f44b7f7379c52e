"""ctypes binding of libcisor.so (argument marshalling only).

Every function here forwards to the C ABI declared in ``include/cisor.h``;
all computation happens in the HIP library.  Loading fails loudly when the
library has not been built: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcisor.so")

OK, NOT_CONVERGED = 0, 1
E_ARG, E_NOMEM, E_DEVICE, E_NONFINITE, E_UNSUPPORTED, E_SIZE = -1, -2, -3, -4, -6, -7


class Geometry(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int), ("h", C.c_double), ("wavelength", C.c_double),
                ("eps_b", C.c_double), ("T", C.c_int), ("M", C.c_int),
                ("tx_dir", C.POINTER(C.c_double)), ("rx_pos", C.POINTER(C.c_double)),
                ("precision", C.c_int), ("tx_kind", C.c_int), ("tx_pos", C.POINTER(C.c_double))]


class LsOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("start", C.c_int),
                ("replace_every", C.c_int), ("check_every", C.c_int)]


class FistaState(C.Structure):
    _fields_ = [("f", C.c_void_p), ("f_prev", C.c_void_p), ("s", C.c_void_p),
                ("t", C.c_double), ("k", C.c_int)]


class StepInfo(C.Structure):
    _fields_ = [("D", C.c_double), ("fwd_iters_max", C.c_int), ("adj_iters_max", C.c_int),
                ("fwd_iters_sum", C.c_longlong), ("adj_iters_sum", C.c_longlong),
                ("max_true_relres", C.c_double), ("status", C.c_int)]


class ApgState(C.Structure):
    _fields_ = [("x", C.c_void_p), ("x_prev", C.c_void_p), ("z", C.c_void_p), ("t", C.c_double),
                ("t_prev", C.c_double), ("k", C.c_int)]


class ApgInfo(C.Structure):
    _fields_ = [("F", C.c_double), ("F_z", C.c_double), ("F_v", C.c_double), ("D_y", C.c_double),
                ("D_x", C.c_double), ("took_z", C.c_int), ("fwd_solves", C.c_int), ("adj_solves", C.c_int),
                ("fwd_iters_sum", C.c_longlong), ("adj_iters_sum", C.c_longlong),
                ("max_true_relres", C.c_double), ("status", C.c_int)]


_vp, _i, _d = C.c_void_p, C.c_int, C.c_double
_SIGS = {
    "cisor_create": (_i, [C.POINTER(Geometry), _vp, C.POINTER(_vp)]),
    "cisor_destroy": (_i, [_vp]),
    "cisor_set_stream": (_i, [_vp, _vp]),
    "cisor_get_sizes": (_i, [_vp, C.POINTER(_i), C.POINTER(_i), C.POINTER(_i), C.POINTER(_i), C.POINTER(_i)]),
    "cisor_get_uin": (_i, [_vp, _vp]),
    "cisor_get_H": (_i, [_vp, _vp]),
    "cisor_forward": (_i, [_vp, _vp, _vp, _vp, C.POINTER(LsOpts), C.POINTER(_i)]),
    "cisor_grad": (_i, [_vp, _vp, _vp, _vp, C.POINTER(_d), _vp, _vp, C.POINTER(LsOpts), C.POINTER(_i)]),
    "cisor_vjp": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(LsOpts), C.POINTER(_i)]),
    "cisor_tv_prox": (_i, [_vp, _vp, _vp, _d, _d, _d, _i]),
    "cisor_tv_prox_noalloc": (_i, [_i, _i, _i, _vp, _vp, _d, _d, _d, _i, _vp]),
    "cisor_set_rx_mask": (_i, [_vp, _vp]),
    "cisor_tv_value": (_i, [_vp, _vp, C.POINTER(_d)]),
    "cisor_fista_step": (_i, [_vp, C.POINTER(FistaState), _vp, _d, _d, _d, _d, _d, _i,
                              C.POINTER(LsOpts), C.POINTER(StepInfo)]),
    "cisor_apg_step": (_i, [_vp, C.POINTER(ApgState), _vp, _d, _d, _d, _d, _d, _i, C.POINTER(LsOpts),
                            C.POINTER(ApgInfo)]),
    "cisor_apply_A": (_i, [_vp, _vp, _vp, _vp, _i]),
    "cisor_born_field": (_i, [_vp, _vp, _vp]),
    "cisor_apply_A_stage": (_i, [_vp, _vp, _vp, _vp, _i, _i]),
    "cisor_solve": (_i, [_vp, _vp, _vp, _vp, _i, C.POINTER(LsOpts), C.POINTER(_i)]),
    "cisor_project": (_i, [_vp, _vp, _vp, _vp, _vp, C.POINTER(_d)]),
    "cisor_backproject": (_i, [_vp, _vp, _vp]),
    "cisor_born_lipschitz": (_i, [_vp, _i, C.POINTER(_d)]),
    "cisor_get_start_choice": (_i, [_vp, C.POINTER(_i)]),
    "cisor_autotune": (_i, [_vp, _i, C.POINTER(_i), C.POINTER(C.c_float)]),
    "cisor_set_col_variant": (_i, [_vp, _i]),
    "cisor_batch_create": (_i, [C.POINTER(Geometry), _i, _vp, C.POINTER(_vp)]),
    "cisor_batch_destroy": (_i, [_vp]),
    "cisor_batch_set_stream": (_i, [_vp, _vp]),
    "cisor_batch_get_sizes": (_i, [_vp, _i, C.POINTER(_i), C.POINTER(_i), C.POINTER(_i), C.POINTER(_i),
                                   C.POINTER(_i)]),
    "cisor_batch_num_groups": (_i, [_vp, C.POINTER(_i)]),
    "cisor_batch_set_problem": (_i, [_vp, _i, _vp, _d, _d]),
    "cisor_batch_fista_step": (_i, [_vp, _d, _d, _d, _i, C.POINTER(LsOpts), C.POINTER(StepInfo)]),
    "cisor_batch_get_f": (_i, [_vp, _i, _vp]),
    "cisor_batch_forward": (_i, [_vp, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(LsOpts),
                                 C.POINTER(_i)]),
    "cisor_batch_autotune": (_i, [_vp, _i, C.POINTER(_i), C.POINTER(C.c_float)]),
    "cisor_batch_born_lipschitz": (_i, [_vp, _i, _i, C.POINTER(_d)]),
    "cisor_net_create": (_i, [_i, _i, _i, _i, C.c_ulonglong, _vp, C.POINTER(_vp)]),
    "cisor_net_destroy": (_i, [_vp]),
    "cisor_net_set_stream": (_i, [_vp, _vp]),
    "cisor_net_num_params": (_i, [_vp, C.POINTER(C.c_longlong)]),
    "cisor_net_get_params": (_i, [_vp, _vp]),
    "cisor_net_set_params": (_i, [_vp, _vp]),
    "cisor_net_forward": (_i, [_vp, _vp, _vp, _vp, _vp, _i]),
    "cisor_net_loss_grad": (_i, [_vp, _vp, _vp, _vp, _vp, _i, C.POINTER(_d), _vp]),
    "cisor_net_train_step": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _d, _d, C.POINTER(_d)]),
    "cisor_nn_conv3x3": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _i, _i, _vp]),
    "cisor_nn_conv3x3_wgrad": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _vp]),
    "cisor_nn_conv3x3_ex": (_i, [_vp, _vp, _i, _vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _i, _i, _i, _vp, C.c_size_t,
                                  _vp]),
    "cisor_vec_create": (_i, [C.POINTER(Geometry), _vp, C.POINTER(_vp)]),
    "cisor_vec_destroy": (_i, [_vp]),
    "cisor_vec_set_stream": (_i, [_vp, _vp]),
    "cisor_vec_get_sizes": (_i, [_vp, C.POINTER(_i), C.POINTER(_i), C.POINTER(_i)]),
    "cisor_vec_get_uin": (_i, [_vp, _vp]),
    "cisor_vec_set_rx_mask": (_i, [_vp, _vp]),
    "cisor_vec_get_H": (_i, [_vp, _vp]),
    "cisor_vec_apply_A": (_i, [_vp, _vp, _vp, _vp, _i]),
    "cisor_vec_forward": (_i, [_vp, _vp, C.POINTER(LsOpts), _vp, _vp, C.POINTER(_i), C.POINTER(_d)]),
    "cisor_vec_project": (_i, [_vp, _vp, _vp, _vp]),
    "cisor_vec_grad": (_i, [_vp, _vp, _vp, _vp, C.POINTER(_d), C.POINTER(LsOpts), C.POINTER(_i), C.POINTER(_d)]),
    "cisor_vec_fista_step": (_i, [_vp, C.POINTER(FistaState), _vp, _d, _d, _d, _d, _d, _i, C.POINTER(LsOpts),
                                  C.POINTER(StepInfo)]),
    "cisor_status_string": (C.c_char_p, [_i]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libcisor.so and declare every exported signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libcisor.so not found at {path}; build it with "
            "`python -m paper_1708_01663_amd.build` (there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


class CisorError(RuntimeError):
    def __init__(self, code, where):
        msg = load().cisor_status_string(code).decode()
        super().__init__(f"{where}: {msg} (status {code})")
        self.code = code


def check(code, where, allow_not_converged=True):
    if code == OK or (code == NOT_CONVERGED and allow_not_converged):
        return code
    raise CisorError(code, where)
