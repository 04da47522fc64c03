"""ctypes binding of libfastalign.so: the C-ABI entry points under the same names.

This module only marshals arguments; every step of the method runs in the HIP
library.  Loading raises if the library has not been built - there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfastalign.so")

FA_OK, FA_WARN_NOT_CONVERGED = 0, 1
FA_ERR_ARG, FA_ERR_SHAPE, FA_ERR_CSR, FA_ERR_WORKSPACE = -1, -2, -3, -4
FA_ERR_NUMERIC, FA_ERR_HIP, FA_ERR_DEVICE, FA_ERR_SYNC = -6, -7, -8, -9
FA_F32, FA_BF16, FA_F64 = 0, 1, 2
FA_START_ZERO, FA_START_CARRY, FA_START_MEAN = 0, 1, 2
FA_SINKHORN_NOALLOC_SCRATCH = 16 << 20

EXPORTS = [
    "fa_last_error", "fa_default_params", "fa_device_check", "fa_csr_build", "fa_row_normalize",
    "fa_positional", "fa_sddmm", "fa_l2_normalize", "fa_feature_sim", "fa_cost_workspace_size",
    "fa_propagate", "fa_cost", "fa_sinkhorn_workspace_size", "fa_sinkhorn", "fa_plan",
    "fa_align_workspace_size", "fa_align", "fa_node_feature_dim", "fa_node_features_workspace_size",
    "fa_node_features", "fa_mlp_param_count", "fa_mlp_act_floats", "fa_mlp_forward",
    "fa_mlp_backward", "fa_adam_step", "fa_stream_read", "fa_plan_topk",
    "fa_align_begin", "fa_align_step", "fa_align_end", "fa_sinkhorn_noalloc_need", "fa_sinkhorn_noalloc",
    "fa_sinkhorn_fused_workspace_size", "fa_sinkhorn_fused", "fa_sinkhorn_fused_grid", "fa_set_sync_spin_limit",
]


class fa_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("colidx", C.c_void_p)]


class fa_params(C.Structure):
    _fields_ = [
        ("eps", C.c_double), ("alpha", C.c_double), ("beta", C.c_double), ("lambda_e", C.c_double),
        ("lambda_n", C.c_double), ("lambda_a", C.c_double), ("lambda_p", C.c_double),
        ("eps_anchor", C.c_double), ("delta_nbr", C.c_double), ("tol", C.c_double),
        ("k_r", C.c_int32), ("k_node", C.c_int32), ("outer_iters", C.c_int32), ("inner_iters", C.c_int32),
        ("check_every", C.c_int32), ("plan_dtype", C.c_int32), ("feat_dtype", C.c_int32),
        ("feat_l2norm", C.c_int32), ("warm_start", C.c_int32), ("chunk_rows", C.c_int32),
        ("profile", C.c_int32),
        ("dual_start", C.c_int32),
        ("transpose_cost", C.c_int32),
        ("plan_in_ct", C.c_int32),
        ("warm_fallback", C.c_int32),
        ("warm_probe", C.c_int32),
        ("sink_fused", C.c_int32),
    ]


class fa_stats(C.Structure):
    _fields_ = [
        ("outer_done", C.c_int32), ("inner_total", C.c_int32), ("fell_back", C.c_int32),
        ("converged_all", C.c_int32), ("marg_err", C.c_double),
        ("warm_iters", C.c_int32), ("cold_iters", C.c_int32), ("warm_err", C.c_double), ("cold_err", C.c_double),
        ("phase_ms", C.c_double * 4),
        ("inner_iters", C.c_int32 * 64), ("inner_err", C.c_double * 64),
        ("kernel_ms", C.c_double * 11), ("kernel_calls", C.c_int32 * 11),
    ]


class FastAlignError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} returned {status}: {msg}")
        self.status = status


_P, _I32, _I64, _D, _SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
_SIGS = {
    "fa_last_error": (C.c_char_p, []),
    "fa_default_params": (None, [C.POINTER(fa_params)]),
    "fa_device_check": (C.c_int, []),
    "fa_csr_build": (C.c_int, [_I32, _I64, _P, _P, _P, _I64, _P]),
    "fa_row_normalize": (C.c_int, [C.POINTER(fa_csr), _P, _P]),
    "fa_positional": (C.c_int, [C.POINTER(fa_csr), _P, _P, _I32, _D, _I32, _P, _P, _P]),
    "fa_sddmm": (C.c_int, [C.POINTER(fa_csr), _P, _P, _I32, _I32, _P, _P]),
    "fa_l2_normalize": (C.c_int, [_P, _I32, _I32, _P, _I32, _P]),
    "fa_feature_sim": (C.c_int, [_P, _P, _I32, _I32, _I32, _I32, _P, _P, _I32, _I32, _D, _P, _P]),
    "fa_cost_workspace_size": (_SZ, [_I32, _I32, _I32, _I32]),
    "fa_propagate": (C.c_int, [C.POINTER(fa_csr), _P, C.POINTER(fa_csr), _P, _P, _P, _I32, _I32, _P, _SZ, _P]),
    "fa_cost": (C.c_int, [C.POINTER(fa_csr), C.POINTER(fa_csr), _P, _P, _P, _P, _P, _I32, _P, _P, _P, _P,
                          C.POINTER(fa_params), _P, _P, _P, _SZ, _P]),
    "fa_sinkhorn_workspace_size": (_SZ, [_I32, _I32]),
    "fa_sinkhorn": (C.c_int, [_P, _P, _I32, _I32, _D, _P, _P, _I32, _D, _I32, _P, _P, _P, _P, _P, _SZ, _P]),
    "fa_sinkhorn_noalloc_need": (_SZ, [_I32, _I32, _I32]),
    "fa_sinkhorn_noalloc": (C.c_int, [_P, _P, _I32, _I32, _D, _P, _P, _I32, _D, _I32, _P, _P, _P]),
    "fa_sinkhorn_fused_workspace_size": (_SZ, [_I32, _I32]),
    "fa_sinkhorn_fused": (C.c_int, [_P, _I32, _I32, _D, _P, _P, _I32, _D, _I32, _P, _P, _P, _P, _P, _SZ, _P]),
    "fa_sinkhorn_fused_grid": (C.c_int, [_I32, _I32, _P, _P]),
    "fa_set_sync_spin_limit": (_I32, [_I32]),
    "fa_plan": (C.c_int, [_P, _I32, _I32, _D, _P, _P, _P, _I32, _P, _P, _P, _P]),
    "fa_plan_topk": (C.c_int, [_P, _I32, _I32, _D, _P, _P, _I32, _P, _P, _P]),
    "fa_align_workspace_size": (_SZ, [_I32, _I32, _I32, _I32, _I64, _I64, C.POINTER(fa_params)]),
    "fa_align": (C.c_int, [C.POINTER(fa_csr), C.POINTER(fa_csr), _P, _P, _I32, _P, _I32, C.POINTER(fa_params),
                           _P, _P, _P, _P, _P, _P, _P, _I32, _P, _P, C.POINTER(fa_stats), _P, _SZ, _P]),
    "fa_align_begin": (C.c_int, [C.POINTER(fa_csr), C.POINTER(fa_csr), _P, _P, _I32, _P, _I32,
                                 C.POINTER(fa_params), _P, _P, _P, C.POINTER(fa_stats), _P, _SZ, _P]),
    "fa_align_step": (C.c_int, [C.POINTER(fa_csr), C.POINTER(fa_csr), _I32, _I32, C.POINTER(fa_params), _P, _I32,
                                _P, _P, _P, _P, _P, _P, C.POINTER(fa_stats), _P, _SZ, _P]),
    "fa_align_end": (C.c_int, [C.POINTER(fa_csr), C.POINTER(fa_csr), _I32, _I32, C.POINTER(fa_params), _I32, _P, _P,
                               _P, _P, _P, _P, _I32, _P, _P, C.POINTER(fa_stats), _P, _SZ, _P]),
    "fa_node_feature_dim": (_I32, []),
    "fa_node_features_workspace_size": (_SZ, [_I32]),
    "fa_node_features": (C.c_int, [C.POINTER(fa_csr), _P, _P, _I32, _P, _P, _I32, _P, _P, _SZ, _P]),
    "fa_mlp_param_count": (_I32, []),
    "fa_mlp_act_floats": (_SZ, [_I32]),
    "fa_mlp_forward": (C.c_int, [_P, _P, _I32, _P, _P, _P]),
    "fa_mlp_backward": (C.c_int, [_P, _P, _P, _I32, _P, _P, _P, _P]),
    "fa_adam_step": (C.c_int, [_P, _P, _P, _P, _I32, _D, _D, _D, _D, _I32, _P]),
    "fa_stream_read": (C.c_int, [_P, _SZ, _P, _I32, _P]),
}


class Lib:
    """The loaded library; attribute access returns checked wrappers."""

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2607_11952_amd.build`")
        self.path = path
        self._dll = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(self._dll, name)
            fn.restype = res
            fn.argtypes = args

    def raw(self, name: str):
        return getattr(self._dll, name)

    def last_error(self) -> str:
        return (self._dll.fa_last_error() or b"").decode()

    def call(self, name: str, *args, allow_warn: bool = True) -> int:
        st = getattr(self._dll, name)(*args)
        if st < 0 or (st > 0 and not allow_warn):
            raise FastAlignError(name, st, self.last_error())
        return st

    def default_params(self) -> fa_params:
        p = fa_params()
        self._dll.fa_default_params(C.byref(p))
        return p


_LIB = None


def load(path: str = LIB_PATH) -> Lib:
    global _LIB
    if _LIB is None or _LIB.path != path:
        _LIB = Lib(path)
    return _LIB
