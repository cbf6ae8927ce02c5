"""ctypes binding of libcfdhip.so: the C entry points under the same names.

Argument marshalling only.  Loading fails loudly when the library has not
been built; there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcfdhip.so")

CFD_OK = 0
STATUS = {0: "CFD_OK", -1: "CFD_ERR_ARG", -2: "CFD_ERR_STATE", -3: "CFD_ERR_TOPOLOGY", -4: "CFD_ERR_GRID",
          -5: "CFD_ERR_HIP", -6: "CFD_ERR_NONFINITE", -7: "CFD_ERR_UNSUPPORTED"}
LIM = {"none": 0, "vanleer": 1, "vanalbada": 2}
FLUX = {"roe": 0, "vanleer_fvs": 1, "steger_warming": 2}
RK = {"mstage": 0, "classic4": 1}
BC = {"slip_wall": 1, "sup_inflow": 2, "extrap_outflow": 3, "farfield": 4, "sub_inflow": 5, "sub_outflow": 6,
      "noslip_wall": 7}
DT_CFL, DT_FIXED, DT_LOCAL = 0, 1, 2
EXEC_BATCHED, EXEC_PER_BLOCK, EXEC_PERSISTENT = 0, 1, 2
GHOSTS_DIRECT, GHOSTS_PACKED = 0, 1
CHECK_FINITE, NAN_GHOSTS = 1, 2  # cfd_config.debug_flags
Q = {"nblocks": 0, "ncells": 1, "nvar": 2, "nvariants": 3, "variant": 4, "ntiles": 5, "ntransfers": 6,
     "npatches": 7, "nnodes": 8, "exchange_doubles": 9, "workspace_bytes": 10, "tile_x": 11, "tile_y": 12}


class CfdConfig(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("gamma", ctypes.c_double), ("limiter", ctypes.c_int),
                ("muscl_eps", ctypes.c_double), ("muscl_kappa", ctypes.c_double),
                ("lim_eps", ctypes.c_double * 5), ("efix", ctypes.c_double), ("rk_stages", ctypes.c_int),
                ("dt_mode", ctypes.c_int), ("cfl", ctypes.c_double), ("dt_fixed", ctypes.c_double),
                ("flux", ctypes.c_int), ("viscosity", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("debug_flags", ctypes.c_int), ("rk_scheme", ctypes.c_int)]


class CfdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_IA = ctypes.POINTER(ctypes.c_int)
_DP = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "cfd_version": ([], ctypes.c_char_p),
    "cfd_status_string": ([_I], ctypes.c_char_p),
    "cfd_last_error": ([_P], ctypes.c_char_p),
    "cfd_create": ([ctypes.POINTER(CfdConfig), _P, ctypes.POINTER(_P)], _I),
    "cfd_destroy": ([_P], _I),
    "cfd_add_block": ([_P, _I, _I, _I, _DP, _IA], _I),
    "cfd_set_bc": ([_P, _I, _I, _IA, _IA, _I, _DP, _IA], _I),
    "cfd_connect": ([_P, _I, _I, _IA, _IA, _I, _I, _IA, _IA, _I], _I),
    "cfd_finalize": ([_P, ctypes.POINTER(ctypes.c_size_t)], _I),
    "cfd_bind_workspace": ([_P, _P, ctypes.c_size_t], _I),
    "cfd_set_nodes": ([_P, _P], _I),
    "cfd_set_bc_params": ([_P, _I, _DP], _I),
    "cfd_set_state": ([_P, _P], _I),
    "cfd_set_state_primitive": ([_P, _P], _I),
    "cfd_get_state": ([_P, _P], _I),
    "cfd_residual": ([_P, _P], _I),
    "cfd_time_step": ([_P, _P], _I),
    "cfd_rk_step": ([_P, _I, _P], _I),
    "cfd_padded_primitives": ([_P, _P], _I),
    "cfd_padded_size": ([_P, ctypes.POINTER(ctypes.c_size_t)], _I),
    "cfd_set_exec": ([_P, _I, _I], _I),
    "cfd_set_ghost_exchange": ([_P, _I], _I),
    "cfd_autotune": ([_P, _I, _IA], _I),
    "cfd_set_variant": ([_P, _I], _I),
    "cfd_profile": ([_P, _I], _I),
    "cfd_kernel_time": ([_P, _DP, ctypes.POINTER(ctypes.c_longlong)], _I),
    "cfd_query": ([_P, _I, ctypes.POINTER(ctypes.c_longlong)], _I),
    "cfd_enable_adjoint": ([_P, _I], _I),
    "cfd_residual_vjp": ([_P, _P, _P, _P, _P], _I),
    "cfd_adjoint_reset": ([_P], _I),
    "cfd_rk_step_vjp": ([_P, _P], _I),
    "cfd_residual_norms": ([_P, _P, _P], _I),
    "cfd_residual_norms_noalloc": ([_P, _P, _P], _I),
    "cfd_enable_limiter_freezing": ([_P, _I], _I),
    "cfd_freeze_limiter": ([_P, _I], _I),
    "cfd_rk_step_record": ([_P, _P], _I),
    "cfd_stream_probe": ([_I, _I, _I, _P, _P, ctypes.c_longlong, _I, _P, _DP], _I),
    "cfd_rk_step_vjp_recorded": ([_P, _P, _P], _I),
    "cfd_objective_wall_pressure": ([_P, _P, _P], _I),
    "cfd_adjoint_result": ([_P, _P, _P], _I),
    "cfd_uniform_state_vjp": ([_P, _DP, _P, _P], _I),
    "cfd_state_size": ([_P, ctypes.POINTER(ctypes.c_size_t)], _I),
    "cfd_save_state": ([_P, _P], _I),
    "cfd_load_state": ([_P, _P], _I),
}

_lib = None


def load():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcfdhip.so is not built (run __graft_entry__.build() or "
                              "python -m paper_2012_02925_amd.build); no fallback exists")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def check(status, ctx=None):
    if status != CFD_OK:
        msg = ""
        if ctx:
            msg = load().cfd_last_error(ctx).decode()
        raise CfdError(status, msg or load().cfd_status_string(status).decode())
    return status


def int2(vals):
    a = (ctypes.c_int * 2)(0, 0)
    for t, v in enumerate(list(vals)[:2]):
        a[t] = int(v)
    return a


def dptr(t):
    """Device (or host) address of a contiguous torch tensor as a void pointer."""
    return ctypes.c_void_p(t.data_ptr())
