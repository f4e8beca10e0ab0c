"""ctypes binding of the C ABI declared in include/lbm.h (argument marshalling only).

Every compute step runs in the HIP library ``liblbm.so``; this module only mirrors the C
structs and loads the library.  Importing it does not touch the GPU.  If the library has
not been built the loader raises: there is no fallback path.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBM_LIBRARY", os.path.join(_HERE, "liblbm.so"))

# enums of lbm.h
LBM_OK, LBM_ERR_ARG, LBM_ERR_UNSUPPORTED, LBM_ERR_CFL, LBM_ERR_LAUNCH = range(5)
LBM_F32_SHIFTED, LBM_F16_SHIFTED, LBM_F64_PLAIN = range(3)
LBM_LOGNH, LBM_NH, LBM_SVK, LBM_MR, LBM_YEOH, LBM_GENT = range(6)
LBM_PERIODIC, LBM_VELOCITY, LBM_TRACTION = range(3)
LBM_XMIN, LBM_XMAX, LBM_YMIN, LBM_YMAX = range(4)
LBM_FAULT_J, LBM_FAULT_NONFINITE, LBM_FAULT_NEWTON, LBM_FAULT_PROBE = 1, 2, 4, 8
LBM_DIAG_COUNT = 10

STORAGE = {"f32": LBM_F32_SHIFTED, "f16": LBM_F16_SHIFTED, "f64": LBM_F64_PLAIN}
MATERIAL = {"lognh": LBM_LOGNH, "nh": LBM_NH, "svk": LBM_SVK, "mr": LBM_MR, "yeoh": LBM_YEOH,
            "gent": LBM_GENT}
# law_k used when a caller gives none: Appendix A fixes c10 + c01 = mu/2 (Mooney-Rivlin) and
# c1 = mu/2 (Yeoh); the split, c2, c3 and the Gent limit J_m are choices of this binding.
LAW_K_DEFAULT = {"mr": (0.3, 0.2, 0.0), "yeoh": (0.5, 0.05, 0.01), "gent": (20.0, 0.0, 0.0)}
BC = {"periodic": LBM_PERIODIC, "velocity": LBM_VELOCITY, "traction": LBM_TRACTION}

c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", c_i32), ("ny", c_i32), ("material", c_i32), ("storage", c_i32),
        ("bc", c_i32 * 4), ("newton_max_iter", c_i32), ("force_unstable", c_i32),
        ("dx", c_dbl), ("c", c_dbl), ("omega", c_dbl), ("newton_tol", c_dbl),
        ("law_k", c_dbl * 3),
    ]


class lbm_state(ctypes.Structure):
    _fields_ = [
        ("pop", c_vp * 2), ("cur", c_i32), ("ustar", c_vp), ("mu", c_vp), ("lam", c_vp),
        ("mu0", c_dbl), ("lam0", c_dbl), ("mu_max", c_dbl), ("lam_max", c_dbl),
        ("body", c_vp), ("body_prev", c_vp), ("b0", c_dbl * 2), ("aux", c_vp), ("fault", c_vp),
    ]


class lbm_edge_data(ctypes.Structure):
    _fields_ = [("value", (c_dbl * 2) * 4), ("field", c_vp * 4)]


class lbm_adj_state(ctypes.Structure):
    _fields_ = [
        ("adj", c_vp * 2), ("cur", c_i32), ("g_mu", c_vp), ("g_lam", c_vp), ("g_body", c_vp),
        ("probe", c_vp), ("ubar", c_vp), ("nprobe", c_i32), ("nsteps", c_i64), ("aux", c_vp),
        ("gsum", c_vp), ("probe_mask", c_vp), ("probe_field", c_vp),
    ]


P = ctypes.POINTER
SIGNATURES = {
    "lbm_tile_width": (ctypes.c_size_t, []),
    "lbm_padded_nodes": (ctypes.c_size_t, [P(lbm_params)]),
    "lbm_pop_bytes": (ctypes.c_size_t, [P(lbm_params)]),
    "lbm_ustar_bytes": (ctypes.c_size_t, [P(lbm_params)]),
    "lbm_aux_bytes": (ctypes.c_size_t, [P(lbm_params)]),
    "lbm_record_bytes": (ctypes.c_size_t, [P(lbm_params)]),
    "lbm_adj_bytes": (ctypes.c_size_t, [P(lbm_params)]),
    "lbm_adj_sum_bytes": (ctypes.c_size_t, [P(lbm_params)]),
    "lbm_diag_scratch_bytes": (ctypes.c_size_t, [P(lbm_params)]),
    "lbm_check_params": (c_i32, [P(lbm_params)]),
    "lbm_check_cfl": (c_i32, [P(lbm_params), c_dbl, c_dbl]),
    "lbm_wall_mode_growth": (c_dbl, [P(lbm_params), c_dbl, c_dbl]),
    "lbm_init": (c_i32, [P(lbm_params), P(lbm_state), c_vp, c_vp, c_vp, c_dbl, c_vp]),
    "lbm_init_state": (c_i32, [P(lbm_params), P(lbm_state), c_vp, c_vp, c_vp, c_vp, c_dbl, c_vp]),
    "lbm_step": (c_i32, [P(lbm_params), P(lbm_state), c_i64, c_dbl, c_dbl, P(lbm_edge_data), c_vp, c_vp]),
    "lbm_step2": (c_i32, [P(lbm_params), P(lbm_state), c_i64, c_dbl, c_dbl, c_dbl, P(lbm_edge_data),
                          P(lbm_edge_data), c_vp, c_vp, c_vp]),
    "lbm_step_multi": (c_i32, [P(lbm_params), P(lbm_state), c_i64, c_i32, c_vp, c_vp, c_i32, c_vp]),
    "lbm_probe_mask_bytes": (ctypes.c_size_t, [P(lbm_params)]),
    "lbm_adjoint_probe_table": (c_i32, [P(lbm_params), P(lbm_adj_state), c_vp, c_vp, c_vp]),
    "lbm_adjoint_step_multi": (c_i32, [P(lbm_params), P(lbm_state), P(lbm_adj_state), c_i64, c_i32, c_vp, c_vp,
                                       c_vp, c_vp, c_vp]),
    "lbm_adjoint_step2": (c_i32, [P(lbm_params), P(lbm_state), P(lbm_adj_state), c_i64, c_dbl, c_dbl,
                                  P(lbm_edge_data), P(lbm_edge_data), c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lbm_displacement": (c_i32, [P(lbm_params), P(lbm_state), c_dbl, c_vp, c_vp]),
    "lbm_moments": (c_i32, [P(lbm_params), P(lbm_state), c_dbl, c_vp, c_vp]),
    "lbm_stress": (c_i32, [P(lbm_params), P(lbm_state), c_dbl, c_vp, c_vp, c_vp]),
    "lbm_diagnostics": (c_i32, [P(lbm_params), P(lbm_state), c_dbl, c_vp, c_vp, c_vp]),
    "lbm_diagnostics_noalloc": (c_i32, [P(lbm_params), P(lbm_state), c_dbl, c_vp, c_vp]),
    "lbm_adjoint_step": (c_i32, [P(lbm_params), P(lbm_state), P(lbm_adj_state), c_i64, c_dbl,
                                 P(lbm_edge_data), c_vp, c_vp]),
    "lbm_adjoint_init": (c_i32, [P(lbm_params), P(lbm_state), P(lbm_adj_state), c_vp, c_vp, c_vp,
                                 c_dbl, c_vp, c_vp]),
    "lbm_record_state": (c_i32, [P(lbm_params), P(lbm_state), c_dbl, c_vp, c_vp]),
    "lbm_status_string": (ctypes.c_char_p, [c_i32]),
    "lbm_version": (ctypes.c_char_p, []),
}

_lib = None


class LBMError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = lib().lbm_status_string(status).decode()
        super().__init__(f"{where}: {msg} (status {status})" if where else msg)


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is not built; run `python -m paper_2605_26677_amd.build` "
                "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, where=""):
    if status != LBM_OK:
        raise LBMError(status, where)
    return status
