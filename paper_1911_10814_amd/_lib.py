"""ctypes view of the C ABI declared in ``include/ns_api.h`` (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libns_hip.so")

NS_OK, NS_NOT_CONVERGED = 0, 1
STATUS_NAMES = {0: "NS_OK", 1: "NS_NOT_CONVERGED", -1: "NS_ERR_ARG", -2: "NS_ERR_HIP", -3: "NS_ERR_NAN",
                -4: "NS_ERR_BREAKDOWN", -5: "NS_ERR_WORKSPACE", -6: "NS_ERR_STATE"}

KERNEL_CLASSES = {"spmv_A": 0, "cheb_A0": 1, "spmv_full": 2, "sfact": 3, "cgs2": 4, "cheb_S1": 5}

OPS = {"full": 0, "A": 1, "B": 2, "C": 3, "D": 4, "shat": 5, "vcycle_A": 6, "vcycle_S": 7, "schur": 8,
       "pscr": 9, "solve_A": 10, "psimple": 11}

PD = C.POINTER(C.c_double)
PI = C.POINTER(C.c_int32)


class NsMesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_elems", C.c_int32), ("n_outlets", C.c_int32),
                ("h_xyz", PD), ("h_tets", PI), ("h_outlet_ptr", PI), ("h_faces", PI),
                ("h_dirichlet", C.POINTER(C.c_uint8))]


class NsCtxOpts(C.Structure):
    _fields_ = [("max_m", C.c_int32), ("max_m_A", C.c_int32), ("max_m_S", C.c_int32),
                ("coarse_nodes", C.c_int32), ("max_levels", C.c_int32), ("coarse_matchings", C.c_int32)]


class NsPhys(C.Structure):
    _fields_ = [("rho", C.c_double), ("mu", C.c_double), ("dt", C.c_double), ("rho_inf", C.c_double),
                ("beta_bf", C.c_double), ("c_t", C.c_double), ("c_i", C.c_double), ("h_m", PD), ("h_P_af", PD),
                ("h_R", PD), ("h_P_n", PD), ("h_Q", PD)]


class NsSolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("rtol_A", C.c_double), ("rtol_S", C.c_double),
                ("rtol_I", C.c_double), ("cheb_ratio", C.c_double), ("cc_scale_A", C.c_double),
                ("cc_scale_S", C.c_double), ("m", C.c_int32), ("nmax", C.c_int32), ("m_A", C.c_int32),
                ("nmax_A", C.c_int32), ("m_S", C.c_int32), ("nmax_S", C.c_int32), ("pc_A", C.c_int32),
                ("precision", C.c_int32), ("cheb_degree", C.c_int32), ("cycles_S", C.c_int32),
                ("pc", C.c_int32), ("cheb_degree_S", C.c_int32), ("pc_I", C.c_int32), ("cycle_index_A", C.c_int32),
                ("cycle_index_S", C.c_int32), ("reserved", C.c_int32),
                ("h_sched", PI), ("sched_len", C.c_int32), ("sched_cap", C.c_int32), ("h_sched_out", PI)]


class NsStats(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("a_solves", C.c_int32), ("a_iters", C.c_int32),
                ("s_solves", C.c_int32), ("s_iters", C.c_int32), ("inner_solves", C.c_int32),
                ("inner_iters", C.c_int32), ("n_calls", C.c_int32), ("amg_levels_A", C.c_int32),
                ("amg_levels_S", C.c_int32), ("true_rel_res", C.c_double), ("setup_ms", C.c_double),
                ("solve_ms", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class NsOutletModel(C.Structure):
    _fields_ = [("h_Rp", PD), ("h_C", PD), ("h_Rd", PD), ("h_Pd", PD), ("h_Pi", PD), ("h_P", PD), ("h_Q", PD),
                ("n_ts", C.c_int32), ("reserved", C.c_int32)]


class NsNewtonOpts(C.Structure):
    _fields_ = [("tol_R", C.c_double), ("tol_A", C.c_double), ("eps_abs", C.c_double), ("eps_rel", C.c_double),
                ("l_max", C.c_int32), ("reserved", C.c_int32)]


class NsStepStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("res0", C.c_double), ("res", C.c_double),
                ("res_hist", C.c_double * 32), ("lin_outer", C.c_int32), ("lin_a", C.c_int32),
                ("lin_s", C.c_int32), ("lin_inner", C.c_int32), ("assemble_ms", C.c_double),
                ("solve_ms", C.c_double), ("total_ms", C.c_double)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "res_hist"}
        d["res_hist"] = list(self.res_hist[:min(self.iterations + 1, 32)])
        return d


# name -> (restype, argtypes)
SIGNATURES = {
    "ns_ctx_create": (C.c_int, [C.POINTER(NsMesh), C.POINTER(NsCtxOpts), C.POINTER(C.c_void_p),
                                C.POINTER(C.c_size_t)]),
    "ns_ctx_bind": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "ns_ctx_destroy": (None, [C.c_void_p]),
    "ns_last_error": (C.c_char_p, [C.c_void_p]),
    "ns_outlet_flow": (C.c_int, [C.c_void_p, C.c_void_p, PD, C.c_void_p]),
    "ns_rank_one_dots": (C.c_int, [C.c_void_p, C.c_void_p, PD, C.c_void_p]),
    "ns_resistance_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, PD, C.c_void_p]),
    "ns_resistance_gradient_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ns_gen_alpha": (C.c_int, [C.c_double, PD]),
    "ns_stream_bench": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, PD]),
    "ns_assemble_tangent": (C.c_int, [C.c_void_p, C.POINTER(NsPhys), C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p]),
    "ns_nested_solve": (C.c_int, [C.c_void_p, C.POINTER(NsSolveOpts), C.c_void_p, C.c_void_p,
                                  C.POINTER(NsStats), C.c_void_p]),
    "ns_adjoint_solve": (C.c_int, [C.c_void_p, C.POINTER(NsSolveOpts), C.c_void_p, C.c_void_p,
                                   C.POINTER(NsStats), C.c_void_p]),
    "ns_newton_update": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ns_time_step": (C.c_int, [C.c_void_p, C.POINTER(NsPhys), C.POINTER(NsOutletModel), C.POINTER(NsNewtonOpts),
                               C.POINTER(NsSolveOpts), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.POINTER(NsStepStats), C.c_void_p]),
    "ns_query": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "ns_query_layout": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "ns_kernel_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "ns_kernel_timing_period": (C.c_int, [C.c_void_p, C.c_int32]),
    "ns_kernel_timing_read": (C.c_int, [C.c_void_p, C.c_int32, PD]),
    "ns_export_pattern": (C.c_int, [C.c_void_p, PI, PI]),
    "ns_export_fixed_width_offsets": (C.c_int, [C.c_void_p, C.POINTER(C.c_int16)]),
    "ns_export_aggregates": (C.c_int, [C.c_void_p, C.c_int32, PI]),
    "ns_export_colors": (C.c_int, [C.c_void_p, PI]),
    "ns_export_bsr": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "ns_export_shat": (C.c_int, [C.c_void_p, PI, PI, C.c_void_p, C.c_void_p]),
    "ns_export_outlet_vectors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ns_apply": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(NsSolveOpts), C.c_void_p, C.c_void_p, C.c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built (there is no
    other implementation to fall back to)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: run `python -m paper_1911_10814_amd.build` "
                           "(or __graft_entry__.build()) first")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class NsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
