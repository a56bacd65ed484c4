"""ctypes declarations of the C ABI in include/hdg.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libhdg.so")
HEADER = os.path.join(HERE, "..", "include", "hdg.h")

HDG_FP64, HDG_FP32, HDG_BF16 = 0, 1, 2
HDG_OK, HDG_EINVAL, HDG_EUNSUPPORTED, HDG_ENONPHYS, HDG_ESINGULAR, HDG_EHIP, HDG_ENOMEM = 0, -1, -2, -3, -4, -5, -6
ERROR_NAMES = {0: "HDG_OK", -1: "HDG_EINVAL", -2: "HDG_EUNSUPPORTED", -3: "HDG_ENONPHYS",
               -4: "HDG_ESINGULAR", -5: "HDG_EHIP", -6: "HDG_ENOMEM"}
ETYPES = {"tri": 0, "quad": 1, "tet": 2, "hex": 3}
PHASES = ["points", "contract", "lu", "solve", "schur", "backsolve", "matvec", "rhs", "condense", "condense_lp",
          "lp_solve", "jvp", "condense_lu", "condense_rhs"]
FLAG_SPLIT_DENSE = 1
FLAG_NARROW_BLOCK = 2
FLAG_ELIMINATE_Q = 4
FLAG_GHAT_INTERIOR = 8
FLAG_SIGMA_S = 16
FLAG_SIGMA_MV = 32
FLAG_GHAT_PROJ = 64


class hdg_phys(ctypes.Structure):
    _fields_ = [("viscous", ctypes.c_int), ("gamma", ctypes.c_double), ("mu", ctypes.c_double),
                ("Pr", ctypes.c_double), ("alpha", ctypes.c_double)]


class hdg_mesh(ctypes.Structure):
    _fields_ = [("elem_type", ctypes.c_int), ("order", ctypes.c_int), ("n_elem", ctypes.c_int),
                ("elem_xyz", ctypes.c_void_p), ("face_bc", ctypes.c_void_p),
                ("trace_map", ctypes.c_void_p), ("n_trace", ctypes.c_int)]


class hdg_opts(ctypes.Structure):
    _fields_ = [("chunk_elems", ctypes.c_int), ("precision", ctypes.c_int), ("flags", ctypes.c_int)]


class hdg_solve_opts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("maxit", ctypes.c_int), ("tol", ctypes.c_double),
                ("precond", ctypes.c_int), ("s_dtype", ctypes.c_int)]


class hdg_refine_opts(ctypes.Structure):
    _fields_ = [("max_outer", ctypes.c_int), ("tol", ctypes.c_double), ("reuse_points", ctypes.c_int),
                ("gmres", hdg_solve_opts)]


HDG_NEWTON_HIST = 32


class hdg_newton_opts(ctypes.Structure):
    _fields_ = [("maxit", ctypes.c_int), ("tol", ctypes.c_double), ("atol", ctypes.c_double),
                ("lin", hdg_solve_opts)]


class hdg_newton_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("lin_iterations", ctypes.c_int),
                ("lin_converged", ctypes.c_int), ("res", ctypes.c_double * HDG_NEWTON_HIST), ("ms", ctypes.c_double)]


class hdg_refine_info(ctypes.Structure):
    _fields_ = [("outer_iterations", ctypes.c_int), ("gmres_iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("total_ms", ctypes.c_double), ("gmres_ms", ctypes.c_double),
                ("history", ctypes.c_double * 16), ("fallback_elements", ctypes.c_int)]


class hdg_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("solve_ms", ctypes.c_double)]


class hdg_tuning(ctypes.Structure):
    _fields_ = [("contract_threads", ctypes.c_int), ("condense_width", ctypes.c_int),
                ("condense_width_lp", ctypes.c_int), ("condense_launches", ctypes.c_int),
                ("lu_waves", ctypes.c_int), ("lp_operands", ctypes.c_int)]


class hdg_batch_io(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("v", "q", "vhat", "u_star", "v_bc", "S", "g", "Y", "z",
                                                "elem_status")]


class hdg_dims(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("dim", "m", "Np", "nf", "Nfp", "Nq", "Nfq", "n", "k", "n_pad",
                                             "k_pad", "n_elem", "n_trace", "chunk_elems")]


P = ctypes.c_void_p
I = ctypes.c_int
SIGNATURES = {
    "hdg_plan_create": (I, [ctypes.POINTER(P), ctypes.POINTER(hdg_mesh), ctypes.POINTER(hdg_phys),
                            ctypes.POINTER(hdg_opts)]),
    "hdg_plan_destroy": (None, [P]),
    "hdg_plan_set_phys": (I, [P, ctypes.POINTER(hdg_phys)]),
    "hdg_plan_dims": (I, [P, ctypes.POINTER(hdg_dims)]),
    "hdg_plan_workspace_bytes": (I, [P, ctypes.POINTER(ctypes.c_size_t)]),
    "hdg_plan_bind_workspace": (I, [P, P, ctypes.c_size_t, P]),
    "hdg_node_coords": (I, [P, P, P, P]),
    "hdg_prepare_state": (I, [P, I, P, P, P, P, P, P]),
    "hdg_assemble": (I, [P, P, P, P, P, P, P, P, P, P, P, P, P, P]),
    "hdg_condense_blocks": (I, [P, P, P, P, P, P, P, P, P, P, P, P, P]),
    "hdg_assemble_condense": (I, [P, P, P, P, P, P, P, P, P, P, P, P, P, P]),
    "hdg_backsolve": (I, [P, P, P, P, P, P, P]),
    "hdg_trace_matvec": (I, [P, P, P, P, P]),
    "hdg_trace_rhs": (I, [P, P, P, P]),
    "hdg_solver_workspace_bytes": (I, [P, ctypes.POINTER(hdg_solve_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "hdg_precond_setup": (I, [P, P, P, ctypes.c_size_t, ctypes.POINTER(hdg_solve_opts), P]),
    "hdg_precond_apply": (I, [P, P, ctypes.c_size_t, ctypes.POINTER(hdg_solve_opts), P, P, P]),
    "hdg_trace_solve": (I, [P, P, P, P, P, ctypes.c_size_t, ctypes.POINTER(hdg_solve_opts),
                            ctypes.POINTER(hdg_solve_info), P]),
    "hdg_lp_factor_bytes": (I, [P, ctypes.POINTER(ctypes.c_size_t)]),
    "hdg_assemble_condense_lp": (I, [P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]),
    "hdg_lp_solve": (I, [P, P, P, P, P]),
    "hdg_jacobian_apply": (I, [P, P, P, P, P, P, I, P, P, P, P, P, P]),
    "hdg_refine_workspace_bytes": (I, [P, ctypes.POINTER(hdg_refine_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "hdg_backsolve_elements": (I, [P, P, P, P, P, P]),
    "hdg_refine_local_workspace_bytes": (I, [P, ctypes.POINTER(ctypes.c_size_t)]),
    "hdg_refine_local": (I, [P, P, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, I, ctypes.c_double, I,
                             ctypes.POINTER(hdg_refine_info), P, P]),
    "hdg_refine_solve": (I, [P, P, P, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_size_t,
                             ctypes.POINTER(hdg_refine_opts), ctypes.POINTER(hdg_refine_info), P, P]),
    "hdg_newton_workspace_bytes": (I, [P, ctypes.POINTER(hdg_newton_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "hdg_newton_solve": (I, [P, P, P, P, P, P, P, ctypes.c_size_t, ctypes.POINTER(hdg_newton_opts),
                             ctypes.POINTER(hdg_newton_info), P]),
    "hdg_dirk_workspace_bytes": (I, [P, ctypes.POINTER(hdg_newton_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "hdg_dirk_step": (I, [P, P, P, P, P, ctypes.c_double, P, ctypes.c_size_t, ctypes.POINTER(hdg_newton_opts),
                          ctypes.POINTER(hdg_newton_info), P]),
    "hdg_plan_set_source": (I, [P, P]),
    "hdg_plan_set_source_points": (I, [P, P]),
    "hdg_quad_coords": (I, [P, P, P]),
    "hdg_l2_error": (I, [P, I, P, P, P, P]),
    "hdg_face_quad_coords": (I, [P, P, P]),
    "hdg_trace_project": (I, [P, P, P, P]),
    "hdg_entropy_integral": (I, [P, P, P, P]),
    "hdg_flow_statistics": (I, [P, P, P, P]),
    "hdg_learn_nparams": (I, []),
    "hdg_learn_outputs": (I, []),
    "hdg_learn_extract": (I, [P, P, ctypes.c_size_t, ctypes.POINTER(hdg_solve_opts), P, P, P, I, P, I,
                              ctypes.c_size_t, ctypes.c_size_t, P, P, P, P, P]),
    "hdg_learn_forward_rows": (I, [P, P, ctypes.c_size_t, P, P]),
    "hdg_learn_rows_scratch_floats": (I, [ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "hdg_learn_backward_rows": (I, [P, P, P, ctypes.c_size_t, P, P, P]),
    "hdg_learn_pool_loss_grad": (I, [I, I, P, P, P, P, ctypes.c_size_t, I, ctypes.c_double, P, P, P]),
    "hdg_learn_setup": (I, [P, P, P, P, P, ctypes.c_size_t, ctypes.POINTER(hdg_solve_opts), P]),
    "hdg_learn_forward": (I, [P, P, P, P, P]),
    "hdg_learn_apply": (I, [P, P, P, ctypes.c_size_t, ctypes.POINTER(hdg_solve_opts), P]),
    "hdg_learn_loss_grad": (I, [P, P, ctypes.c_size_t, ctypes.POINTER(hdg_solve_opts), P, P, P, I,
                                ctypes.c_double, P, P, P]),
    "hdg_learn_scratch_floats": (I, [P, ctypes.POINTER(ctypes.c_size_t)]),
    "hdg_learn_backward": (I, [P, P, P, P, P, P, P]),
    "hdg_learn_backward_noalloc": (I, [P, P, P, P, P, P]),
    "hdg_learn_adam": (I, [P, P, P, P, I, ctypes.c_float, P]),
    "hdg_learn_train_step": (I, [P, P, P, P, I, ctypes.c_float, P, P, ctypes.c_size_t,
                                 ctypes.POINTER(hdg_solve_opts), P, P, I, ctypes.c_double, P, P, P, P, P, P]),
    "hdg_plan_set_tuning": (I, [P, ctypes.POINTER(hdg_tuning)]),
    "hdg_plan_get_tuning": (I, [P, ctypes.POINTER(hdg_tuning)]),
    "hdg_batch_create": (I, [ctypes.POINTER(P), ctypes.POINTER(P), I, I]),
    "hdg_batch_destroy": (None, [P]),
    "hdg_batch_workspace_bytes": (I, [P, ctypes.POINTER(ctypes.c_size_t)]),
    "hdg_batch_bind_workspace": (I, [P, P, ctypes.c_size_t, P]),
    "hdg_batch_set_groups": (I, [P, I]),
    "hdg_batch_set_streams": (I, [P, I]),
    "hdg_batch_set_io": (I, [P, ctypes.POINTER(hdg_batch_io), P]),
    "hdg_batch_run": (I, [P, P]),
    "hdg_batch_capture": (I, [P, P]),
    "hdg_batch_replay": (I, [P, P]),
    "hdg_batch_info": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(ctypes.c_size_t)]),
    "hdg_selftest": (I, [ctypes.POINTER(ctypes.c_double)]),
    "hdg_plan_set_timing": (I, [P, I]),
    "hdg_plan_phase_times": (I, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_long), I]),
    "hdg_status": (I, [P, P, P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "hdg_last_error": (ctypes.c_char_p, []),
}

_lib = None


def header_symbols():
    """Function names declared in include/hdg.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hdg_[a-z_]+)\s*\(", txt)))


def load():
    """Load libhdg.so; raises if it was not built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhdg.so not found at %s; build it with "
                           "`python paper_1808_05066_amd/build.py`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class HdgError(RuntimeError):
    def __init__(self, code, where):
        msg = load().hdg_last_error().decode(errors="replace")
        super().__init__("%s failed with %s: %s" % (where, ERROR_NAMES.get(code, code), msg))
        self.code = code


def check(code, where):
    if code != HDG_OK:
        raise HdgError(code, where)
