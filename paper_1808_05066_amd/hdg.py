"""Thin Python binding of the C ABI.  Torch provides device memory and streams.

Every step of the hot path runs in libhdg.so; this module only allocates
tensors, passes pointers and checks return codes.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import check


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """One mesh (single element type and order) with bound device workspace.

    elem_xyz: (E, nv, d) float64 vertex coordinates; trace_map: (E, nf, Nfp)
    int32; face_bc: (E, nf) int32 (1 = Dirichlet-trace face) or None.
    """

    def __init__(self, etype, order, elem_xyz, trace_map, n_trace, face_bc=None, *, viscous=False,
                 gamma=1.4, mu=0.0, Pr=0.72, alpha=0.0, chunk_elems=0, split_dense=False, narrow_block=False,
                 eliminate_q=False, ghat_interior=False, sigma="slf", ghat_proj=False,
                 device="cuda"):
        torch = _torch()
        self.lib = _lib.load()
        self._xyz = np.ascontiguousarray(elem_xyz, dtype=np.float64)
        self._tmap = np.ascontiguousarray(trace_map, dtype=np.int32)
        self._fbc = None if face_bc is None else np.ascontiguousarray(face_bc, dtype=np.int32)
        mesh = _lib.hdg_mesh(_lib.ETYPES[etype] if isinstance(etype, str) else int(etype), int(order),
                             int(self._xyz.shape[0]), self._xyz.ctypes.data,
                             None if self._fbc is None else self._fbc.ctypes.data,
                             self._tmap.ctypes.data, int(n_trace))
        phys = _lib.hdg_phys(int(bool(viscous)), float(gamma), float(mu), float(Pr), float(alpha))
        flags = ((_lib.FLAG_SPLIT_DENSE if split_dense else 0) | (_lib.FLAG_NARROW_BLOCK if narrow_block else 0) |
                 (_lib.FLAG_ELIMINATE_Q if eliminate_q else 0) | (_lib.FLAG_GHAT_INTERIOR if ghat_interior else 0) |
                 (_lib.FLAG_SIGMA_S if sigma == "s" else 0) | (_lib.FLAG_SIGMA_MV if sigma == "mv" else 0) |
                 (_lib.FLAG_GHAT_PROJ if ghat_proj else 0))
        opts = _lib.hdg_opts(int(chunk_elems), 0, flags)
        h = ctypes.c_void_p()
        check(self.lib.hdg_plan_create(ctypes.byref(h), ctypes.byref(mesh), ctypes.byref(phys),
                                       ctypes.byref(opts)), "hdg_plan_create")
        self.h = h
        d = _lib.hdg_dims()
        check(self.lib.hdg_plan_dims(h, ctypes.byref(d)), "hdg_plan_dims")
        self.dims = {f: getattr(d, f) for f, _ in _lib.hdg_dims._fields_}
        for key, val in self.dims.items():
            setattr(self, key, val)
        self.viscous = bool(viscous)
        self.device = torch.device(device)
        nb = ctypes.c_size_t()
        check(self.lib.hdg_plan_workspace_bytes(h, ctypes.byref(nb)), "hdg_plan_workspace_bytes")
        self.workspace = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = ctypes.c_void_p(self.workspace.data_ptr() + off)
        check(self.lib.hdg_plan_bind_workspace(h, self._ws_ptr, ctypes.c_size_t(nb.value), _stream()),
              "hdg_plan_bind_workspace")

    def set_phys(self, gamma=1.4, mu=0.0, Pr=0.72, alpha=0.0):
        phys = _lib.hdg_phys(int(self.viscous), float(gamma), float(mu), float(Pr), float(alpha))
        check(self.lib.hdg_plan_set_phys(self.h, ctypes.byref(phys)), "hdg_plan_set_phys")

    def tuning(self):
        t = _lib.hdg_tuning()
        check(self.lib.hdg_plan_get_tuning(self.h, ctypes.byref(t)), "hdg_plan_get_tuning")
        return {f: getattr(t, f) for f, _ in _lib.hdg_tuning._fields_}

    def set_tuning(self, contract_threads=0, condense_width=0, condense_width_lp=0, condense_launches=0,
                   lu_waves=0, lp_operands=0):
        t = _lib.hdg_tuning(int(contract_threads), int(condense_width), int(condense_width_lp),
                            int(condense_launches), int(lu_waves), int(lp_operands))
        check(self.lib.hdg_plan_set_tuning(self.h, ctypes.byref(t)), "hdg_plan_set_tuning")

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.hdg_plan_destroy(h)
            self.h = None

    # -- helpers -------------------------------------------------------------
    def _empty(self, *shape, dtype=None):
        torch = _torch()
        return torch.empty(*shape, dtype=torch.float64 if dtype is None else dtype, device=self.device)

    @property
    def n_nodes(self):
        return self.n_elem * self.Np

    def node_coords(self):
        x = self._empty(self.dim, self.n_nodes)
        xt = self._empty(self.dim, self.n_trace)
        check(self.lib.hdg_node_coords(self.h, _ptr(x), _ptr(xt), _stream()), "hdg_node_coords")
        return x, xt

    def prepare_state(self, prim, grad=None, want_u=False):
        N = prim.shape[1]
        v = self._empty(self.m, N)
        q = self._empty(self.m * self.dim, N) if grad is not None else None
        u = self._empty(self.m, N) if want_u else None
        check(self.lib.hdg_prepare_state(self.h, N, _ptr(prim), _ptr(grad), _ptr(v), _ptr(q), _ptr(u),
                                         _stream()), "hdg_prepare_state")
        return v, q, u

    def assemble(self, v, q, vhat, ustar=None, vbc=None):
        E, n, k = self.n_elem, self.n, self.k
        out = dict(A=self._empty(E, n, n), B=self._empty(E, k, n), C=self._empty(E, n, k),
                   D=self._empty(E, k, k), R_loc=self._empty(E, n), R_tr=self._empty(E, k))
        torch = _torch()
        status = torch.empty(E, dtype=torch.int32, device=self.device)
        check(self.lib.hdg_assemble(self.h, _ptr(v), _ptr(q), _ptr(vhat), _ptr(ustar), _ptr(vbc),
                                    _ptr(out["A"]), _ptr(out["B"]), _ptr(out["C"]), _ptr(out["D"]),
                                    _ptr(out["R_loc"]), _ptr(out["R_tr"]), _ptr(status), _stream()),
              "hdg_assemble")
        out["status"] = status
        return out

    def alloc_outputs(self, residuals=False):
        """Output tensors of assemble_condense (column-major blocks as (E, cols, rows))."""
        torch = _torch()
        E, n, k = self.n_elem, self.n, self.k
        out = dict(S=self._empty(E, k, k), g=self._empty(E, k), Y=self._empty(E, k, n), z=self._empty(E, n),
                   status=torch.empty(E, dtype=torch.int32, device=self.device))
        if residuals:
            out["R_loc"] = self._empty(E, n)
            out["R_tr"] = self._empty(E, k)
        return out

    def assemble_condense(self, v, q, vhat, ustar=None, vbc=None, out=None, residuals=False):
        if out is None:
            out = self.alloc_outputs(residuals)
        check(self.lib.hdg_assemble_condense(
            self.h, _ptr(v), _ptr(q), _ptr(vhat), _ptr(ustar), _ptr(vbc), _ptr(out["S"]), _ptr(out["g"]),
            _ptr(out["Y"]), _ptr(out["z"]), _ptr(out.get("R_loc")), _ptr(out.get("R_tr")), _ptr(out["status"]),
            _stream()), "hdg_assemble_condense")
        return out

    def condense_blocks(self, blocks, out=None):
        """Condensation of caller blocks (dict with A, B, C, D, R_loc, R_tr in the layout of
        assemble()) with the hot path's kernels (hdg_condense_blocks)."""
        if out is None:
            out = self.alloc_outputs()
        check(self.lib.hdg_condense_blocks(self.h, *(_ptr(blocks[key]) for key in ("A", "B", "C", "D", "R_loc", "R_tr")),
                                           _ptr(out["S"]), _ptr(out["g"]), _ptr(out["Y"]), _ptr(out["z"]),
                                           _ptr(out["status"]), _stream()), "hdg_condense_blocks")
        return out

    def backsolve(self, Y, z, dvhat, dv=None, dq=None):
        if dv is None:
            dv = self._empty(self.m, self.n_nodes)
        if dq is None and self.viscous:
            dq = self._empty(self.m * self.dim, self.n_nodes)
        check(self.lib.hdg_backsolve(self.h, _ptr(Y), _ptr(z), _ptr(dvhat), _ptr(dv), _ptr(dq), _stream()),
              "hdg_backsolve")
        return dv, dq

    def trace_matvec(self, S, x, y=None):
        if y is None:
            y = self._empty(self.m, self.n_trace)
        check(self.lib.hdg_trace_matvec(self.h, _ptr(S), _ptr(x), _ptr(y), _stream()), "hdg_trace_matvec")
        return y

    def set_timing(self, enable=True):
        check(self.lib.hdg_plan_set_timing(self.h, int(bool(enable))), "hdg_plan_set_timing")

    def phase_times(self):
        """{phase: (total ms, calls)} accumulated since timing was enabled."""
        n = len(_lib.PHASES)
        ms = (ctypes.c_double * n)()
        calls = (ctypes.c_long * n)()
        check(self.lib.hdg_plan_phase_times(self.h, ms, calls, n), "hdg_plan_phase_times")
        return {name: (ms[i], calls[i]) for i, name in enumerate(_lib.PHASES)}

    def status(self, elem_status):
        """(first element whose status is not HDG_OK, its code), (-1, 0) if none; synchronizes."""
        first, code = ctypes.c_int(), ctypes.c_int()
        check(self.lib.hdg_status(self.h, ctypes.c_void_p(elem_status.data_ptr()), _stream(), ctypes.byref(first),
                                  ctypes.byref(code)), "hdg_status")
        return first.value, code.value

    # -- mixed precision -----------------------------------------------------
    def lp_factor_bytes(self):
        nb = ctypes.c_size_t()
        check(self.lib.hdg_lp_factor_bytes(self.h, ctypes.byref(nb)), "hdg_lp_factor_bytes")
        return int(nb.value)

    def alloc_outputs_lp(self, residuals=True):
        """Outputs of assemble_condense_lp: FP32 S, Y; FP64 g, z; FP32 factor records."""
        torch = _torch()
        E, n, k = self.n_elem, self.n, self.k
        f32 = torch.float32
        out = dict(S=self._empty(E, k, k, dtype=f32), g=self._empty(E, k), Y=self._empty(E, k, n, dtype=f32),
                   z=self._empty(E, n), factors=self._empty(self.lp_factor_bytes() // 4, dtype=f32),
                   status=torch.empty(E, dtype=torch.int32, device=self.device))
        if residuals:
            out["R_loc"] = self._empty(E, n)
            out["R_tr"] = self._empty(E, k)
        return out

    def assemble_condense_lp(self, v, q, vhat, ustar=None, vbc=None, out=None, residuals=True):
        if out is None:
            out = self.alloc_outputs_lp(residuals)
        check(self.lib.hdg_assemble_condense_lp(
            self.h, _ptr(v), _ptr(q), _ptr(vhat), _ptr(ustar), _ptr(vbc), _ptr(out["S"]), _ptr(out["g"]),
            _ptr(out["Y"]), _ptr(out["z"]), _ptr(out["factors"]), _ptr(out.get("R_loc")), _ptr(out.get("R_tr")),
            _ptr(out["status"]), _stream()), "hdg_assemble_condense_lp")
        return out

    def lp_solve(self, factors, r, x=None):
        if x is None:
            x = self._empty(self.n_elem, self.n)
        check(self.lib.hdg_lp_solve(self.h, _ptr(factors), _ptr(r), _ptr(x), _stream()), "hdg_lp_solve")
        return x

    def jacobian_apply(self, v, q, vhat, dx, dlam, ustar=None, vbc=None, reuse_points=False, y_loc=None,
                       y_tr=None, status=None):
        torch = _torch()
        if y_loc is None:
            y_loc = self._empty(self.n_elem, self.n)
        if y_tr is None:
            y_tr = self._empty(self.n_elem, self.k)
        if status is None:
            status = torch.zeros(self.n_elem, dtype=torch.int32, device=self.device)
        check(self.lib.hdg_jacobian_apply(self.h, _ptr(v), _ptr(q), _ptr(vhat), _ptr(ustar), _ptr(vbc),
                                          int(bool(reuse_points)), _ptr(dx), _ptr(dlam), _ptr(y_loc), _ptr(y_tr),
                                          _ptr(status), _stream()), "hdg_jacobian_apply")
        return y_loc, y_tr

    def refine_solve(self, v, q, vhat, lp, ustar=None, vbc=None, tol=1e-10, max_outer=10, reuse_points=False,
                     gmres_restart=50, gmres_maxit=2000, gmres_tol=1e-6, precond="block_jacobi"):
        """Outer FP64 refinement of the full Newton system with the low-precision outputs `lp`.

        Returns (dx [E][n], dlam [m][n_trace], info dict)."""
        torch = _torch()
        go = _lib.hdg_solve_opts(int(gmres_restart), int(gmres_maxit), float(gmres_tol),
                                 TraceSolver.PRECONDS[precond], _lib.HDG_FP32)
        opts = _lib.hdg_refine_opts(int(max_outer), float(tol), int(bool(reuse_points)), go)
        nb = ctypes.c_size_t()
        check(self.lib.hdg_refine_workspace_bytes(self.h, ctypes.byref(opts), ctypes.byref(nb)),
              "hdg_refine_workspace_bytes")
        work = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        wp = ctypes.c_void_p(work.data_ptr() + (-work.data_ptr()) % 256)
        dx = self._empty(self.n_elem, self.n)
        dlam = self._empty(self.m, self.n_trace)
        info = _lib.hdg_refine_info()
        status = torch.zeros(self.n_elem, dtype=torch.int32, device=self.device)
        check(self.lib.hdg_refine_solve(self.h, _ptr(v), _ptr(q), _ptr(vhat), _ptr(ustar), _ptr(vbc), _ptr(lp["S"]),
                                        _ptr(lp["Y"]), _ptr(lp["factors"]), _ptr(lp["R_loc"]), _ptr(lp["R_tr"]),
                                        _ptr(dx), _ptr(dlam), wp, ctypes.c_size_t(nb.value), ctypes.byref(opts),
                                        ctypes.byref(info), _ptr(status), _stream()), "hdg_refine_solve")
        res = {f: getattr(info, f) for f, _ in _lib.hdg_refine_info._fields_ if f != "history"}
        res["history"] = [info.history[i] for i in range(min(16, info.outer_iterations))]
        return dx, dlam, res

    def backsolve_elements(self, Y, z, dvhat, dx=None):
        """dx [E][n] = -z - Y P dvhat in the element-local ordering (FP64 Y, z)."""
        if dx is None:
            dx = self._empty(self.n_elem, self.n)
        check(self.lib.hdg_backsolve_elements(self.h, _ptr(Y), _ptr(z), _ptr(dvhat), _ptr(dx), _stream()),
              "hdg_backsolve_elements")
        return dx

    def refine_local(self, v, q, vhat, lp, dvhat, ustar=None, vbc=None, tol=1e-10, max_iter=10,
                     reuse_points=False):
        """Element-level refinement A dx = -(R_loc + B P dvhat) with the low-precision factors of
        `lp` (hdg_refine_local).  Returns (dx [E][n], info dict)."""
        torch = _torch()
        nb = ctypes.c_size_t()
        check(self.lib.hdg_refine_local_workspace_bytes(self.h, ctypes.byref(nb)), "hdg_refine_local_workspace_bytes")
        work = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        wp = ctypes.c_void_p(work.data_ptr() + (-work.data_ptr()) % 256)
        dx = self._empty(self.n_elem, self.n)
        info = _lib.hdg_refine_info()
        status = torch.zeros(self.n_elem, dtype=torch.int32, device=self.device)
        check(self.lib.hdg_refine_local(self.h, _ptr(v), _ptr(q), _ptr(vhat), _ptr(ustar), _ptr(vbc),
                                        _ptr(lp["factors"]), _ptr(lp["R_loc"]), _ptr(dvhat), _ptr(dx), wp,
                                        ctypes.c_size_t(nb.value), int(max_iter), float(tol), int(bool(reuse_points)),
                                        ctypes.byref(info), _ptr(status), _stream()), "hdg_refine_local")
        res = {f: getattr(info, f) for f, _ in _lib.hdg_refine_info._fields_ if f != "history"}
        res["history"] = [info.history[i] for i in range(min(16, info.outer_iterations))]
        return dx, res

    def newton_solve(self, v, q, vhat, ustar=None, vbc=None, maxit=10, tol=1e-10, atol=0.0, lin_tol=1e-12,
                     lin_restart=50, lin_maxit=2000, precond="block_jacobi"):
        """Newton iterations on the nonlinear system (hdg_newton_solve): v, q, vhat updated in
        place.  Returns the info as a dict (residual history in "res")."""
        torch = _torch()
        lo = _lib.hdg_solve_opts(int(lin_restart), int(lin_maxit), float(lin_tol), TraceSolver.PRECONDS[precond],
                                 _lib.HDG_FP64)
        opts = _lib.hdg_newton_opts(int(maxit), float(tol), float(atol), lo)
        nb = ctypes.c_size_t()
        check(self.lib.hdg_newton_workspace_bytes(self.h, ctypes.byref(opts), ctypes.byref(nb)),
              "hdg_newton_workspace_bytes")
        work = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        wp = ctypes.c_void_p(work.data_ptr() + (-work.data_ptr()) % 256)
        info = _lib.hdg_newton_info()
        check(self.lib.hdg_newton_solve(self.h, _ptr(v), _ptr(q), _ptr(vhat), _ptr(ustar), _ptr(vbc), wp,
                                        ctypes.c_size_t(nb.value), ctypes.byref(opts), ctypes.byref(info),
                                        _stream()), "hdg_newton_solve")
        res = {f: getattr(info, f) for f, _ in _lib.hdg_newton_info._fields_ if f != "res"}
        res["res"] = [info.res[i] for i in range(min(_lib.HDG_NEWTON_HIST, info.iterations + 1))]
        return res

    def dirk_step(self, v, q, vhat, dt, vbc=None, maxit=10, tol=1e-10, atol=0.0, lin_tol=1e-12, lin_restart=50,
                  lin_maxit=2000, precond="block_jacobi"):
        """One DIRK(3,3) step (hdg_dirk_step): v, q, vhat replaced in place by the step's end state;
        sets the plan's alpha to 1/(a_ii dt).  Returns one info dict per stage."""
        torch = _torch()
        lo = _lib.hdg_solve_opts(int(lin_restart), int(lin_maxit), float(lin_tol), TraceSolver.PRECONDS[precond],
                                 _lib.HDG_FP64)
        opts = _lib.hdg_newton_opts(int(maxit), float(tol), float(atol), lo)
        nb = ctypes.c_size_t()
        check(self.lib.hdg_dirk_workspace_bytes(self.h, ctypes.byref(opts), ctypes.byref(nb)),
              "hdg_dirk_workspace_bytes")
        work = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        wp = ctypes.c_void_p(work.data_ptr() + (-work.data_ptr()) % 256)
        infos = (_lib.hdg_newton_info * 3)()
        check(self.lib.hdg_dirk_step(self.h, _ptr(v), _ptr(q), _ptr(vhat), _ptr(vbc), ctypes.c_double(dt), wp,
                                     ctypes.c_size_t(nb.value), ctypes.byref(opts), infos, _stream()),
              "hdg_dirk_step")
        out = []
        for info in infos:
            res = {f: getattr(info, f) for f, _ in _lib.hdg_newton_info._fields_ if f != "res"}
            res["res"] = [info.res[i] for i in range(min(_lib.HDG_NEWTON_HIST, info.iterations + 1))]
            out.append(res)
        return out

    def set_source(self, src):
        """Nodal source [m][E*Np] of the conservation law (a device tensor kept alive by the
        plan), or None to remove it."""
        self._src = src
        check(self.lib.hdg_plan_set_source(self.h, _ptr(src)), "hdg_plan_set_source")

    def set_source_points(self, src):
        """Source [m][E*Nq] at the volume quadrature points (quad_coords order), a device tensor
        kept alive by the plan, or None to remove it."""
        self._src = src
        check(self.lib.hdg_plan_set_source_points(self.h, _ptr(src)), "hdg_plan_set_source_points")

    def quad_coords(self):
        """Physical coordinates of the volume quadrature points [dim][E*Nq]."""
        xq = self._empty(self.dim, self.n_elem * self.Nq)
        check(self.lib.hdg_quad_coords(self.h, _ptr(xq), _stream()), "hdg_quad_coords")
        return xq

    def face_quad_coords(self):
        """Physical coordinates of the face quadrature points [dim][E*nf*Nfq]."""
        xf = self._empty(self.dim, self.n_elem * self.nf * self.Nfq)
        check(self.lib.hdg_face_quad_coords(self.h, _ptr(xf), _stream()), "hdg_face_quad_coords")
        return xf

    def trace_project(self, g, vbc):
        """Face L2 projection of Dirichlet data g [m][E*nf*Nfq] (entropy variables at the face
        quadrature points) into the Dirichlet faces' nodes of vbc [m][n_trace] (in place)."""
        check(self.lib.hdg_trace_project(self.h, _ptr(g), _ptr(vbc), _stream()), "hdg_trace_project")
        return vbc

    def l2_error(self, f, exact, kind="u"):
        """Per-component squared L2 errors summed over the elements (hdg_l2_error): kind "u"
        compares u(v_h) from v with exact conserved variables, kind "q" the gradient unknowns,
        kind "v" the entropy variables, kind "stress" the viscous stress and heat flux formed
        from f = [v; q] stacked against exact = [v; q] stacked at the quadrature points."""
        k = {"u": 0, "q": 1, "v": 2, "stress": 3}[kind]
        nc = self.m * self.dim if k == 1 else (self.dim * self.dim + self.dim if k == 3 else self.m)
        out = self._empty(self.n_elem, nc)
        check(self.lib.hdg_l2_error(self.h, k, _ptr(f), _ptr(exact), _ptr(out), _stream()), "hdg_l2_error")
        return out.sum(dim=0)

    def entropy_integral(self, v):
        """Per-element (int_K rho s, int_K rho), s = ln(p / rho^gamma), as [E][2]
        (hdg_entropy_integral)."""
        out = self._empty(self.n_elem, 2)
        check(self.lib.hdg_entropy_integral(self.h, _ptr(v), _ptr(out), _stream()), "hdg_entropy_integral")
        return out

    def flow_statistics(self, v):
        """Per-element integrals [E][8] of (rho s, rho, rho |V|^2 / 2, |omega|^2, theta,
        theta^2, T, T^2) (hdg_flow_statistics)."""
        out = self._empty(self.n_elem, 8)
        check(self.lib.hdg_flow_statistics(self.h, _ptr(v), _ptr(out), _stream()), "hdg_flow_statistics")
        return out

    def trace_rhs(self, g, r=None):
        if r is None:
            r = self._empty(self.m, self.n_trace)
        check(self.lib.hdg_trace_rhs(self.h, _ptr(g), _ptr(r), _stream()), "hdg_trace_rhs")
        return r


class TraceSolver:
    """Restarted GMRES on the condensed trace system of one plan.

    precond: "none" or "block_jacobi".  setup(S) builds the preconditioner
    from the Schur blocks; solve(S, rhs) returns (x, info dict).
    """

    PRECONDS = {"none": 0, "block_jacobi": 1}

    def __init__(self, plan, restart=50, maxit=2000, tol=1e-10, precond="block_jacobi", s_dtype="fp64"):
        torch = _torch()
        self.plan = plan
        self.opts = _lib.hdg_solve_opts(int(restart), int(maxit), float(tol), self.PRECONDS[precond],
                                        {"fp64": _lib.HDG_FP64, "fp32": _lib.HDG_FP32}[s_dtype])
        nb = ctypes.c_size_t()
        check(plan.lib.hdg_solver_workspace_bytes(plan.h, ctypes.byref(self.opts), ctypes.byref(nb)),
              "hdg_solver_workspace_bytes")
        self.nbytes = int(nb.value)
        self.workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=plan.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ptr = ctypes.c_void_p(self.workspace.data_ptr() + off)

    def setup(self, S):
        if self.opts.precond:
            check(self.plan.lib.hdg_precond_setup(self.plan.h, _ptr(S), self._ptr, ctypes.c_size_t(self.nbytes),
                                                  ctypes.byref(self.opts), _stream()), "hdg_precond_setup")

    def apply(self, r, z=None):
        if z is None:
            z = self.plan._empty(self.plan.m, self.plan.n_trace)
        check(self.plan.lib.hdg_precond_apply(self.plan.h, self._ptr, ctypes.c_size_t(self.nbytes),
                                              ctypes.byref(self.opts), _ptr(r), _ptr(z), _stream()),
              "hdg_precond_apply")
        return z

    def solve(self, S, rhs, x=None):
        if x is None:
            x = self.plan._empty(self.plan.m, self.plan.n_trace)
        info = _lib.hdg_solve_info()
        check(self.plan.lib.hdg_trace_solve(self.plan.h, _ptr(S), _ptr(rhs), _ptr(x), self._ptr,
                                            ctypes.c_size_t(self.nbytes), ctypes.byref(self.opts),
                                            ctypes.byref(info), _stream()), "hdg_trace_solve")
        return x, {f: getattr(info, f) for f, _ in _lib.hdg_solve_info._fields_}


class LearnedPrecond:
    """Learned rescaling of the block-Jacobi inverses of one TraceSolver (see include/hdg.h).

    setup(S, vhat) computes the features and the plain block-Jacobi inverses;
    apply(theta) rescales the inverses with the network's outputs, after which
    the solver's preconditioner is the learned one.  train_step() runs one Adam
    step of the network on (X, W = K X) with the unscaled inverses.
    """

    def __init__(self, solver):
        torch = _torch()
        self.ts = solver
        self.plan = solver.plan
        lib = self.plan.lib
        self.nparams = lib.hdg_learn_nparams()
        self.no = lib.hdg_learn_outputs()
        self.N = self.plan.m * self.plan.n_trace
        dev = self.plan.device
        self.feat = torch.empty(self.N, 16, dtype=torch.float32, device=dev)
        self.out = torch.zeros(self.N, self.no, dtype=torch.float32, device=dev)
        self.dO = torch.empty(self.N, self.no, dtype=torch.float32, device=dev)
        self.grad = torch.empty(self.nparams, dtype=torch.float32, device=dev)
        n = ctypes.c_size_t()
        check(lib.hdg_learn_scratch_floats(self.plan.h, ctypes.byref(n)), "hdg_learn_scratch_floats")
        self.scratch = torch.empty(int(n.value), dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)

    def _w(self):
        return self.ts._ptr, ctypes.c_size_t(self.ts.nbytes), ctypes.byref(self.ts.opts)

    def setup(self, S, vhat):
        w, nb, op = self._w()
        check(self.plan.lib.hdg_learn_setup(self.plan.h, _ptr(S), _ptr(vhat), _ptr(self.feat), w, nb, op,
                                            _stream()), "hdg_learn_setup")

    def forward(self, theta):
        check(self.plan.lib.hdg_learn_forward(self.plan.h, _ptr(theta), _ptr(self.feat), _ptr(self.out),
                                              _stream()), "hdg_learn_forward")
        return self.out

    def apply(self, theta):
        self.forward(theta)
        w, nb, op = self._w()
        check(self.plan.lib.hdg_learn_apply(self.plan.h, _ptr(self.out), w, nb, op, _stream()), "hdg_learn_apply")

    def loss_grad(self, X, Wv, out=None):
        out = self.out if out is None else out
        w, nb, op = self._w()
        x2 = float((X * X).sum())
        check(self.plan.lib.hdg_learn_loss_grad(self.plan.h, w, nb, op, _ptr(out), _ptr(X), _ptr(Wv), X.shape[0],
                                                x2, _ptr(self.dO), _ptr(self.loss), _stream()),
              "hdg_learn_loss_grad")
        return self.loss, self.dO

    def backward(self, theta, dO=None):
        dO = self.dO if dO is None else dO
        check(self.plan.lib.hdg_learn_backward(self.plan.h, _ptr(theta), _ptr(self.feat), _ptr(dO),
                                               _ptr(self.grad), _ptr(self.scratch), _stream()), "hdg_learn_backward")
        return self.grad

    def backward_noalloc(self, theta, dO=None, grad=None):
        """backward() through hdg_learn_backward_noalloc (no scratch argument)."""
        dO = self.dO if dO is None else dO
        grad = self.grad if grad is None else grad
        check(self.plan.lib.hdg_learn_backward_noalloc(self.plan.h, _ptr(theta), _ptr(self.feat), _ptr(dO),
                                                       _ptr(grad), _stream()), "hdg_learn_backward_noalloc")
        return grad

    def extract(self, X, Wv, sel, pool, b0):
        """Blocks sel (device int32) of this system into pool (a LearnPool) from block b0 on."""
        w, nb, op = self._w()
        check(self.plan.lib.hdg_learn_extract(self.plan.h, w, nb, op, _ptr(self.feat), _ptr(X), _ptr(Wv), X.shape[0],
                                              _ptr(sel), int(sel.numel()), int(b0), int(pool.ld), _ptr(pool.B),
                                              _ptr(pool.feat), _ptr(pool.X), _ptr(pool.W), _stream()),
              "hdg_learn_extract")

    def train_step(self, theta, m, v, t, lr, X, Wv, x2):
        w, nb, op = self._w()
        check(self.plan.lib.hdg_learn_train_step(self.plan.h, _ptr(theta), _ptr(m), _ptr(v), int(t),
                                                 ctypes.c_float(lr), _ptr(self.feat), w, nb, op, _ptr(X), _ptr(Wv),
                                                 X.shape[0], float(x2), _ptr(self.out), _ptr(self.dO),
                                                 _ptr(self.grad), _ptr(self.scratch), _ptr(self.loss), _stream()),
              "hdg_learn_train_step")
        return self.loss


class LearnPool:
    """Face blocks sampled from many systems for training the learned correction (caller-owned
    device arrays of the library's pool layout; see hdg_learn_extract in include/hdg.h)."""

    def __init__(self, capacity, bs, nvec, device="cuda"):
        torch = _torch()
        lib = _lib.load()
        self.lib, self.cap, self.bs, self.nvec = lib, int(capacity), int(bs), int(nvec)
        self.no, self.nparams = lib.hdg_learn_outputs(), lib.hdg_learn_nparams()
        self.ld = self.cap * self.bs
        self.n = 0                                    # blocks filled
        self.B = torch.empty(self.cap, bs, bs, dtype=torch.float64, device=device)
        self.feat = torch.empty(self.ld, 16, dtype=torch.float32, device=device)
        self.X = torch.empty(nvec, self.ld, dtype=torch.float64, device=device)
        self.W = torch.empty(nvec, self.ld, dtype=torch.float64, device=device)
        self.out = torch.zeros(self.ld, self.no, dtype=torch.float32, device=device)
        self.dO = torch.empty(self.ld, self.no, dtype=torch.float32, device=device)
        self.grad = torch.empty(self.nparams, dtype=torch.float32, device=device)
        n = ctypes.c_size_t()
        check(lib.hdg_learn_rows_scratch_floats(self.ld, ctypes.byref(n)), "hdg_learn_rows_scratch_floats")
        self.scratch = torch.empty(int(n.value), dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)

    def add(self, lp, X, Wv, sel):
        """Append blocks sel of the system behind LearnedPrecond lp (after lp.setup)."""
        k = int(sel.numel())
        if self.n + k > self.cap:
            raise ValueError("pool full")
        lp.extract(X, Wv, sel, self, self.n)
        self.n += k

    def _rows(self, b0, nb):
        return b0 * self.bs, nb * self.bs

    def loss_grad(self, theta, b0, nb):
        """Forward, loss and dL/do over pool blocks b0 .. b0 + nb - 1; returns the loss tensor."""
        r0, nr = self._rows(b0, nb)
        feat, out, dO = self.feat[r0:r0 + nr], self.out[r0:r0 + nr], self.dO[r0:r0 + nr]
        X, W = self.X[:, r0:], self.W[:, r0:]
        x2 = float((self.X[:, r0:r0 + nr] ** 2).sum())
        check(self.lib.hdg_learn_forward_rows(_ptr(theta), _ptr(feat), nr, _ptr(out), _stream()),
              "hdg_learn_forward_rows")
        check(self.lib.hdg_learn_pool_loss_grad(nb, self.bs, _ptr(self.B[b0]), _ptr(out), _ptr(X), _ptr(W),
                                                self.ld, self.nvec, x2, _ptr(dO), _ptr(self.loss), _stream()),
              "hdg_learn_pool_loss_grad")
        return self.loss

    def train_step(self, theta, m, v, t, lr, b0, nb):
        """One Adam step on pool blocks b0 .. b0 + nb - 1; returns the loss before the step."""
        loss = self.loss_grad(theta, b0, nb).clone()
        r0, nr = self._rows(b0, nb)
        check(self.lib.hdg_learn_backward_rows(_ptr(theta), _ptr(self.feat[r0:r0 + nr]), _ptr(self.dO[r0:r0 + nr]),
                                               nr, _ptr(self.grad), _ptr(self.scratch), _stream()),
              "hdg_learn_backward_rows")
        adam(theta, self.grad, m, v, t, lr)
        return loss


def adam(theta, grad, m, v, t, lr):
    """One device Adam step (the library's kernel)."""
    lib = _lib.load()
    check(lib.hdg_learn_adam(_ptr(theta), _ptr(grad), _ptr(m), _ptr(v), int(t), ctypes.c_float(lr), _stream()),
          "hdg_learn_adam")


class Batch:
    """Condensation of several plans in two launches (LU items, then right-hand-side items),
    optionally replayed from a hipGraph.

    io: list (one per plan) of dicts with v, q, vhat, ustar, vbc and outputs S, g, Y, z, status.
    order: "lpt" (largest blocks first) or "plan".
    """

    def __init__(self, plans, order="lpt"):
        torch = _torch()
        self.lib = _lib.load()
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.h.value for p in self.plans])
        h = ctypes.c_void_p()
        check(self.lib.hdg_batch_create(ctypes.byref(h), arr, len(self.plans), 0 if order == "lpt" else 1),
              "hdg_batch_create")
        self.h = h
        nb = ctypes.c_size_t()
        check(self.lib.hdg_batch_workspace_bytes(h, ctypes.byref(nb)), "hdg_batch_workspace_bytes")
        self.workspace = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.plans[0].device)
        ptr = ctypes.c_void_p(self.workspace.data_ptr() + (-self.workspace.data_ptr()) % 256)
        check(self.lib.hdg_batch_bind_workspace(h, ptr, ctypes.c_size_t(nb.value), _stream()),
              "hdg_batch_bind_workspace")
        self._io = None

    def info(self):
        n, g, lds = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        check(self.lib.hdg_batch_info(self.h, ctypes.byref(n), ctypes.byref(g), ctypes.byref(lds)), "hdg_batch_info")
        return {"items": n.value, "groups": g.value, "lds_bytes": lds.value}

    def set_groups(self, groups):
        """0 (default): one workgroup per item; > 0: a persistent grid of that many workgroups."""
        check(self.lib.hdg_batch_set_groups(self.h, int(groups)), "hdg_batch_set_groups")

    def set_streams(self, n):
        """n >= 1: every plan's own assemble + condense on n concurrent streams; 0: item lists."""
        check(self.lib.hdg_batch_set_streams(self.h, int(n)), "hdg_batch_set_streams")

    def set_io(self, io):
        arr = (_lib.hdg_batch_io * len(io))()
        for i, d in enumerate(io):
            arr[i] = _lib.hdg_batch_io(*[None if d.get(k) is None else d[k].data_ptr()
                                         for k in ("v", "q", "vhat", "ustar", "vbc", "S", "g", "Y", "z",
                                                   "status")])
        self._io = io
        check(self.lib.hdg_batch_set_io(self.h, arr, _stream()), "hdg_batch_set_io")

    def run(self):
        check(self.lib.hdg_batch_run(self.h, _stream()), "hdg_batch_run")

    def capture(self):
        """Capture on a stream of its own (the default stream cannot be captured)."""
        torch = _torch()
        self._gstream = torch.cuda.Stream()
        self._gstream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self._gstream):
            check(self.lib.hdg_batch_capture(self.h, _stream()), "hdg_batch_capture")
        torch.cuda.current_stream().wait_stream(self._gstream)

    def replay(self):
        torch = _torch()
        s = self._gstream
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            check(self.lib.hdg_batch_replay(self.h, _stream()), "hdg_batch_replay")
        torch.cuda.current_stream().wait_stream(s)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.hdg_batch_destroy(h)
            self.h = None


def selftest():
    """Largest error of the device matrix-core layout self-check."""
    lib = _lib.load()
    e = ctypes.c_double(-1.0)
    check(lib.hdg_selftest(ctypes.byref(e)), "hdg_selftest")
    return e.value
