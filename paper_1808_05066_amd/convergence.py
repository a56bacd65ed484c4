"""Convergence study of the Couette flow with a source term (the Navier-Stokes convergence
example of Section 5) on the GPU path: steady Newton iterations (hdg_newton_solve) on uniform
n x n triangle meshes with the exact solution as Dirichlet data on the whole boundary, then
element L2 errors at the volume quadrature points (hdg_quad_coords, hdg_l2_error).

Reported quantities, with rho0 = V0 = L = 1: the conserved variables (rho, momentum, rho E)
and the gradient unknowns q (the entropy-variable gradients from which the stresses and heat
fluxes are formed), as L2 norms and rates log2(e_n / e_2n)."""
from __future__ import annotations

import numpy as np


def couette_run(n, p, scheme="hdg", tol=1e-9, atol=1e-10, maxit=20, lin_tol=1e-13):
    """Solve the Couette problem on an n x n mesh of order p; returns the error dict."""
    import torch

    from workloads import meshes as M
    from workloads.fields import Couette

    from .hdg import Plan

    f = Couette()
    mesh = M.tri_square(n, 0.0, 0, periodic=False)
    tmap, nt = M.trace_map(mesh, p, scheme)
    plan = Plan(mesh.etype, p, mesh.elem_xyz, tmap, nt, mesh.boundary.astype(np.int32), viscous=True,
                gamma=f.gamma, mu=f.mu, Pr=f.Pr, alpha=0.0)
    dev = plan.device
    xn, xt = (t.cpu().numpy() for t in plan.node_coords())

    def state(x, grad):
        prim, g = f.prim_and_grad(x)
        tp = torch.from_numpy(np.ascontiguousarray(prim)).to(dev)
        tg = torch.from_numpy(np.ascontiguousarray(g)).to(dev) if grad else None
        return plan.prepare_state(tp, tg, want_u=True)

    v, q, _ = state(xn, True)
    vhat, _, _ = state(xt, False)
    vbc = vhat.clone()
    plan.set_source(torch.from_numpy(np.ascontiguousarray(f.source(xn))).to(dev))
    info = plan.newton_solve(v, q, vhat, None, vbc, maxit=maxit, tol=tol, atol=atol, lin_tol=lin_tol)
    xq = plan.quad_coords().cpu().numpy()
    _, qex, uex = state(xq, True)
    eu = torch.sqrt(plan.l2_error(v, uex, "u")).cpu().numpy()
    eq = torch.sqrt(plan.l2_error(q, qex, "q")).cpu().numpy()
    return {"n": n, "p": p, "elements": mesh.n_elem, "newton_iterations": info["iterations"],
            "converged": info["converged"], "res": info["res"][-1],
            "rho": float(eu[0]), "momentum": float(np.hypot(eu[1], eu[2])), "rhoE": float(eu[3]),
            "q": float(np.sqrt(np.sum(eq ** 2)))}


def couette_table(ns=(4, 8, 16), ps=(1, 2)):
    """Errors and rates for every (p, n); rates against the next finer mesh."""
    rows = []
    for p in ps:
        prev = None
        for n in ns:
            r = couette_run(n, p)
            if prev is not None:
                for key in ("rho", "momentum", "rhoE", "q"):
                    r["rate_" + key] = float(np.log2(prev[key] / r[key]))
            rows.append(r)
            prev = r
    return rows
