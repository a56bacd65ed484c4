"""Convergence studies of Section 5 on the GPU path: steady Newton iterations
(hdg_newton_solve) on uniform n x n squares split into 2 n^2 triangles, the exact solution
as Dirichlet data on the whole boundary, then element L2 errors at the volume quadrature
points (hdg_quad_coords, hdg_l2_error).

* Couette flow with a source term (Navier-Stokes, Table 6): reported as the table reports it,
  with rho0 = V0 = L = 1: the conserved variables (rho, momentum, rho E) and the stress and heat
  flux formed from v_h and q_h (tau* = tau / mu, f* = f / mu), besides the raw gradient
  unknowns q.  The Dirichlet data is the exact solution tested on each boundary face (its face
  L2 projection, hdg_trace_project) and the source is evaluated at the volume quadrature points;
  bc="nodal" takes the nodal interpolants of both instead.
* Ringleb flow (Euler, Tables 3-5): the square (-5, -1) x (1, 5), h = 4 / n, the
  [L2(Omega)]^m norm of the error in the conserved variables, for HDG, IEDG and EDG traces.

Rates are log2(e_n / e_2n)."""
from __future__ import annotations

import numpy as np


def couette_run(n, p, scheme="hdg", tol=1e-9, atol=1e-10, maxit=20, lin_tol=1e-13, ghat_proj=False,
                bc="projection"):
    """Solve the Couette problem on an n x n mesh of order p; returns the error dict."""
    import torch

    from workloads import meshes as M
    from workloads.fields import Couette

    from .hdg import Plan

    f = Couette()
    mesh = M.tri_square(n, 0.0, 0, periodic=False)
    tmap, nt = M.trace_map(mesh, p, scheme)
    plan = Plan(mesh.etype, p, mesh.elem_xyz, tmap, nt, mesh.boundary.astype(np.int32), viscous=True,
                gamma=f.gamma, mu=f.mu, Pr=f.Pr, alpha=0.0, ghat_proj=ghat_proj)
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
    if bc == "projection":
        gf, _, _ = state(plan.face_quad_coords().cpu().numpy(), False)
        plan.trace_project(gf, vbc)
        vhat = vbc.clone()
    xq = plan.quad_coords().cpu().numpy()
    if bc == "projection":
        plan.set_source_points(torch.from_numpy(np.ascontiguousarray(f.source(xq))).to(dev))
    else:
        plan.set_source(torch.from_numpy(np.ascontiguousarray(f.source(xn))).to(dev))
    info = plan.newton_solve(v, q, vhat, None, vbc, maxit=maxit, tol=tol, atol=atol, lin_tol=lin_tol)
    vex, qex, uex = state(xq, True)
    eu = torch.sqrt(plan.l2_error(v, uex, "u")).cpu().numpy()
    eq = torch.sqrt(plan.l2_error(q, qex, "q")).cpu().numpy()
    es = plan.l2_error(torch.cat([v, q]), torch.cat([vex, qex]), "stress").cpu().numpy()
    d = 2
    return {"n": n, "p": p, "bc": bc, "elements": mesh.n_elem, "newton_iterations": info["iterations"],
            "converged": info["converged"], "res": info["res"][-1],
            "rho": float(eu[0]), "momentum": float(np.hypot(eu[1], eu[2])), "rhoE": float(eu[3]),
            "tau": float(np.sqrt(es[:d * d].sum())) / f.mu, "f": float(np.sqrt(es[d * d:].sum())) / f.mu,
            "q": float(np.sqrt(np.sum(eq ** 2)))}


COUETTE_KEYS = ("rho", "momentum", "rhoE", "tau", "f", "q")


def couette_table(ns=(4, 8, 16), ps=(1, 2), scheme="hdg", ghat_proj=False, bc="projection"):
    """Errors and rates for every (p, n); rates against the next finer mesh."""
    rows = []
    for p in ps:
        prev = None
        for n in ns:
            r = couette_run(n, p, scheme, ghat_proj=ghat_proj, bc=bc)
            r["scheme"] = scheme
            r["ghat_proj"] = ghat_proj
            if prev is not None:
                for key in COUETTE_KEYS:
                    r["rate_" + key] = float(np.log2(prev[key] / r[key]))
            rows.append(r)
            prev = r
    return rows


def ringleb_run(n, p, scheme="hdg", tol=1e-10, atol=1e-13, maxit=20, lin_tol=1e-13):
    """Solve the Ringleb problem on an n x n mesh of (-5, -1) x (1, 5) of order p."""
    import torch

    from workloads import meshes as M
    from workloads.fields import Ringleb

    from .hdg import Plan

    f = Ringleb()
    mesh = M.tri_square(n, 0.0, 0, periodic=False, lo=0.0, length=4.0)
    mesh.elem_xyz[..., 0] -= 5.0
    mesh.elem_xyz[..., 1] += 1.0
    tmap, nt = M.trace_map(mesh, p, scheme)
    plan = Plan(mesh.etype, p, mesh.elem_xyz, tmap, nt, mesh.boundary.astype(np.int32), viscous=False,
                gamma=f.gamma, alpha=0.0)
    dev = plan.device
    xn, xt = (t.cpu().numpy() for t in plan.node_coords())

    def state(x):
        tp = torch.from_numpy(np.ascontiguousarray(f.prim(x))).to(dev)
        return plan.prepare_state(tp, None, want_u=True)

    v, _, _ = state(xn)
    vhat, _, _ = state(xt)
    vbc = vhat.clone()
    info = plan.newton_solve(v, None, vhat, None, vbc, maxit=maxit, tol=tol, atol=atol, lin_tol=lin_tol)
    _, _, uex = state(plan.quad_coords().cpu().numpy())
    err = float(torch.sqrt(plan.l2_error(v, uex, "u").sum()))
    return {"n": n, "inv_h": n / 4.0, "p": p, "scheme": scheme, "elements": mesh.n_elem, "n_trace": nt,
            "newton_iterations": info["iterations"], "converged": info["converged"], "res": info["res"][-1],
            "error": err}


def ringleb_table(ns=(8, 16, 32, 64), ps=(1, 2, 3, 4), schemes=("hdg", "iedg", "edg"), **kw):
    """Errors and rates for every (scheme, p, n); rates against the next finer mesh."""
    rows = []
    for scheme in schemes:
        for p in ps:
            prev = None
            for n in ns:
                r = ringleb_run(n, p, scheme, **kw)
                if prev is not None:
                    r["rate"] = float(np.log2(prev["error"] / r["error"]))
                rows.append(r)
                prev = r
    return rows


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Ringleb (Euler) or Couette (Navier-Stokes) convergence on the GPU")
    ap.add_argument("--problem", default="ringleb", choices=("ringleb", "couette"))
    ap.add_argument("--ns", default=None, help="comma-separated n (default 8,16,32,64 / 4,8,16)")
    ap.add_argument("--ps", default="1,2,3,4")
    ap.add_argument("--schemes", default="hdg,iedg,edg")
    ap.add_argument("--ghat-proj", action="store_true", help="couette: projection viscous flux")
    ap.add_argument("--bc", default="projection", choices=("projection", "nodal"),
                    help="couette: Dirichlet data as the face L2 projection or the nodal interpolant")
    a = ap.parse_args(argv)
    ps = tuple(int(x) for x in a.ps.split(","))
    if a.problem == "ringleb":
        ns = tuple(int(x) for x in (a.ns or "8,16,32,64").split(","))
        for scheme in a.schemes.split(","):
            for r in ringleb_table(ns, ps, (scheme,)):
                print(json.dumps(r), flush=True)
    else:
        ns = tuple(int(x) for x in (a.ns or "4,8,16").split(","))
        for scheme in a.schemes.split(","):
            for r in couette_table(ns, ps, scheme, a.ghat_proj, a.bc):
                print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
