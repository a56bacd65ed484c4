"""The Shu vortex of Section 5 on the GPU path: a homentropic vortex advected by a uniform
stream through the doubly periodic square (-5L, 5L)^2, 10 x 10 squares cut into 200
triangles, entropy-variable HDG of degree k = 4, DIRK(3,3) steps of dt = 0.05 L / V_inf
(hdg_dirk_step), psi = 5, M_inf = gamma^-1/2, rho_inf = V_inf = L = 1.

Recorded after every step: the change of the total thermodynamic entropy int rho s since
t = 0 (hdg_entropy_integral; Proposition 1 makes int H = -int rho s non-increasing for the
semi-discrete scheme on a periodic domain, and the paper reports the total entropy of the
entropy-variable scheme as non-decreasing), the total mass, the L2 errors of u(v_h) and of
v_h against the exact solution (the initial vortex translated by V_inf t, wrapped to the
periodic square), and the Newton iteration counts of the three stages."""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def shu_vortex_run(steps, dt=0.05, p=4, n=10, sigma="slf", record_every=1, tol=1e-12, atol=1e-13,
                   lin_tol=1e-13, psi=5.0, gamma=1.4, progress=False):
    import torch

    from workloads import meshes as M
    from workloads.fields import ShuVortex

    from .hdg import Plan

    L, half = 1.0, 5.0
    f = ShuVortex(psi=psi, mach=gamma ** -0.5, L=L, center=(0.0, 0.0), gamma=gamma)
    mesh = M.tri_square(n, 0.0, 0, periodic=True, lo=-half * L, length=2 * half * L)
    tmap, nt = M.trace_map(mesh, p, "hdg")
    plan = Plan(mesh.etype, p, mesh.elem_xyz, tmap, nt, np.zeros((mesh.n_elem, 3), np.int32), viscous=False,
                gamma=gamma, sigma=sigma)
    dev = plan.device
    xn, xt = (t.cpu().numpy() for t in plan.node_coords())
    xq = plan.quad_coords().cpu().numpy()

    def exact_prim(x, t):
        xs = np.array(x, copy=True)
        xs[0] = np.mod(xs[0] - f.v_inf * t + half * L, 2 * half * L) - half * L
        return f.prim(xs)

    def state(x, t):
        tp = torch.from_numpy(np.ascontiguousarray(exact_prim(x, t))).to(dev)
        return plan.prepare_state(tp, None, want_u=True)

    v, _, _ = state(xn, 0.0)
    vhat, _, _ = state(xt, 0.0)
    S0, m0 = (float(a) for a in plan.entropy_integral(v).sum(0).cpu())

    def record(t, infos):
        vex, _, uex = state(xq, t)
        S, mass = (float(a) for a in plan.entropy_integral(v).sum(0).cpu())
        eu = float(torch.sqrt(plan.l2_error(v, uex, "u").sum()))
        ev = float(torch.sqrt(plan.l2_error(v, vex, "v").sum()))
        return {"t": t, "dS": S - S0, "mass": mass, "err_u": eu, "err_v": ev,
                "newton": [i["iterations"] for i in infos], "converged": all(i["converged"] for i in infos)}

    hist = [record(0.0, [])]
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        infos = plan.dirk_step(v, None, vhat, dt, tol=tol, atol=atol, lin_tol=lin_tol)
        if k % record_every == 0 or k == steps:
            hist.append(record(k * dt, infos))
            if progress:
                print(json.dumps(hist[-1]), flush=True)
            if not hist[-1]["converged"]:
                break
    torch.cuda.synchronize()
    return {"elements": mesh.n_elem, "p": p, "dt": dt, "sigma": sigma, "S0": S0, "mass0": m0,
            "seconds": time.perf_counter() - t0, "history": hist}


def tgv_run(steps, dt=5.71e-2, p=2, n=16, scheme="edg", sigma="slf", mach=0.8, record_every=1, tol=1e-9,
            atol=1e-12, lin_tol=1e-12, gamma=1.4, progress=False):
    """Inviscid Taylor-Green vortex of Section 5 (the periodic cube (-pi L, pi L)^3 in n^3
    hexahedra, degree p, M0 = 0.8, dt = 0.0571 L / V0, entropy-variable EDG by default;
    the paper uses n = 32).  Recorded (hdg_flow_statistics): the change of the mean
    thermodynamic entropy (int rho s - int rho s at t = 0) / |Omega|, the mass drift, the mean
    kinetic energy, the mean-square vorticity <omega . omega>, the dilatation variance
    <theta' theta'> and the temperature variance <T' T'> / T0^2 (T = p / rho, T0 = P0 / rho0),
    with the stages' Newton and GMRES iteration counts and convergence flags."""
    import torch

    from workloads import meshes as M
    from workloads.fields import TaylorGreen

    from .hdg import Plan

    f = TaylorGreen(mach=mach, gamma=gamma)
    mesh = M.hex_cube(n, 0.0, 0, periodic=True, lo=-np.pi, length=2 * np.pi)
    tmap, nt = M.trace_map(mesh, p, scheme)
    plan = Plan(mesh.etype, p, mesh.elem_xyz, tmap, nt, np.zeros((mesh.n_elem, 6), np.int32), viscous=False,
                gamma=gamma, sigma=sigma)
    dev = plan.device
    xn, xt = (t.cpu().numpy() for t in plan.node_coords())

    def state(x):
        tp = torch.from_numpy(np.ascontiguousarray(f.prim(x))).to(dev)
        return plan.prepare_state(tp)[0]

    v, vhat = state(xn), state(xt)
    vol = (2 * np.pi) ** 3
    T0 = f.p0 / f.rho0
    S0, m0 = (float(a) for a in plan.entropy_integral(v).sum(0).cpu())

    def record(t, infos):
        st = plan.flow_statistics(v).sum(0).cpu().numpy() / vol
        S, mass = st[0] * vol, st[1] * vol
        return {"t": t, "ds_mean": (S - S0) / vol, "mass_drift": mass / m0 - 1.0,
                "kinetic_energy": float(st[2]), "vorticity_ms": float(st[3]),
                "dilatation_var": float(st[5] - st[4] ** 2), "temperature_var": float((st[7] - st[6] ** 2) / T0 ** 2),
                "newton": [i["iterations"] for i in infos], "gmres": [i["lin_iterations"] for i in infos],
                "converged": all(i["converged"] for i in infos)}

    hist = [record(0.0, [])]
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        infos = plan.dirk_step(v, None, vhat, dt, tol=tol, atol=atol, lin_tol=lin_tol)
        if k % record_every == 0 or k == steps:
            hist.append(record(k * dt, infos))
            if progress:
                print(json.dumps(hist[-1]), flush=True)
    torch.cuda.synchronize()
    return {"elements": mesh.n_elem, "p": p, "scheme": scheme, "dt": dt, "sigma": sigma, "n_trace": nt,
            "S0_mean": S0 / vol, "seconds": time.perf_counter() - t0, "history": hist}


def main(argv=None):
    ap = argparse.ArgumentParser(description="Shu vortex or inviscid Taylor-Green vortex entropy history on the GPU "
                                             "(one JSON line per record)")
    ap.add_argument("--problem", default="shu", choices=("shu", "tgv"))
    ap.add_argument("--t-end", type=float, default=None, help="default 500 (shu), 10 (tgv)")
    ap.add_argument("--dt", type=float, default=None, help="default 0.05 (shu), 0.0571 (tgv)")
    ap.add_argument("--n", type=int, default=16, help="tgv: hexahedra per side")
    ap.add_argument("--sigma", default="slf", choices=("slf", "s", "mv"))
    ap.add_argument("--record-every", type=int, default=100)
    ap.add_argument("--out", default=None, help="write the whole history as JSON here")
    a = ap.parse_args(argv)
    if a.problem == "tgv":
        dt = a.dt or 5.71e-2
        r = tgv_run(int(round((a.t_end or 10.0) / dt)), dt=dt, n=a.n, sigma=a.sigma, record_every=a.record_every,
                    progress=True)
        h = r["history"]
        ds = np.array([x["ds_mean"] for x in h])
        print(json.dumps({"elements": r["elements"], "p": r["p"], "scheme": r["scheme"], "n_trace": r["n_trace"],
                          "dt": r["dt"], "t_end": h[-1]["t"], "seconds": r["seconds"],
                          "min_record_ds": float(np.diff(ds).min()), "ds_end": float(ds[-1]),
                          "mass_drift": max(abs(x["mass_drift"]) for x in h),
                          "all_converged": all(x["converged"] for x in h)}), flush=True)
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(r, fh)
        return
    a.t_end, a.dt = a.t_end or 500.0, a.dt or 0.05
    r = shu_vortex_run(int(round(a.t_end / a.dt)), dt=a.dt, sigma=a.sigma, record_every=a.record_every,
                       progress=True)
    dS = np.array([h["dS"] for h in r["history"]])
    summary = {"elements": r["elements"], "p": r["p"], "dt": r["dt"], "sigma": r["sigma"], "t_end": r["history"][-1]["t"],
               "seconds": r["seconds"], "min_step_dS": float(np.diff(dS).min()), "dS_end": float(dS[-1]),
               "mass_drift": max(abs(h["mass"] / r["mass0"] - 1.0) for h in r["history"]),
               "max_err_u": max(h["err_u"] for h in r["history"]), "max_err_v": max(h["err_v"] for h in r["history"])}
    print(json.dumps(summary), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(r, fh)


if __name__ == "__main__":
    main()
