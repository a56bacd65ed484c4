"""Newton driver on the condensed trace system (oracle, small meshes): the steady
problem, or one implicit stage when the discretization's alpha > 0 and u* is given
(the mass term alpha (u(v) - u*, w) of the stage residual).

Each iteration assembles every element (complex-step Jacobian), condenses,
solves the global trace system with a sparse direct solver and back-solves
the element unknowns:  v, q += dx;  v_hat += dlambda.  Used only to check the
order of accuracy of the discretization on manufactured solutions (the
paper reports k+1 convergence for smooth problems in its Ringleb and Couette
examples).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import hdg


def newton_steady(disc: hdg.Discretization, v, q, vhat, vbc=None, source=None, tol=1e-11,
                  maxit=12, verbose=False, ustar=None):
    v, vhat = v.copy(), vhat.copy()
    q = None if q is None else q.copy()
    m, d, Np = disc.m, disc.d, disc.Np
    hist = []
    for it in range(maxit):
        Ys, zs, Ss, gs, rn = [], [], [], [], 0.0
        rt = np.zeros(m * disc.n_trace)
        for e in range(disc.mesh.n_elem):
            x, lam, us, vb = disc.elem_inputs(e, v, q, vhat, ustar, vbc)
            s = disc.element_system(e, x, lam, us, vb, source)
            c = hdg.condense(s)
            Ys.append(c["Y"]); zs.append(c["z"]); Ss.append(c["S"]); gs.append(c["g"])
            rn += np.sum(s["R_loc"] ** 2)
            np.add.at(rt, hdg.element_trace_index(disc, e), s["R_tr"])
        res = np.sqrt(rn + np.sum(rt ** 2))
        hist.append(res)
        if verbose:
            print(it, res)
        if res < tol:
            break
        K = hdg.trace_matrix(disc, Ss).tocsc()
        dl = spla.spsolve(K, hdg.trace_rhs(disc, gs))
        dx = hdg.backsolve(disc, Ys, zs, dl)
        vhat = vhat + dl.reshape(m, disc.n_trace)
        for e in range(disc.mesh.n_elem):
            sl = slice(e * Np, (e + 1) * Np)
            v[:, sl] += dx[e][:m * Np].reshape(m, Np)
            if disc.phys.viscous:
                q[:, sl] += dx[e][m * Np:].reshape(m * d, Np)
    return v, q, vhat, hist


def l2_error_u(disc: hdg.Discretization, v, u_exact):
    """sqrt(sum_K int |u(v_h) - u_exact|^2) with the element quadrature."""
    from . import physics as ph
    err = 0.0
    for e in range(disc.mesh.n_elem):
        G = disc.geom(e)
        vq = disc.ref.phi @ v[:, e * disc.Np:(e + 1) * disc.Np].T
        du = ph.u_of_v(vq, disc.phys.gamma) - u_exact(G.xq)
        err += np.sum(G.W[:, None] * du ** 2)
    return np.sqrt(err)


def l2_error_v(disc: hdg.Discretization, v, v_exact):
    """sqrt(sum_K int |v_h - v_exact|^2) with the element quadrature."""
    err = 0.0
    for e in range(disc.mesh.n_elem):
        G = disc.geom(e)
        dv = disc.ref.phi @ v[:, e * disc.Np:(e + 1) * disc.Np].T - v_exact(G.xq)
        err += np.sum(G.W[:, None] * dv ** 2)
    return np.sqrt(err)


def l2_error_components(disc: hdg.Discretization, v, u_exact):
    """Per conserved component c: sqrt(sum_K int_K (u(v_h) - u_exact)_c^2), element quadrature."""
    from . import physics as ph
    err = np.zeros(disc.m)
    for e in range(disc.mesh.n_elem):
        G = disc.geom(e)
        vq = disc.ref.phi @ v[:, e * disc.Np:(e + 1) * disc.Np].T
        du = ph.u_of_v(vq, disc.phys.gamma) - u_exact(G.xq)
        err += np.sum(G.W[:, None] * du ** 2, axis=0)
    return np.sqrt(err)


def l2_error_stress_heat(disc: hdg.Discretization, v, q, v_exact, q_exact):
    """L2(Omega) norms of the errors in the viscous stress and the heat flux formed from
    (v_h, q_h) against those formed from the exact state and its gradient (the quantities of
    the Couette example of Section 5: the approximate stresses and heat fluxes come from the
    approximate solution and the approximate gradients).  v_exact: x (N, d) -> (N, m),
    q_exact: x (N, d) -> (N, m, d).  Returns (||tau_h - tau||, ||f_h - f||)."""
    from . import physics as ph
    ph_, d, m = disc.phys, disc.d, disc.m
    et = ef = 0.0
    for e in range(disc.mesh.n_elem):
        G = disc.geom(e)
        sl = slice(e * disc.Np, (e + 1) * disc.Np)
        vq = disc.ref.phi @ v[:, sl].T
        qq = (disc.ref.phi @ q[:, sl].T).reshape(len(G.W), m, d)
        th, fh = ph.stress_heat_flux(vq, qq, ph_.gamma, ph_.mu, ph_.Pr)
        te, fe = ph.stress_heat_flux(v_exact(G.xq), q_exact(G.xq), ph_.gamma, ph_.mu, ph_.Pr)
        et += np.sum(G.W[:, None, None] * (th - te) ** 2)
        ef += np.sum(G.W[:, None] * (fh - fe) ** 2)
    return np.sqrt(et), np.sqrt(ef)


def project_boundary_data(disc: hdg.Discretization, v_exact):
    """Dirichlet data of the trace equation <v_hat - v_bc, mu>_F = 0 on the boundary faces as
    the L2(F) projection of the boundary function onto the face's trace space: per Dirichlet
    face, M_F c = <v_exact, mu>_F with M_F the face mass matrix of the trace basis, by the face
    quadrature.  (Testing the trace equation against every mu with the boundary function itself
    gives exactly this projection; a nodal interpolant of it is a different, O(h^{k+1}) nearby
    datum.)  v_exact: x (N, d) -> (N, m).  Returns (m, n_trace): the projection on the nodes of
    Dirichlet faces, zero elsewhere.  A trace node shared by two Dirichlet faces (a continuous
    trace at a boundary corner) has no face-local projection and raises ValueError."""
    out = np.zeros((disc.m, disc.n_trace))
    seen = np.zeros(disc.n_trace, dtype=bool)
    for e in range(disc.mesh.n_elem):
        for f in range(disc.nf):
            if disc.face_bc[e, f] != 1:
                continue
            nodes = disc.tmap[e, f]
            if np.any(seen[nodes]):
                raise ValueError("trace node shared by two Dirichlet faces")
            seen[nodes] = True
            F = disc.geom(e).faces[f]
            Mf = F["psi"].T @ (F["W"][:, None] * F["psi"])
            rhs = F["psi"].T @ (F["W"][:, None] * v_exact(F["x"]))
            out[:, nodes] = np.linalg.solve(Mf, rhs).T
    return out


def entropy_integral(disc: hdg.Discretization, v):
    """Per element (int_K rho s, int_K rho) with s = ln(p / rho^gamma) at u(v_h), by the
    element quadrature: the total thermodynamic entropy, the negative of the integral of
    the generalized entropy H = -rho s that Proposition 1 follows (entropy-variable section)."""
    from . import physics as ph
    out = np.zeros((disc.mesh.n_elem, 2))
    for e in range(disc.mesh.n_elem):
        G = disc.geom(e)
        vq = disc.ref.phi @ v[:, e * disc.Np:(e + 1) * disc.Np].T
        H, _ = ph.entropy_pair(vq, disc.phys.gamma)
        rho = ph.prim_of_v(vq, disc.phys.gamma)[0]
        out[e] = (np.sum(G.W * -H), np.sum(G.W * rho))
    return out


def flow_statistics(disc: hdg.Discretization, v):
    """Per element the integrals of (rho s, rho, rho |V|^2 / 2, |omega|^2, theta, theta^2, T,
    T^2) by the element quadrature, at u(v_h) and the velocity gradient of v_h: the quantities
    whose means and variances the Taylor-Green example of Section 5 follows.  s = ln(p/rho^gamma),
    omega = curl V (a scalar in 2D), theta = div V, T = p / rho.  The velocity gradient comes from
    V(v) = -v_{2..d+1} / v_m differentiated by the chain rule."""
    from . import physics as ph
    d, m, g = disc.d, disc.m, disc.phys.gamma
    out = np.zeros((disc.mesh.n_elem, 8))
    for e in range(disc.mesh.n_elem):
        G = disc.geom(e)
        ve = v[:, e * disc.Np:(e + 1) * disc.Np]              # (m, Np)
        vq = disc.ref.phi @ ve.T                              # (nq, m)
        gv = np.einsum("naj,ca->ncj", G.gphi, ve)              # (nq, m, d): d v_c / d x_j
        rho, V, p = ph.prim_of_v(vq, g)
        vm = vq[:, m - 1]
        dV = -(gv[:, 1:d + 1, :] + V[:, :, None] * gv[:, None, m - 1, :]) / vm[:, None, None]   # [q, i, j]
        if d == 2:
            om2 = (dV[:, 1, 0] - dV[:, 0, 1]) ** 2
        else:
            om = np.stack([dV[:, 2, 1] - dV[:, 1, 2], dV[:, 0, 2] - dV[:, 2, 0], dV[:, 1, 0] - dV[:, 0, 1]], axis=1)
            om2 = np.sum(om ** 2, axis=1)
        th = np.trace(dV, axis1=1, axis2=2)
        T = p / rho
        cols = [rho * np.log(p / rho ** g), rho, 0.5 * rho * np.sum(V ** 2, axis=1), om2, th, th ** 2, T, T ** 2]
        out[e] = [np.sum(G.W * c) for c in cols]
    return out


# ---- one step of Alexander's three-stage L-stable DIRK(3,3) (the time integration of
# the paper's numerical examples, Section 5).  Stage i solves
#   alpha (u(v_i) - u*_i, w) + s(v_i; w) = 0,   alpha = 1 / (a_ii dt),
# with (u*_i, w) = (u_n, w) - dt sum_{j<i} a_ij s(v_j; w).  A converged stage j gives
# s(v_j; w) = -alpha (u(v_j) - u*_j, w); on the element L2 products b(v) = (u(v), phi_a)_K
# this is b*_i = b(v_n) + sum_{j<i} (a_ij / a_jj) (b(v_j) - b*_j), and u*_i = M_K^-1 b*_i
# as nodal values.  Stiffly accurate: the step ends in the last stage's state.

DIRK33_G = 0.435866521508459   # root of x^3 - 3x^2 + 3x/2 - 1/6 in (1/6, 1/2)


def dirk33_tableau():
    g = DIRK33_G
    return np.array([[g, 0.0, 0.0],
                     [0.5 * (1.0 - g), g, 0.0],
                     [-0.25 * (6 * g * g - 16 * g + 1), 0.25 * (6 * g * g - 20 * g + 5), g]])


def weak_u(disc: hdg.Discretization, v):
    """b[c][e Np + a] = (u_c(v_h), phi_a)_K by the element quadrature."""
    from . import physics as ph
    Np, phi = disc.Np, disc.ref.phi
    b = np.zeros_like(v)
    for e in range(disc.mesh.n_elem):
        sl = slice(e * Np, (e + 1) * Np)
        uq = ph.u_of_v(phi @ v[:, sl].T, disc.phys.gamma)
        b[:, sl] = (phi.T @ (disc.geom(e).W[:, None] * uq)).T
    return b


def mass_solve(disc: hdg.Discretization, b):
    """u[:, K] = M_K^-1 b[:, K], M_K the element mass matrix (phi_a, phi_b)_K."""
    Np, phi = disc.Np, disc.ref.phi
    u = np.zeros_like(b)
    for e in range(disc.mesh.n_elem):
        sl = slice(e * Np, (e + 1) * Np)
        Mk = phi.T @ (disc.geom(e).W[:, None] * phi)
        u[:, sl] = np.linalg.solve(Mk, b[:, sl].T).T
    return u


def dirk33_step(disc: hdg.Discretization, v, q, vhat, dt, vbc=None, tol=1e-11, maxit=12):
    """One DIRK(3,3) step; the discretization's alpha must be 1 / (a_ii dt)."""
    A = dirk33_tableau()
    assert abs(disc.phys.alpha * A[0, 0] * dt - 1.0) < 1e-12
    bn = weak_u(disc, v)
    d, hists = [], []
    for i in range(3):
        bs = bn.copy()
        for j in range(i):
            bs = bs + (A[i, j] / A[j, j]) * d[j]
        v, q, vhat, hist = newton_steady(disc, v, q, vhat, vbc=vbc, tol=tol, maxit=maxit,
                                         ustar=mass_solve(disc, bs))
        hists.append(hist)
        d.append(weak_u(disc, v) - bs)
    return v, q, vhat, hists
