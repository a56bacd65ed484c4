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
