"""Conversion of primitive workload fields to the method's unknowns (oracle).

v = v(u(rho, V, p)) by the paper's entropy-variable map; q = grad v by the
chain rule, taken as a complex-step directional derivative of that map along
the primitive gradient (exact to rounding); u* = u(prim) by the perfect-gas
relations of the Euler section.
"""
from __future__ import annotations

import numpy as np

from . import physics as ph

CS_H = 1e-30


def _v_of_prim_cols(prim, gamma):
    """prim (m, N) -> v (m, N)."""
    m = prim.shape[0]
    rho, V, p = prim[0], prim[1:m - 1].T, prim[m - 1]
    return ph.v_of_prim(rho, V, p, gamma).T


def entropy_state(prim, grad, gamma):
    """(v (m, N), q (m*d, N) or None) from primitives and their gradients."""
    prim = np.asarray(prim, float)
    v = np.real(_v_of_prim_cols(prim.astype(complex), gamma))
    if grad is None:
        return v, None
    m, d, N = grad.shape
    q = np.empty((m, d, N))
    for k in range(d):
        pc = prim.astype(complex) + 1j * CS_H * grad[:, k, :]
        q[:, k, :] = np.imag(_v_of_prim_cols(pc, gamma)) / CS_H
    return v, q.reshape(m * d, N)


def conservative_state(prim, gamma):
    m = prim.shape[0]
    return ph.u_of_prim(prim[0], prim[1:m - 1].T, prim[m - 1], gamma).T.copy()


def oracle_inputs(wl, disc):
    """All method inputs of a workload, computed with the oracle's own geometry."""
    xn = disc.node_coords()
    xt = disc.trace_coords()
    s = wl.sample(xn, xt)
    v, q = entropy_state(s["prim"], s["grad"], wl.gamma)
    vhat, _ = entropy_state(s["prim_hat"], None, wl.gamma)
    ustar = conservative_state(s["prim_star"], wl.gamma)
    vbc, _ = entropy_state(s["prim_bc"], None, wl.gamma)
    return dict(v=v, q=q, vhat=vhat, ustar=ustar, vbc=vbc, xn=xn, xt=xt, **s)


def node_coords(disc):
    """(d, E*Np) element node coordinates via the oracle's vertex maps (all elements at once)."""
    from .geometry import shape_functions
    N, _ = shape_functions(disc.ref.etype, disc.ref.nodes)          # (Np, nv)
    x = np.einsum("av,evi->eai", N, disc.mesh.elem_xyz)             # (E, Np, d)
    return x.reshape(-1, disc.d).T.copy()


def trace_coords(disc, xn):
    """(d, n_trace) trace node coordinates from the element node coordinates."""
    X = np.full((disc.d, disc.n_trace), np.nan)
    fn = np.stack(disc.ref.face_nodes)                               # (nf, Nfp)
    idx = (np.arange(disc.mesh.n_elem)[:, None, None] * disc.Np + fn[None]).reshape(-1)
    X[:, disc.tmap.reshape(-1)] = xn[:, idx]
    return X


def oracle_inputs_fast(wl, disc):
    """oracle_inputs without per-element geometry objects (large meshes)."""
    xn = node_coords(disc)
    xt = trace_coords(disc, xn)
    s = wl.sample(xn, xt)
    v, q = entropy_state(s["prim"], s["grad"], wl.gamma)
    vhat, _ = entropy_state(s["prim_hat"], None, wl.gamma)
    ustar = conservative_state(s["prim_star"], wl.gamma)
    vbc, _ = entropy_state(s["prim_bc"], None, wl.gamma)
    return dict(v=v, q=q, vhat=vhat, ustar=ustar, vbc=vbc, xn=xn, xt=xt, **s)
