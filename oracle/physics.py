"""Pointwise physics in entropy variables (oracle).

Every function accepts complex arrays (so that the element Jacobian can be
taken by complex step) and broadcasts over leading axes.  The state vector
has m = d + 2 components; the last axis of ``v`` / ``u`` is the component.

References to the paper:

* conservation variables, inviscid flux F and the perfect-gas pressure:
  the compressible Euler section (flux equation and the EOS after it);
* viscous flux G, Newtonian stress with beta = 0 and Fourier heat flux with
  kappa = c_p mu / Pr: the compressible Navier-Stokes section;
* entropy pair H = -rho s, F_H = -rho s V with s = log(p / rho^gamma) - s0
  and the entropy variables v(u): the section on entropy pairs and
  symmetrization (the map equation there);
* G in entropy variables, G(v, q) = G(u(v), grad u) with grad u = A0(v) q:
  the NS hybridized DG section;
* trace flux f_hat = 1/2 (F(v_hat) + F(v)).n + 1/2 sigma (v - v_hat): the
  numerical flux equation of the Euler hybridized DG section;
* symmetric Lax-Friedrichs stabilization sigma = lambda_max(v*) A0(v*) with
  v* = v_hat: its definition in the stability section and the choice stated
  at the start of the numerical examples;
* viscous trace flux g_hat = G(v_hat, q).n: second option of the viscous
  numerical flux equations, the one used in the numerical examples.

Gas constant R = 1 (T = p / rho), c_v = 1/(gamma-1), c_p = gamma/(gamma-1),
s0 = 0.
"""
from __future__ import annotations

import numpy as np


def abs_cs(x):
    """|x| continued analytically for complex step; derivative +1 at 0."""
    return np.where(np.real(x) >= 0, x, -x)


def split_v(v):
    m = v.shape[-1]
    return v[..., 0], v[..., 1:m - 1], v[..., m - 1]


def prim_of_v(v, gamma):
    """Density, velocity (..., d) and pressure from entropy variables."""
    v1, w, vm = split_v(v)
    s = gamma - v1 + (w * w).sum(-1) / (2.0 * vm)
    rho = ((gamma - 1.0) / (-vm) * np.exp(-s)) ** (1.0 / (gamma - 1.0))
    p = (gamma - 1.0) * rho / (-vm)
    V = -w / vm[..., None]
    return rho, V, p


def u_of_v(v, gamma):
    """Conservation variables u(v) (inverse of the entropy-variable map)."""
    rho, V, p = prim_of_v(v, gamma)
    rE = p / (gamma - 1.0) + 0.5 * rho * (V * V).sum(-1)
    return np.concatenate([rho[..., None], rho[..., None] * V, rE[..., None]], axis=-1)


def prim_of_u(u, gamma):
    m = u.shape[-1]
    rho = u[..., 0]
    V = u[..., 1:m - 1] / rho[..., None]
    p = (gamma - 1.0) * (u[..., m - 1] - 0.5 * rho * (V * V).sum(-1))
    return rho, V, p


def u_of_prim(rho, V, p, gamma):
    rE = p / (gamma - 1.0) + 0.5 * rho * (V * V).sum(-1)
    return np.concatenate([rho[..., None], rho[..., None] * V, rE[..., None]], axis=-1)


def v_of_u(u, gamma):
    """Entropy variables from the paper's closed form for H = -rho s (s0 = 0)."""
    m = u.shape[-1]
    rho, V, p = prim_of_u(u, gamma)
    s = np.log(p / rho ** gamma)
    rE = u[..., m - 1]
    v1 = (gamma - 1.0) * (-s / (gamma - 1.0) + (gamma + 1.0) / (gamma - 1.0) - rE / p)
    w = (gamma - 1.0) * u[..., 1:m - 1] / p[..., None]
    vm = -(gamma - 1.0) * rho / p
    return np.concatenate([v1[..., None], w, vm[..., None]], axis=-1)


def v_of_prim(rho, V, p, gamma):
    return v_of_u(u_of_prim(rho, V, p, gamma), gamma)


def entropy_pair(v, gamma):
    """Generalized entropy H = -rho s and entropy flux F_H = -rho s V."""
    rho, V, p = prim_of_v(v, gamma)
    s = np.log(p / rho ** gamma)
    H = -rho * s
    return H, H[..., None] * V


def A0(v, gamma):
    """Closed form of dU/dV for H = -rho s (symmetric positive definite).

    The paper defers the expression to its reference on symmetrization; this
    is that matrix written with E = rho E / rho, H_t = E + p / rho and
    c^2 = gamma p / rho, scaled by 1/(gamma - 1).  Pinned in tests against the
    complex-step derivative of ``u_of_v``.
    """
    rho, V, p = prim_of_v(v, gamma)
    d = V.shape[-1]
    m = d + 2
    E = p / ((gamma - 1.0) * rho) + 0.5 * (V * V).sum(-1)
    Ht = E + p / rho
    c2 = gamma * p / rho
    out = np.zeros(v.shape[:-1] + (m, m), dtype=np.result_type(v, float))
    out[..., 0, 0] = rho
    out[..., 0, 1:m - 1] = rho[..., None] * V
    out[..., 1:m - 1, 0] = rho[..., None] * V
    out[..., 0, m - 1] = rho * E
    out[..., m - 1, 0] = rho * E
    out[..., 1:m - 1, 1:m - 1] = rho[..., None, None] * V[..., :, None] * V[..., None, :] \
        + p[..., None, None] * np.eye(d)
    out[..., 1:m - 1, m - 1] = (rho * Ht)[..., None] * V
    out[..., m - 1, 1:m - 1] = (rho * Ht)[..., None] * V
    out[..., m - 1, m - 1] = rho * Ht * Ht - c2 * p / (gamma - 1.0)
    return out / (gamma - 1.0)


def flux_F(v, gamma):
    """Inviscid flux F(u(v)), shape (..., m, d)."""
    rho, V, p = prim_of_v(v, gamma)
    d = V.shape[-1]
    m = d + 2
    rE = p / (gamma - 1.0) + 0.5 * rho * (V * V).sum(-1)
    F = np.zeros(v.shape[:-1] + (m, d), dtype=np.result_type(v, float))
    F[..., 0, :] = rho[..., None] * V
    F[..., 1:m - 1, :] = rho[..., None, None] * V[..., :, None] * V[..., None, :] \
        + p[..., None, None] * np.eye(d)
    F[..., m - 1, :] = V * (rE + p)[..., None]
    return F


def stress_heat_flux(v, q, gamma, mu, Pr):
    """Viscous stress tau (..., d, d) and heat flux f (..., d) of the state v with gradient
    unknowns q (..., m, d) (the Navier-Stokes section: Newtonian stress with beta = 0, Fourier
    heat flux f = -kappa grad T, kappa = c_p mu / Pr).

    grad u = A0(v) q per direction, then the velocity and temperature gradients from grad u.
    """
    rho, V, p = prim_of_v(v, gamma)
    d = V.shape[-1]
    m = d + 2
    gu = np.einsum("...ab,...bk->...ak", A0(v, gamma), q)        # (..., m, d)
    grho = gu[..., 0, :]
    gV = (gu[..., 1:m - 1, :] - V[..., :, None] * grho[..., None, :]) / rho[..., None, None]
    gp = (gamma - 1.0) * (gu[..., m - 1, :] - np.einsum("...i,...ik->...k", V, gu[..., 1:m - 1, :])
                          + 0.5 * (V * V).sum(-1)[..., None] * grho)
    T = p / rho
    gT = (gp - T[..., None] * grho) / rho[..., None]
    div = np.einsum("...ii->...", gV)
    tau = mu * (gV + np.swapaxes(gV, -1, -2) - (2.0 / 3.0) * div[..., None, None] * np.eye(d))
    kappa = gamma / (gamma - 1.0) * mu / Pr
    return tau, -kappa * gT


def flux_G(v, q, gamma, mu, Pr):
    """Viscous flux G(v, q), shape (..., m, d); q has shape (..., m, d):
    G = -(0, tau, V.tau - f) with the stress and heat flux of ``stress_heat_flux``."""
    rho, V, p = prim_of_v(v, gamma)
    d = V.shape[-1]
    m = d + 2
    tau, f = stress_heat_flux(v, q, gamma, mu, Pr)
    G = np.zeros(v.shape[:-1] + (m, d), dtype=np.result_type(v, q, float))
    G[..., 1:m - 1, :] = -tau
    G[..., m - 1, :] = -(np.einsum("...i,...ij->...j", V, tau) - f)
    return G


def lam_max(v, n, gamma):
    """Largest |eigenvalue| of A_n: |V.n| + c (n unit)."""
    rho, V, p = prim_of_v(v, gamma)
    vn = (V * n).sum(-1)
    return abs_cs(vn) + np.sqrt(gamma * p / rho)


def sigma_slf(vh, n, gamma):
    """Symmetric Lax-Friedrichs stabilization lambda_max(v_hat) A0(v_hat)."""
    return lam_max(vh, n, gamma)[..., None, None] * A0(vh, gamma)


def abs_An_apply(v, n, gamma, du):
    """|A_n(v)| du for perturbations du (..., m) of the conservation variables, from the
    eigen-decomposition of the Euler flux Jacobian along the unit normal n: acoustic waves
    u_n -/+ c with strengths (dp -/+ rho c du_n) / (2 c^2) on (1, V -/+ c n, H -/+ c u_n), the
    entropy wave (speed u_n) with strength drho - dp / c^2 on (1, V, |V|^2 / 2) and the shear
    waves (speed u_n) rho (0, dV_t, V . dV_t), dV_t = dV - du_n n; dprim linearized from du."""
    rho, V, p = prim_of_v(v, gamma)
    m = du.shape[-1]
    d = m - 2
    drho = du[..., 0]
    dV = (du[..., 1:m - 1] - V * drho[..., None]) / rho[..., None]
    dp = (gamma - 1.0) * (du[..., m - 1] - 0.5 * (V * V).sum(-1) * drho - rho * (V * dV).sum(-1))
    c = np.sqrt(gamma * p / rho)
    un = (V * n).sum(-1)
    H = c * c / (gamma - 1.0) + 0.5 * (V * V).sum(-1)
    dun = (dV * n).sum(-1)
    dVt = dV - dun[..., None] * n
    a1 = (dp - rho * c * dun) / (2 * c * c)
    a4 = (dp + rho * c * dun) / (2 * c * c)
    a2 = drho - dp / (c * c)

    def vec(s0, sV, sE):
        return np.concatenate([s0[..., None], sV, sE[..., None]], axis=-1)

    one = np.ones_like(rho)
    r1 = vec(one, V - c[..., None] * n, H - c * un)
    r4 = vec(one, V + c[..., None] * n, H + c * un)
    r2 = vec(one, V, 0.5 * (V * V).sum(-1))
    sh = vec(0 * rho, rho[..., None] * dVt, rho * (V * dVt).sum(-1))
    return (abs_cs(un - c)[..., None] * a1[..., None] * r1
            + abs_cs(un)[..., None] * (a2[..., None] * r2 + sh)
            + abs_cs(un + c)[..., None] * a4[..., None] * r4)


def sigma_s_apply(vh, n, gamma, dv):
    """Symmetric variable stabilization |A_n(v_hat)| A0(v_hat) applied to dv (v* = v_hat)."""
    return abs_An_apply(vh, n, gamma, np.einsum("...ab,...b->...a", A0(vh, gamma), dv))


def _path_speeds(vh, v, th, n, gamma):
    """Real wave speeds u_n - c, u_n, u_n + c (last axis) at the states vh + th (v - vh) (real
    parts; th broadcasts against the leading axes)."""
    vt = np.real(vh) + th[..., None] * (np.real(v) - np.real(vh))
    rho, V, p = prim_of_v(vt, gamma)
    un = (V * n).sum(-1)
    c = np.sqrt(gamma * p / rho)
    return np.stack([un - c, un, un + c], axis=-1)


MV_SAMPLES = 32       # sub-intervals of [0, 1] searched for sign changes of the wave speeds
MV_GAUSS = 12         # Gauss-Legendre points on every smooth piece


def mv_breakpoints(vh, v, n, gamma):
    """Sorted breakpoints (..., MV_SAMPLES + 4) in [0, 1] of the mean-value integrand along the
    straight path vh + th (v - vh): 0, 1 and every root of u_n - c, u_n and u_n + c (where |A_n|
    has a kink), found by bisection in the sub-intervals where a speed changes sign; unused
    slots repeat 1.  At most one root per speed and sub-interval is resolved (a second one in
    the same 1/32 of the path would be missed)."""
    lead = np.broadcast_shapes(np.shape(np.real(vh))[:-1], np.shape(np.real(v))[:-1], np.shape(n)[:-1])
    ts = np.linspace(0.0, 1.0, MV_SAMPLES + 1)
    g = _path_speeds(vh[..., None, :], v[..., None, :], np.broadcast_to(ts, lead + ts.shape),
                     n[..., None, :], gamma)                        # (..., S+1, 3)
    sa, sb = g[..., :-1, :], g[..., 1:, :]
    bracket = (sa * sb < 0) | ((sb == 0) & (sa != 0))
    lo = np.broadcast_to(ts[:-1, None], bracket.shape).copy()
    hi = np.broadcast_to(ts[1:, None], bracket.shape).copy()
    flo = sa.copy()
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        gm = np.empty_like(mid)
        for k in range(3):
            gm[..., k] = _path_speeds(vh[..., None, :], v[..., None, :], mid[..., k], n[..., None, :], gamma)[..., k]
        left = np.sign(gm) == np.sign(flo)
        lo = np.where(left, mid, lo)
        flo = np.where(left, gm, flo)
        hi = np.where(left, hi, mid)
    roots = np.where(bracket, 0.5 * (lo + hi), 1.0).reshape(lead + (-1,))
    roots = np.sort(roots, axis=-1)[..., :3]                           # at most 3 kinks kept
    if np.any(bracket.sum(axis=(-2, -1)) > 3):
        raise ValueError("more than three wave-speed sign changes along a mean-value path")
    ends = np.broadcast_to(np.array([0.0, 1.0]), lead + (2,))
    return np.sort(np.concatenate([ends, roots], axis=-1), axis=-1)


def sigma_mv_apply(vh, v, n, gamma, dv):
    """Mean-value stabilization of Section 4 on the straight path in entropy variables,
    sigma_MV(v_hat, v) = int_0^1 |A_n| A0 (v_hat + theta (v - v_hat)) d theta (the definition's two
    (1 - theta) weighted integrals along the path and its reverse add up to this), applied to dv.
    The integrand is smooth except where a wave speed u_n - c, u_n, u_n + c changes sign along
    the path; the integral is split there (mv_breakpoints, on the real parts) and every piece is
    integrated with MV_GAUSS-point Gauss-Legendre, exact to rounding.  Complex-step derivatives
    pass through: the integrand is continuous at the breakpoints, so their motion adds nothing."""
    br = mv_breakpoints(vh, v, n, gamma)                               # (..., 5)
    x, w = np.polynomial.legendre.leggauss(MV_GAUSS)
    out = 0.0
    for i in range(br.shape[-1] - 1):
        a, b = br[..., i], br[..., i + 1]
        for xg, wg in zip(x, w):
            th = a + (b - a) * 0.5 * (1.0 + xg)
            out = out + (0.5 * wg * (b - a))[..., None] * \
                sigma_s_apply(vh + th[..., None] * (v - vh), n, gamma, dv)
    return out


def fhat(vh, v, n, gamma, sigma="slf"):
    """Inviscid trace flux with sigma_SLF (default), sigma_S (v* = v_hat) or sigma_MV."""
    Fn = np.einsum("...cj,...j->...c", flux_F(vh, gamma) + flux_F(v, gamma), n)
    if sigma == "s":
        return 0.5 * Fn + 0.5 * sigma_s_apply(vh, n, gamma, v - vh)
    if sigma == "mv":
        return 0.5 * Fn + 0.5 * sigma_mv_apply(vh, v, n, gamma, v - vh)
    sig = sigma_slf(vh, n, gamma)
    return 0.5 * Fn + 0.5 * np.einsum("...ab,...b->...a", sig, v - vh)


def ghat(vh, q, n, gamma, mu, Pr):
    """Viscous trace flux G(v_hat, q).n."""
    return np.einsum("...cj,...j->...c", flux_G(vh, q, gamma, mu, Pr), n)


def jac_cs(f, x, h=1e-30):
    """Complex-step Jacobian of f at real x: (..., out, in)."""
    x = np.asarray(x, dtype=complex)
    n = x.shape[-1]
    cols = []
    for i in range(n):
        xp = x.copy()
        xp[..., i] += 1j * h
        cols.append(np.imag(f(xp)) / h)
    return np.stack(cols, axis=-1)
