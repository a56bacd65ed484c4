"""Primitive flow fields (density, velocity, pressure) at caller-given points.

Every field returns primitives ``(rho, V_1..V_d, p)`` as an (m, N) array and,
through a complex-step derivative of its own analytic formula, the spatial
gradient as an (m, d, N) array.  Formulas are written so that they accept
complex coordinates.  Nothing here converts to conservation or entropy
variables: that belongs to the method and is done by each consumer.

Fields:

* ``ShuVortex`` -- the homentropic vortex of the paper's Shu-vortex example,
  with the density amplitude written with the square of the free-stream Mach
  number (the printed formula drops the square; radial equilibrium
  dp/dr = rho u_theta^2 / r only holds with it, see tests).
* ``TaylorGreen`` -- the Taylor-Green initial condition of the paper's TGV
  example (constant density, pressure from the incompressible solution).
* ``Uniform`` -- a constant state (free-stream tests).
* ``Couette`` -- the steady compressible Couette flow with a source term of the
  paper's Navier-Stokes convergence example (exact solution and source).
* ``Ringleb`` -- the Ringleb flow of the paper's steady Euler convergence
  example (hodograph solution; speed of sound from a scalar root find per point,
  written with the corrected forms of two garbled formulas, see tests).
* ``SmoothNoise`` wraps a field and perturbs it with seeded periodic
  sinusoids (relative for rho and p, scaled by a reference speed for V).
* ``node_noise`` draws the per-node i.i.d. perturbation.
"""
from __future__ import annotations

import numpy as np

_CS_H = 1e-30


class Field:
    dim: int

    def prim(self, x):  # pragma: no cover - interface
        raise NotImplementedError

    def prim_and_grad(self, x: np.ndarray):
        """x: (d, N) real points -> prim (m, N), grad (m, d, N) (exact complex step)."""
        x = np.asarray(x, dtype=float)
        d = x.shape[0]
        p0 = np.real(self.prim(x.astype(complex)))
        g = np.empty((p0.shape[0], d, x.shape[1]))
        for k in range(d):
            xc = x.astype(complex)
            xc[k] += 1j * _CS_H
            g[:, k, :] = np.imag(self.prim(xc)) / _CS_H
        return p0, g


class Uniform(Field):
    def __init__(self, rho, V, p):
        self.dim = len(V)
        self.vals = np.array([rho, *V, p], dtype=float)

    def prim(self, x):
        return self.vals[:, None] * np.ones_like(x[0])[None, :]


class Couette(Field):
    """Steady compressible Couette flow on (0, L)^2 (the Navier-Stokes convergence example of
    Section 5): V_x = V0 y' log(1 + y'), V_y = 0, p = P0,
    T = T0 (a + y' (b - a)) + V0^2 Pr / (2 c_v gamma) y' (1 - y'), rho = p / ((gamma - 1) c_v T),
    y' = y / L, T0 = V0^2 / ((gamma - 1) gamma M0^2 c_v).  Units: R = 1 (c_v = 1 / (gamma - 1)),
    rho0 = V0 = L = 1, so P0 = 1 / (gamma M0^2) and mu = 1 / Re0.  ``source`` is the right-hand side
    s of the conservation law that this field satisfies exactly (same section)."""

    def __init__(self, gamma=1.4, Pr=0.71, M0=0.15, a=0.8, b=0.85, Re0=0.1):
        self.dim = 2
        self.gamma, self.Pr, self.M0, self.a, self.b = gamma, Pr, M0, a, b
        self.cv = 1.0 / (gamma - 1.0)
        self.V0, self.L = 1.0, 1.0
        self.P0 = 1.0 / (gamma * M0 ** 2)
        self.mu = 1.0 / Re0
        self.T0 = self.V0 ** 2 / ((gamma - 1.0) * gamma * M0 ** 2 * self.cv)

    def prim(self, x):
        y = x[1] / self.L
        g, cv = self.gamma, self.cv
        T = self.T0 * (self.a + y * (self.b - self.a)) + self.V0 ** 2 * self.Pr / (2 * cv * g) * y * (1 - y)
        p = self.P0 * np.ones_like(y)
        rho = p / ((g - 1.0) * cv * T)
        return np.stack([rho, self.V0 * y * np.log(1 + y), 0 * y, p])

    def source(self, x):
        """(4, N) right-hand side of the conservation law (mass, x and y momentum, energy)."""
        y = np.asarray(x[1]) / self.L
        lg = np.log(1 + y)
        mu, V0, L = self.mu, self.V0, self.L
        sx = -mu * V0 / L ** 2 * (2 + y) / (1 + y) ** 2
        se = -mu * V0 ** 2 / L ** 2 * (lg ** 2 + y * lg / (1 + y) + (y * (3 + 2 * y) * lg - 2 * y - 1) / (1 + y) ** 2)
        z = 0 * y
        return np.stack([z, sx, z, se])


class Ringleb(Field):
    """Steady Ringleb flow (real points only; gamma = 1.4 is built into its hodograph).

    With c the speed of sound and V the speed, c^2 = 1 - V^2 / 5 and
    A(c) = 1/c + 1/(3c^3) + 1/(5c^5) - ln((1 + c) / (1 - c)) / 2, the point (x, y) lies on
    (x - A/2)^2 + y^2 = 1 / (4 c^10 V^4); its streamline parameter is
    psi^2 = 1 / (2V^2) - c^5 (x - A/2) and the flow angle theta = arcsin(psi V).  Then
    rho = c^5, p = c^7 / gamma and V = V (cos theta, sin theta).  The root in c is unique
    in (1/2, 1) on the example's square (-5, -1) x (1, 5) (subsonic there, c > 0.95) and is
    found by bisection."""

    gamma = 1.4

    def __init__(self):
        self.dim = 2

    @staticmethod
    def _A(c):
        return 1.0 / c + 1.0 / (3.0 * c ** 3) + 1.0 / (5.0 * c ** 5) - 0.5 * np.log((1.0 + c) / (1.0 - c))

    def _f(self, c, x, y):
        V2 = 5.0 * (1.0 - c * c)
        return (x - 0.5 * self._A(c)) ** 2 + y * y - 1.0 / (4.0 * c ** 10 * V2 * V2)

    def speed_of_sound(self, x):
        x0, y0 = np.asarray(x[0], float), np.asarray(x[1], float)
        lo = np.full(x0.shape, 0.5)
        hi = np.full(x0.shape, 1.0 - 1e-14)
        if np.any(self._f(lo, x0, y0) <= 0.0) or np.any(self._f(hi, x0, y0) >= 0.0):
            raise ValueError("point outside the bracketed Ringleb region")
        for _ in range(64):
            mid = 0.5 * (lo + hi)
            pos = self._f(mid, x0, y0) > 0.0
            lo = np.where(pos, mid, lo)
            hi = np.where(pos, hi, mid)
        return 0.5 * (lo + hi)

    def prim(self, x):
        c = self.speed_of_sound(x)
        V = np.sqrt(5.0 * (1.0 - c * c))
        psi = np.sqrt(1.0 / (2.0 * V * V) - c ** 5 * (np.asarray(x[0], float) - 0.5 * self._A(c)))
        th = np.arcsin(np.clip(psi * V, -1.0, 1.0))
        return np.stack([c ** 5, V * np.cos(th), V * np.sin(th), c ** 7 / self.gamma])


class ShuVortex(Field):
    """Homentropic vortex advected by a uniform stream, at t = 0."""

    def __init__(self, psi=5.0, mach=0.5, L=0.1, center=(0.5, 0.5), rho_inf=1.0,
                 v_inf=1.0, gamma=1.4):
        self.dim = 2
        self.psi, self.mach, self.L = psi, mach, L
        self.center = np.asarray(center, float)
        self.rho_inf, self.v_inf, self.gamma = rho_inf, v_inf, gamma

    def prim(self, x):
        g = self.gamma
        X = x[0] - self.center[0]
        Y = x[1] - self.center[1]
        r2 = (X * X + Y * Y) / self.L ** 2
        e1 = np.exp(1.0 - r2)
        amp = self.psi ** 2 * self.mach ** 2 * (g - 1.0) / (16.0 * np.pi ** 2)
        rho = self.rho_inf * (1.0 - amp * e1 * e1) ** (1.0 / (g - 1.0))
        vx = self.v_inf * (1.0 - self.psi * Y / (2 * np.pi * self.L) * e1)
        vy = self.v_inf * self.psi * X / (2 * np.pi * self.L) * e1
        p = self.rho_inf ** (1.0 - g) * self.v_inf ** 2 / (g * self.mach ** 2) * rho ** g
        return np.stack([rho, vx, vy, p])


class TaylorGreen(Field):
    """Taylor-Green vortex initial state on a 2*pi*L periodic box."""

    def __init__(self, mach=0.1, rho0=1.0, v0=1.0, L=1.0, gamma=1.4, phase=(0.0, 0.0, 0.0)):
        self.dim = 3
        self.mach, self.rho0, self.v0, self.L, self.gamma = mach, rho0, v0, L, gamma
        self.p0 = rho0 * v0 ** 2 / (gamma * mach ** 2)
        self.phase = np.asarray(phase, float)

    def prim(self, x):
        X = x[0] / self.L + self.phase[0]
        Y = x[1] / self.L + self.phase[1]
        Z = x[2] / self.L + self.phase[2]
        rho = self.rho0 * np.ones_like(X)
        vx = self.v0 * np.sin(X) * np.cos(Y) * np.cos(Z)
        vy = -self.v0 * np.cos(X) * np.sin(Y) * np.cos(Z)
        vz = 0.0 * X
        p = self.p0 + self.rho0 * self.v0 ** 2 / 16.0 * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
        return np.stack([rho, vx, vy, vz, p])


class OctantTaylorGreen(TaylorGreen):
    """Taylor-Green velocity with a background pressure set by a Mach number per octant.

    Octant o = 4 b_z + 2 b_y + b_x with b = 1 on (pi L, 2 pi L) of an axis.  The
    squared octant Mach numbers are blended with the periodic, analytic
    indicator s(x) = (1 - tanh(sin(x / L) / delta)) / 2 per axis (delta = 0.5)
    and the background pressure is 1 / (gamma M^2(x)): the entropy variable
    v_m is proportional to M^2, so it varies smoothly between the octant values
    and high-order interpolation stays physical (a pressure jump of up to
    (0.8 / 0.1)^2 would not).
    """

    def __init__(self, machs, rho0=1.0, v0=1.0, L=1.0, gamma=1.4, delta=0.5):
        super().__init__(mach=float(np.min(machs)), rho0=rho0, v0=v0, L=L, gamma=gamma)
        self.machs = np.asarray(machs, float)
        self.delta = delta

    def prim(self, x):
        base = super().prim(x)
        s = [0.5 * (1.0 - np.tanh(np.sin(x[a] / self.L) / self.delta)) for a in range(3)]
        m2 = 0.0
        for o in range(8):
            w = 1.0
            for a in range(3):
                w = w * (s[a] if (o >> a) & 1 else 1.0 - s[a])
            m2 = m2 + w * self.machs[o] ** 2
        p0 = self.rho0 * self.v0 ** 2 / (self.gamma * m2)
        return np.concatenate([base[:4], (base[4] - self.p0 + p0)[None]])


class SmoothNoise(Field):
    """base * (1 + eps*eta) for rho and p; V + eps*vref*eta for velocity.

    eta is a sum of 4 seeded sinusoids per component with integer wave numbers
    1..3 on the box [lo, lo+length]^d and amplitudes summing to 1, so |eta| <= 1.
    """

    def __init__(self, base: Field, eps: float, rng, lo, length, vref=1.0, nmodes=4):
        self.base, self.eps, self.vref = base, eps, vref
        self.dim = base.dim
        self.lo = np.asarray(lo, float)
        self.length = np.asarray(length, float)
        m = self.dim + 2
        self.k = rng.integers(1, 4, size=(m, nmodes, self.dim)) * rng.choice([-1, 1], size=(m, nmodes, self.dim))
        self.phi = rng.uniform(0, 2 * np.pi, size=(m, nmodes))
        a = rng.uniform(0.5, 1.0, size=(m, nmodes))
        self.a = a / a.sum(axis=1, keepdims=True)

    def eta(self, x):
        m = self.dim + 2
        out = []
        for c in range(m):
            acc = 0.0 * x[0]
            for s in range(self.k.shape[1]):
                arg = self.phi[c, s]
                for ax in range(self.dim):
                    arg = arg + 2 * np.pi * self.k[c, s, ax] * (x[ax] - self.lo[ax]) / self.length[ax]
                acc = acc + self.a[c, s] * np.sin(arg)
            out.append(acc)
        return np.stack(out)

    def prim(self, x):
        b = self.base.prim(x)
        e = self.eta(x)
        m = b.shape[0]
        out = [b[0] * (1 + self.eps * e[0])]
        for c in range(1, m - 1):
            out.append(b[c] + self.eps * self.vref * e[c])
        out.append(b[m - 1] * (1 + self.eps * e[m - 1]))
        return np.stack(out)


def node_noise(prim, grad, eps, rng, vref=1.0):
    """Add the per-node i.i.d. U(-eps, eps) perturbation to primitives (and gradients).

    rho and p are perturbed relatively, V by eps*vref.  Gradients get a
    perturbation of eps times the RMS of each gradient component over the
    points (so that q differs from the gradient of v at the nodes).
    """
    m, N = prim.shape
    xi = rng.uniform(-1.0, 1.0, size=(m, N))
    out = prim.copy()
    out[0] *= 1 + eps * xi[0]
    out[1:m - 1] += eps * vref * xi[1:m - 1]
    out[m - 1] *= 1 + eps * xi[m - 1]
    gout = None
    if grad is not None:
        scale = np.sqrt(np.mean(grad ** 2, axis=2, keepdims=True)) + 1e-300
        gout = grad + eps * scale * rng.uniform(-1.0, 1.0, size=grad.shape)
    return out, gout
