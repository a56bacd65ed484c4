"""Named synthetic workloads with seeded meshes, states and physical parameters.

The recipes follow the paper's own test states (Shu vortex, Taylor-Green
vortex) on the element counts and orders of the measured configurations:

* ``euler2d_tri_p2``  -- unit square, 8x8 squares split SW-NE (128 triangles),
  interior vertices jittered by up to 10% of h, p = 2, Euler, gamma = 1.4,
  Shu vortex (psi = 5, M = 0.5, L = 0.1, centred) + 1% noise, steady
  (alpha = 0), Dirichlet-trace boundary faces with the noise-free vortex.
  ``periodic=True`` gives the doubly periodic variant.
* ``ns3d_hex``        -- [0, 2 pi]^3 periodic, n^3 trilinear hexes jittered by
  up to ``jitter`` of h, order p, Navier-Stokes with Re = 1600 (mu = 1/Re with
  rho0 = V0 = L = 1), Pr = 0.72, gamma = 1.4, Taylor-Green state at Mach 0.1
  plus ``eps`` noise; mass coefficient alpha = 1/(a_ii dt) with the paper's
  TGV step dt = 5.71e-2 and the DIRK(3,3) diagonal a_ii.
  n = 16, p = 2, eps = 2% is the 4096-element measured case; n = 32, p = 3,
  eps = 5% the large mixed-precision case.

Seeds: ``numpy.random.default_rng([config_id, purpose])`` with purpose
0 mesh jitter, 1 smooth noise, 2 node noise of v and q, 3 node noise of v_hat.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fields as F
from . import meshes as M

DIRK33_AII = 0.435866521508459   # diagonal of Alexander's L-stable DIRK(3,3)
TGV_DT = 5.71e-2


@dataclass
class Workload:
    name: str
    config_id: int
    mesh: M.Mesh
    p: int
    scheme: str
    gamma: float
    mu: float
    Pr: float
    alpha: float
    viscous: bool
    field_clean: F.Field
    eps: float
    vref: float
    face_bc: np.ndarray
    tmap: np.ndarray = None
    n_trace: int = 0
    extra: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.tmap is None:
            self.tmap, self.n_trace = M.trace_map(self.mesh, self.p, self.scheme)

    @property
    def dim(self):
        return self.mesh.dim

    @property
    def m(self):
        return self.mesh.dim + 2

    def noisy_field(self):
        rng = np.random.default_rng([self.config_id, 1])
        return F.SmoothNoise(self.field_clean, self.eps, rng, self.mesh.extent, self.mesh.length,
                             vref=self.vref)

    def sample(self, x_nodes: np.ndarray, x_trace: np.ndarray):
        """Primitive inputs at the given coordinates.

        x_nodes: (d, E*Np) element node coordinates; x_trace: (d, n_trace).
        Returns dict with
          prim (m, E*Np), grad (m, d, E*Np) or None  -- noisy state for v, q
          prim_hat (m, n_trace)                       -- noisy state for v_hat
          prim_star (m, E*Np)                         -- noise-free state for u*
          prim_bc (m, n_trace)                        -- noise-free state for v_bc
        """
        nf = self.noisy_field()
        prim, grad = nf.prim_and_grad(x_nodes)
        rng = np.random.default_rng([self.config_id, 2])
        prim, grad = F.node_noise(prim, grad if self.viscous else None, self.eps / 10, rng, self.vref)
        ph, _ = nf.prim_and_grad(x_trace)
        rng = np.random.default_rng([self.config_id, 3])
        ph, _ = F.node_noise(ph, None, self.eps / 10, rng, self.vref)
        pstar = np.real(self.field_clean.prim(x_nodes.astype(complex)))
        pbc = np.real(self.field_clean.prim(x_trace.astype(complex)))
        return dict(prim=prim, grad=grad, prim_hat=ph, prim_star=pstar, prim_bc=pbc)


def euler2d_tri_p2(n=8, p=2, periodic=False, scheme="hdg", eps=0.01, jitter=0.1, config_id=1):
    mesh = M.tri_square(n, jitter, seed=[config_id, 0], periodic=periodic)
    face_bc = mesh.boundary.astype(np.int32)
    fld = F.ShuVortex(psi=5.0, mach=0.5, L=0.1, center=(0.5, 0.5))
    return Workload("euler2d_tri_p%d_%dx%d%s" % (p, n, n, "_periodic" if periodic else ""),
                    config_id, mesh, p, scheme, 1.4, 0.0, 0.72, 0.0, False, fld, eps, 1.0, face_bc)


def ns3d_hex(n=16, p=2, eps=0.02, jitter=0.05, mach=0.1, re=1600.0, scheme="hdg", config_id=2,
             alpha=None):
    mesh = M.hex_cube(n, jitter, seed=[config_id, 0], periodic=True)
    face_bc = np.zeros((mesh.n_elem, 6), dtype=np.int32)
    fld = F.TaylorGreen(mach=mach)
    a = 1.0 / (DIRK33_AII * TGV_DT) if alpha is None else alpha
    return Workload("ns3d_hex_p%d_%d^3" % (p, n), config_id, mesh, p, scheme, 1.4, 1.0 / re, 0.72,
                    a, True, fld, eps, 1.0, face_bc)


def euler3d_hex(n=2, p=2, eps=0.02, jitter=0.05, mach=0.3, config_id=6):
    mesh = M.hex_cube(n, jitter, seed=[config_id, 0], periodic=True)
    face_bc = np.zeros((mesh.n_elem, 6), dtype=np.int32)
    fld = F.TaylorGreen(mach=mach)
    return Workload("euler3d_hex_p%d_%d^3" % (p, n), config_id, mesh, p, "hdg", 1.4, 0.0, 0.72,
                    0.0, False, fld, eps, 1.0, face_bc)


def ns2d_tri(n=3, p=2, eps=0.02, jitter=0.1, mach=0.3, re=100.0, config_id=7, alpha=5.0):
    """Small 2D Navier-Stokes case on periodic split squares (parity / brute force)."""
    mesh = M.tri_square(n, jitter, seed=[config_id, 0], periodic=True, lo=0.0, length=2 * np.pi)
    face_bc = np.zeros((mesh.n_elem, 3), dtype=np.int32)

    class TG2(F.Field):
        dim = 2

        def prim(self, x):
            X, Y = x[0], x[1]
            p0 = 1.0 / (1.4 * mach ** 2)
            return np.stack([1.0 + 0.0 * X, np.sin(X) * np.cos(Y), -np.cos(X) * np.sin(Y),
                             p0 + 0.25 * (np.cos(2 * X) + np.cos(2 * Y))])
    return Workload("ns2d_tri_p%d_%dx%d" % (p, n, n), config_id, mesh, p, "hdg", 1.4, 1.0 / re, 0.72,
                    alpha, True, TG2(), eps, 1.0, face_bc)


def ns3d_tet(n=2, p=2, eps=0.02, jitter=0.05, mach=0.3, re=1.0e4, config_id=8, alpha=None):
    """Periodic Kuhn tetrahedra (6 per cube) with the Taylor-Green state."""
    mesh = M.kuhn_tets(n, jitter, seed=[config_id, 0], periodic=True)
    face_bc = np.zeros((mesh.n_elem, 4), dtype=np.int32)
    fld = F.TaylorGreen(mach=mach)
    a = 1.0 / (DIRK33_AII * TGV_DT) if alpha is None else alpha
    return Workload("ns3d_tet_p%d_%d^3x6" % (p, n), config_id, mesh, p, "hdg", 1.4, 1.0 / re, 0.72, a, True, fld,
                    eps, 1.0, face_bc)


def mixed_batch(n_tet=15, n_hex=16, orders=(1, 2, 3, 4), jitter=0.05, eps=0.02, re=1.0e4, config_id=3,
                with_hex=True):
    """Mixed batch of Navier-Stokes elements for one persistent launch.

    n_tet^3 x 6 periodic Kuhn tetrahedra (15 -> 20,250) with the order of each
    element drawn uniformly from `orders` (seed [config_id, 4]), plus the
    n_hex^3 periodic p = 2 hex mesh (16 -> 4,096); Taylor-Green velocity with
    the background pressure of a Mach number per octant, M ~ U(0.1, 0.8)
    (seed [config_id, 6]); Re = 1e4, Pr = 0.72, DIRK stage mass term.  Each
    element uses a trace space of its own order, so the batch is one workload
    per order: the tetrahedra of order p form a sub-mesh whose faces towards
    elements of another order are Dirichlet-trace faces (v_bc from the clean
    state).  Returns a list of Workloads.
    """
    rng = np.random.default_rng([config_id, 4])
    tets = M.kuhn_tets(n_tet, jitter, seed=[config_id, 0], periodic=True)
    pk = np.asarray(orders)[rng.integers(0, len(orders), size=tets.n_elem)]
    machs = np.random.default_rng([config_id, 6]).uniform(0.1, 0.8, size=8)
    fld = F.OctantTaylorGreen(machs)
    a = 1.0 / (DIRK33_AII * TGV_DT)
    out = []
    for p in orders:
        sel = np.nonzero(pk == p)[0]
        if len(sel) == 0:
            continue
        sub = M.subset_mesh(tets, sel)
        out.append(Workload("mixed_tet_p%d" % p, config_id, sub, int(p), "hdg", 1.4, 1.0 / re, 0.72, a, True, fld,
                            eps, 1.0, sub.boundary.astype(np.int32)))
    if with_hex:
        hexes = M.hex_cube(n_hex, jitter, seed=[config_id, 5], periodic=True)
        out.append(Workload("mixed_hex_p2", config_id, hexes, 2, "hdg", 1.4, 1.0 / re, 0.72, a, True, fld, eps, 1.0,
                            np.zeros((hexes.n_elem, 6), dtype=np.int32)))
    return out
