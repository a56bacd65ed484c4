"""Element geometry at quadrature points (oracle).

Straight-sided simplices use the affine map from the reference simplex;
quads / hexes use the bi- / trilinear map of their 2^d corners.  (The paper
allows p-th degree curved elements; the workloads here are straight or
multilinear, which is this implementation's reading of the mesh.)

Face normals are built from the cross product (3D) or rotation (2D) of the
physical tangent vectors of the face parametrization, oriented with the
reference outward normal; the surface measure is the norm of that vector.
"""
from __future__ import annotations

import numpy as np

from .refelem import RefElem


def shape_functions(etype: str, xi: np.ndarray):
    """Vertex shape functions (N, nv) and their reference gradients (N, nv, d)."""
    N, d = xi.shape
    if etype in ("tri", "tet"):
        val = np.empty((N, d + 1))
        val[:, 0] = 1.0 - xi.sum(axis=1)
        val[:, 1:] = xi
        grad = np.zeros((N, d + 1, d))
        grad[:, 0, :] = -1.0
        for r in range(d):
            grad[:, r + 1, r] = 1.0
        return val, grad
    nv = 2 ** d
    val = np.ones((N, nv))
    grad = np.ones((N, nv, d))
    for c in range(nv):
        for a in range(d):
            sgn = 1.0 if (c >> a) & 1 else -1.0
            fac = 0.5 * (1.0 + sgn * xi[:, a])
            val[:, c] *= fac
            for b in range(d):
                grad[:, c, b] *= (0.5 * sgn) if b == a else fac
    return val, grad


def map_points(ref: RefElem, xyz: np.ndarray, xi: np.ndarray):
    """Physical points (N, d) and Jacobians J[n, i, r] = dx_i / dxi_r."""
    val, grad = shape_functions(ref.etype, xi)
    x = val @ xyz
    J = np.einsum("nvr,vi->nir", grad, xyz)
    return x, J


class ElemGeom:
    """Volume and face quadrature data of one element."""

    def __init__(self, ref: RefElem, xyz: np.ndarray):
        self.ref = ref
        d = ref.dim
        self.xq, J = map_points(ref, xyz, ref.xq)
        detJ = np.linalg.det(J)
        if np.any(detJ <= 0):
            raise ValueError("element with non-positive Jacobian determinant")
        Jinv = np.linalg.inv(J)                       # [n, r, i] = dxi_r / dx_i
        self.W = ref.wq * detJ                        # volume weights
        self.gphi = np.einsum("nar,nri->nai", ref.dphi, Jinv)   # physical gradients
        self.faces = []
        for F in ref.faces:
            xf, Jf = map_points(ref, xyz, F["xi"])
            Tphys = np.einsum("nir,rs->nis", Jf, F["T"])     # physical tangents
            if d == 2:
                raw = np.stack([Tphys[:, 1, 0], -Tphys[:, 0, 0]], axis=1)
            else:
                raw = np.cross(Tphys[:, :, 0], Tphys[:, :, 1])
            raw = F["sign"] * raw
            dS = np.linalg.norm(raw, axis=1)
            self.faces.append(dict(x=xf, n=raw / dS[:, None], W=F["w"] * dS,
                                   phi=F["phi"], psi=F["psi"], nodes=F["nodes"]))

    def node_coords(self, xyz):
        x, _ = map_points(self.ref, xyz, self.ref.nodes)
        return x
