"""Reference elements: nodes, quadrature and nodal Lagrange bases (oracle).

The paper fixes only the polynomial spaces (section on finite element spaces:
P_k on simplices; the tensor space on quads / hexes is the usual Q_k reading).
The node sets and quadrature are this implementation's reading:

* nodes: Gauss-Lobatto-Legendre tensor lattice on [-1,1]^d (quad / hex),
  equispaced barycentric lattice on the unit simplex (tri / tet); node order as
  in ``workloads.meshes``;
* volume quadrature: tensor Gauss-Legendre with p+2 points per direction;
  on simplices the collapsed (Duffy) map of that tensor rule;
* face quadrature: the same rules in d-1 dimensions on the face
  parametrization.

The Lagrange basis is built from the inverse of the monomial Vandermonde
matrix (plain and obviously correct for p <= 4).
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
from numpy.polynomial import legendre as npleg

from workloads.meshes import ETYPE_DIM, face_nodes, node_multi_indices


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule on [-1, 1]."""
    x, w = npleg.leggauss(n)
    return x, w


def gll_points(p: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points: -1, roots of P_p', +1 (ascending)."""
    if p == 0:
        return np.array([0.0])
    if p == 1:
        return np.array([-1.0, 1.0])
    dP = npleg.Legendre.basis(p).deriv()
    r = np.sort(np.real(dP.roots()))
    # one Newton polish on P_p'
    d2P = dP.deriv()
    r = r - dP(r) / d2P(r)
    return np.concatenate([[-1.0], r, [1.0]])


def exponents(etype: str, p: int) -> np.ndarray:
    """Monomial exponents spanning P_p (simplices) or Q_p (tensor elements)."""
    d = ETYPE_DIM[etype]
    out = []
    if etype in ("quad", "hex"):
        rng = range(p + 1)
        for e in np.ndindex(*([p + 1] * d)):
            out.append(e)
    else:
        for e in np.ndindex(*([p + 1] * d)):
            if sum(e) <= p:
                out.append(e)
    return np.array(out, dtype=np.int64)


def monomials(x: np.ndarray, ex: np.ndarray):
    """Values (N, M) and gradients (N, M, d) of monomials x^ex at points x (N, d)."""
    N, d = x.shape
    val = np.ones((N, ex.shape[0]))
    for a in range(d):
        val = val * x[:, a:a + 1] ** ex[None, :, a]
    grad = np.zeros((N, ex.shape[0], d))
    for a in range(d):
        g = np.ones((N, ex.shape[0]))
        for b in range(d):
            if b == a:
                e = ex[None, :, b]
                g = g * np.where(e > 0, e * x[:, b:b + 1] ** np.maximum(e - 1, 0), 0.0)
            else:
                g = g * x[:, b:b + 1] ** ex[None, :, b]
        grad[:, :, a] = g
    return val, grad


def ref_vertices(etype: str) -> np.ndarray:
    if etype == "tri":
        return np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    if etype == "tet":
        return np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0], [0.0, 0, 1]])
    d = ETYPE_DIM[etype]
    return np.array([[(-1.0 if (c >> a) & 1 == 0 else 1.0) for a in range(d)]
                     for c in range(2 ** d)])


def ref_nodes(etype: str, p: int) -> np.ndarray:
    mi = node_multi_indices(etype, p).astype(float)
    if etype in ("quad", "hex"):
        r = gll_points(p)
        return r[mi.astype(int)]
    return mi / p


def simplex_rule(d: int, n: int):
    """Collapsed Gauss-Legendre rule on the unit simplex with n points per direction."""
    g, w = gauss_legendre(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    pts, wts = [], []
    if d == 1:
        return g[:, None], w
    if d == 2:
        for ib in range(n):
            for ia in range(n):
                a, b = g[ia], g[ib]
                pts.append((a * (1 - b), b))
                wts.append(w[ia] * w[ib] * (1 - b))
    else:
        for ic in range(n):
            for ib in range(n):
                for ia in range(n):
                    a, b, c = g[ia], g[ib], g[ic]
                    pts.append((a * (1 - b) * (1 - c), b * (1 - c), c))
                    wts.append(w[ia] * w[ib] * w[ic] * (1 - b) * (1 - c) ** 2)
    return np.array(pts), np.array(wts)


def tensor_rule(d: int, n: int):
    g, w = gauss_legendre(n)
    pts, wts = [], []
    for idx in np.ndindex(*([n] * d)):
        idx = idx[::-1]  # first coordinate fastest
        pts.append([g[i] for i in idx])
        wts.append(np.prod([w[i] for i in idx]))
    return np.array(pts), np.array(wts)


class RefElem:
    """Tables of one reference element of type ``etype`` and order ``p``."""

    def __init__(self, etype: str, p: int, nquad: int | None = None):
        self.etype, self.p = etype, p
        self.dim = d = ETYPE_DIM[etype]
        self.nquad = nquad if nquad is not None else p + 2
        self.nodes = ref_nodes(etype, p)
        self.np_ = self.nodes.shape[0]
        self.ex = exponents(etype, p)
        V, _ = monomials(self.nodes, self.ex)
        self.coef = np.linalg.inv(V)              # phi(x) = mono(x) @ coef
        self.verts = ref_vertices(etype)
        self.face_nodes = face_nodes(etype, p)
        self.nf = len(self.face_nodes)
        self.nfp = len(self.face_nodes[0])
        # volume rule
        if etype in ("quad", "hex"):
            self.xq, self.wq = tensor_rule(d, self.nquad)
        else:
            self.xq, self.wq = simplex_rule(d, self.nquad)
        self.phi, self.dphi = self.basis(self.xq)
        # faces: parametrization xi(s) = o + T s, reference outward normal
        self.faces = [self._face(f) for f in range(self.nf)]

    def basis(self, x):
        val, grad = monomials(np.atleast_2d(x), self.ex)
        return val @ self.coef, np.einsum("nmd,ma->nad", grad, self.coef)

    def _face(self, f):
        d, et = self.dim, self.etype
        if et in ("quad", "hex"):
            ax, side = divmod(f, 2)
            free = [a for a in range(d) if a != ax]
            o = np.zeros(d)
            o[ax] = -1.0 if side == 0 else 1.0
            T = np.zeros((d, d - 1))
            for r, a in enumerate(free):
                T[a, r] = 1.0
            s, w = tensor_rule(d - 1, self.nquad)
            nref = np.zeros(d)
            nref[ax] = -1.0 if side == 0 else 1.0
        else:
            vs = [r for r in range(d + 1) if r != f]
            V = self.verts
            o = V[vs[0]].copy()
            T = np.stack([V[vs[r]] - V[vs[0]] for r in range(1, d)], axis=1)
            s, w = simplex_rule(d - 1, self.nquad)
            if f == 0:
                nref = np.ones(d) / np.sqrt(d)
            else:
                nref = np.zeros(d)
                nref[f - 1] = -1.0
        xi = o[None, :] + s @ T.T
        # orientation of the raw normal built from the parametrization tangents
        if d == 2:
            raw = np.array([T[1, 0], -T[0, 0]])
        else:
            raw = np.cross(T[:, 0], T[:, 1])
        sign = 1.0 if raw @ nref > 0 else -1.0
        phi, dphi = self.basis(xi)
        fn = self.face_nodes[f]
        return dict(xi=xi, w=w, T=T, sign=sign, nref=nref, phi=phi, dphi=dphi,
                    psi=phi[:, fn], nodes=fn)


@lru_cache(maxsize=None)
def get_refelem(etype: str, p: int, nquad: int | None = None) -> RefElem:
    return RefElem(etype, p, nquad)
