"""Element residual, Jacobian and static condensation (oracle).

Weak forms (paper, sections on the entropy-variable hybridized DG methods for
Euler and for Navier-Stokes).  With nodal test functions phi_a, trace test
functions mu_b and the local ordering

    x_K = [ v (c*Np + a) ; q (m*Np + (c*d + j)*Np + a) ],
    lambda_K = v_hat on the element faces (f*(m*Nfp) + c*Nfp + b),

the element rows are

    R_v[c,a]   = alpha (u(v_h) - u*, phi_a)_K - (F + G, grad phi_a)_K
                 + <f_hat + g_hat, phi_a>_dK                      (element eq.)
    R_q[c,j,a] = (q_cj, phi_a)_K + (v_c, d phi_a / dx_j)_K
                 - <v_hat_c n_j, phi_a>_dK                       (gradient eq.)

and the element's share of the trace equation is

    R_tr[f,c,b] = <f_hat + g_hat, mu_b>_F       (interior / periodic faces)
    R_tr[f,c,b] = <v_hat - v_bc, mu_b>_F        (Dirichlet-trace faces)
    R_tr[f,c,b] = 0                             (other faces at a node of a Dirichlet face)

The last case only arises with a continuous trace (EDG): a trace node shared by a
Dirichlet face and interior faces keeps the Dirichlet condition alone, so the
boundary value is imposed at the node rather than mixed with flux balances of
other faces (the paper leaves the boundary operator open; HDG and IEDG traces
never share a node across a Dirichlet face).

The mass term alpha (u(v_h) - u*, w) stands in for the time derivative of a
backward-Euler or DIRK stage (alpha = 1 / (a_ii dt); alpha = 0 is steady);
Euler drops q, G and R_q.  The Newton system per element is

    [A B; C D] [dx; dlambda] = -[R_loc; R_tr],

A = dR_loc/dx, B = dR_loc/dlambda, C = dR_tr/dx, D = dR_tr/dlambda, all taken
here by complex step of the whole element residual (exact to rounding).
Static condensation (the paper notes the element equations eliminate q_h and
v_h locally, leaving v_hat globally coupled):

    Y = A^-1 B,  z = A^-1 R_loc,  S = D - C Y,  g = -R_tr + C z,
    (sum_K P_K^T S_K P_K) dlambda = sum_K P_K^T g_K,   dx_K = -z_K - Y_K P_K dlambda.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import physics as ph
from .geometry import ElemGeom
from .refelem import get_refelem

CS_H = 1e-30


@dataclass
class Phys:
    gamma: float = 1.4
    mu: float = 0.0
    Pr: float = 0.72
    alpha: float = 0.0
    viscous: bool = False
    # viscous numerical flux: G(v_hat, q) . n (the one used in the paper's examples) or, with
    # ghat_interior, G(v, q) . n with the element's v (the first of the two choices of Section 3.3)
    ghat_interior: bool = False
    # stabilization matrix: "slf" (symmetric Lax-Friedrichs, the paper's examples), "s"
    # (symmetric variable |A_n| A0), both at v* = v_hat, or "mv" (mean value between v_hat and v)
    sigma: str = "slf"
    # projection viscous numerical flux of Section 4: (Pi G(v_h, q_h)) . n with Pi the element L2
    # projection onto the polynomial space of q_h (overrides ghat_interior)
    ghat_proj: bool = False


class Discretization:
    """Oracle discretization of one mesh (single element type and order)."""

    def __init__(self, mesh, p: int, phys: Phys, tmap: np.ndarray, n_trace: int,
                 face_bc: np.ndarray | None = None, nquad: int | None = None):
        self.mesh, self.p, self.phys = mesh, p, phys
        self.ref = get_refelem(mesh.etype, p, nquad)
        self.d = d = self.ref.dim
        self.m = m = d + 2
        self.Np, self.nf, self.Nfp = self.ref.np_, self.ref.nf, self.ref.nfp
        self.tmap = np.asarray(tmap)
        self.n_trace = n_trace
        self.face_bc = (np.zeros((mesh.n_elem, self.nf), dtype=np.int32)
                        if face_bc is None else np.asarray(face_bc))
        # trace nodes of Dirichlet-trace faces
        self.dir_node = np.zeros(n_trace, dtype=bool)
        self.dir_node[self.tmap[self.face_bc == 1].ravel()] = True
        self.n = m * self.Np * (1 + d) if phys.viscous else m * self.Np
        self.k = self.nf * m * self.Nfp
        self._geo = {}

    # -- geometry ------------------------------------------------------------
    def geom(self, e) -> ElemGeom:
        if e not in self._geo:
            self._geo[e] = ElemGeom(self.ref, self.mesh.elem_xyz[e])
        return self._geo[e]

    def node_coords(self):
        """(d, E*Np) element node coordinates, element-major."""
        out = np.stack([self.geom(e).node_coords(self.mesh.elem_xyz[e])
                        for e in range(self.mesh.n_elem)])
        return out.reshape(-1, self.d).T.copy()

    def trace_coords(self):
        """(d, n_trace) coordinates of the global trace nodes."""
        X = np.full((self.d, self.n_trace), np.nan)
        for e in range(self.mesh.n_elem):
            xn = self.geom(e).node_coords(self.mesh.elem_xyz[e])
            for f in range(self.nf):
                X[:, self.tmap[e, f]] = xn[self.ref.face_nodes[f]].T
        return X

    # -- packing ---------------------------------------------------------------
    def pack_local(self, v, q, e):
        """x_K from global SoA v (m, E*Np) and q (m*d, E*Np)."""
        sl = slice(e * self.Np, (e + 1) * self.Np)
        parts = [v[:, sl].reshape(-1)]
        if self.phys.viscous:
            parts.append(q[:, sl].reshape(-1))
        return np.concatenate(parts)

    def gather_trace(self, vhat, e):
        """lambda_K from the global trace field (m, n_trace)."""
        return vhat[:, self.tmap[e]].transpose(1, 0, 2).reshape(-1)

    def scatter_trace(self, r, e, out):
        """Add an element trace vector (k,) into a global (m, n_trace) array."""
        rr = r.reshape(self.nf, self.m, self.Nfp).transpose(1, 0, 2)
        for c in range(self.m):
            np.add.at(out[c], self.tmap[e].reshape(-1), rr[c].reshape(-1))

    # -- residual ----------------------------------------------------------------
    def element_residual(self, e, X, L, ustar_nodes=None, vbc_nodes=None, source=None):
        """Residual of element e for a batch of inputs.

        X: (P, n) local unknowns, L: (P, k) element trace unknowns (real or
        complex); ustar_nodes: (m, Np) nodal u* or None; vbc_nodes:
        (nf, m, Nfp) Dirichlet data at the face nodes or None; source: callable
        x (N, d) -> (N, m) right-hand side s of the strong form
        (du/dt + div(F + G) = s), tested against phi_a and subtracted.
        Returns R_loc (P, n), R_tr (P, k).
        """
        ph_, G = self.phys, self.geom(e)
        gam = ph_.gamma
        m, d, Np, Nfp, nf = self.m, self.d, self.Np, self.Nfp, self.nf
        P = X.shape[0]
        vN = X[:, :m * Np].reshape(P, m, Np)
        qN = X[:, m * Np:].reshape(P, m, d, Np) if ph_.viscous else None
        LN = L.reshape(P, nf, m, Nfp)
        phi, gphi, W = self.ref.phi, G.gphi, G.W

        vq = np.einsum("qa,pca->pqc", phi, vN)
        flux = ph.flux_F(vq, gam)
        if ph_.viscous:
            qq = np.einsum("qa,pcja->pqcj", phi, qN)
            flux = flux + ph.flux_G(vq, qq, gam, ph_.mu, ph_.Pr)
        Rv = -np.einsum("q,pqcj,qaj->pca", W, flux, gphi)
        if ph_.viscous and ph_.ghat_proj:
            # nodal coefficients of the element L2 projection of G(v_h, q_h): M Gpi = (phi_a, G)_K
            Gq = ph.flux_G(vq, qq, gam, ph_.mu, ph_.Pr)
            Mk = phi.T @ (W[:, None] * phi)
            rhs = np.einsum("q,qa,pqcj->apcj", W, phi, Gq)
            Gpi = np.linalg.solve(Mk, rhs.reshape(Np, -1)).reshape(Np, P, m, d).transpose(1, 0, 2, 3)
        if ph_.alpha != 0.0:
            us = np.zeros((phi.shape[0], m)) if ustar_nodes is None else phi @ ustar_nodes.T
            Rv = Rv + ph_.alpha * np.einsum("q,pqc,qa->pca", W, ph.u_of_v(vq, gam) - us, phi)
        if source is not None:
            Rv = Rv - np.einsum("q,qc,qa->ca", W, source(G.xq), phi)[None]
        if ph_.viscous:
            Rq = np.einsum("q,pqcj,qa->pcja", W, qq, phi) + np.einsum("q,pqc,qaj->pcja", W, vq, gphi)
        Rtr = []
        for f in range(nf):
            F = G.faces[f]
            vf = np.einsum("qa,pca->pqc", F["phi"], vN)
            vhf = np.einsum("qb,pcb->pqc", F["psi"], LN[:, f])
            nrm = F["n"]
            tf = ph.fhat(vhf, vf, nrm, gam, ph_.sigma)
            if ph_.viscous:
                if ph_.ghat_proj:
                    tf = tf + np.einsum("qa,pacj,qj->pqc", F["phi"], Gpi, nrm)
                else:
                    qf = np.einsum("qa,pcja->pqcj", F["phi"], qN)
                    tf = tf + ph.ghat(vf if ph_.ghat_interior else vhf, qf, nrm, gam, ph_.mu, ph_.Pr)
                Rq = Rq - np.einsum("q,pqc,qj,qa->pcja", F["W"], vhf, nrm, F["phi"])
            Rv = Rv + np.einsum("q,pqc,qa->pca", F["W"], tf, F["phi"])
            if self.face_bc[e, f] == 1:
                vb = np.zeros((m, Nfp)) if vbc_nodes is None else vbc_nodes[f]
                vbq = F["psi"] @ vb.T
                Rtr.append(np.einsum("q,pqc,qb->pcb", F["W"], vhf - vbq[None], F["psi"]))
            else:
                keep = ~self.dir_node[self.tmap[e, f]]
                Rtr.append(np.einsum("q,pqc,qb->pcb", F["W"], tf, F["psi"]) * keep)
        Rloc = Rv.reshape(P, -1)
        if ph_.viscous:
            Rloc = np.concatenate([Rloc, Rq.reshape(P, -1)], axis=1)
        return Rloc, np.stack(Rtr, axis=1).reshape(P, -1)

    def element_system(self, e, x, lam, ustar_nodes=None, vbc_nodes=None, source=None):
        """Residual and complex-step Jacobian blocks of element e.

        Returns dict with R_loc, R_tr, A, B, C, D.
        """
        n, k = self.n, self.k
        R0, T0 = self.element_residual(e, x[None], lam[None], ustar_nodes, vbc_nodes, source)
        I = np.eye(n + k)
        Xc = x[None, :].astype(complex) + 1j * CS_H * I[:, :n]
        Lc = lam[None, :].astype(complex) + 1j * CS_H * I[:, n:]
        Rc, Tc = self.element_residual(e, Xc, Lc, ustar_nodes, vbc_nodes, source)
        Jl = np.imag(Rc).T / CS_H          # (n, n+k)
        Jt = np.imag(Tc).T / CS_H          # (k, n+k)
        return dict(R_loc=R0[0], R_tr=T0[0], A=Jl[:, :n], B=Jl[:, n:], C=Jt[:, :n], D=Jt[:, n:])

    # -- per-element inputs --------------------------------------------------------
    def elem_inputs(self, e, v, q, vhat, ustar=None, vbc=None):
        x = self.pack_local(v, q, e)
        lam = self.gather_trace(vhat, e)
        us = None if ustar is None else ustar[:, e * self.Np:(e + 1) * self.Np]
        vb = None
        if vbc is not None:
            vb = vbc[:, self.tmap[e]].transpose(1, 0, 2)   # (nf, m, Nfp)
        return x, lam, us, vb


def condense(sysd):
    """Static condensation of one element (LAPACK solve with partial pivoting)."""
    A, B, C, D = sysd["A"], sysd["B"], sysd["C"], sysd["D"]
    rhs = np.concatenate([B, sysd["R_loc"][:, None]], axis=1)
    sol = np.linalg.solve(A, rhs)
    Y, z = sol[:, :-1], sol[:, -1]
    return dict(S=D - C @ Y, g=-sysd["R_tr"] + C @ z, Y=Y, z=z)


def assemble_condense(disc: Discretization, v, q, vhat, ustar=None, vbc=None, elems=None,
                      keep_blocks=False):
    """Per-element residual, Jacobian and condensed blocks for ``elems``."""
    elems = range(disc.mesh.n_elem) if elems is None else elems
    out = []
    for e in elems:
        x, lam, us, vb = disc.elem_inputs(e, v, q, vhat, ustar, vbc)
        s = disc.element_system(e, x, lam, us, vb)
        c = condense(s)
        if keep_blocks:
            c.update(s)
        else:
            c.update(R_loc=s["R_loc"], R_tr=s["R_tr"])
        out.append(c)
    return out


# ----------------------------------------------------------------------------
# global trace operator, solves
# ----------------------------------------------------------------------------
def element_trace_index(disc: Discretization, e):
    """Flat global index (c*n_trace + t) of each element trace row (k,)."""
    t = disc.tmap[e]                                     # (nf, Nfp)
    c = np.arange(disc.m)[None, :, None]
    return (c * disc.n_trace + t[:, None, :]).reshape(-1)


def trace_matvec(disc: Discretization, S_list, x):
    """y = sum_K P_K^T S_K P_K x on the flattened (m*n_trace) trace vector."""
    y = np.zeros_like(x)
    for e, S in enumerate(S_list):
        idx = element_trace_index(disc, e)
        np.add.at(y, idx, S @ x[idx])
    return y


def trace_matrix(disc: Discretization, S_list):
    rows, cols, vals = [], [], []
    for e, S in enumerate(S_list):
        idx = element_trace_index(disc, e)
        rows.append(np.repeat(idx, len(idx)))
        cols.append(np.tile(idx, len(idx)))
        vals.append(S.reshape(-1))
    N = disc.m * disc.n_trace
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def trace_rhs(disc: Discretization, g_list):
    r = np.zeros(disc.m * disc.n_trace)
    for e, g in enumerate(g_list):
        np.add.at(r, element_trace_index(disc, e), g)
    return r


def backsolve(disc: Discretization, Y_list, z_list, dlam):
    """dx_K = -z_K - Y_K P_K dlambda for every element."""
    return [-z - Y @ dlam[element_trace_index(disc, e)] for e, (Y, z) in enumerate(zip(Y_list, z_list))]


def brute_force_solve(disc: Discretization, blocks):
    """Solve the uncondensed global Newton system J delta = -R directly.

    ``blocks``: per element dict with A, B, C, D, R_loc, R_tr.  Returns
    (dx list, dlambda).
    """
    E, n = len(blocks), disc.n
    Nt = disc.m * disc.n_trace
    rows, cols, vals = [], [], []
    rhs = np.zeros(E * n + Nt)

    def add(r, c, M):
        rr, cc = np.meshgrid(r, c, indexing="ij")
        rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(M.ravel())

    for e, b in enumerate(blocks):
        li = e * n + np.arange(n)
        ti = E * n + element_trace_index(disc, e)
        add(li, li, b["A"]); add(li, ti, b["B"]); add(ti, li, b["C"]); add(ti, ti, b["D"])
        rhs[li] -= b["R_loc"]
        np.add.at(rhs, ti, -b["R_tr"])
    J = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(E * n + Nt, E * n + Nt))
    sol = spla.spsolve(J, rhs)
    return [sol[e * n:(e + 1) * n] for e in range(E)], sol[E * n:]
