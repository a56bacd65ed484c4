"""GMRES(m) with right preconditioning and block-Jacobi (oracle; test infrastructure only).

Not in the paper (which does not describe its linear solver); the global trace
system sum_K P_K^T S_K P_K dlambda = sum_K P_K^T g_K is solved here with
restarted GMRES (Saad & Schultz) in its textbook form: Arnoldi with modified
Gram-Schmidt, Givens rotations on the Hessenberg matrix, right
preconditioning x = x0 + M^-1 V y.  Block-Jacobi takes the diagonal blocks of
the assembled operator over a partition of the unknowns and inverts them.
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, b, precond=None, restart=50, tol=1e-10, maxit=1000, x0=None):
    """Returns (x, iterations, history of relative residual estimates)."""
    n = b.shape[0]
    M = (lambda v: v) if precond is None else precond
    x = np.zeros(n) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, [0.0]
    hist = []
    it = 0
    while it < maxit:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta / bnorm <= tol:
            break
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        gvec = np.zeros(restart + 1)
        gvec[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(restart):
            w = matvec(M(V[j]))
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            it += 1
            j_done = j + 1
            hist.append(abs(gvec[j + 1]) / bnorm)
            if abs(gvec[j + 1]) / bnorm <= tol or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), gvec[:j_done])
        x = x + M(V[:j_done].T @ y)
    return x, it, hist


def block_jacobi(K, groups):
    """Inverses of the diagonal blocks of sparse K over index groups (list of index arrays)."""
    Kc = K.tocsr()
    invs = [np.linalg.inv(Kc[g][:, g].toarray()) for g in groups]

    def apply(v):
        out = np.zeros_like(v)
        for g, Bi in zip(groups, invs):
            out[g] = Bi @ v[g]
        return out
    return apply, invs


def face_groups(disc):
    """Unknown index groups of the faces (HDG: every trace node on exactly one face)."""
    seen = {}
    for e in range(disc.mesh.n_elem):
        for f in range(disc.nf):
            key = tuple(sorted(disc.tmap[e, f]))
            seen.setdefault(key, None)
    groups = []
    for key in seen:
        nodes = np.array(key)
        groups.append((np.arange(disc.m)[:, None] * disc.n_trace + nodes[None, :]).reshape(-1))
    return groups


def point_groups(disc):
    """Unknown index groups of single trace nodes (all m components of one node)."""
    comps = np.arange(disc.m) * disc.n_trace
    return [comps + t for t in range(disc.n_trace)]


def faces_are_disjoint(disc):
    """True when every trace node lies on exactly one mesh face (HDG trace spaces)."""
    owner = {}
    for e in range(disc.mesh.n_elem):
        for f in range(disc.nf):
            key = tuple(sorted(disc.tmap[e, f]))
            for t in key:
                if owner.setdefault(int(t), key) != key:
                    return False
    return True


def trace_groups(disc):
    """Face groups where faces are disjoint, point groups otherwise."""
    return face_groups(disc) if faces_are_disjoint(disc) else point_groups(disc)
