"""Shared helpers for GPU parity tests: oracle inputs and GPU plans of a workload."""
import numpy as np

from oracle import hdg as ohdg
from oracle import state as ostate
from workloads import configs as C


def oracle_disc(wl, nquad=None, ghat_interior=False, sigma="slf", ghat_proj=False):
    return ohdg.Discretization(wl.mesh, wl.p, ohdg.Phys(wl.gamma, wl.mu, wl.Pr, wl.alpha, wl.viscous,
                                                        ghat_interior, sigma, ghat_proj),
                               wl.tmap, wl.n_trace, wl.face_bc, nquad)


def oracle_case(wl):
    disc = oracle_disc(wl)
    return disc, ostate.oracle_inputs(wl, disc)


def gpu_plan(wl, chunk_elems=0, split_dense=False, narrow_block=False, eliminate_q=False, ghat_interior=False,
             sigma="slf", ghat_proj=False):
    from paper_1808_05066_amd.hdg import Plan
    return Plan(wl.mesh.etype, wl.p, wl.mesh.elem_xyz, wl.tmap, wl.n_trace, wl.face_bc, viscous=wl.viscous,
                gamma=wl.gamma, mu=wl.mu, Pr=wl.Pr, alpha=wl.alpha, chunk_elems=chunk_elems,
                split_dense=split_dense, narrow_block=narrow_block, eliminate_q=eliminate_q,
                ghat_interior=ghat_interior, sigma=sigma, ghat_proj=ghat_proj)


def smooth_periodic_case(dt, n=2, p=2, mu=0.02, Pr=0.72, gamma=1.4):
    """Smooth periodic Navier-Stokes state on an n x n triangle mesh (seeded jitter); the
    discretization carries the DIRK(3,3) stage coefficient alpha = 1 / (a_ii dt).
    Returns (mesh data for a GPU plan, oracle discretization, v, q = 0, vhat)."""
    from oracle import newton, physics as ph
    from workloads import meshes as M
    mesh = M.tri_square(n, 0.05, 7, periodic=True)
    tmap, nt = M.trace_map(mesh, p, "hdg")
    alpha = 1.0 / (newton.DIRK33_G * dt)
    face_bc = np.zeros((mesh.n_elem, 3), dtype=np.int32)
    disc = ohdg.Discretization(mesh, p, ohdg.Phys(gamma, mu, Pr, alpha, True), tmap, nt, face_bc)

    def v_of(x):
        r = 1 + 0.1 * np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1])
        V = np.stack([0.3 + 0.05 * np.cos(2 * np.pi * x[1]), -0.2 + 0.05 * np.sin(2 * np.pi * x[0])], axis=-1)
        pp = 1 + 0.05 * np.cos(2 * np.pi * (x[0] + x[1]))
        return ph.v_of_prim(r, V, pp, gamma).T.copy()

    v0, vh0 = v_of(disc.node_coords()), v_of(disc.trace_coords())
    md = dict(mesh=mesh, p=p, tmap=tmap, n_trace=nt, face_bc=face_bc, mu=mu, Pr=Pr, gamma=gamma, alpha=alpha)
    return md, disc, v0, np.zeros((4 * 2, v0.shape[1])), vh0


def to_dev(inp):
    import torch
    out = {}
    for key in ("v", "q", "vhat", "ustar", "vbc"):
        a = inp.get(key)
        out[key] = None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return out


def rel_err_per_elem(gpu, ref):
    """max over elements of ||gpu - ref||_F / ||ref||_F (elements along axis 0)."""
    g = np.asarray(gpu).reshape(gpu.shape[0], -1)
    r = np.asarray(ref).reshape(ref.shape[0], -1)
    num = np.linalg.norm(g - r, axis=1)
    den = np.linalg.norm(r, axis=1)
    return float(np.max(num / np.where(den > 0, den, 1.0)))


def colmajor(mats):
    """Stack (rows x cols) numpy matrices into the (E, cols, rows) column-major layout."""
    return np.stack([np.asarray(M).T for M in mats])


SMALL_CASES = {
    "euler2d_tri_p2": lambda: C.euler2d_tri_p2(),
    "euler2d_tri_p2_periodic_edg": lambda: C.euler2d_tri_p2(n=4, periodic=True, scheme="edg"),
    "euler2d_tri_p2_iedg": lambda: C.euler2d_tri_p2(n=4, scheme="iedg"),
    "ns2d_tri_p2": lambda: C.ns2d_tri(n=3, p=2),
    "ns2d_tri_p3": lambda: C.ns2d_tri(n=2, p=3),
    "ns3d_hex_p1": lambda: C.ns3d_hex(n=3, p=1),
    "ns3d_hex_p2": lambda: C.ns3d_hex(n=2, p=2),
    "euler3d_hex_p2": lambda: C.euler3d_hex(n=2, p=2),
}


def residual_term_scale(disc, e, x, lam, ustar=None):
    """Norm of the element residual with every quadrature contribution in absolute value.

    R_loc is a sum of volume and face contributions that nearly cancel for
    states close to a discrete steady state; its floating-point error is
    bounded by eps times this sum of magnitudes, so parity of R_loc is stated
    relative to it.
    """
    return float(np.linalg.norm(residual_term_magnitudes(disc, e, x, lam, ustar)))


def residual_term_magnitudes(disc, e, x, lam, ustar=None):
    """Per row of R_loc, the sum of its quadrature contributions in absolute value."""
    from oracle import physics as ph
    G = disc.geom(e)
    m, d, Np, Nfp, nf = disc.m, disc.d, disc.Np, disc.Nfp, disc.nf
    gam, P = disc.phys.gamma, disc.phys
    vN = x[:m * Np].reshape(m, Np)
    qN = x[m * Np:].reshape(m, d, Np) if P.viscous else None
    LN = lam.reshape(nf, m, Nfp)
    phi, gphi, W = disc.ref.phi, G.gphi, np.abs(G.W)
    vq = phi @ vN.T
    flux = np.abs(ph.flux_F(vq, gam))
    if P.viscous:
        qq = np.einsum("qa,cja->qcj", phi, qN)
        flux = flux + np.abs(ph.flux_G(vq, qq, gam, P.mu, P.Pr))
    Tv = np.einsum("q,qcj,qaj->ca", W, flux, np.abs(gphi))
    if P.alpha:
        us = 0.0 if ustar is None else np.abs(phi @ ustar.T)
        Tv = Tv + P.alpha * np.einsum("q,qc,qa->ca", W, np.abs(ph.u_of_v(vq, gam)) + us, np.abs(phi))
    if P.viscous:
        Tq = np.einsum("q,qcj,qa->cja", W, np.abs(qq), np.abs(phi)) + \
            np.einsum("q,qc,qaj->cja", W, np.abs(vq), np.abs(gphi))
    for f in range(nf):
        F = G.faces[f]
        vf = F["phi"] @ vN.T
        vhf = F["psi"] @ LN[f].T
        tf = np.abs(0.5 * np.einsum("qcj,qj->qc", ph.flux_F(vhf, gam) + ph.flux_F(vf, gam), F["n"])) + \
            np.abs(0.5 * np.einsum("qab,qb->qa", ph.sigma_slf(vhf, F["n"], gam), vf - vhf))
        if P.viscous:
            qf = np.einsum("qa,cja->qcj", F["phi"], qN)
            tf = tf + np.abs(ph.ghat(vhf, qf, F["n"], gam, P.mu, P.Pr))
            Tq = Tq + np.einsum("q,qc,qj,qa->cja", np.abs(F["W"]), np.abs(vhf), np.abs(F["n"]), np.abs(F["phi"]))
        Tv = Tv + np.einsum("q,qc,qa->ca", np.abs(F["W"]), tf, np.abs(F["phi"]))
    out = Tv.reshape(-1)
    if P.viscous:
        out = np.concatenate([out, Tq.reshape(-1)])
    return out


def rloc_err(disc, inp, gpu_R, ref_R):
    """max over elements of ||R_gpu - R_oracle|| / (sum-of-magnitudes scale)."""
    worst = 0.0
    for e in range(gpu_R.shape[0]):
        x, lam, us, _ = disc.elem_inputs(e, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"])
        s = residual_term_scale(disc, e, x, lam, us)
        worst = max(worst, float(np.linalg.norm(gpu_R[e] - ref_R[e])) / s)
    return worst


def z_backward_err(disc, inp, e, A, R_loc, z_gpu):
    """||A z_gpu - R_loc|| over the summation scale of R_loc (element e, oracle A and R_loc).

    z = A^-1 R_loc inherits the cancellation of R_loc; two correct FP64 codes agree
    on z only to the rounding of R_loc amplified by A^-1, so z is judged by how
    well it solves A z = R_loc measured in R_loc's own scale.
    """
    x, lam, us, _ = disc.elem_inputs(e, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"])
    s = residual_term_scale(disc, e, x, lam, us)
    return float(np.linalg.norm(A @ z_gpu - R_loc)) / s


def z_forward_bound(disc, inp, e, A, R_loc, z):
    """Forward-error bound of z = A^-1 R_loc for element e, derived from the element's own data.

    Both codes form R_loc with a componentwise rounding error of at most about m eps t, t the
    per-row sum of magnitudes of its m quadrature contributions (residual_term_magnitudes), and
    solve with LU and partial pivoting, whose backward error is componentwise at most about
    3 n eps |A| (for moderate growth).  To first order the two solutions then differ by at most
        eps (2 * 3n |A^-1| |A| |z| + 2 m |A^-1| t)
    per component (Skeel's componentwise condition, insensitive to the row and column scaling
    that makes the normwise kappa(A) large on these blocks).  Returned relative to ||z||."""
    x, lam, us, _ = disc.elem_inputs(e, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"])
    t = residual_term_magnitudes(disc, e, x, lam, us)
    n = A.shape[0]
    m = disc.ref.phi.shape[0] + disc.nf * disc.geom(e).faces[0]["W"].shape[0]
    Ai = np.abs(np.linalg.inv(A))
    dz = np.finfo(float).eps * (6 * n * (Ai @ (np.abs(A) @ np.abs(z))) + 2 * m * (Ai @ t))
    return float(np.linalg.norm(dz) / np.linalg.norm(z))


def z_forward_report(disc, inp, elems, A, R_loc, z_ref, z_gpu):
    """Forward errors ||z_gpu - z_oracle|| / ||z_oracle|| of the given elements and their ratios to
    the elements' derived bounds (z_forward_bound).  Returns (largest error, largest ratio) and
    prints the distribution."""
    errs, ratios = [], []
    for e, a, r, zr, zg in zip(elems, A, R_loc, z_ref, z_gpu):
        err = float(np.linalg.norm(zg - zr) / np.linalg.norm(zr))
        errs.append(err)
        ratios.append(err / z_forward_bound(disc, inp, e, a, r, zr))
    print("z forward error: max %.2e median %.2e; error / derived bound: max %.2e median %.2e"
          % (max(errs), float(np.median(errs)), max(ratios), float(np.median(ratios))))
    return max(errs), max(ratios)
