"""Pins of the oracle's residual, Jacobian and condensation.

P1 free-stream preservation; P5 complex-step Jacobian vs finite differences;
P6 condensed solve + back-solve == brute-force full solve; P7 element-level
u-conservation; P8 the total-entropy identity of Proposition 1 (exact for
piecewise-constant states, converging under over-integration otherwise);
P9 Tables 1-2 (global trace DOFs and Jacobian nonzeros); P10 order k+1 on
manufactured solutions (Euler and Navier-Stokes, HDG).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import hdg, newton, physics as ph, state
from workloads import configs as C
from workloads import meshes as M

from cases import smooth_periodic_case

GAM = 1.4
HERE = os.path.dirname(os.path.abspath(__file__))


def _disc(wl, nquad=None):
    return hdg.Discretization(wl.mesh, wl.p, hdg.Phys(wl.gamma, wl.mu, wl.Pr, wl.alpha, wl.viscous),
                              wl.tmap, wl.n_trace, wl.face_bc, nquad)


# --------------------------------------------------------------------------- P1
@pytest.mark.parametrize("case", ["tri_dirichlet", "tri_ns", "hex_ns"])
def test_free_stream(case):
    if case == "tri_dirichlet":
        wl = C.euler2d_tri_p2(n=4)
    elif case == "tri_ns":
        wl = C.ns2d_tri(n=3, p=2)
    else:
        wl = C.ns3d_hex(n=3, p=1)
    disc = _disc(wl)
    m, d = disc.m, disc.d
    vc = ph.v_of_prim(np.array([1.3]), np.array([[0.4, -0.25, 0.1][:d]]), np.array([2.1]), GAM)[0]
    NN = wl.mesh.n_elem * disc.Np
    v = np.tile(vc[:, None], (1, NN))
    q = np.zeros((m * d, NN)) if wl.viscous else None
    vhat = np.tile(vc[:, None], (1, wl.n_trace))
    ustar = np.tile(ph.u_of_v(vc[None], GAM)[0][:, None], (1, NN))
    rtr = np.zeros(m * wl.n_trace)
    scale = 0.0
    for e in range(wl.mesh.n_elem):
        x, lam, us, vb = disc.elem_inputs(e, v, q, vhat, ustar, vhat)
        R, T = disc.element_residual(e, x[None], lam[None], us, vb)
        scale = max(scale, np.abs(T).max())
        assert np.abs(R).max() < 1e-13 * max(1.0, scale)
        np.add.at(rtr, hdg.element_trace_index(disc, e), T[0])
    assert np.abs(rtr).max() < 1e-13 * scale


# --------------------------------------------------------------------------- P5
@pytest.mark.parametrize("case", ["c1", "ns2d"])
def test_jacobian_complex_step_vs_finite_difference(case):
    wl = C.euler2d_tri_p2() if case == "c1" else C.ns2d_tri(n=2, p=2)
    disc = _disc(wl)
    inp = state.oracle_inputs(wl, disc)
    e = 3
    x, lam, us, vb = disc.elem_inputs(e, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"])
    s = disc.element_system(e, x, lam, us, vb)
    J = np.block([[s["A"], s["B"]], [s["C"], s["D"]]])
    z = np.concatenate([x, lam])
    n = disc.n
    Jf = np.empty_like(J)
    for i in range(len(z)):
        h = 1e-6 * max(1.0, abs(z[i]))
        zp, zm = z.copy(), z.copy()
        zp[i] += h
        zm[i] -= h
        Rp, Tp = disc.element_residual(e, zp[None, :n], zp[None, n:], us, vb)
        Rm, Tm = disc.element_residual(e, zm[None, :n], zm[None, n:], us, vb)
        Jf[:, i] = np.concatenate([Rp[0] - Rm[0], Tp[0] - Tm[0]]) / (2 * h)
    assert np.linalg.norm(J - Jf) <= 1e-6 * np.linalg.norm(J)


# --------------------------------------------------------------------------- P6
@pytest.mark.parametrize("case", ["c1", "ns2d", "hex_ns_p1"])
def test_condensation_equals_brute_force(case):
    if case == "c1":
        wl = C.euler2d_tri_p2()
    elif case == "ns2d":
        wl = C.ns2d_tri(n=3, p=2)
    else:
        wl = C.ns3d_hex(n=3, p=1)
    disc = _disc(wl)
    inp = state.oracle_inputs(wl, disc)
    blocks = hdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"],
                                   keep_blocks=True)
    K = hdg.trace_matrix(disc, [b["S"] for b in blocks]).tocsc()
    dl = spla.spsolve(K, hdg.trace_rhs(disc, [b["g"] for b in blocks]))
    dx = hdg.backsolve(disc, [b["Y"] for b in blocks], [b["z"] for b in blocks], dl)
    bx, bl = hdg.brute_force_solve(disc, blocks)
    assert np.linalg.norm(dl - bl) <= 1e-10 * np.linalg.norm(bl)
    num = np.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(dx, bx)))
    den = np.sqrt(sum(np.sum(b ** 2) for b in bx))
    assert num <= 1e-10 * den
    # the matrix-free trace operator equals the assembled one
    xr = np.random.default_rng(0).normal(size=K.shape[0])
    assert np.allclose(hdg.trace_matvec(disc, [b["S"] for b in blocks], xr), K @ xr, rtol=1e-13, atol=1e-13 * np.abs(K).max())


# --------------------------------------------------------------------------- P7
@pytest.mark.parametrize("case", ["ns2d", "hex_ns_p1", "c1"])
def test_element_u_conservation(case):
    """sum_a R_v[c,a] - sum_{f,b} R_tr[f,c,b] = alpha int (u - u*)_c on flux faces."""
    wl = {"ns2d": lambda: C.ns2d_tri(n=2, p=2), "hex_ns_p1": lambda: C.ns3d_hex(n=3, p=1),
          "c1": lambda: C.euler2d_tri_p2(n=3)}[case]()
    disc = _disc(wl)
    inp = state.oracle_inputs(wl, disc)
    m, Np = disc.m, disc.Np
    for e in range(wl.mesh.n_elem):
        x, lam, us, vb = disc.elem_inputs(e, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"])
        R, T = disc.element_residual(e, x[None], lam[None], us, vb)
        Rv = R[0, :m * Np].reshape(m, Np).sum(1)
        Tr = T[0].reshape(disc.nf, m, disc.Nfp)
        flux_faces = wl.face_bc[e] == 0
        lhs = Rv - Tr[flux_faces].sum(axis=(0, 2))
        if not np.all(flux_faces):
            # Dirichlet faces: the element still sees <f_hat, 1>; add it back
            G = disc.geom(e)
            for f in np.nonzero(~flux_faces)[0]:
                F = G.faces[f]
                vf = F["phi"] @ x[:m * Np].reshape(m, Np).T
                vhf = F["psi"] @ lam.reshape(disc.nf, m, disc.Nfp)[f].T
                lhs = lhs - F["W"] @ ph.fhat(vhf, vf, F["n"], GAM)
        G = disc.geom(e)
        vq = disc.ref.phi @ x[:m * Np].reshape(m, Np).T
        uq = ph.u_of_v(vq, GAM)
        rhs = wl.alpha * (G.W @ (uq - disc.ref.phi @ us.T))
        scale = np.abs(R).max() + np.abs(T).max() + wl.alpha * (G.W @ np.abs(uq)).max()
        assert np.abs(lhs - rhs).max() <= 1e-13 * scale


# --------------------------------------------------------------------------- P8
def _sigma_quadratic_form(vh, v, n, nth=120):
    """(v - vh)^T [sigma(vh) - Sigma(vh, v; n)] (v - vh), pointwise, straight path."""
    x, w = np.polynomial.legendre.leggauss(nth)
    th, wt = 0.5 * (x + 1), 0.5 * w
    dv = v - vh
    out = np.empty(vh.shape[0])
    for i in range(vh.shape[0]):
        Fn = lambda z: np.einsum("...cj,j->...c", ph.flux_F(z, GAM), n[i])
        path = vh[i][None, :] + th[:, None] * dv[i][None, :]
        An = ph.jac_cs(Fn, path)
        Sig = np.einsum("t,tab->ab", wt * (1 - 2 * th), An)
        sig = ph.sigma_slf(vh[i][None], n[i][None], GAM)[0]
        out[i] = dv[i] @ (sig - Sig) @ dv[i]
    return out


def _entropy_identity_gap(wl, v, vhat, nquad=None):
    disc = _disc(wl, nquad)
    m, Np = disc.m, disc.Np
    lhs, rhs, scale = 0.0, 0.0, 0.0
    rtr = np.zeros((m, wl.n_trace))
    for e in range(wl.mesh.n_elem):
        x, lam, _, _ = disc.elem_inputs(e, v, None, vhat)
        R, T = disc.element_residual(e, x[None], lam[None])
        lhs += x @ R[0]
        scale += np.abs(x * R[0]).sum()
        disc.scatter_trace(T[0], e, rtr)
        G = disc.geom(e)
        for f, F in enumerate(G.faces):
            vf = F["phi"] @ x.reshape(m, Np).T
            vhf = F["psi"] @ lam.reshape(disc.nf, m, disc.Nfp)[f].T
            rhs += 0.5 * F["W"] @ _sigma_quadratic_form(vhf, vf, F["n"])
    lhs -= np.sum(vhat * rtr)
    return abs(lhs - rhs), scale


@pytest.mark.parametrize("etype", ["tri", "hex"])
def test_total_entropy_identity_piecewise_constant(etype):
    """Proposition 1 (periodic, steady part): exact for constant v per element, v_hat per face."""
    if etype == "tri":
        wl = C.euler2d_tri_p2(n=3, periodic=True)
    else:
        wl = C.euler3d_hex(n=3, p=1)
    disc = _disc(wl)
    rng = np.random.default_rng(7)
    E, Np, m, d = wl.mesh.n_elem, disc.Np, disc.m, disc.d

    def rand_states(k):
        rho = rng.uniform(0.8, 1.3, k)
        V = rng.uniform(-0.4, 0.4, (k, d))
        p = rng.uniform(0.8, 1.4, k)
        return ph.v_of_prim(rho, V, p, GAM)

    ve = rand_states(E)
    v = np.repeat(ve.T, Np, axis=1)
    # one constant state per mesh face (HDG: each face owns its trace nodes)
    face_of_trace = np.arange(wl.n_trace) // disc.Nfp
    vf = rand_states(face_of_trace.max() + 1)
    vhat = vf[face_of_trace].T.copy()
    gap, scale = _entropy_identity_gap(wl, v, vhat)
    assert gap <= 1e-12 * scale


def test_total_entropy_identity_converges_with_over_integration():
    wl = C.euler2d_tri_p2(n=2, periodic=True, eps=0.05)
    disc = _disc(wl)
    inp = state.oracle_inputs(wl, disc)
    gaps = [_entropy_identity_gap(wl, inp["v"], inp["vhat"], nq)[0] for nq in (4, 6, 8)]
    assert gaps[1] < gaps[0] and gaps[2] < gaps[1]


# --------------------------------------------------------------------------- P9
def _alphas(mesh, k, scheme):
    tmap, nt = M.trace_map(mesh, k, scheme)
    nv = int(np.prod(mesh.period))
    E = tmap.shape[0]
    nodes = tmap.reshape(E, -1)
    pairs = set()
    enc = []
    for e in range(E):
        u = np.unique(nodes[e])
        enc.append((u[:, None] * nt + u[None, :]).ravel())
    npairs = len(np.unique(np.concatenate(enc)))
    return nt / nv, npairs / nv


@pytest.mark.parametrize("dim", ["2d", "3d"])
@pytest.mark.parametrize("scheme", ["hdg", "edg"])
def test_tables_1_2_dof_and_nnz(dim, scheme):
    tab = json.load(open(os.path.join(HERE, "golden", "paper_tables_1_2.json")))
    ks = [1, 2, 3, 4] if dim == "3d" else [1, 2, 3, 4, 5]
    mesh = M.tri_square(4, 0.0, 0, periodic=True) if dim == "2d" else M.kuhn_tets(3, 0.0, 0, periodic=True)
    for k in ks:
        a_dof, a_nnz = _alphas(mesh, k, scheme)
        assert a_dof == tab["alpha_dof"][dim][scheme][k - 1]
        assert a_nnz == tab["alpha_nnz"][dim][scheme][k - 1]


def test_condensed_matrix_nonzeros_match_table2():
    """Nonzeros of the assembled sum P^T S P from actual oracle blocks (2D HDG, k = 1, 2)."""
    tab = json.load(open(os.path.join(HERE, "golden", "paper_tables_1_2.json")))
    for k in (1, 2):
        wl = C.euler2d_tri_p2(n=3, p=k, periodic=True)
        wl.mesh.info["n"] = 3
        disc = _disc(wl)
        inp = state.oracle_inputs(wl, disc)
        blocks = hdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"])
        K = hdg.trace_matrix(disc, [b["S"] for b in blocks])
        K.eliminate_zeros()
        nv = 9
        assert K.nnz == nv * disc.m ** 2 * tab["alpha_nnz"]["2d"]["hdg"][k - 1]
        assert wl.n_trace * disc.m == nv * disc.m * tab["alpha_dof"]["2d"]["hdg"][k - 1]


# --------------------------------------------------------------------------- P10
def _mms_prim(x):
    X, Y = x[..., 0], x[..., 1]
    rho = 1 + 0.1 * np.sin(np.pi * X + 0.3) * np.cos(np.pi * Y)
    vx = 0.4 + 0.1 * np.cos(np.pi * X) * np.sin(np.pi * Y)
    vy = 0.2 + 0.1 * np.sin(np.pi * X + 1.0)
    p = 1 + 0.1 * np.cos(np.pi * X) * np.cos(np.pi * Y + 0.5)
    return rho, np.stack([vx, vy], -1), p


def _vex(x):
    r, V, p = _mms_prim(x)
    return ph.v_of_prim(r, V, p, GAM)


def _uex(x):
    r, V, p = _mms_prim(x)
    return ph.u_of_prim(r, V, p, GAM)


def _qex(x):
    out = []
    for j in range(2):
        xc = x.astype(complex)
        xc[:, j] += 1e-30j
        out.append(np.imag(_vex(xc)) / 1e-30)
    return np.stack(out, -1)    # (N, m, d)


def _source(x, mu, Pr):
    if mu == 0.0:
        s = 0.0
        for j in range(2):
            xc = x.astype(complex)
            xc[:, j] += 1e-30j
            s = s + np.imag(ph.flux_F(_vex(xc), GAM)[..., j]) / 1e-30
        return s
    s = 0.0
    for j in range(2):
        h = 1e-5
        e = np.zeros(2)
        e[j] = h
        fl = lambda y: (ph.flux_F(_vex(y), GAM) + ph.flux_G(_vex(y), _qex(y), GAM, mu, Pr))[..., j]
        s = s + (8 * (fl(x + e) - fl(x - e)) - (fl(x + 2 * e) - fl(x - 2 * e))) / (12 * h)
    return s


@pytest.mark.parametrize("viscous,p", [(False, 1), (False, 2), (True, 1), (True, 2)])
def test_convergence_order_k_plus_1(viscous, p):
    """Euler: L2 error of u at rate >= k+1-0.3.  NS (mu = 0.05): u at >= k+1-0.45 and the
    temperature-gradient component of q (the last entropy variable) at >= k+1-0.3.

    The other components of q are not pinned at k+1: the viscous flux sees q only through
    K~(v) q, whose null space holds the density gradient at fixed velocity and temperature and
    the skew part of the velocity gradient; the scheme controls those directions of q only
    through the inviscid stabilization, and they converge at about k (Couette, k = 1: first
    component 0.98, momentum components 0.7 to 1.6, last component 2.0).  What Table 6 prints,
    the stress and heat flux formed from (v_h, q_h), lies in the range of K~ and converges at
    k+1: test_couette_against_table_6.
    """
    mu = 0.05 if viscous else 0.0
    Pr = 0.72
    errs, qerrs = [], []
    for n in (4, 8):
        mesh = M.tri_square(n, 0.05, 3, periodic=False)
        tmap, nt = M.trace_map(mesh, p, "hdg")
        disc = hdg.Discretization(mesh, p, hdg.Phys(GAM, mu, Pr, 0.0, viscous), tmap, nt,
                                  mesh.boundary.astype(np.int32))
        xn, xt = disc.node_coords(), disc.trace_coords()
        v0, vh0 = _vex(xn.T).T.copy(), _vex(xt.T).T.copy()
        q0 = _qex(xn.T).transpose(1, 2, 0).reshape(-1, xn.shape[1]).copy() if viscous else None
        v, q, vh, hist = newton.newton_steady(disc, v0, q0, vh0, vbc=vh0,
                                              source=lambda x: _source(x, mu, Pr))
        assert hist[-1] < 1e-10
        errs.append(newton.l2_error_u(disc, v, _uex))
        if viscous:
            qe = 0.0
            for e in range(mesh.n_elem):
                G = disc.geom(e)
                qq = (disc.ref.phi @ q[:, e * disc.Np:(e + 1) * disc.Np].T).reshape(len(G.W), 4, 2)
                dq = qq[:, 3, :] - _qex(G.xq)[:, 3, :]
                qe += np.sum(G.W[:, None] * dq ** 2)
            qerrs.append(np.sqrt(qe))
    rate = np.log2(errs[0] / errs[1])
    assert rate >= p + 1 - (0.45 if viscous else 0.3), (errs, rate)
    if viscous:
        qrate = np.log2(qerrs[0] / qerrs[1])
        assert qrate >= p + 1 - 0.3, (qerrs, qrate)


def test_implicit_stage_newton_returns_to_uniform_flow():
    """One implicit stage (alpha > 0) whose previous-stage state u* is a uniform flow: the
    uniform flow (v constant, q = 0, vhat = v) solves it exactly (free-stream preservation
    and alpha (u - u*) = 0), and it is the solution Newton finds from a perturbed start,
    with the residual falling quadratically."""
    mu, Pr, alpha, p = 0.01, 0.72, 5.0, 2
    mesh = M.tri_square(2, 0.05, 7, periodic=True)
    tmap, nt = M.trace_map(mesh, p, "hdg")
    disc = hdg.Discretization(mesh, p, hdg.Phys(GAM, mu, Pr, alpha, True), tmap, nt,
                              np.zeros((mesh.n_elem, 3), dtype=np.int32))
    vc = ph.v_of_prim(np.array(1.1), np.array([0.3, -0.2]), np.array(0.9), GAM)
    nn = mesh.n_elem * disc.Np
    v_ex = np.repeat(vc[:, None], nn, axis=1)
    vh_ex = np.repeat(vc[:, None], nt, axis=1)
    ustar = ph.u_of_v(v_ex.T, GAM).T.copy()
    rng = np.random.default_rng(11)
    v0 = v_ex * (1 + 1e-2 * rng.standard_normal(v_ex.shape))
    vh0 = vh_ex * (1 + 1e-2 * rng.standard_normal(vh_ex.shape))
    q0 = 1e-3 * rng.standard_normal((4 * 2, nn))
    v, q, vh, hist = newton.newton_steady(disc, v0, q0, vh0, ustar=ustar, tol=1e-12, maxit=8)
    assert hist[-1] < 1e-12 * max(1.0, hist[0]), hist
    assert len(hist) <= 6, hist
    for i in range(1, len(hist) - 1):
        assert hist[i + 1] <= 10 * hist[i] ** 2 / hist[0] + 1e-13, hist   # quadratic decrease
    assert np.max(np.abs(v - v_ex)) < 1e-10 * np.max(np.abs(vc))
    assert np.max(np.abs(q)) < 1e-9
    assert np.max(np.abs(vh - vh_ex)) < 1e-10 * np.max(np.abs(vc))


def test_dirk33_tableau_order_conditions():
    """Alexander's DIRK(3,3): a_ii is the root of x^3 - 3x^2 + 3x/2 - 1/6 in (1/6, 1/2); the
    stiffly accurate weights (last row) satisfy the third-order conditions."""
    A = newton.dirk33_tableau()
    g = A[0, 0]
    assert abs(g ** 3 - 3 * g ** 2 + 1.5 * g - 1.0 / 6.0) < 1e-15
    b, c = A[2], A.sum(axis=1)
    assert abs(c[2] - 1.0) < 1e-15
    for lhs, rhs in ((b.sum(), 1.0), (b @ c, 0.5), (b @ c ** 2, 1.0 / 3.0), (b @ A @ c, 1.0 / 6.0)):
        assert abs(lhs - rhs) < 1e-14


def test_dirk33_step_temporal_order():
    """Self-convergence in time of the oracle's DIRK(3,3) steps on a smooth periodic flow (T = 0.2
    in 2, 4, 8 steps): the error ratio must show third order (rate >= 2.5; a wrong stage
    coefficient drops it to 2 or below)."""
    out = {}
    for nsteps in (2, 4, 8):
        dt = 0.2 / nsteps
        _, disc, v, q, vh = smooth_periodic_case(dt)
        for _ in range(nsteps):
            v, q, vh, hists = newton.dirk33_step(disc, v, q, vh, dt)
            assert all(h[-1] < 1e-11 for h in hists), hists
        out[nsteps] = v
    e1 = np.linalg.norm(out[2] - out[4])
    e2 = np.linalg.norm(out[4] - out[8])
    assert np.log2(e1 / e2) >= 2.5, (e1, e2)


def _ringleb_oracle_error(n, p, scheme):
    from workloads.fields import Ringleb
    f = Ringleb()
    mesh = M.tri_square(n, 0.0, 0, periodic=False, lo=0.0, length=4.0)
    mesh.elem_xyz[..., 0] -= 5.0
    mesh.elem_xyz[..., 1] += 1.0
    tmap, nt = M.trace_map(mesh, p, scheme)
    disc = hdg.Discretization(mesh, p, hdg.Phys(f.gamma, 0.0, 0.72, 0.0, False), tmap, nt,
                               mesh.boundary.astype(np.int32))

    def v_of(x):
        pr = f.prim(x)
        return ph.v_of_prim(pr[0], pr[1:3].T, pr[3], f.gamma).T.copy()

    def u_ex(xq):
        pr = f.prim(xq.T)
        return ph.u_of_prim(pr[0], pr[1:3].T, pr[3], f.gamma)

    vh = v_of(disc.trace_coords())
    v, _, _, hist = newton.newton_steady(disc, v_of(disc.node_coords()), None, vh, vbc=vh.copy(), tol=1e-12)
    assert hist[-1] < 1e-12 and len(hist) <= 6
    return newton.l2_error_u(disc, v, u_ex)


def test_ringleb_errors_match_tables_3_to_5():
    """Steady Ringleb flow (Section 5) by the oracle's Newton iteration, p = 1: the errors on
    1/h = 2 for HDG, IEDG and EDG traces within 40% of Tables 3-5 (the diagonal of the split is
    not stated; measured 5% / 20% / 36% above), and HDG on 1/h = 4 within 5% of Table 3 (1%
    below).  A Dirichlet-trace node of a continuous trace that kept the flux rows of the
    interior faces meeting it would leave the EDG error 30x larger (0.18)."""
    tab = json.load(open(os.path.join(HERE, "golden", "paper_tables_3_5_ringleb.json")))
    for scheme in ("hdg", "iedg", "edg"):
        err = _ringleb_oracle_error(8, 1, scheme)
        ref = tab["error"][scheme][0][0]
        print(scheme, err, ref)
        assert ref / 1.4 < err < ref * 1.4, (scheme, err, ref)
    err = _ringleb_oracle_error(16, 1, "hdg")
    assert abs(err / tab["error"]["hdg"][0][1] - 1.0) < 0.05, err


def _proj_case(seed, const_v):
    """A 2x2 jittered periodic triangle mesh, p = 2, Navier-Stokes; v either one constant state or
    a smooth field, q seeded random nodal values."""
    mesh = M.tri_square(2, 0.1, seed, periodic=True)
    tmap, nt = M.trace_map(mesh, 2, "hdg")
    fbc = np.zeros((mesh.n_elem, 3), dtype=np.int32)
    rng = np.random.default_rng(seed)
    discs = {k: hdg.Discretization(mesh, 2, hdg.Phys(1.4, 0.05, 0.72, 0.0, True, k == "int", "slf", k == "proj"),
                                   tmap, nt, fbc) for k in ("int", "proj")}
    d0 = discs["int"]
    x = d0.node_coords()
    rho = np.ones(x.shape[1]) if const_v else 1.0 + 0.2 * np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1])
    V = np.stack([0.3 + (0 if const_v else 0.2) * np.cos(2 * np.pi * x[1]), -0.2 + 0 * x[0]], axis=1)
    v = ph.v_of_prim(rho, V, 1.0 + 0 * x[0], 1.4).T.copy()
    q = rng.standard_normal((8, x.shape[1]))
    vh = rng.standard_normal((4, nt)) * 0.01 + v[:, :1]
    return discs, v, q, vh


def test_projection_viscous_flux_reduces_to_interior_flux():
    """With one constant state v_h, G(v_h, q_h) is linear in q_h with constant coefficients, so it
    lies in the polynomial space of q_h and its projection is itself: the projection viscous flux
    (Section 4) equals the interior flux G(v_h, q_h).n, element residuals to 1e-13."""
    discs, v, q, vh = _proj_case(3, True)
    for e in range(discs["int"].mesh.n_elem):
        out = []
        for k in ("int", "proj"):
            dk = discs[k]
            xl, lam = dk.pack_local(v, q, e), dk.gather_trace(vh, e)
            out.append(dk.element_residual(e, xl[None], lam[None]))
        for a, b in zip(*out):
            assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_projection_viscous_flux_against_least_squares_projection():
    """With a varying v_h the projection flux differs from the interior one by
    <(Pi G - G) . n, phi_i> on the element boundary; Pi is computed here independently as the
    weighted least-squares fit of G(v_h, q_h) at the volume quadrature points (numpy lstsq), and
    the face integrals with the face quadrature: R_v(proj) - R_v(int) matches to 1e-11."""
    discs, v, q, vh = _proj_case(5, False)
    di, dp = discs["int"], discs["proj"]
    Np, m, d = di.Np, di.m, di.d
    for e in range(di.mesh.n_elem):
        xl, lam = di.pack_local(v, q, e), di.gather_trace(vh, e)
        Ri = di.element_residual(e, xl[None], lam[None])[0][0][:m * Np].reshape(m, Np)
        Rp = dp.element_residual(e, xl[None], lam[None])[0][0][:m * Np].reshape(m, Np)
        G = di.geom(e)
        sl = slice(e * Np, (e + 1) * Np)
        vq = di.ref.phi @ v[:, sl].T
        qq = np.einsum("qa,cja->qcj", di.ref.phi, q[:, sl].reshape(m, d, Np))
        Gq = ph.flux_G(vq, qq, 1.4, 0.05, 0.72).reshape(len(G.W), m * d)
        sw = np.sqrt(G.W)[:, None]
        coef = np.linalg.lstsq(sw * di.ref.phi, sw * Gq, rcond=None)[0]          # (Np, m d)
        diff = np.zeros((m, Np))
        for F in G.faces:
            vf = F["phi"] @ v[:, sl].T
            qf = np.einsum("qa,cja->qcj", F["phi"], q[:, sl].reshape(m, d, Np))
            Gf = ph.flux_G(vf, qf, 1.4, 0.05, 0.72)
            Pf = (F["phi"] @ coef).reshape(-1, m, d)
            diff += np.einsum("q,qcj,qj,qa->ca", F["W"], Pf - Gf, F["n"], F["phi"])
        assert np.abs(diff).max() > 1e-4
        assert np.abs((Rp - Ri) - diff).max() <= 1e-11 * np.abs(diff).max()


# ------------------------------------------------- Dirichlet data, Table 6 (Couette)
def _couette_exact():
    from workloads.fields import Couette
    f = Couette()

    def v_ex(x):                                   # x (N, d) -> (N, m)
        pr = f.prim(x.T)
        return ph.v_of_prim(pr[0], pr[1:3].T, pr[3], f.gamma)

    def q_ex(x):                                   # grad v by complex step: (N, m, d)
        cols = []
        for j in range(2):
            xc = x.astype(complex)
            xc[:, j] += 1e-30j
            pr = f.prim(xc.T)
            cols.append(np.imag(ph.v_of_prim(pr[0], pr[1:3].T, pr[3], f.gamma)) / 1e-30)
        return np.stack(cols, -1)

    def u_ex(x):
        pr = f.prim(x.T)
        return ph.u_of_prim(pr[0], pr[1:3].T, pr[3], f.gamma)

    return f, v_ex, q_ex, u_ex


def test_boundary_projection_reproduces_face_polynomials_and_is_best():
    """The face L2 projection of the Dirichlet data reproduces, at the trace nodes, a field that
    is a polynomial of degree <= k along every boundary face (here one of total degree k on
    straight faces), and for a non-polynomial field its L2(F) error is no larger than that of the
    nodal interpolant, measured with an independent 12-point Gauss rule on each face."""
    for p in (1, 2, 3):
        mesh = M.tri_square(3, 0.08, 4, periodic=False)
        tmap, nt = M.trace_map(mesh, p, "hdg")
        disc = hdg.Discretization(mesh, p, hdg.Phys(GAM, 0.0, 0.72, 0.0, False), tmap, nt,
                                  mesh.boundary.astype(np.int32))
        xt = disc.trace_coords().T
        bnd = disc.dir_node
        c = np.random.default_rng(p).normal(size=(4, 3))
        poly = lambda x: np.stack([(c[i, 0] + c[i, 1] * x[:, 0] + c[i, 2] * x[:, 1]) ** p
                                   for i in range(4)], -1)
        vb = newton.project_boundary_data(disc, poly)
        assert np.allclose(vb[:, bnd], poly(xt[bnd]).T, rtol=1e-12, atol=1e-12)
        smooth = lambda x: np.stack([np.sin(3 * x[:, 0] + 2 * x[:, 1] + i) for i in range(4)], -1)
        vb = newton.project_boundary_data(disc, smooth)
        vi = smooth(xt).T
        s, t = np.polynomial.legendre.leggauss(12)
        worse = 0
        for e in range(mesh.n_elem):
            xyz = mesh.elem_xyz[e]
            for f in range(3):
                if disc.face_bc[e, f] != 1:
                    continue
                a, b = xyz[(f + 1) % 3], xyz[(f + 2) % 3]   # the face opposite vertex f
                nodes = tmap[e, f]
                xn = xt[nodes]
                # 1D Lagrange basis in the face's arc parameter through its nodes
                tn = (xn - a) @ (b - a) / ((b - a) @ (b - a))
                tq = 0.5 * (s + 1.0)
                L = np.ones((len(tq), len(tn)))
                for i in range(len(tn)):
                    for j in range(len(tn)):
                        if j != i:
                            L[:, i] *= (tq - tn[j]) / (tn[i] - tn[j])
                gq = smooth(a + tq[:, None] * (b - a))
                ep = np.sum(t[:, None] * (L @ vb[:, nodes].T - gq) ** 2)
                ei = np.sum(t[:, None] * (L @ vi[:, nodes].T - gq) ** 2)
                worse += ep > ei * (1 + 1e-9)
        assert worse == 0


def _couette_oracle_errors(n, p):
    f, v_ex, q_ex, u_ex = _couette_exact()
    mesh = M.tri_square(n, 0.0, 0, periodic=False)
    tmap, nt = M.trace_map(mesh, p, "hdg")
    disc = hdg.Discretization(mesh, p, hdg.Phys(f.gamma, f.mu, f.Pr, 0.0, True), tmap, nt,
                              mesh.boundary.astype(np.int32))
    xn, xt = disc.node_coords().T, disc.trace_coords().T
    vbc = newton.project_boundary_data(disc, v_ex)
    vh0 = v_ex(xt).T.copy()
    vh0[:, disc.dir_node] = vbc[:, disc.dir_node]
    q0 = q_ex(xn).transpose(1, 2, 0).reshape(-1, xn.shape[0]).copy()
    v, q, vh, hist = newton.newton_steady(disc, v_ex(xn).T.copy(), q0, vh0, vbc=vbc,
                                          source=lambda x: f.source(x.T).T, tol=1e-11)
    assert hist[-1] < 1e-10, hist
    eu = newton.l2_error_components(disc, v, u_ex)
    et, ef = newton.l2_error_stress_heat(disc, v, q, v_ex, q_ex)
    # non-dimensional as printed: rho0 = V0 = L = 1, so tau* = tau / mu and f* = f / mu
    return {"rho": eu[0], "momentum": np.hypot(eu[1], eu[2]), "rhoE": eu[3],
            "tau": et / f.mu, "f": ef / f.mu}


@pytest.mark.parametrize("p,ns", [(1, (16, 32)), (2, (8, 16))])
def test_couette_against_table_6(p, ns):
    """Table 6 (Couette flow, entropy-variable HDG, Dirichlet data = the exact solution, tested
    on each boundary face, i.e. its face L2 projection): the density, momentum, total energy,
    stress tau* and heat flux f* (formed from v_h and q_h) errors within a factor 6 of the printed
    ones, and every rate on the mesh pair within 0.3 of the printed rate.  The factor covers what
    the paper leaves unstated (the diagonal of the split, the quadrature, the nodes); the rate
    window the scatter of the printed rates themselves."""
    tab = json.load(open(os.path.join(HERE, "golden", "paper_table_6_couette.json")))
    hs = tab["L_over_h"]
    i0, i1 = hs.index(ns[0]), hs.index(ns[1])
    e0, e1 = _couette_oracle_errors(ns[0], p), _couette_oracle_errors(ns[1], p)
    for key in tab["quantities"]:
        for e, i in ((e0, i0), (e1, i1)):
            ref = tab["error"][key][p - 1][i]
            assert ref / 6 <= e[key] <= 6 * ref, (key, p, hs[i], e[key], ref)
        rate = np.log2(e0[key] / e1[key])
        ref_rate = tab["rate"][key][p - 1][i1 - 1]
        assert abs(rate - ref_rate) <= 0.3, (key, p, rate, ref_rate)
