"""Pins of the oracle's pointwise physics.

* U <-> V round trip and the closed-form A0 against the complex-step dU/dV
  (entropy variables of the section on entropy pairs and symmetrization);
* symmetrization: A0 SPD, A_n A0 symmetric (the stability section's notation);
* Lemma 1 / Corollary 3 (jump entropy identity) pointwise;
* the dissipation identity of the viscous flux written with grad v
  (the paper's identity for q^T K q in terms of Phi / T and |grad T|^2),
  with T and V gradients taken from q directly, not through A0;
* complex step against central finite differences.
"""
import numpy as np
import pytest

from oracle import physics as P

GAM = 1.4


def _states(rng, n, d):
    rho = rng.uniform(0.3, 3.0, n)
    V = rng.normal(size=(n, d)) * rng.uniform(0.1, 2.0, (n, 1))
    p = rng.uniform(0.3, 5.0, n)
    return rho, V, p


@pytest.mark.parametrize("d", [2, 3])
def test_round_trip_and_A0(d):
    rng = np.random.default_rng(10 + d)
    rho, V, p = _states(rng, 50, d)
    u = P.u_of_prim(rho, V, p, GAM)
    v = P.v_of_u(u, GAM)
    assert np.abs(P.u_of_v(v, GAM) - u).max() <= 1e-14 * np.abs(u).max()
    # printed closed form of v (section on entropy pairs): v_m = -(gamma-1) rho / p
    assert np.allclose(v[:, -1], -(GAM - 1) * rho / p, rtol=1e-15)
    assert np.allclose(v[:, 1:-1], (GAM - 1) * rho[:, None] * V / p[:, None], rtol=1e-14)
    J = P.jac_cs(lambda x: P.u_of_v(x, GAM), v)
    A0 = P.A0(v, GAM)
    assert np.abs(J - A0).max() <= 1e-14 * np.abs(J).max()
    assert np.abs(A0 - np.swapaxes(A0, 1, 2)).max() <= 1e-14 * np.abs(A0).max()
    assert np.all(np.linalg.eigvalsh(A0) > 0)
    # A0 times dv/du is the identity
    dvdu = P.jac_cs(lambda x: P.v_of_u(x, GAM), u)
    assert np.abs(np.einsum("nab,nbc->nac", A0, dvdu) - np.eye(d + 2)).max() < 1e-12


@pytest.mark.parametrize("d", [2, 3])
def test_symmetrized_flux_jacobian(d):
    rng = np.random.default_rng(20 + d)
    rho, V, p = _states(rng, 30, d)
    v = P.v_of_prim(rho, V, p, GAM)
    n = rng.normal(size=(30, d))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    An = P.jac_cs(lambda x: np.einsum("...cj,...j->...c", P.flux_F(x, GAM), n), v)
    assert np.abs(An - np.swapaxes(An, 1, 2)).max() <= 1e-13 * np.abs(An).max()
    # lambda_max is the spectral radius of A_n = dF_n/du
    Au = P.jac_cs(lambda x: np.einsum("...cj,...j->...c", P.flux_F(P.v_of_u(x, GAM), GAM), n),
                  P.u_of_v(v, GAM))
    rad = np.abs(np.linalg.eigvals(Au)).max(1)
    assert np.allclose(rad, np.real(P.lam_max(v, n, GAM)), rtol=1e-10)


@pytest.mark.parametrize("d", [2, 3])
def test_entropy_flux_identity(d):
    # dF_H/dv = v^T dF/dv (the identity defining the entropy pair, written in v)
    rng = np.random.default_rng(30 + d)
    rho, V, p = _states(rng, 20, d)
    v = P.v_of_prim(rho, V, p, GAM)
    for j in range(d):
        dFH = P.jac_cs(lambda x: P.entropy_pair(x, GAM)[1][..., j][..., None], v)[:, 0]
        dF = P.jac_cs(lambda x: P.flux_F(x, GAM)[..., j], v)
        assert np.abs(dFH - np.einsum("na,nab->nb", v, dF)).max() < 1e-12 * np.abs(dFH).max()


def _gauss01(nq):
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (x + 1), 0.5 * w


@pytest.mark.parametrize("d", [2, 3])
def test_lemma1_jump_entropy_identity(d):
    """-[F_H.n] + 1/2 (v1+v2)^T [F_n] = 1/2 dv^T Sigma(v1,v2;n) dv, straight path."""
    rng = np.random.default_rng(40 + d)
    th, wt = _gauss01(200)
    for _ in range(20):
        r1, V1, p1 = _states(rng, 1, d)
        r2, V2, p2 = _states(rng, 1, d)
        v1, v2 = P.v_of_prim(r1, V1, p1, GAM)[0], P.v_of_prim(r2, V2, p2, GAM)[0]
        n = rng.normal(size=d)
        n /= np.linalg.norm(n)
        Fn = lambda x: np.einsum("...cj,j->...c", P.flux_F(x, GAM), n)
        FHn = lambda x: P.entropy_pair(x, GAM)[1] @ n
        dv = v2 - v1
        path = v1[None, :] + th[:, None] * dv[None, :]
        An = P.jac_cs(Fn, path)
        Sigma = np.einsum("t,tab->ab", wt * (1 - 2 * th), An)
        lhs = -(FHn(v2[None])[0] - FHn(v1[None])[0]) + 0.5 * (v1 + v2) @ (Fn(v2[None])[0] - Fn(v1[None])[0])
        rhs = 0.5 * dv @ Sigma @ dv
        scale = abs(FHn(v2[None])[0]) + abs(FHn(v1[None])[0]) + abs(rhs)
        assert abs(lhs - rhs) <= 1e-12 * scale


@pytest.mark.parametrize("d", [2, 3])
def test_viscous_dissipation_identity(d):
    """-sum q:G(v,q) = (gamma-1) (Phi/T + kappa |grad T|^2 / T^2) with q = grad v."""
    rng = np.random.default_rng(50 + d)
    mu, Pr = 0.37, 0.72
    rho, V, p = _states(rng, 40, d)
    v = P.v_of_prim(rho, V, p, GAM)
    q = rng.normal(size=(40, d + 2, d))
    G = P.flux_G(v, q, GAM, mu, Pr)
    lhs = -(q * G).sum((1, 2))
    # primitive gradients straight from grad v: T = -(gamma-1)/v_m, V = -w / v_m
    vm, w = v[:, -1], v[:, 1:-1]
    T = -(GAM - 1) / vm
    gT = (GAM - 1) * q[:, -1, :] / vm[:, None] ** 2
    gV = -q[:, 1:-1, :] / vm[:, None, None] + w[:, :, None] * q[:, -1, None, :] / vm[:, None, None] ** 2
    div = np.einsum("nii->n", gV)
    tau = mu * (gV + gV.transpose(0, 2, 1) - 2.0 / 3.0 * div[:, None, None] * np.eye(d))
    Phi = (tau * gV).sum((1, 2))
    kappa = GAM / (GAM - 1) * mu / Pr
    rhs = (GAM - 1) * (Phi / T + kappa * (gT ** 2).sum(1) / T ** 2)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()
    # G is linear in q and annihilates the mass row
    assert np.abs(G[:, 0, :]).max() == 0.0
    G2 = P.flux_G(v, 2.0 * q, GAM, mu, Pr)
    assert np.allclose(G2, 2 * G, rtol=1e-14, atol=0)


def test_complex_step_matches_finite_differences():
    rng = np.random.default_rng(60)
    rho, V, p = _states(rng, 5, 3)
    v = P.v_of_prim(rho, V, p, GAM)
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    vh = v + 0.01 * rng.normal(size=v.shape) * np.abs(v)
    f = lambda x: P.fhat(x, v, n, GAM)
    Jc = P.jac_cs(f, vh)
    Jf = np.empty_like(Jc)
    for i in range(5):
        h = 1e-6 * max(1.0, abs(vh[0, i]))
        e = np.zeros(5)
        e[i] = h
        Jf[:, :, i] = (f(vh + e) - f(vh - e)) / (2 * h)
    assert np.abs(Jc - Jf).max() <= 1e-6 * np.abs(Jc).max()


def test_abs_An_matches_the_eigen_decomposition():
    """|A_n| du from the closed-form wave decomposition against V |Lambda| V^-1 du, A_n = dF_n/du
    by complex step and V, Lambda from a general eigen-solver, at random states (2D and 3D);
    sigma_S = |A_n| A0 is symmetric positive semi-definite."""
    rng = np.random.default_rng(3)
    for d in (2, 3):
        m = d + 2
        for _ in range(4):
            v = P.v_of_prim(np.array(1 + 0.3 * rng.random()), 0.6 * rng.standard_normal(d),
                             np.array(1 + 0.5 * rng.random()), GAM)
            n = rng.standard_normal(d)
            n /= np.linalg.norm(n)
            u = P.u_of_v(v, GAM)
            J = np.zeros((m, m))
            for k in range(m):
                uc = u.astype(complex)
                uc[k] += 1e-30j
                J[:, k] = np.imag(np.einsum("cj,j->c", P.flux_F(P.v_of_u(uc, GAM), GAM), n)) / 1e-30
            w, R = np.linalg.eig(J)
            absA = np.real(R @ np.diag(np.abs(w)) @ np.linalg.inv(R))
            du = rng.standard_normal(m)
            assert np.max(np.abs(absA @ du - P.abs_An_apply(v, n, GAM, du))) <= 1e-12 * np.max(np.abs(absA @ du))
            S = np.stack([P.sigma_s_apply(v, n, GAM, e) for e in np.eye(m)], axis=1)
            assert np.max(np.abs(S - S.T)) <= 1e-12 * np.max(np.abs(S))
            assert np.min(np.linalg.eigvalsh(0.5 * (S + S.T))) >= -1e-12 * np.max(np.abs(S))


def test_mean_value_stabilization():
    """sigma_MV: equal to sigma_S when v = v_hat (the path is a point), symmetric positive
    semi-definite, symmetric in its two states (the definition's two path integrals), and equal
    to a 64-point rule of the same integral between nearby states where no wave speed changes
    sign along the path (the integrand is then smooth; n along the velocity keeps V.n > 0)."""
    rng = np.random.default_rng(5)
    for d in (2, 3):
        m = d + 2
        Vh = np.array([0.4, -0.2, 0.1][:d])
        vh = P.v_of_prim(np.array(1.1), Vh, np.array(0.9), GAM)
        v = P.v_of_prim(np.array(1.15), np.array([0.45, -0.15, 0.12][:d]), np.array(0.95), GAM)
        n = Vh / np.linalg.norm(Vh)
        dv = rng.standard_normal(m)
        assert np.allclose(P.sigma_mv_apply(vh, vh, n, GAM, dv), P.sigma_s_apply(vh, n, GAM, dv), rtol=1e-13,
                           atol=1e-13)
        S = np.stack([P.sigma_mv_apply(vh, v, n, GAM, e) for e in np.eye(m)], axis=1)
        assert np.max(np.abs(S - S.T)) <= 1e-12 * np.max(np.abs(S))
        assert np.min(np.linalg.eigvalsh(0.5 * (S + S.T))) >= -1e-12 * np.max(np.abs(S))
        assert np.allclose(P.sigma_mv_apply(v, vh, n, GAM, dv), P.sigma_mv_apply(vh, v, n, GAM, dv),
                           rtol=1e-13, atol=1e-13)
        th, w = np.polynomial.legendre.leggauss(64)
        fine = sum(0.5 * wi * P.sigma_s_apply(vh + 0.5 * (1 + ti) * (v - vh), n, GAM, dv) for ti, wi in zip(th, w))
        assert np.max(np.abs(P.sigma_mv_apply(vh, v, n, GAM, dv) - fine)) <= 1e-13 * np.max(np.abs(fine))


@pytest.mark.parametrize("case", ["u_n", "u_n - c", "u_n + c", "two"])
def test_mean_value_stabilization_across_sign_changes(case):
    """Where a wave speed changes sign along the path, the integrand has a kink; the split
    integral agrees with a composite trapezoidal rule on 40,000 intervals (error O(h^2) at a
    kink, about 1e-10 of the integral here) to 1e-8, while a single 4-point Gauss rule across
    the kink misses by more than 1e-5: a missed or misplaced breakpoint fails the first bound."""
    rng = np.random.default_rng(11)
    for d in (2, 3):
        m = d + 2
        n = np.zeros(d)
        n[0] = 1.0
        c0 = np.sqrt(GAM * 0.9 / 1.1)
        u0, u1 = {"u_n": (-0.3, 0.4), "u_n - c": (c0 - 0.35, c0 + 0.3), "u_n + c": (-c0 - 0.3, -c0 + 0.25),
                  "two": (-c0 - 0.2, 0.3)}[case]
        V0 = np.array([u0, 0.2, -0.1][:d])
        V1 = np.array([u1, -0.1, 0.15][:d])
        vh = P.v_of_prim(np.array(1.1), V0, np.array(0.9), GAM)
        v = P.v_of_prim(np.array(1.1), V1, np.array(0.9), GAM)
        br = P.mv_breakpoints(vh, v, n, GAM)
        inner = br[(br > 0) & (br < 1)]
        assert len(inner) == (2 if case == "two" else 1), br
        dv = rng.standard_normal(m)
        got = P.sigma_mv_apply(vh, v, n, GAM, dv)
        N = 40000
        ts = np.linspace(0.0, 1.0, N + 1)
        vals = P.sigma_s_apply(vh + ts[:, None] * (v - vh), n, GAM, dv)
        trap = (vals[0] + vals[-1]) / (2 * N) + vals[1:-1].sum(0) / N
        scale = np.max(np.abs(trap))
        assert np.max(np.abs(got - trap)) <= 1e-8 * scale, (case, d, got, trap)
        x4, w4 = np.polynomial.legendre.leggauss(4)
        g4 = sum(0.5 * wi * P.sigma_s_apply(vh + 0.5 * (1 + ti) * (v - vh), n, GAM, dv) for ti, wi in zip(x4, w4))
        assert np.max(np.abs(g4 - trap)) > 1e-5 * scale, (case, d)


def test_stress_and_heat_flux_closed_form():
    """tau and f formed from (v, q = grad v) equal the Newtonian stress (beta = 0) and the Fourier
    heat flux of a flow with a given affine velocity, density and pressure, written in closed form
    from the primitive gradients (the Navier-Stokes section)."""
    gam, mu, Pr = 1.4, 0.03, 0.72
    rng = np.random.default_rng(5)
    for d in (2, 3):
        x0 = rng.normal(size=d)
        gV = rng.normal(size=(d, d))                     # dV_i / dx_j
        grho, gp = rng.normal(size=d) * 0.1, rng.normal(size=d) * 0.2
        rho0, p0, V0 = 1.1, 0.9, rng.normal(size=d) * 0.3

        def prim(x):
            dx = x - x0
            return rho0 + grho @ dx, V0 + gV @ dx, p0 + gp @ dx

        def v_at(x):
            r, V, p = prim(x)
            return P.v_of_prim(np.asarray(r), V, np.asarray(p), gam)

        q = np.stack([np.imag(v_at(x0 + 1e-30j * np.eye(d)[j])) / 1e-30 for j in range(d)], -1)
        tau, f = P.stress_heat_flux(v_at(x0)[None].real, q[None], gam, mu, Pr)
        div = np.trace(gV)
        tau_ex = mu * (gV + gV.T - 2.0 / 3.0 * div * np.eye(d))
        gT = (gp - p0 / rho0 * grho) / rho0               # T = p / rho
        f_ex = -gam / (gam - 1.0) * mu / Pr * gT
        assert np.allclose(tau[0], tau_ex, rtol=1e-12, atol=1e-14)
        assert np.allclose(f[0], f_ex, rtol=1e-12, atol=1e-14)
