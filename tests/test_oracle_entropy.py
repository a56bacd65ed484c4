"""Pins of the oracle's element entropy integrals (int_K rho s, int_K rho), s = ln(p / rho^gamma),
the quantity of Proposition 1 and of the Shu vortex entropy history (Section 5), and of its
flow statistics (kinetic energy, |curl V|^2, div V, T = p / rho; the Taylor-Green example):

* a uniform state: closed form rho ln(p / rho^gamma) |Omega| and rho |Omega| on jittered
  triangle and hexahedron meshes (weights, sign and the gamma exponent);
* the homentropic Shu vortex: p / rho^gamma = 1 / (gamma M^2) everywhere, so the
  mass-weighted mean of s equals ln(1 / (gamma M^2)) up to the interpolation error of v_h
  (1e-5 relative at p = 4, h = 0.83 L), although rho varies by a quarter over the vortex
  (an exponent other than gamma fails);
* rigid rotations, a uniform expansion and a 3D shear whose velocity is linear (so v_h is
  exact at p = 2): curl, divergence and kinetic energy in closed form (a wrong sign or index
  in the chain rule V = -w / v_m or in the curl fails)."""
import numpy as np

from oracle import hdg as ohdg, newton, physics as ph
from workloads import fields as F, meshes as M


def disc_of(mesh, p, gamma=1.4):
    tmap, nt = M.trace_map(mesh, p, "hdg")
    fbc = np.zeros((mesh.n_elem, mesh.nf), dtype=np.int32)
    return ohdg.Discretization(mesh, p, ohdg.Phys(gamma, 0.0, 0.72, 0.0, False), tmap, nt, fbc)


def test_entropy_integral_uniform_state():
    rho, p, gamma = 1.3, 0.9, 1.4
    for mesh, V in ((M.tri_square(3, 0.1, 5, periodic=True), [0.2, -0.1]),
                    (M.hex_cube(2, 0.05, 3, periodic=True), [0.2, -0.1, 0.3])):
        disc = disc_of(mesh, 2, gamma)
        N = disc.node_coords().shape[1]
        v = np.repeat(ph.v_of_prim(np.array(rho), np.array(V), np.array(p), gamma)[:, None], N, axis=1)
        out = newton.entropy_integral(disc, v)
        vol = float(np.prod(mesh.length))
        assert out.shape == (mesh.n_elem, 2)
        np.testing.assert_allclose(out.sum(0), [rho * np.log(p / rho ** gamma) * vol, rho * vol], rtol=1e-13)


def test_entropy_integral_homentropic_vortex():
    gamma, mach = 1.4, 0.5
    f = F.ShuVortex(mach=mach, gamma=gamma)
    disc = disc_of(M.tri_square(12, 0.0, 0, periodic=True), 4, gamma)
    prim = f.prim(disc.node_coords())
    v = ph.v_of_prim(prim[0], prim[1:3].T, prim[3], gamma).T.copy()
    rho = prim[0]
    assert rho.min() < 0.75 * rho.max()
    S, mass = newton.entropy_integral(disc, v).sum(0)
    s_exact = np.log(1.0 / (gamma * mach ** 2))
    assert abs(S / mass - s_exact) < 1e-5 * abs(s_exact)   # 1.4e-6 measured (interpolation of v_h)


def _v_of(f_prim, x, gamma=1.4):
    rho, V, p = f_prim(x)
    return ph.v_of_prim(rho, V, p, gamma).T.copy()


def test_flow_statistics_closed_forms_2d():
    """Rigid rotation V = Omega (-(y - 1/2), x - 1/2) and uniform expansion V = a (x - 1/2, y - 1/2)
    with constant rho, p on the unit square (p = 2: v_h is the field itself): |omega|^2 = 4 Omega^2,
    theta = 0, int rho |V|^2 / 2 = rho Omega^2 / 12; theta = 2a, omega = 0; T = p / rho."""
    rho, p, Om, a = 1.2, 0.8, 0.7, 0.3
    disc = disc_of(M.tri_square(3, 0.1, 5, periodic=False), 2)
    x = disc.node_coords()
    one = np.ones(x.shape[1])
    rot = newton.flow_statistics(disc, _v_of(lambda x: (rho * one, np.stack([-Om * (x[1] - .5), Om * (x[0] - .5)], 1),
                                                        p * one), x)).sum(0)
    np.testing.assert_allclose(rot[[1, 2, 3, 6, 7]], [rho, rho * Om ** 2 / 12, 4 * Om ** 2, p / rho, (p / rho) ** 2],
                               rtol=1e-12)
    assert abs(rot[4]) < 1e-13 and abs(rot[5]) < 1e-13
    exp = newton.flow_statistics(disc, _v_of(lambda x: (rho * one, np.stack([a * (x[0] - .5), a * (x[1] - .5)], 1),
                                                        p * one), x)).sum(0)
    np.testing.assert_allclose(exp[[4, 5]], [2 * a, 4 * a * a], rtol=1e-12)
    assert abs(exp[3]) < 1e-13


def test_flow_statistics_curl_3d():
    """V = (-Omega y', Omega x', beta x') (x' = x - pi, y' = y - pi) on hexahedra of [0, 2 pi]^3:
    omega = (0, -beta, 2 Omega), |omega|^2 = beta^2 + 4 Omega^2 everywhere, theta = 0."""
    rho, p, Om, be = 1.0, 1.1, 0.4, 0.25
    mesh = M.hex_cube(2, 0.05, 3, periodic=False)
    disc = disc_of(mesh, 2)
    x = disc.node_coords()
    one = np.ones(x.shape[1])
    st = newton.flow_statistics(disc, _v_of(lambda x: (rho * one, np.stack([-Om * (x[1] - np.pi), Om * (x[0] - np.pi),
                                                                           be * (x[0] - np.pi)], 1), p * one), x)).sum(0)
    vol = (2 * np.pi) ** 3
    np.testing.assert_allclose(st[[1, 3]], [rho * vol, (be ** 2 + 4 * Om ** 2) * vol], rtol=1e-12)
    assert abs(st[4]) < 1e-12 * vol and abs(st[5]) < 1e-12 * vol
