"""Pins of the oracle's element entropy integrals (int_K rho s, int_K rho), s = ln(p / rho^gamma),
the quantity of Proposition 1 and of the Shu vortex entropy history (Section 5):

* a uniform state: closed form rho ln(p / rho^gamma) |Omega| and rho |Omega| on jittered
  triangle and hexahedron meshes (weights, sign and the gamma exponent);
* the homentropic Shu vortex: p / rho^gamma = 1 / (gamma M^2) everywhere, so the
  mass-weighted mean of s equals ln(1 / (gamma M^2)) up to the interpolation error of v_h
  (1e-5 relative at p = 4, h = 0.83 L),
  although rho varies by a quarter over the vortex (an exponent other than gamma fails)."""
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
