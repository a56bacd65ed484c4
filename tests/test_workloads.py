"""Input generators: the paper's analytic states and mesh conformity."""
import numpy as np

from workloads import configs as C
from workloads import fields as F
from workloads import meshes as M


def test_shu_vortex_radial_equilibrium():
    """dp/dr = rho u_theta^2 / r holds with the squared Mach number in the density law."""
    f = F.ShuVortex(psi=5.0, mach=0.5, L=0.1, center=(0.5, 0.5))
    r = np.linspace(0.005, 0.3, 50)
    x = np.stack([0.5 + r, 0.5 + 0 * r])
    prim, grad = f.prim_and_grad(x)
    rho, vx, vy, p = prim
    dpdr = grad[3, 0]                     # along +x from the centre
    # relative to the uniform stream, the swirl is vy at these points
    assert np.allclose(dpdr, rho * vy ** 2 / r, rtol=1e-10, atol=1e-12)


def test_tgv_initial_state():
    f = F.TaylorGreen(mach=0.1)
    x = np.random.default_rng(0).uniform(0, 2 * np.pi, (3, 20))
    prim, grad = f.prim_and_grad(x)
    assert np.allclose(prim[0], 1.0)
    assert np.allclose(f.p0, 1 / (1.4 * 0.01))
    # incompressible initial velocity: div V = 0
    assert np.abs(grad[1, 0] + grad[2, 1] + grad[3, 2]).max() < 1e-13


def test_periodic_fields_are_periodic():
    wl = C.ns3d_hex(n=2)
    nf = wl.noisy_field()
    x = np.random.default_rng(1).uniform(0, 2 * np.pi, (3, 10))
    a = nf.prim(x.astype(complex))
    b = nf.prim((x + 2 * np.pi * np.array([1, 0, 0])[:, None]).astype(complex))
    assert np.allclose(a, b, rtol=1e-12)


def test_meshes_conforming_and_counts():
    m = M.hex_cube(4, 0.05, 0)
    tmap, nt = M.trace_map(m, 2, "hdg")
    assert nt == 3 * 64 * 9                     # 3 faces per periodic hex
    counts = np.bincount(tmap.ravel(), minlength=nt)
    assert np.all(counts == 2)                  # every HDG trace node seen by two elements
    nb, nbf = M.face_neighbors(m, 2)
    assert np.all(nb >= 0)
    t = M.tri_square(8, 0.1, 1)
    tm, nt = M.trace_map(t, 2, "hdg")
    assert nt == 208 * 3 and t.boundary.sum() == 32


def test_couette_source_is_the_divergence_of_the_fluxes():
    """The printed source of the Couette example equals div(F(v) + G(v, grad v)) of the printed
    exact solution under the oracle's flux functions (4th-order central differences of the
    flux divergence, gradients of v by differences as well): a check of the formula reading
    and of the flux conventions (stress, heat flux with kappa = mu gamma c_v / Pr)."""
    from oracle import physics as ph
    from workloads.fields import Couette
    c = Couette()
    gam = c.gamma

    def v_at(X):
        pr, _ = c.prim_and_grad(X)
        return ph.v_of_prim(pr[0], pr[1:3].T, pr[3], gam)

    def d4(f, X, k, h):
        e = np.zeros((2, 1))
        e[k] = h
        return (8 * (f(X + e) - f(X - e)) - (f(X + 2 * e) - f(X - 2 * e))) / (12 * h)

    def flux(X):
        v = v_at(X)
        q = np.stack([d4(v_at, X, k, 1e-3) for k in range(2)], axis=-1)
        return ph.flux_F(v, gam) + ph.flux_G(v, q, gam, c.mu, c.Pr)

    ys = np.array([0.05, 0.3, 0.5, 0.8, 0.97])
    X = np.stack([np.full_like(ys, 0.4), ys])
    div = sum(d4(lambda Y: flux(Y)[:, :, k], X, k, 2e-3) for k in range(2)).T
    s = c.source(X)
    assert np.max(np.abs(div - s)) <= 1e-5 * np.max(np.abs(s))


def test_ringleb_field_is_a_steady_euler_solution():
    """The Ringleb field, read with (x - A/2)^2 + y^2 = 1/(4 c^10 V^4) and the 1/(3c^3) term of A
    (both printed garbled), is a steady Euler solution on the example's square: the central
    difference divergence of its inviscid fluxes (written out here) falls as h^2 (below 1e-7
    at h = 1e-3, 100x smaller at h = 1e-4), while the mirrored flow angle leaves an O(1)
    residual; the root solves the hodograph relation, the flow is subsonic, and p = rho^gamma / gamma
    (the hodograph flow is homentropic)."""
    from workloads.fields import Ringleb
    f = Ringleb()
    g = f.gamma
    rng = np.random.default_rng(0)
    pts = np.stack([rng.uniform(-4.9, -1.1, 60), rng.uniform(1.1, 4.9, 60)])

    def fluxes(X, flip=1.0):
        r, u, v, p = f.prim(X)
        v = flip * v
        E = p / (g - 1) + 0.5 * r * (u * u + v * v)
        return (np.stack([r * u, r * u * u + p, r * u * v, u * (E + p)]),
                np.stack([r * v, r * u * v, r * v * v + p, v * (E + p)]))

    def div(h, flip=1.0):
        ex, ey = np.array([[h], [0.0]]), np.array([[0.0], [h]])
        return np.abs((fluxes(pts + ex, flip)[0] - fluxes(pts - ex, flip)[0]) / (2 * h)
                      + (fluxes(pts + ey, flip)[1] - fluxes(pts - ey, flip)[1]) / (2 * h)).max()

    r3, r4 = div(1e-3), div(1e-4)
    assert r3 < 1e-7 and r4 < r3 / 50
    assert div(1e-4, flip=-1.0) > 0.1
    c = f.speed_of_sound(pts)
    assert np.abs(f._f(c, pts[0], pts[1])).max() < 1e-9
    r, u, v, p = f.prim(pts)
    assert np.all(np.hypot(u, v) < np.sqrt(g * p / r))
    np.testing.assert_allclose(p, r ** g / g, rtol=1e-13)
