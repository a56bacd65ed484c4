"""Pins of the oracle's reference elements and geometry against closed forms."""
import itertools

import numpy as np
import pytest

from oracle import geometry as G
from oracle import refelem as R
from workloads import meshes as M

ETYPES = ["tri", "quad", "tet", "hex"]


def test_gll_points_closed_forms():
    # P_2' root at 0; P_3' roots at +-1/sqrt(5); P_4' roots at 0, +-sqrt(3/7)
    assert np.allclose(R.gll_points(2), [-1, 0, 1], atol=1e-15)
    assert np.allclose(R.gll_points(3), [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], atol=1e-15)
    assert np.allclose(R.gll_points(4), [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], atol=1e-15)


@pytest.mark.parametrize("etype", ETYPES)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lagrange_kronecker_and_partition(etype, p):
    ref = R.get_refelem(etype, p)
    phi, dphi = ref.basis(ref.nodes)
    assert np.allclose(phi, np.eye(ref.np_), atol=1e-11)
    val, grad = ref.basis(ref.xq)
    assert np.allclose(val.sum(1), 1.0, atol=1e-12)
    assert np.allclose(grad.sum(1), 0.0, atol=1e-10)


def _exact_monomial_integral(etype, e):
    """Integral of x^e over the reference element (closed forms)."""
    from math import factorial
    if etype in ("quad", "hex"):
        return np.prod([0.0 if k % 2 else 2.0 / (k + 1) for k in e])
    d = len(e)
    # Dirichlet integral over the unit simplex: prod(e_i!) / (d + sum e)!
    return np.prod([factorial(k) for k in e]) / factorial(d + sum(e))


@pytest.mark.parametrize("etype", ETYPES)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_volume_quadrature_exactness(etype, p):
    ref = R.get_refelem(etype, p)
    d = ref.dim
    deg = 2 * (p + 2) - 1 if etype in ("quad", "hex") else 2 * (p + 2) - 1 - (d - 1)
    for e in itertools.product(range(deg + 1), repeat=d):
        if etype in ("quad", "hex") and max(e) > deg:
            continue
        if etype in ("tri", "tet") and sum(e) > deg:
            continue
        num = np.sum(ref.wq * np.prod(ref.xq ** np.array(e)[None, :], axis=1))
        assert abs(num - _exact_monomial_integral(etype, e)) < 1e-13


@pytest.mark.parametrize("etype", ETYPES)
def test_face_nodes_lie_on_faces_and_basis_vanishes_off_face(etype):
    p = 3
    ref = R.get_refelem(etype, p)
    for f, F in enumerate(ref.faces):
        # face quadrature points lie on the face: only the face nodes' basis is non-zero
        off = np.setdiff1d(np.arange(ref.np_), F["nodes"])
        assert np.abs(F["phi"][:, off]).max() < 1e-12
        assert np.allclose(F["psi"].sum(1), 1.0, atol=1e-12)


def _mesh(etype, periodic):
    if etype == "tri":
        return M.tri_square(3, 0.15, 5, periodic=periodic)
    if etype == "quad":
        return M.quad_square(3, 0.15, 5, periodic=periodic)
    if etype == "tet":
        return M.kuhn_tets(2, 0.08, 5, periodic=periodic)
    return M.hex_cube(2, 0.08, 5, periodic=periodic)


@pytest.mark.parametrize("etype", ETYPES)
def test_geometry_volume_and_closed_surface(etype):
    mesh = _mesh(etype, False)
    ref = R.get_refelem(etype, 2)
    vol = 0.0
    for e in range(mesh.n_elem):
        g = G.ElemGeom(ref, mesh.elem_xyz[e])
        vol += g.W.sum()
        # closed surface: sum of n dS vanishes
        tot = sum((F["W"][:, None] * F["n"]).sum(0) for F in g.faces)
        assert np.abs(tot).max() < 1e-13
        # divergence theorem for every basis function: int grad phi = oint phi n
        lhs = np.einsum("q,qaj->aj", g.W, g.gphi)
        rhs = sum(np.einsum("q,qa,qj->aj", F["W"], F["phi"], F["n"]) for F in g.faces)
        assert np.abs(lhs - rhs).max() < 1e-12
    assert abs(vol - np.prod(mesh.length)) < 1e-12 * np.prod(mesh.length)


@pytest.mark.parametrize("etype", ETYPES)
def test_face_normals_outward(etype):
    mesh = _mesh(etype, False)
    ref = R.get_refelem(etype, 1)
    for e in range(mesh.n_elem):
        g = G.ElemGeom(ref, mesh.elem_xyz[e])
        cen = mesh.elem_xyz[e].mean(0)
        for F in g.faces:
            assert np.all(((F["x"] - cen) * F["n"]).sum(1) > 0)
