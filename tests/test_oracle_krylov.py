"""Pins of the oracle GMRES and block-Jacobi against mathematics, not against themselves.

* exactness: with restart >= n GMRES reaches the solution np.linalg.solve gives;
* finite termination: a diagonalizable matrix with k distinct eigenvalues is
  solved in at most k Arnoldi steps (minimal polynomial of degree k);
* minimal residual: the residual estimate never grows within a cycle, and the
  estimate at the end of a cycle equals the true residual of the update;
* right preconditioning with the exact inverse converges in one step;
* block Jacobi is the exact inverse of a block-diagonal matrix;
* the face / point groups of real trace spaces partition the unknowns.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import krylov
from workloads import configs as C

from cases import oracle_disc


def _rand_system(n, seed, shift=4.0):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n)) / np.sqrt(n) + shift * np.eye(n)
    b = rng.normal(size=n)
    return A, b


def test_gmres_full_restart_gives_the_solution():
    A, b = _rand_system(60, 1, shift=1.5)
    x, it, hist = krylov.gmres(lambda v: A @ v, b, restart=60, tol=1e-13, maxit=60)
    x_ref = np.linalg.solve(A, b)
    assert it <= 60
    assert np.linalg.norm(x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)


def test_gmres_finite_termination_with_k_distinct_eigenvalues():
    rng = np.random.default_rng(2)
    n, eig = 40, np.array([1.0, 3.0, -2.0])
    Q = rng.normal(size=(n, n)) + 4 * np.eye(n)
    lam = eig[rng.integers(0, 3, size=n)]
    A = Q @ np.diag(lam) @ np.linalg.inv(Q)
    b = rng.normal(size=n)
    x, it, hist = krylov.gmres(lambda v: A @ v, b, restart=20, tol=1e-9, maxit=20)
    assert it <= 3, (it, hist)
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)


def test_gmres_restarted_residual_is_monotone_and_estimate_is_true():
    A, b = _rand_system(80, 3, shift=1.2)
    x, it, hist = krylov.gmres(lambda v: A @ v, b, restart=7, tol=1e-11, maxit=400)
    assert np.all(np.diff(hist) <= 1e-14), "GMRES residual increased"
    assert it > 7, "test must exercise restarts"
    assert np.linalg.norm(b - A @ x) <= 1.0001e-11 * np.linalg.norm(b) + 1e-15
    # a single cycle: estimate == true residual of the update
    x1, it1, hist1 = krylov.gmres(lambda v: A @ v, b, restart=5, tol=1e-30, maxit=5)
    true1 = np.linalg.norm(b - A @ x1) / np.linalg.norm(b)
    assert abs(hist1[-1] - true1) <= 1e-12


def test_gmres_exact_right_preconditioner_one_step():
    A, b = _rand_system(50, 4, shift=0.5)
    Ainv = np.linalg.inv(A)
    x, it, _ = krylov.gmres(lambda v: A @ v, b, precond=lambda v: Ainv @ v, restart=10, tol=1e-12)
    assert it == 1
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)


def test_block_jacobi_inverts_block_diagonal_matrix():
    rng = np.random.default_rng(5)
    sizes = [3, 5, 4, 6]
    perm = rng.permutation(sum(sizes))
    groups, start = [], 0
    for s in sizes:
        groups.append(np.sort(perm[start:start + s]))
        start += s
    K = np.zeros((18, 18))
    for g in groups:
        K[np.ix_(g, g)] = rng.normal(size=(len(g), len(g))) + 3 * np.eye(len(g))
    apply, invs = krylov.block_jacobi(sp.csr_matrix(K), groups)
    r = rng.normal(size=18)
    assert np.linalg.norm(apply(r) - np.linalg.solve(K, r)) <= 1e-12 * np.linalg.norm(r)
    x, it, _ = krylov.gmres(lambda v: K @ v, r, precond=apply, restart=5, tol=1e-12)
    assert it == 1


@pytest.mark.parametrize("wl,disjoint", [
    (lambda: C.euler2d_tri_p2(n=3), True),
    (lambda: C.ns3d_hex(n=3, p=1), True),
    (lambda: C.euler2d_tri_p2(n=4, periodic=True, scheme="edg"), False),
])
def test_trace_groups_partition_the_unknowns(wl, disjoint):
    w = wl()
    disc = oracle_disc(w)
    assert krylov.faces_are_disjoint(disc) == disjoint
    groups = krylov.trace_groups(disc)
    allidx = np.sort(np.concatenate(groups))
    assert np.array_equal(allidx, np.arange(disc.m * disc.n_trace))
    size = disc.m * disc.Nfp if disjoint else disc.m
    assert all(len(g) == size for g in groups)
