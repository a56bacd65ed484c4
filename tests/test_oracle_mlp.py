"""Pins of the NumPy MLP and preconditioner-loss oracle.

* backward() and precond_loss()'s gradient against central finite differences
  of the forward functions (FP64, step 1e-6, relative agreement 1e-6);
* layer algebra against closed forms: with zero hidden weights the network is
  the constant tanh-free output b3; a zero output layer gives M = block Jacobi
  (loss equals the plain block-Jacobi residual);
* Adam's first step moves every parameter by lr * sign(grad) (bias correction);
* with exact block inverses of a block-diagonal K the loss is zero.
"""
import numpy as np

from oracle import mlp


def _rand_theta(seed):
    return np.random.default_rng(seed).normal(scale=0.3, size=mlp.N_PARAMS)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(7, mlp.NF))
    dO = rng.normal(size=(7, mlp.NO))
    theta = _rand_theta(2)
    o, cache = mlp.forward(theta, X)
    g = mlp.backward(theta, cache, dO)
    h = 1e-6
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (np.sum(dO * mlp.forward(tp, X)[0]) - np.sum(dO * mlp.forward(tm, X)[0])) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_constant_network_and_block_jacobi_start():
    X = np.random.default_rng(3).normal(size=(5, mlp.NF))
    parts = mlp.unpack(np.zeros(mlp.N_PARAMS))
    b3 = np.linspace(-0.7, 0.7, mlp.NO)
    parts["b3"] = b3
    o, _ = mlp.forward(mlp.pack(parts), X)
    assert np.allclose(o, [b3] * 5, rtol=0, atol=0)
    theta = mlp.init_params(0)
    o, _ = mlp.forward(theta, X)
    assert np.all(o == 0.0)


def _block_system(seed, nblk=4, bs=5, coupling=0.2):
    rng = np.random.default_rng(seed)
    N = nblk * bs
    K = coupling * rng.normal(size=(N, N))
    for F in range(nblk):
        s = slice(F * bs, (F + 1) * bs)
        K[s, s] = rng.normal(size=(bs, bs)) + 4 * np.eye(bs)
    Binv = np.stack([np.linalg.inv(K[F * bs:(F + 1) * bs, F * bs:(F + 1) * bs]) for F in range(nblk)])
    return K, Binv


def test_loss_gradient_matches_finite_differences():
    K, Binv = _block_system(4)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(3, K.shape[0]))
    Wv = X @ K.T
    o = rng.normal(scale=0.5, size=(K.shape[0], mlp.NO))
    L, dO = mlp.precond_loss(Binv, o, X, Wv)
    h = 1e-6
    for i in range(0, K.shape[0], 3):
        for j in range(mlp.NO):
            op, om = o.copy(), o.copy()
            op[i, j] += h
            om[i, j] -= h
            fd = (mlp.precond_loss(Binv, op, X, Wv)[0] - mlp.precond_loss(Binv, om, X, Wv)[0]) / (2 * h)
            assert abs(fd - dO[i, j]) <= 1e-6 * max(1e-3, abs(fd)), (i, j, fd, dO[i, j])
    # loss is the plain residual of the scaled preconditioner
    Y = np.stack([mlp.apply_scaled(Binv, o, Wv[v]) for v in range(3)])
    assert abs(L - np.sum((X - Y) ** 2) / np.sum(X ** 2)) <= 1e-12


def test_exact_inverse_gives_zero_loss_and_zero_output_is_block_jacobi():
    K, Binv = _block_system(6, coupling=0.0)
    X = np.random.default_rng(7).normal(size=(2, K.shape[0]))
    Wv = X @ K.T
    L, dO = mlp.precond_loss(Binv, np.zeros((K.shape[0], mlp.NO)), X, Wv)
    assert L <= 1e-24 and np.max(np.abs(dO)) <= 1e-12


def test_corrected_block_is_scaling_plus_rank_r():
    """The corrected block against its definition written out entry by entry: row and column
    rescaling of B + sum_k c_i c_j U_ik V_jk, of rank at most R in the correction."""
    rng = np.random.default_rng(9)
    bs = 6
    BF = rng.normal(size=(bs, bs)) + 3 * np.eye(bs)
    oF = rng.normal(scale=0.7, size=(bs, mlp.NO))
    M = mlp.corrected_block(BF, oF)
    for i in range(bs):
        for j in range(bs):
            ai, bj = 0.5 * np.tanh(oF[i, 0]), 0.5 * np.tanh(oF[j, 1])
            ci, cj = np.sqrt(abs(BF[i, i])), np.sqrt(abs(BF[j, j]))
            corr = sum(ci * cj * np.tanh(oF[i, 2 + k]) * np.tanh(oF[j, 2 + mlp.R + k]) for k in range(mlp.R))
            assert abs(M[i, j] - np.exp(ai) * (BF[i, j] + corr) * np.exp(bj)) <= 1e-13 * (1 + abs(M[i, j]))
    a, b = mlp.scalings(oF)
    D = np.exp(-a)[:, None] * M * np.exp(-b)[None, :] - BF
    assert np.linalg.matrix_rank(D, tol=1e-10) <= mlp.R


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(8)
    theta = rng.normal(size=20)
    grad = rng.normal(size=20)
    t2, m, v = mlp.adam_step(theta, grad, np.zeros(20), np.zeros(20), 1, lr=1e-2, eps=0.0)
    assert np.allclose(theta - t2, 1e-2 * np.sign(grad), rtol=0, atol=1e-15)
