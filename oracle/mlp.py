"""NumPy reference of the learned block-Jacobi correction (oracle; test infrastructure only).

Not in the paper.  The learned preconditioner corrects every block-Jacobi
inverse B_F of the condensed trace operator K by a row and column rescaling
and a rank-R term,

    M_F^-1 = diag(e^a) (B_F + (c U)(c V)^T) diag(e^b),
    a_i = 0.5 tanh(o_i0),  b_i = 0.5 tanh(o_i1),
    U_ik = tanh(o_i,2+k),  V_ik = tanh(o_i,2+R+k),  c_i = |B_F,ii|^(1/2),

(c U meaning diag(c) U), with o_i the output of a small multilayer perceptron
applied to per-unknown features (16 -> 32 -> 32 -> 2 + 2R, tanh hidden layers,
linear output).  Row i of U and V comes from row i's own features, so the
rank-R term couples the unknowns of a block with one another.  It is trained
to make M^-1 K close to the identity on random vectors,

    L = sum_v ||x_v - M^-1 K x_v||^2 / sum_v ||x_v||^2,

with Adam (Kingma & Ba).  Everything here is FP64 and written for checking:
plain loops over blocks, explicit chain rule, no fusion.

Parameter vector layout (shared with the device kernels):
    W1 [32][16], b1 [32], W2 [32][32], b2 [32], W3 [2+2R][32], b3 [2+2R].
"""
from __future__ import annotations

import numpy as np

NF, NH, R = 16, 32, 4
NO = 2 + 2 * R
SHAPES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NO, NH)), ("b3", (NO,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[o:o + size].reshape(shape)
        o += size
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def init_params(seed, zero_output=True):
    """Glorot-uniform hidden layers; the output layer starts at zero (M = block Jacobi)."""
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            parts[name] = rng.uniform(-lim, lim, size=shape)
        else:
            parts[name] = np.zeros(shape)
    if zero_output:
        parts["W3"] = np.zeros((NO, NH))
    return pack(parts)


def forward(theta, X):
    """o = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3 for every row x of X (N x 16)."""
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.tanh(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.tanh(z2)
    o = h2 @ p["W3"].T + p["b3"]
    return o, (X, h1, h2)


def backward(theta, cache, dO):
    """Gradient of sum(dO * o) with respect to the parameters (chain rule, layer by layer)."""
    p = unpack(theta)
    X, h1, h2 = cache
    g = {"W3": dO.T @ h2, "b3": dO.sum(0)}
    d2 = (dO @ p["W3"]) * (1.0 - h2 ** 2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 ** 2)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(0)
    return pack(g)


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad ** 2
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def scalings(o):
    return 0.5 * np.tanh(o[:, 0]), 0.5 * np.tanh(o[:, 1])


def low_rank(o):
    """U, V (rows x R) of the rank-R term."""
    return np.tanh(o[:, 2:2 + R]), np.tanh(o[:, 2 + R:2 + 2 * R])


def corrected_block(BF, oF):
    """M_F^-1 of one block (bs x bs) from its inverse BF and the outputs oF (bs x NO)."""
    a, b = scalings(oF)
    U, V = low_rank(oF)
    c = np.sqrt(np.abs(np.diag(BF)))
    return np.exp(a)[:, None] * (BF + (c[:, None] * U) @ (c[:, None] * V).T) * np.exp(b)[None, :]


def precond_loss(Binv, o, X, Wv):
    """Loss L and dL/do for block inverses Binv (nblk x bs x bs), outputs o (nblk*bs x NO).

    X, Wv: (nvec, nblk*bs) random vectors and their images w = K x, both in the
    block-row order (block F, position i -> row F*bs + i).  Per block and vector,
    with e = e^b w, t = (cV)^T e, u = B e + (cU) t, y = e^a u, r = x - y:
    dL/dy = -2 r / |X|^2, and the chain rule back through u, t, e to a, b, U, V.
    """
    nblk, bs, _ = Binv.shape
    a, b = scalings(o)
    U, V = low_rank(o)
    ea, eb = np.exp(a), np.exp(b)
    x2 = float(np.sum(X ** 2))
    loss = 0.0
    ga, gb = np.zeros_like(a), np.zeros_like(b)
    gU, gV = np.zeros_like(U), np.zeros_like(V)
    for F in range(nblk):
        rows = slice(F * bs, (F + 1) * bs)
        BF = Binv[F]
        c = np.sqrt(np.abs(np.diag(BF)))
        cU, cV = c[:, None] * U[rows], c[:, None] * V[rows]
        for v in range(X.shape[0]):
            e = eb[rows] * Wv[v, rows]
            t = cV.T @ e
            u = BF @ e + cU @ t
            y = ea[rows] * u
            r = X[v, rows] - y
            loss += float(r @ r)
            dy = -2.0 * r / x2
            ga[rows] += dy * y
            du = ea[rows] * dy
            gU[rows] += np.outer(du, t) * c[:, None]
            dt = cU.T @ du
            gV[rows] += np.outer(e, dt) * c[:, None]
            de = BF.T @ du + cV @ dt
            gb[rows] += de * e
    th = np.tanh(o)
    dO = np.zeros_like(o)
    dO[:, 0] = ga * 0.5 * (1.0 - th[:, 0] ** 2)
    dO[:, 1] = gb * 0.5 * (1.0 - th[:, 1] ** 2)
    dO[:, 2:2 + R] = gU * (1.0 - th[:, 2:2 + R] ** 2)
    dO[:, 2 + R:] = gV * (1.0 - th[:, 2 + R:] ** 2)
    return loss / x2, dO


def apply_scaled(Binv, o, w):
    """M^-1 w with the corrected blocks (block-row order)."""
    nblk, bs, _ = Binv.shape
    out = np.zeros_like(w)
    for F in range(nblk):
        rows = slice(F * bs, (F + 1) * bs)
        out[rows] = corrected_block(Binv[F], o[rows]) @ w[rows]
    return out
