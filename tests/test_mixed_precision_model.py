"""Refinement with low-precision factors of an element block (CPU model of the arithmetic).

The mixed-precision path factors each element block in low precision after the symmetric
power-of-two scaling D A D (d_i = 2^-round(log2 sqrt|a_ii|)) and refines in FP64.  Whether a
precision can drive the refinement to the 1e-10 criterion is a property of the arithmetic, not
of the kernels, so it is measured here on an oracle element block (3D Navier-Stokes, p = 2
hexahedron, n = 540, cond(A) ~ 1e9, cond(DAD) ~ 2e2) with a plain right-looking LU with partial
pivoting whose update operands are rounded as the matrix cores would take them:

* FP32 operands, FP32 accumulation (the built FP32 path);
* BF16 operands (round to nearest even), FP32 accumulation, factors stored in BF16;
* split BF16: hi + lo operands, three products (hi hi, hi lo, lo hi), FP32 accumulation.

Refinement x += F^-1 (b - A x) with the residual in FP64.  Measured: FP32 and split BF16 reach
1e-13 in two steps; plain BF16 contracts by ~1e-2 per step and reaches 1e-10 in five.
"""
import numpy as np

from oracle import hdg as ohdg
from oracle import state as ostate
from workloads import configs as C


def _bf16(x):
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _lu(A, mode):
    n = A.shape[0]
    M = A.astype(np.float32)
    piv = np.arange(n)
    for k in range(n):
        p = k + int(np.argmax(np.abs(M[k:, k])))
        if p != k:
            M[[k, p]] = M[[p, k]]
            piv[[k, p]] = piv[[p, k]]
        M[k + 1:, k] /= M[k, k]
        l, u = M[k + 1:, k], M[k, k + 1:]
        if mode == "fp32":
            prod = np.outer(l.astype(np.float64), u)
        elif mode == "bf16":
            prod = np.outer(_bf16(l).astype(np.float64), _bf16(u))
        else:
            lh, uh = _bf16(l), _bf16(u)
            ll, ul = _bf16(l - lh), _bf16(u - uh)
            lh64 = lh.astype(np.float64)
            prod = np.outer(lh64, uh) + np.outer(lh64, ul) + np.outer(ll.astype(np.float64), uh)
        M[k + 1:, k + 1:] -= prod.astype(np.float32)
    if mode == "bf16":
        M = _bf16(M)
    return M.astype(np.float64), piv


def _solve(F, piv, b):
    y = b[piv].copy()
    n = len(y)
    for i in range(n):
        y[i] -= F[i, :i] @ y[:i]
    for i in range(n - 1, -1, -1):
        y[i] = (y[i] - F[i, i + 1:] @ y[i + 1:]) / F[i, i]
    return y


def _refine(As, bs, F, piv, steps):
    x = np.zeros_like(bs)
    hist = []
    for _ in range(steps):
        r = bs - As @ x
        hist.append(np.linalg.norm(r) / np.linalg.norm(bs))
        x = x + _solve(F, piv, r)
    return hist


def test_low_precision_factors_and_fp64_refinement():
    wl = C.ns3d_hex(n=2, p=2)
    disc = ohdg.Discretization(wl.mesh, wl.p, ohdg.Phys(wl.gamma, wl.mu, wl.Pr, wl.alpha, wl.viscous), wl.tmap,
                               wl.n_trace, wl.face_bc)
    inp = ostate.oracle_inputs(wl, disc)
    A = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], elems=[3],
                               keep_blocks=True)[0]["A"]
    d = 2.0 ** (-np.rint(0.5 * np.log2(np.abs(np.diag(A)))))
    As = d[:, None] * A * d[None, :]
    assert np.linalg.cond(As) < 1e3 < 1e6 < np.linalg.cond(A)
    bs = d * np.random.default_rng(0).normal(size=A.shape[0])
    h = {m: _refine(As, bs, *_lu(As, m), steps=6) for m in ("fp32", "bf16x3", "bf16")}
    print({m: ["%.1e" % v for v in hs] for m, hs in h.items()})
    assert h["fp32"][2] <= 1e-12 and h["bf16x3"][2] <= 1e-10
    assert max(h["bf16"][i + 1] / h["bf16"][i] for i in range(4)) <= 0.05
    assert h["bf16"][5] <= 1e-10
