"""Learned block-Jacobi correction on the GPU vs the NumPy oracle (oracle/mlp.py).

* network forward and backward (FP32 kernels) against the FP64 NumPy network on
  the same parameters and features: relative error <= 1e-5;
* Adam step against the NumPy step on the same FP32-rounded inputs: <= 2e-5
  relative (beta2 = 0.999 is not exact in FP32: 1 - beta2 carries a 1.3e-5
  relative representation error into the second moment);
* loss and dL/do (row and column rescaling and rank-R term) with the GPU block
  inverses against the oracle's inverses of the oracle's assembled operator on
  identical vectors: <= 1e-9 relative (the inverses agree to cond * 1e-12);
* the pool of sampled blocks: extracting every block of a system gives the
  same loss and dL/do as the whole-system kernel; the corrected blocks that
  hdg_learn_apply forms act as the oracle's corrected blocks of the extracted
  inverses;
* features: the block-statistics columns against the oracle operator;
* a short training run lowers the proxy loss below its block-Jacobi start, the
  learned GMRES solve reaches the true 1e-10 residual, and the comparison with
  plain block Jacobi is reported (no gain is asserted; the fallback covers a loss).
"""
import numpy as np
import pytest

from oracle import hdg as ohdg
from oracle import krylov
from oracle import mlp as omlp

from cases import SMALL_CASES, gpu_plan, oracle_case, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def case(torch):
    from paper_1808_05066_amd.hdg import LearnedPrecond, TraceSolver
    wl = SMALL_CASES["ns3d_hex_p1"]()
    disc, inp = oracle_case(wl)
    blocks = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"])
    K = ohdg.trace_matrix(disc, [b["S"] for b in blocks]).tocsr()
    plan = gpu_plan(wl)
    d = to_dev(inp)
    out = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    ts = TraceSolver(plan, restart=10, precond="block_jacobi")
    lp = LearnedPrecond(ts)
    lp.setup(out["S"], d["vhat"])
    torch.cuda.synchronize()
    return dict(wl=wl, disc=disc, inp=inp, K=K, plan=plan, d=d, out=out, ts=ts, lp=lp)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_forward_backward_match_numpy(torch, case):
    lp = case["lp"]
    rng = np.random.default_rng(21)
    theta = rng.normal(scale=0.3, size=omlp.N_PARAMS).astype(np.float32)
    feat = rng.normal(size=(lp.N, 16)).astype(np.float32)
    lp.feat.copy_(torch.from_numpy(feat))
    th = torch.from_numpy(theta).cuda()
    o = lp.forward(th).cpu().numpy()
    o_ref, cache = omlp.forward(theta.astype(np.float64), feat.astype(np.float64))
    assert _rel(o, o_ref) <= 1e-5
    dO = rng.normal(size=(lp.N, omlp.NO)).astype(np.float32)
    g = lp.backward(th, torch.from_numpy(dO).cuda()).cpu().numpy()
    g_ref = omlp.backward(theta.astype(np.float64), cache, dO.astype(np.float64))
    assert _rel(g, g_ref) <= 1e-5
    # restore the real features for the other tests
    case["lp"].setup(case["out"]["S"], case["d"]["vhat"])


def test_adam_matches_numpy(torch):
    from paper_1808_05066_amd.hdg import adam
    rng = np.random.default_rng(22)
    n = omlp.N_PARAMS
    theta, g = rng.normal(size=n), rng.normal(size=n)
    m, v = rng.normal(size=n) * 0.1, np.abs(rng.normal(size=n)) * 0.01
    theta, g, m, v = (a.astype(np.float32).astype(np.float64) for a in (theta, g, m, v))
    t_ref, m_ref, v_ref = omlp.adam_step(theta, g, m, v, 3, lr=1e-3)
    tt = [torch.from_numpy(a.astype(np.float32)).cuda() for a in (theta, g, m, v)]
    adam(tt[0], tt[1], tt[2], tt[3], 3, 1e-3)
    assert _rel(tt[0].cpu().numpy(), t_ref) <= 2e-5
    assert _rel(tt[2].cpu().numpy(), m_ref) <= 2e-5 and _rel(tt[3].cpu().numpy(), v_ref) <= 2e-5


def test_loss_gradient_matches_numpy(torch, case):
    disc, K, lp, plan = case["disc"], case["K"], case["lp"], case["plan"]
    groups = krylov.trace_groups(disc)
    Binv = np.stack([np.linalg.inv(K[g][:, g].toarray()) for g in groups])
    cond = max(np.linalg.cond(B) for B in Binv)
    order = np.concatenate(groups)            # block-row r -> global unknown order[r]
    rng = np.random.default_rng(23)
    nvec = 3
    X = rng.normal(size=(nvec, K.shape[0]))
    Wv = np.stack([K @ X[v] for v in range(nvec)])
    o = rng.normal(scale=0.5, size=(len(order), omlp.NO)).astype(np.float32)
    L_ref, dO_ref = omlp.precond_loss(Binv, o.astype(np.float64), X[:, order], Wv[:, order])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    loss, dO = lp.loss_grad(dev(X.reshape(nvec, disc.m, -1)), dev(Wv.reshape(nvec, disc.m, -1)), out=dev(o))
    loss, dO = float(loss), dO.cpu().numpy()
    print("loss", loss, L_ref, "cond", cond)
    assert abs(loss - L_ref) <= max(1e-9, 1e-12 * cond) * abs(L_ref)
    assert _rel(dO, dO_ref) <= max(1e-6, 1e-12 * cond)


def test_pool_matches_whole_system_and_correction_matches_oracle(torch, case):
    from paper_1808_05066_amd.hdg import LearnPool
    disc, lp, plan, ts = case["disc"], case["lp"], case["plan"], case["ts"]
    bs = plan.m * plan.dims["Nfp"]
    nblk = lp.N // bs
    rng = np.random.default_rng(24)
    nvec = 2
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    X = dev(rng.normal(size=(nvec, plan.m, plan.n_trace)))
    Wv = torch.stack([plan.trace_matvec(case["out"]["S"], X[v]) for v in range(nvec)])
    o = dev(rng.normal(scale=0.5, size=(lp.N, omlp.NO)).astype(np.float32))
    loss_w, dO_w = lp.loss_grad(X, Wv, out=o)
    loss_w, dO_w = float(loss_w), dO_w.cpu().numpy().copy()
    # every block into a pool, in two parts, in reverse block order
    pool = LearnPool(nblk, bs, nvec)
    perm = np.arange(nblk)[::-1].copy()
    half = nblk // 2
    pool.add(lp, X, Wv, dev(perm[:half].astype(np.int32)))
    pool.add(lp, X, Wv, dev(perm[half:].astype(np.int32)))
    assert pool.n == nblk
    rows = (perm[:, None] * bs + np.arange(bs)[None, :]).reshape(-1)   # pool row -> system block row
    pool.out.copy_(o[dev(rows)])
    x2 = float((X * X).sum())
    from paper_1808_05066_amd.hdg import _ptr, _stream
    from paper_1808_05066_amd._lib import check
    check(pool.lib.hdg_learn_pool_loss_grad(nblk, bs, _ptr(pool.B), _ptr(pool.out), _ptr(pool.X), _ptr(pool.W),
                                            pool.ld, nvec, x2, _ptr(pool.dO), _ptr(pool.loss), _stream()), "pool")
    torch.cuda.synchronize()
    assert abs(float(pool.loss) - loss_w) <= 1e-12 * abs(loss_w)
    assert _rel(pool.dO.cpu().numpy(), dO_w[rows]) <= 1e-6
    # the corrected blocks of hdg_learn_apply against the oracle's on the extracted inverses:
    # a pool of the index vector maps every block row to its global unknown
    Bsys = np.empty_like(pool.B.cpu().numpy())
    Bsys[perm] = pool.B.cpu().numpy()                        # pool block q = system block perm[q]
    idx = dev(np.arange(plan.m * plan.n_trace, dtype=np.float64).reshape(1, plan.m, plan.n_trace))
    imap = LearnPool(nblk, bs, 1)
    imap.add(lp, idx, idx, dev(np.arange(nblk, dtype=np.int32)))
    gidx = imap.X.cpu().numpy()[0].astype(np.int64)          # block row r -> global unknown
    lp.apply(dev(rng.normal(scale=0.3, size=omlp.N_PARAMS).astype(np.float32)))
    out_sys = lp.out.cpu().numpy().astype(np.float64)
    w_sys = rng.normal(size=(plan.m, plan.n_trace))
    z = ts.apply(dev(w_sys)).cpu().numpy().reshape(-1)
    # stored blocks are column-major: pool block [j][i] is entry (i, j)
    zr = omlp.apply_scaled(Bsys.transpose(0, 2, 1), out_sys, w_sys.reshape(-1)[gidx])
    print("corrected apply vs oracle", _rel(z[gidx], zr))
    assert _rel(z[gidx], zr) <= 1e-12
    # restore the plain inverses and features for the other tests
    lp.setup(case["out"]["S"], case["d"]["vhat"])


def test_features_match_oracle_block_statistics(torch, case):
    disc, K, lp = case["disc"], case["K"], case["lp"]
    groups = krylov.trace_groups(disc)
    f = lp.feat.cpu().numpy().astype(np.float64)
    Kd = K.toarray()
    r = 0
    for g in groups[:20]:
        mask = np.ones(K.shape[0], bool)
        mask[g] = False
        for i, gi in enumerate(g):
            row = f[r]
            assert abs(row[0] - 0.25 * np.log10(abs(Kd[gi, gi]))) <= 1e-5
            assert abs(row[1] - 0.25 * np.log10(np.linalg.norm(Kd[gi, g]))) <= 1e-5
            assert abs(row[2] - 0.25 * np.log10(np.linalg.norm(Kd[gi, mask]))) <= 1e-5
            assert row[4 + i // disc.Nfp] == 1.0 and row[4:9].sum() == 1.0
            assert row[9:12].sum() == 1.0 and row[15] == 1.0
            r += 1
    assert np.all(np.isfinite(f))


def test_training_lowers_loss_and_learned_gmres_converges(torch):
    from paper_1808_05066_amd import learn
    plan, systems = learn.make_training_set(4, n=3, nvec=2, log=print)
    theta, hist = learn.train(systems, 15, lr=3e-3, log=print)
    print("loss history", hist)
    assert hist[-1] < hist[0]
    res = learn.evaluate(theta.cpu().numpy(), n=4, seeds=(learn.HELDOUT_SEED0,), log=print)
    row = res[0]
    print(row)
    assert row["block_jacobi"]["converged"] == 1 and row["block_jacobi"]["true_rel_residual"] <= 1.01e-10
    assert row["learned"]["converged"] == 1 and row["learned"]["true_rel_residual"] <= 1.01e-10
