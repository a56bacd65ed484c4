"""Full-size parity: the 4096-element 3D Navier-Stokes p=2 mesh, in the launch
configuration bench.py times (one chunk of all elements), checked against the
oracle on sampled elements (first, last and seeded random ones).

S, Y, g, R_tr: relative Frobenius error <= 1e-12.  z: backward error
||A z_gpu - R_loc|| <= 1e-12 times the summation scale of R_loc, and forward
relative error <= 1e-11 and within the element's derived first-order bound
(see cases.z_backward_err, cases.z_forward_bound)."""
import numpy as np
import pytest

from oracle import hdg as ohdg
from oracle import state as ostate
from workloads import configs as C

from cases import gpu_plan, oracle_disc, z_backward_err, z_forward_report

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def full(torch):
    wl = C.ns3d_hex(n=16, p=2)
    disc = oracle_disc(wl)
    inp = ostate.oracle_inputs_fast(wl, disc)
    plan = gpu_plan(wl)
    dev = {k: (None if inp[k] is None else torch.from_numpy(np.ascontiguousarray(inp[k])).cuda())
           for k in ("v", "q", "vhat", "ustar")}
    print("full-size run: %d elements" % wl.mesh.n_elem, flush=True)
    out = plan.assemble_condense(dev["v"], dev["q"], dev["vhat"], dev["ustar"], None, residuals=True)
    torch.cuda.synchronize()
    return wl, disc, inp, plan, out


@pytest.fixture(scope="module")
def sampled_ref(full):
    wl, disc, inp, _, _ = full
    E = wl.mesh.n_elem
    rng = np.random.default_rng(2024)
    sample = [0, E - 1] + list(rng.choice(np.arange(1, E - 1), 2, replace=False))
    ref = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], None, elems=sample,
                                 keep_blocks=True)
    return sample, ref


def check_sampled(disc, inp, out, sample, ref):
    for e, r in zip(sample, ref):
        errs = {}
        zg = out["z"][e].cpu().numpy()
        zf, zr = z_forward_report(disc, inp, [e], [r["A"]], [r["R_loc"]], [r["z"]], [zg])
        assert zf <= 1e-11 and zr <= 1.0, (e, zf, zr)
        errs["z_backward"] = z_backward_err(disc, inp, e, r["A"], r["R_loc"], zg)
        for key, mat in (("S", True), ("Y", True), ("g", False)):
            got = out[key][e].cpu().numpy()
            got = got.T if mat else got
            errs[key] = np.linalg.norm(got - r[key]) / np.linalg.norm(r[key])
        errs["R_tr"] = np.linalg.norm(out["R_tr"][e].cpu().numpy() - r["R_tr"]) / np.linalg.norm(r["R_tr"])
        print("element", e, errs, flush=True)
        for key, err in errs.items():
            assert err <= TOL, (e, key, err)


def test_ns3d_hex_p2_16_sampled(torch, full, sampled_ref):
    wl, disc, inp, plan, out = full
    assert int((out["status"] != 0).sum()) == 0
    check_sampled(disc, inp, out, *sampled_ref)


def test_ns3d_hex_p2_16_eliminate_q(torch, full, sampled_ref):
    """The q-eliminating condensation at full size in the launch configuration bench.py times: sampled
    elements against the oracle, and every element against the full-block condensation."""
    wl, disc, inp, _, out = full
    plan = gpu_plan(wl, eliminate_q=True)
    dev = {k: (None if inp[k] is None else torch.from_numpy(np.ascontiguousarray(inp[k])).cuda())
           for k in ("v", "q", "vhat", "ustar")}
    print("full-size run with q eliminated first", flush=True)
    outq = plan.assemble_condense(dev["v"], dev["q"], dev["vhat"], dev["ustar"], None, residuals=True)
    torch.cuda.synchronize()
    assert int((outq["status"] != 0).sum()) == 0
    check_sampled(disc, inp, outq, *sampled_ref)
    E = wl.mesh.n_elem
    for key in ("S", "Y", "g"):
        a = outq[key].reshape(E, -1)
        b = out[key].reshape(E, -1)
        err = float(((a - b).norm(dim=1) / b.norm(dim=1)).max())
        print(key, "max over elements vs full block", err, flush=True)
        assert err <= TOL, (key, err)
    del plan, outq, dev
    torch.cuda.empty_cache()


def test_ns3d_hex_p2_16_trace_solve(torch, full):
    """GMRES(50) + block Jacobi on the full condensed system.

    Sampled check of the preconditioner: the face block shared by elements
    (e, f) and its neighbour, assembled from the oracle's S of both elements,
    must be inverted by the GPU apply of a vector supported on that face
    (backward error ||B_o z - r|| <= 1e-12 cond-free scale ||B_o|| ||z||).
    The solve must reach its tolerance on the true residual, recomputed here
    with the (parity-tested) trace operator.
    """
    from paper_1808_05066_amd.hdg import TraceSolver
    wl, disc, inp, plan, out = full
    m, nt, Nfp = disc.m, wl.n_trace, disc.Nfp
    ts = TraceSolver(plan, restart=50, maxit=1000, tol=1e-10, precond="block_jacobi")
    ts.setup(out["S"])
    # sampled face blocks
    rng = np.random.default_rng(11)
    for e, f in ((0, 0), (wl.mesh.n_elem - 1, disc.nf - 1), (int(rng.integers(wl.mesh.n_elem)), 2)):
        nodes = np.sort(wl.tmap[e, f])
        owners = [(e2, f2) for e2 in range(wl.mesh.n_elem) for f2 in range(disc.nf)
                  if np.array_equal(np.sort(wl.tmap[e2, f2]), nodes)]
        assert 1 <= len(owners) <= 2
        ref = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], None,
                                     elems=[o[0] for o in owners])
        gidx = (np.arange(m)[:, None] * nt + nodes[None, :]).reshape(-1)
        B = np.zeros((m * Nfp, m * Nfp))
        for (e2, f2), r2 in zip(owners, ref):
            idx = ohdg.element_trace_index(disc, e2)
            pos = {int(t): i for i, t in enumerate(idx)}
            loc = np.array([pos[int(t)] for t in gidx])
            B += r2["S"][np.ix_(loc, loc)]
        rvec = np.zeros(m * nt)
        rvec[gidx] = rng.normal(size=gidx.size)
        z = ts.apply(torch.from_numpy(rvec.reshape(m, nt)).cuda()).cpu().numpy().reshape(-1)
        zg = z[gidx]
        back = np.linalg.norm(B @ zg - rvec[gidx]) / (np.linalg.norm(B) * np.linalg.norm(zg))
        print("face block", e, f, owners, "backward", back, flush=True)
        assert back <= 1e-12
        mask = np.ones(m * nt, bool)
        mask[gidx] = False
        assert np.all(z[mask] == 0.0)
    rhs = plan.trace_rhs(out["g"])
    x, info = ts.solve(out["S"], rhs)
    print("full-size GMRES", info, flush=True)
    assert info["converged"] == 1
    y = plan.trace_matvec(out["S"], x)
    res = float(torch.linalg.norm(rhs - y) / torch.linalg.norm(rhs))
    assert res <= 1.01e-10


def test_p3_hex_fp64_condensation_sampled(torch):
    """FP64 condensation of p = 3 hexahedra (n = 1280, k = 480, the block of the 32^3 mesh): the local
    block does not fit the left-looking kernels' LDS, so the right-looking kernels run, with the
    rows of the first panels beyond 1168 kept in the block itself; S, Y, g and R_tr of sampled
    elements against the oracle to 1e-12, z by its backward error (1e-12) and forward error (1e-11)."""
    wl = C.ns3d_hex(n=2, p=3, eps=0.05, jitter=0.05)
    disc = oracle_disc(wl)
    inp = ostate.oracle_inputs(wl, disc)
    plan = gpu_plan(wl)
    assert plan.dims["n"] == 1280 and plan.tuning()["condense_width"] == 0
    dev = {k: (None if inp[k] is None else torch.from_numpy(np.ascontiguousarray(inp[k])).cuda())
           for k in ("v", "q", "vhat", "ustar", "vbc")}
    out = plan.assemble_condense(dev["v"], dev["q"], dev["vhat"], dev["ustar"], dev["vbc"], residuals=True)
    torch.cuda.synchronize()
    assert int(out["status"].abs().max()) == 0
    sample = [0, 5]
    ref = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"], elems=sample,
                                 keep_blocks=True)
    check_sampled(disc, inp, out, sample, ref)
