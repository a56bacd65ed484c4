"""Mixed-precision path on the GPU vs the FP64 oracle.

* Matrix-free FP64 Jacobian action (hdg_jacobian_apply) against the oracle's
  element blocks: y = [A B; C D][x; P lambda] per element, error relative to
  the magnitude sum |A||x| + |B||P lambda| (resp. C, D) <= 1e-12.
* Low-precision condensation: the error of S, g, Y, z and of the FP32 local
  solve against the oracle is REPORTED (no exact pin exists); the bound
  asserted is the FP32 one, 1e-3, far above the expected kappa_scaled * u32.
* Refinement gate: ||J delta + R|| / ||R|| <= 1e-10 on the full Newton system,
  as reported by the library, recomputed with the oracle's own blocks (to the
  1e-10 gate plus the 1e-12 parity of the blocks times |J| |delta| / ||R||);
  the forward error against the oracle's direct solve is printed and held
  to 1e-4 as a sanity bound (kappa(J) reaches ~1e9 on these blocks, so the
  1e-10 backward error implies nothing sharper).
"""
import numpy as np
import pytest

from oracle import hdg as ohdg

from workloads import configs as C

from cases import SMALL_CASES, gpu_plan, oracle_case, to_dev

pytestmark = pytest.mark.gpu

CASES = ["euler2d_tri_p2", "ns2d_tri_p2", "ns3d_hex_p1", "ns3d_hex_p2"]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


_cache = {}


def _case(name):
    if name not in _cache:
        wl = SMALL_CASES[name]()
        disc, inp = oracle_case(wl)
        blocks = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"],
                                        keep_blocks=True)
        _cache[name] = (wl, disc, inp, blocks)
    return _cache[name]


def _oracle_apply(disc, blocks, dx, dlam):
    """Per element A x + B P lam, and the element trace rows C x + D P lam."""
    yl, yt, sl, st = [], [], [], []
    for e, b in enumerate(blocks):
        lam = dlam[ohdg.element_trace_index(disc, e)]
        yl.append(b["A"] @ dx[e] + b["B"] @ lam)
        yt.append(b["C"] @ dx[e] + b["D"] @ lam)
        sl.append(np.abs(b["A"]) @ np.abs(dx[e]) + np.abs(b["B"]) @ np.abs(lam))
        st.append(np.abs(b["C"]) @ np.abs(dx[e]) + np.abs(b["D"]) @ np.abs(lam))
    return np.array(yl), np.array(yt), np.array(sl), np.array(st)


@pytest.mark.parametrize("name", CASES + ["euler2d_tri_p2_iedg"])
def test_jacobian_apply_matches_oracle_blocks(torch, name):
    wl, disc, inp, blocks = _case(name)
    print("case", name, flush=True)
    plan = gpu_plan(wl)
    d = to_dev(inp)
    rng = np.random.default_rng(17)
    E, n = wl.mesh.n_elem, disc.n
    dx = rng.normal(size=(E, n))
    dlam = rng.normal(size=(disc.m, wl.n_trace))
    yl, yt = plan.jacobian_apply(d["v"], d["q"], d["vhat"], torch.from_numpy(dx).cuda(),
                                 torch.from_numpy(dlam).cuda(), ustar=d["ustar"], vbc=d["vbc"])
    torch.cuda.synchronize()
    yl, yt = yl.cpu().numpy(), yt.cpu().numpy()
    ol, ot, sl, st = _oracle_apply(disc, blocks, dx, dlam.reshape(-1))
    el = max(np.linalg.norm(yl[e] - ol[e]) / np.linalg.norm(sl[e]) for e in range(E))
    et = max(np.linalg.norm(yt[e] - ot[e]) / np.linalg.norm(st[e]) for e in range(E))
    print(name, "jvp err loc", el, "tr", et)
    assert el <= 1e-12 and et <= 1e-12
    # reusing the stored pointwise data gives the same result
    plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    yl2, yt2 = plan.jacobian_apply(None, None, None, torch.from_numpy(dx).cuda(), torch.from_numpy(dlam).cuda(),
                                   reuse_points=True)
    assert np.array_equal(yl2.cpu().numpy(), yl) and np.array_equal(yt2.cpu().numpy(), yt)


@pytest.mark.parametrize("name,narrow", [(c, False) for c in CASES] + [("ns3d_hex_p2", True)])
def test_lp_condensation_error_report(torch, name, narrow):
    wl, disc, inp, blocks = _case(name)
    print("case", name, "narrow", narrow, flush=True)
    plan = gpu_plan(wl, narrow_block=narrow)
    d = to_dev(inp)
    lp = plan.assemble_condense_lp(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    torch.cuda.synchronize()
    assert int(lp["status"].abs().max()) == 0
    E = wl.mesh.n_elem

    def rel(got, key, mat):
        worst = 0.0
        for e in range(E):
            g = got[e].astype(np.float64)
            g = g.T if mat else g
            worst = max(worst, np.linalg.norm(g - blocks[e][key]) / np.linalg.norm(blocks[e][key]))
        return worst

    errs = {"S": rel(lp["S"].cpu().numpy(), "S", True), "Y": rel(lp["Y"].cpu().numpy(), "Y", True),
            "g": rel(lp["g"].cpu().numpy(), "g", False), "z": rel(lp["z"].cpu().numpy(), "z", False)}
    # FP32 local solve of a random right-hand side vs the oracle's A
    rng = np.random.default_rng(5)
    r = rng.normal(size=(E, disc.n))
    x = plan.lp_solve(lp["factors"], torch.from_numpy(r).cuda()).cpu().numpy()
    errs["lp_solve"] = max(np.linalg.norm(x[e] - np.linalg.solve(blocks[e]["A"], r[e])) /
                           np.linalg.norm(np.linalg.solve(blocks[e]["A"], r[e])) for e in range(E))
    # residuals are FP64 and identical to the FP64 path's
    errs["R_tr"] = max(np.linalg.norm(lp["R_tr"][e].cpu().numpy() - blocks[e]["R_tr"]) /
                       np.linalg.norm(blocks[e]["R_tr"]) for e in range(E))
    print(name, "low-precision errors vs oracle", errs)
    for key in ("S", "Y", "g", "z", "lp_solve"):
        assert errs[key] <= 1e-3, (key, errs[key])
    assert errs["R_tr"] <= 1e-12


@pytest.mark.parametrize("name", CASES)
def test_refinement_reaches_full_system_tolerance(torch, name):
    wl, disc, inp, blocks = _case(name)
    print("case", name, flush=True)
    plan = gpu_plan(wl)
    d = to_dev(inp)
    lp = plan.assemble_condense_lp(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    dx, dlam, info = plan.refine_solve(d["v"], d["q"], d["vhat"], lp, ustar=d["ustar"], vbc=d["vbc"], tol=1e-10,
                                       max_outer=12, gmres_tol=1e-8)
    torch.cuda.synchronize()
    print(name, info)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    dx, dlam = dx.cpu().numpy(), dlam.cpu().numpy().reshape(-1)
    # residual of the full system with the oracle's blocks
    yl, yt, sl, st = _oracle_apply(disc, blocks, dx, dlam)
    rl = yl + np.array([b["R_loc"] for b in blocks])
    rt = ohdg.trace_rhs(disc, list(yt)) + ohdg.trace_rhs(disc, [b["R_tr"] for b in blocks])
    R = np.concatenate([np.concatenate([b["R_loc"] for b in blocks]),
                        ohdg.trace_rhs(disc, [b["R_tr"] for b in blocks])])
    res = np.linalg.norm(np.concatenate([rl.reshape(-1), rt])) / np.linalg.norm(R)
    mag = np.linalg.norm(np.concatenate([sl.reshape(-1), ohdg.trace_rhs(disc, list(st))])) / np.linalg.norm(R)
    print(name, "oracle-block residual", res, "magnitude ratio", mag)
    assert res <= 1e-10 + 1e-12 * mag
    # forward error against the oracle's direct solve
    bx, bl = ohdg.brute_force_solve(disc, blocks)
    ref = np.concatenate([np.concatenate(bx), bl])
    got = np.concatenate([dx.reshape(-1), dlam])
    fwd = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(name, "forward error vs oracle", fwd)
    assert fwd <= 1e-4


def test_large_block_p3_hex_fp32_and_refinement(torch):
    """n = 1280 (p = 3 hexes, the per-GPU shape of the 32^3 mesh): the FP32 condensation runs with
    16-column blocks (the FP64 one with the right-looking kernels, test_gpu_fullsize); sampled outputs
    against the oracle and the FP64 GPU outputs, and the refined solve."""
    wl = C.ns3d_hex(n=2, p=3, eps=0.05, jitter=0.05)
    disc, inp = oracle_case(wl)
    plan = gpu_plan(wl)
    assert plan.tuning()["condense_width_lp"] == 16
    d = to_dev(inp)
    f64 = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    lp = plan.assemble_condense_lp(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    torch.cuda.synchronize()
    rel = {k: float(torch.linalg.norm(lp[k].double() - f64[k]) / torch.linalg.norm(f64[k])) for k in ("S", "Y", "g", "z")}
    print("p=3 hex FP32 vs FP64 GPU", rel)
    for k, e in rel.items():
        assert e <= 1e-3, (k, e)
    torch.cuda.synchronize()
    assert int(lp["status"].abs().max()) == 0
    ref = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"], elems=[0],
                                 keep_blocks=True)[0]
    errs = {"S": np.linalg.norm(lp["S"][0].cpu().numpy().astype(np.float64).T - ref["S"]) / np.linalg.norm(ref["S"]),
            "Y": np.linalg.norm(lp["Y"][0].cpu().numpy().astype(np.float64).T - ref["Y"]) / np.linalg.norm(ref["Y"]),
            "g": np.linalg.norm(lp["g"][0].cpu().numpy() - ref["g"]) / np.linalg.norm(ref["g"])}
    print("p=3 hex FP32 errors vs oracle", errs)
    for k, e in errs.items():
        assert e <= 1e-3, (k, e)
    # matrix-free FP64 Jacobian of element 0 against the oracle blocks
    rng = np.random.default_rng(31)
    dx = rng.normal(size=(wl.mesh.n_elem, disc.n))
    dlam = rng.normal(size=(disc.m, wl.n_trace))
    yl, yt = plan.jacobian_apply(d["v"], d["q"], d["vhat"], torch.from_numpy(dx).cuda(),
                                 torch.from_numpy(dlam).cuda(), ustar=d["ustar"], vbc=d["vbc"])
    lam0 = dlam.reshape(-1)[ohdg.element_trace_index(disc, 0)]
    ol = ref["A"] @ dx[0] + ref["B"] @ lam0
    sl = np.abs(ref["A"]) @ np.abs(dx[0]) + np.abs(ref["B"]) @ np.abs(lam0)
    assert np.linalg.norm(yl[0].cpu().numpy() - ol) / np.linalg.norm(sl) <= 1e-12
    dxs, dls, info = plan.refine_solve(d["v"], d["q"], d["vhat"], lp, ustar=d["ustar"], vbc=d["vbc"], tol=1e-10,
                                       max_outer=12, gmres_tol=1e-8)
    print("p=3 hex refinement", info)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10


@pytest.mark.parametrize("name", ["ns3d_hex_p2", "ns3d_hex_p3"])
def test_element_refinement_with_fixed_trace_update(torch, name):
    """hdg_refine_local (the element version of the mixed-precision criterion): with the FP32
    factors, A dx = -(R_loc + B P dvhat) for a seeded dvhat converges to a per-element relative
    residual <= 1e-10, and dx equals the FP64 element back-solve -z - Y P dvhat
    (hdg_backsolve_elements) to 1e-9."""
    wl = SMALL_CASES[name]() if name in SMALL_CASES else C.ns3d_hex(n=2, p=3, eps=0.05, jitter=0.05)
    disc, inp = oracle_case(wl)
    plan = gpu_plan(wl)
    d = to_dev(inp)
    f64 = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    lp = plan.assemble_condense_lp(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    rng = np.random.default_rng(41)
    dl = torch.from_numpy(1e-3 * rng.standard_normal((disc.m, wl.n_trace)) * np.abs(inp["vhat"])).cuda()
    dx, info = plan.refine_local(d["v"], d["q"], d["vhat"], lp, dl, ustar=d["ustar"], vbc=d["vbc"], tol=1e-10)
    dx64 = plan.backsolve_elements(f64["Y"], f64["z"], dl)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(dx - dx64) / torch.linalg.norm(dx64))
    print(name, info, "dx vs FP64 back-solve", err, flush=True)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert err <= 1e-9


def test_element_refinement_falls_back_to_fp64(torch):
    """The FP64 fallback of hdg_refine_local, forced from the host: one refinement step cannot
    reach 1e-10 (the FP32 correction leaves about 1e-5), so every element above the tolerance is
    re-assembled and solved with the FP64 LU; the result then meets the tolerance and equals the
    FP64 element back-solve."""
    wl = SMALL_CASES["ns3d_hex_p2"]()
    disc, inp = oracle_case(wl)
    plan = gpu_plan(wl)
    d = to_dev(inp)
    f64 = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    lp = plan.assemble_condense_lp(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    rng = np.random.default_rng(43)
    dl = torch.from_numpy(1e-3 * rng.standard_normal((disc.m, wl.n_trace)) * np.abs(inp["vhat"])).cuda()
    dx, info = plan.refine_local(d["v"], d["q"], d["vhat"], lp, dl, ustar=d["ustar"], vbc=d["vbc"], tol=1e-10,
                                 max_iter=1)
    dx64 = plan.backsolve_elements(f64["Y"], f64["z"], dl)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(dx - dx64) / torch.linalg.norm(dx64))
    print(info, "dx vs FP64 back-solve", err, flush=True)
    assert info["history"][0] > 1e-10                      # one step alone does not reach tol
    assert info["fallback_elements"] == wl.mesh.n_elem
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert err <= 1e-9


@pytest.mark.parametrize("name,narrow", [("ns3d_hex_p1", False), ("ns3d_hex_p2", False), ("ns3d_hex_p2", True)])
def test_bf16_operands_condensation_and_refinement(torch, name, narrow):
    """BF16 operands on the matrix cores (lp_operands = 2; FP32 data, panels and accumulation):
    S, Y, g, z against the oracle carry BF16-level errors.  To first order an output's error is
    its condition times the unit roundoff of the operands, so against the FP32 operands' errors
    on the same blocks it grows by at most the ratio of the unit roundoffs, 2^-9 / 2^-24 = 2^15
    (asserted with a factor 4 of slack), and by at least 10 (evidence that the BF16 instructions
    run); S within 5e-2.  FP64 refinement then reaches 1e-10 on the full Newton system and on the
    element systems, where dx equals the FP64 element back-solve to 1e-9.  narrow: 16-column
    panels (one 16x16x16 BF16 instruction per k-panel instead of 16x16x32)."""
    wl, disc, inp, blocks = _case(name)
    print("case", name, "narrow", narrow, flush=True)
    plan = gpu_plan(wl, narrow_block=narrow)
    if narrow:
        assert plan.tuning()["condense_width_lp"] == 16
    d = to_dev(inp)
    E = wl.mesh.n_elem

    def errs(lp):
        out = {}
        for key, mat in (("S", True), ("Y", True), ("g", False), ("z", False)):
            got = lp[key].cpu().numpy()
            out[key] = max(np.linalg.norm((got[e].astype(np.float64).T if mat else got[e]) - blocks[e][key]) /
                           np.linalg.norm(blocks[e][key]) for e in range(E))
        return out

    plan.set_tuning(lp_operands=1)
    e32 = errs(plan.assemble_condense_lp(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"]))
    plan.set_tuning(lp_operands=2)
    assert plan.tuning()["lp_operands"] == 2
    lp = plan.assemble_condense_lp(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    torch.cuda.synchronize()
    assert int(lp["status"].abs().max()) == 0
    ebf = errs(lp)
    print(name, "FP32 operands", e32, "BF16 operands", ebf, flush=True)
    assert ebf["S"] <= 5e-2, ebf["S"]
    for key in ("S", "Y", "g", "z"):
        assert 10 * e32[key] <= ebf[key] <= 4 * 2.0 ** 15 * e32[key], (key, ebf[key], e32[key])
    dx, dlam, info = plan.refine_solve(d["v"], d["q"], d["vhat"], lp, ustar=d["ustar"], vbc=d["vbc"], tol=1e-10,
                                       max_outer=16, gmres_tol=1e-8)
    torch.cuda.synchronize()
    print(name, "BF16 full-system refinement", info, flush=True)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    f64 = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    rng = np.random.default_rng(47)
    dl = torch.from_numpy(1e-3 * rng.standard_normal((disc.m, wl.n_trace)) * np.abs(inp["vhat"])).cuda()
    dxl, linfo = plan.refine_local(d["v"], d["q"], d["vhat"], lp, dl, ustar=d["ustar"], vbc=d["vbc"], tol=1e-10,
                                   max_iter=12)
    dx64 = plan.backsolve_elements(f64["Y"], f64["z"], dl)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(dxl - dx64) / torch.linalg.norm(dx64))
    print(name, "BF16 element refinement", linfo, "dx vs FP64 back-solve", err, flush=True)
    assert linfo["converged"] == 1 and linfo["rel_residual"] <= 1e-10
    assert linfo["fallback_elements"] == 0
    assert err <= 1e-9
