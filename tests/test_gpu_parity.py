"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Bar (FP64 path): per element ||X_gpu - X_oracle||_F / ||X_oracle||_F <= 1e-12 for
the pure evaluations R_tr, A, B, C, D and for the condensed outputs S, g, Y, z;
max over elements.  R_loc nearly cancels (states close to a discrete steady
state), so its error is measured against the sum of magnitudes of its
quadrature contributions (cases.residual_term_scale), also at 1e-12; z = A^-1
R_loc inherits that cancellation and is judged by its backward error in the
same scale (cases.z_backward_err) at 1e-12, with a forward error of at most 1e-11 that must
also lie within each element's derived first-order bound (cases.z_forward_bound: LU backward
error and the rounding of R_loc through Skeel's componentwise condition; 4.5e-12 to 9.2e-10 on
these cases).
"""
import numpy as np
import pytest

from oracle import hdg as ohdg
from oracle import state as ostate

from cases import (SMALL_CASES, colmajor, gpu_plan, oracle_case, oracle_disc, rel_err_per_elem, rloc_err, to_dev,
                   z_backward_err, z_forward_report)

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def test_mfma_layout_selftest(torch):
    from paper_1808_05066_amd.hdg import selftest
    assert selftest() == 0.0


_cache = {}


def _case(name):
    if name not in _cache:
        wl = SMALL_CASES[name]()
        disc, inp = oracle_case(wl)
        blocks = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"],
                                        keep_blocks=True)
        _cache[name] = (wl, disc, inp, blocks)
    return _cache[name]


@pytest.mark.parametrize("name,ct", [(c, 1024) for c in SMALL_CASES] +
                         [(c, t) for c in ("ns2d_tri_p2", "ns3d_hex_p1", "ns3d_hex_p2", "euler3d_hex_p2")
                          for t in (256, 512)])
def test_assemble_blocks_match_oracle(torch, name, ct):
    """Every block of the element against the oracle, at each workgroup size of the block
    contraction (each size is its own kernel instantiation)."""
    wl, disc, inp, blocks = _case(name)
    print("case", name, "contract_threads", ct, flush=True)
    plan = gpu_plan(wl)
    plan.set_tuning(contract_threads=ct)
    d = to_dev(inp)
    out = plan.assemble(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    torch.cuda.synchronize()
    assert int(out["status"].abs().max()) == 0
    errs = {
        "R_loc": rloc_err(disc, inp, out["R_loc"].cpu().numpy(), np.stack([b["R_loc"] for b in blocks])),
        "R_tr": rel_err_per_elem(out["R_tr"].cpu().numpy(), np.stack([b["R_tr"] for b in blocks])),
        "A": rel_err_per_elem(out["A"].cpu().numpy(), colmajor([b["A"] for b in blocks])),
        "B": rel_err_per_elem(out["B"].cpu().numpy(), colmajor([b["B"] for b in blocks])),
        "C": rel_err_per_elem(out["C"].cpu().numpy(), colmajor([b["C"] for b in blocks])),
        "D": rel_err_per_elem(out["D"].cpu().numpy(), colmajor([b["D"] for b in blocks])),
    }
    print(name, errs)
    for key, err in errs.items():
        assert err <= TOL, (key, err)


@pytest.mark.parametrize("name", list(SMALL_CASES))
@pytest.mark.parametrize("chunk,split,narrow", [(0, False, False), (3, False, False), (0, True, False),
                                                (0, False, True)])
def test_condense_matches_oracle(torch, name, chunk, split, narrow):
    wl, disc, inp, blocks = _case(name)
    print("case", name, "chunk", chunk, "split", split, "narrow", narrow, flush=True)
    plan = gpu_plan(wl, chunk_elems=chunk, split_dense=split, narrow_block=narrow)
    d = to_dev(inp)
    out = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"], residuals=True)
    torch.cuda.synchronize()
    assert int(out["status"].abs().max()) == 0
    errs = {
        "S": rel_err_per_elem(out["S"].cpu().numpy(), colmajor([b["S"] for b in blocks])),
        "Y": rel_err_per_elem(out["Y"].cpu().numpy(), colmajor([b["Y"] for b in blocks])),
        "g": rel_err_per_elem(out["g"].cpu().numpy(), np.stack([b["g"] for b in blocks])),
        "z_backward": max(z_backward_err(disc, inp, e, b["A"], b["R_loc"], out["z"][e].cpu().numpy())
                          for e, b in enumerate(blocks)),
        "R_loc": rloc_err(disc, inp, out["R_loc"].cpu().numpy(), np.stack([b["R_loc"] for b in blocks])),
        "R_tr": rel_err_per_elem(out["R_tr"].cpu().numpy(), np.stack([b["R_tr"] for b in blocks])),
    }
    print(name, errs)
    for key, err in errs.items():
        assert err <= TOL, (key, err)
    zf, zr = z_forward_report(disc, inp, range(len(blocks)), [b["A"] for b in blocks], [b["R_loc"] for b in blocks],
                              [b["z"] for b in blocks], list(out["z"].cpu().numpy()))
    assert zf <= 1e-11 and zr <= 1.0, (zf, zr)


@pytest.mark.parametrize("name", list(SMALL_CASES))
@pytest.mark.parametrize("lu_waves,chunk", [(2, 0), (4, 0), (8, 0), (4, 3)])
def test_register_lu_matches_oracle(torch, name, lu_waves, chunk):
    """The LU with its working block in registers (2, 4 or 8 waves) in front of the same
    right-hand-side launch: S, Y, g, z against the oracle at the bar of the LDS kernel, and
    against the LDS kernel's outputs on the same plan.  Two waves take n_pad <= 160 only,
    four n_pad <= 192; a larger block must be refused."""
    wl, disc, inp, blocks = _case(name)
    print("case", name, "lu_waves", lu_waves, "chunk", chunk, flush=True)
    plan = gpu_plan(wl, chunk_elems=chunk)
    d = to_dev(inp)
    if plan.n_pad > {2: 160, 4: 192, 8: 640}[lu_waves]:
        with pytest.raises(RuntimeError):
            plan.set_tuning(lu_waves=lu_waves)
        return
    plan.set_tuning(lu_waves=1)
    ref = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    plan.set_tuning(lu_waves=lu_waves)
    assert plan.tuning()["lu_waves"] == lu_waves
    out = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"], residuals=True)
    torch.cuda.synchronize()
    assert int(out["status"].abs().max()) == 0
    errs = {
        "S": rel_err_per_elem(out["S"].cpu().numpy(), colmajor([b["S"] for b in blocks])),
        "Y": rel_err_per_elem(out["Y"].cpu().numpy(), colmajor([b["Y"] for b in blocks])),
        "g": rel_err_per_elem(out["g"].cpu().numpy(), np.stack([b["g"] for b in blocks])),
        "z_backward": max(z_backward_err(disc, inp, e, b["A"], b["R_loc"], out["z"][e].cpu().numpy())
                          for e, b in enumerate(blocks)),
    }
    print(name, errs)
    for key, err in errs.items():
        assert err <= TOL, (key, err)
    zf, zr = z_forward_report(disc, inp, range(len(blocks)), [b["A"] for b in blocks], [b["R_loc"] for b in blocks],
                              [b["z"] for b in blocks], list(out["z"].cpu().numpy()))
    assert zf <= 1e-11 and zr <= 1.0, (zf, zr)
    for key in ("S", "Y", "g"):
        diff = rel_err_per_elem(out[key].cpu().numpy(), ref[key].cpu().numpy())
        assert diff <= TOL, (key, diff)


@pytest.mark.parametrize("name", ["euler2d_tri_p2", "ns2d_tri_p2", "ns3d_hex_p1", "ns3d_hex_p2"])
def test_trace_operator_backsolve_and_brute_force(torch, name):
    """Condensed solve with GPU S, g + GPU back-solve == oracle brute-force full solve.  The p = 2
    hexahedra (k = 270, n = 540) run the operator product and the back-solve at the shapes of the
    measured workload (one row per thread over whole waves)."""
    import scipy.sparse.linalg as spla
    wl, disc, inp, blocks = _case(name)
    plan = gpu_plan(wl)
    d = to_dev(inp)
    out = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    S = out["S"].cpu().numpy()
    g = out["g"].cpu().numpy()
    m, nt = disc.m, wl.n_trace
    # matrix-free operator and right-hand side vs the oracle's
    x = np.random.default_rng(3).normal(size=(m, nt))
    y = plan.trace_matvec(out["S"], torch.from_numpy(x).cuda()).cpu().numpy()
    y_ref = ohdg.trace_matvec(disc, [b["S"] for b in blocks], x.reshape(-1)).reshape(m, nt)
    assert np.linalg.norm(y - y_ref) <= 1e-12 * np.linalg.norm(y_ref)
    r = plan.trace_rhs(out["g"]).cpu().numpy()
    r_ref = ohdg.trace_rhs(disc, [b["g"] for b in blocks]).reshape(m, nt)
    assert np.linalg.norm(r - r_ref) <= 1e-12 * np.linalg.norm(r_ref)
    # global solve on the host from the GPU blocks, then GPU back-solve
    K = ohdg.trace_matrix(disc, [Si.T for Si in S]).tocsc()
    dl = spla.spsolve(K, r.reshape(-1))
    dv, dq = plan.backsolve(out["Y"], out["z"], torch.from_numpy(dl.reshape(m, nt).copy()).cuda())
    bx, bl = ohdg.brute_force_solve(disc, blocks)
    assert np.linalg.norm(dl - bl) <= 1e-10 * np.linalg.norm(bl)
    dv = dv.cpu().numpy()
    Np = disc.Np
    for e in range(0, wl.mesh.n_elem, max(1, wl.mesh.n_elem // 7)):
        ref = bx[e]
        got = dv[:, e * Np:(e + 1) * Np].reshape(-1)
        if wl.viscous:
            got = np.concatenate([got, dq.cpu().numpy()[:, e * Np:(e + 1) * Np].reshape(-1)])
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", ["euler2d_tri_p2", "ns3d_hex_p2"])
def test_prepare_state_and_node_coords(torch, name):
    wl, disc, inp, _ = _case(name)
    plan = gpu_plan(wl)
    x, xt = plan.node_coords()
    assert np.allclose(x.cpu().numpy(), inp["xn"], rtol=0, atol=1e-14 * np.abs(inp["xn"]).max())
    assert np.allclose(xt.cpu().numpy(), inp["xt"], rtol=0, atol=1e-14 * np.abs(inp["xt"]).max())
    prim = torch.from_numpy(inp["prim"]).cuda()
    grad = torch.from_numpy(inp["grad"]).cuda() if inp["grad"] is not None else None
    v, q, u = plan.prepare_state(prim, grad, want_u=True)
    v_ref, q_ref = ostate.entropy_state(inp["prim"], inp["grad"], wl.gamma)
    assert np.abs(v.cpu().numpy() - v_ref).max() <= 1e-13 * np.abs(v_ref).max()
    if q is not None:
        assert np.abs(q.cpu().numpy() - q_ref).max() <= 1e-12 * np.abs(q_ref).max()
    u_ref = ostate.conservative_state(inp["prim"], wl.gamma)
    assert np.abs(u.cpu().numpy() - u_ref).max() <= 1e-14 * np.abs(u_ref).max()


def test_nonphysical_state_is_flagged(torch):
    wl, disc, inp, _ = _case("euler2d_tri_p2")
    plan = gpu_plan(wl)
    d = to_dev(inp)
    bad = 17
    d["v"][-1, bad * disc.Np:(bad + 1) * disc.Np] = 0.5       # v_m >= 0: not a physical state
    out = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    st = out["status"].cpu().numpy()
    assert st[bad] == -3
    assert np.count_nonzero(st) == 1
    # the status reduction of the C-ABI names the same element and code
    assert plan.status(out["status"]) == (bad, -3)
    good = plan.assemble_condense(*(to_dev(inp)[key] for key in ("v", "q", "vhat", "ustar", "vbc")))
    assert plan.status(good["status"]) == (-1, 0)


VISCOUS_CASES = [n for n in SMALL_CASES if n.startswith("ns")]


@pytest.mark.parametrize("name", VISCOUS_CASES)
@pytest.mark.parametrize("chunk,launches", [(0, 2), (3, 1)])
def test_q_elimination_matches_oracle(torch, name, chunk, launches):
    """HDG_FLAG_ELIMINATE_Q: the gradient unknowns eliminated element by element, then the
    m N_p block of v condensed; S, Y (all rows), g, z against the oracle's dense condensation."""
    wl, disc, inp, blocks = _case(name)
    print("case", name, "chunk", chunk, "launches", launches, flush=True)
    plan = gpu_plan(wl, chunk_elems=chunk, eliminate_q=True)
    plan.set_tuning(condense_launches=launches)
    d = to_dev(inp)
    out = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"], residuals=True)
    torch.cuda.synchronize()
    assert int(out["status"].abs().max()) == 0
    errs = {
        "S": rel_err_per_elem(out["S"].cpu().numpy(), colmajor([b["S"] for b in blocks])),
        "Y": rel_err_per_elem(out["Y"].cpu().numpy(), colmajor([b["Y"] for b in blocks])),
        "g": rel_err_per_elem(out["g"].cpu().numpy(), np.stack([b["g"] for b in blocks])),
        "z_backward": max(z_backward_err(disc, inp, e, b["A"], b["R_loc"], out["z"][e].cpu().numpy())
                          for e, b in enumerate(blocks)),
    }
    print(name, errs)
    for key, err in errs.items():
        assert err <= TOL, (key, err)
    zf, zr = z_forward_report(disc, inp, range(len(blocks)), [b["A"] for b in blocks], [b["R_loc"] for b in blocks],
                              [b["z"] for b in blocks], list(out["z"].cpu().numpy()))
    assert zf <= 1e-11 and zr <= 1.0, (zf, zr)
    # the condensation forms only the parts of the q rows of A that the elimination reads; the
    # block export of the same plan afterwards still has the whole of A
    blk = plan.assemble(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    torch.cuda.synchronize()
    ea = rel_err_per_elem(blk["A"].cpu().numpy(), colmajor([b["A"] for b in blocks]))
    assert ea <= TOL, ea


def test_q_elimination_needs_gradient_unknowns(torch):
    from paper_1808_05066_amd import _lib
    wl, _, _, _ = _case("euler2d_tri_p2")
    with pytest.raises(_lib.HdgError):
        gpu_plan(wl, eliminate_q=True)


@pytest.mark.parametrize("name", ["ns2d_tri_p2", "ns3d_hex_p1"])
def test_source_term_matches_oracle(torch, name):
    """hdg_plan_set_source: a source linear in x (its nodal interpolant is exact, so the GPU's
    interpolated source and the oracle's source at the quadrature points are the same
    function); R_loc against the oracle's element residual with that source, R_tr and the
    Jacobian unchanged."""
    wl, disc, inp, blocks = _case(name)
    rng = np.random.default_rng(42)
    coef = rng.standard_normal((disc.m, 1 + disc.d))

    def src(x):   # x (Nq, d) -> (Nq, m)
        return coef[:, 0][None, :] + x @ coef[:, 1:].T

    plan = gpu_plan(wl)
    d = to_dev(inp)
    xn = disc.node_coords()
    plan.set_source(torch.from_numpy(np.ascontiguousarray(src(xn.T).T)).cuda())
    out = plan.assemble(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    torch.cuda.synchronize()
    ref_R, ref_T = [], []
    for e in range(disc.mesh.n_elem):
        x, lam, us, vb = disc.elem_inputs(e, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"])
        R, T = disc.element_residual(e, x[None], lam[None], us, vb, src)
        ref_R.append(R[0]), ref_T.append(T[0])
    err_R = rloc_err(disc, inp, out["R_loc"].cpu().numpy(), np.stack(ref_R))
    err_T = rel_err_per_elem(out["R_tr"].cpu().numpy(), np.stack(ref_T))
    err_A = rel_err_per_elem(out["A"].cpu().numpy(), colmajor([b["A"] for b in blocks]))
    print(name, "source: R_loc", err_R, "R_tr", err_T, "A", err_A, flush=True)
    assert err_R <= TOL and err_T <= TOL and err_A <= TOL


@pytest.mark.parametrize("name", ["ns2d_tri_p2", "ns3d_hex_p1"])
def test_source_at_quadrature_points_matches_oracle(torch, name):
    """hdg_plan_set_source_points: a non-polynomial source given by its values at the GPU's volume
    quadrature points; R_loc against the oracle's element residual with the same function
    evaluated at its own quadrature points."""
    wl, disc, inp, blocks = _case(name)
    rng = np.random.default_rng(43)
    coef = rng.standard_normal((disc.m, disc.d))

    def src(x):   # x (Nq, d) -> (Nq, m)
        return np.sin(x @ coef.T + np.arange(disc.m)[None, :])

    plan = gpu_plan(wl)
    d = to_dev(inp)
    xq = plan.quad_coords().cpu().numpy()
    plan.set_source_points(torch.from_numpy(np.ascontiguousarray(src(xq.T).T)).cuda())
    out = plan.assemble(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    torch.cuda.synchronize()
    ref_R = []
    for e in range(disc.mesh.n_elem):
        x, lam, us, vb = disc.elem_inputs(e, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"])
        R, _ = disc.element_residual(e, x[None], lam[None], us, vb, src)
        ref_R.append(R[0])
    err_R = rloc_err(disc, inp, out["R_loc"].cpu().numpy(), np.stack(ref_R))
    print(name, "source at points: R_loc", err_R, flush=True)
    assert err_R <= TOL


@pytest.mark.parametrize("name", ["ns2d_tri_p2", "ns3d_hex_p1"])
def test_interior_viscous_flux_matches_oracle(torch, name):
    """HDG_FLAG_GHAT_INTERIOR: viscous numerical flux G(v_h, q_h).n (the first of the two choices
    of Section 3.3).  All blocks, the residuals and the condensed outputs against the oracle with
    the same choice; the blocks must differ from the default flux's."""
    wl = SMALL_CASES[name]()
    disc = oracle_disc(wl, ghat_interior=True)
    inp = ostate.oracle_inputs(wl, disc)
    blocks = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"],
                                    keep_blocks=True)
    plan = gpu_plan(wl, ghat_interior=True)
    d = to_dev(inp)
    out = plan.assemble(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    cond = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"], residuals=True)
    torch.cuda.synchronize()
    errs = {
        "R_loc": rloc_err(disc, inp, out["R_loc"].cpu().numpy(), np.stack([b["R_loc"] for b in blocks])),
        "R_tr": rel_err_per_elem(out["R_tr"].cpu().numpy(), np.stack([b["R_tr"] for b in blocks])),
        "S": rel_err_per_elem(cond["S"].cpu().numpy(), colmajor([b["S"] for b in blocks])),
        "Y": rel_err_per_elem(cond["Y"].cpu().numpy(), colmajor([b["Y"] for b in blocks])),
    }
    for key in ("A", "B", "C", "D"):
        errs[key] = rel_err_per_elem(out[key].cpu().numpy(), colmajor([b[key] for b in blocks]))
    print(name, errs, flush=True)
    for key, err in errs.items():
        assert err <= TOL, (key, err)
    _, _, _, base = _case(name)
    assert rel_err_per_elem(np.stack([b["C"] for b in blocks]), np.stack([b["C"] for b in base])) > 1e-6


@pytest.mark.parametrize("eliminate_q", [False, True])
@pytest.mark.parametrize("name", ["ns2d_tri_p2", "ns3d_hex_p1"])
def test_projection_viscous_flux_matches_oracle(torch, name, eliminate_q):
    """HDG_FLAG_GHAT_PROJ: projection viscous flux (Pi G(v_h, q_h)).n of Section 4 (added from the
    volume points after the contraction).  Blocks, residuals and condensed outputs against the
    oracle with the same flux, also through the q-eliminating condensation; the blocks must
    differ from the default flux's."""
    wl = SMALL_CASES[name]()
    disc = oracle_disc(wl, ghat_proj=True)
    inp = ostate.oracle_inputs(wl, disc)
    blocks = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"],
                                    keep_blocks=True)
    plan = gpu_plan(wl, ghat_proj=True, eliminate_q=eliminate_q)
    d = to_dev(inp)
    out = plan.assemble(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    errs = {}
    for rep in range(2):   # the second call runs on the workspace the first one left
        cond = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"], residuals=True)
        torch.cuda.synchronize()
        errs["S%d" % rep] = rel_err_per_elem(cond["S"].cpu().numpy(), colmajor([b["S"] for b in blocks]))
        errs["Y%d" % rep] = rel_err_per_elem(cond["Y"].cpu().numpy(), colmajor([b["Y"] for b in blocks]))
        errs["g%d" % rep] = rel_err_per_elem(cond["g"].cpu().numpy(), np.stack([b["g"] for b in blocks]))
    errs["R_loc"] = rloc_err(disc, inp, out["R_loc"].cpu().numpy(), np.stack([b["R_loc"] for b in blocks]))
    errs["R_tr"] = rel_err_per_elem(out["R_tr"].cpu().numpy(), np.stack([b["R_tr"] for b in blocks]))
    for key in ("A", "B", "C", "D"):
        errs[key] = rel_err_per_elem(out[key].cpu().numpy(), colmajor([b[key] for b in blocks]))
    print(name, eliminate_q, errs, flush=True)
    for key, err in errs.items():
        assert err <= TOL, (key, err)
    _, _, _, base = _case(name)
    # (4.6e-7 on the nearly uniform hexahedron state, whose G is close to its projection)
    assert rel_err_per_elem(np.stack([b["A"] for b in blocks]), np.stack([b["A"] for b in base])) > 1e-8


@pytest.mark.parametrize("sigma", ["s", "mv"])
@pytest.mark.parametrize("name", ["euler2d_tri_p2", "ns3d_hex_p1", "euler3d_hex_p2"])
def test_symmetric_variable_stabilization_matches_oracle(torch, name, sigma):
    """HDG_FLAG_SIGMA_S / HDG_FLAG_SIGMA_MV: stabilization sigma_S = |A_n(v_hat)| A0(v_hat) or the
    mean-value matrix between v_hat and v (Section 4).  Blocks, residuals and condensed outputs
    against the oracle with the same matrix; the blocks must differ from the sigma_SLF ones."""
    wl = SMALL_CASES[name]()
    disc = oracle_disc(wl, sigma=sigma)
    inp = ostate.oracle_inputs(wl, disc)
    blocks = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"],
                                    keep_blocks=True)
    plan = gpu_plan(wl, sigma=sigma)
    d = to_dev(inp)
    out = plan.assemble(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    cond = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"], residuals=True)
    torch.cuda.synchronize()
    errs = {
        "R_loc": rloc_err(disc, inp, out["R_loc"].cpu().numpy(), np.stack([b["R_loc"] for b in blocks])),
        "R_tr": rel_err_per_elem(out["R_tr"].cpu().numpy(), np.stack([b["R_tr"] for b in blocks])),
    }
    for key in ("A", "B", "C", "D"):
        errs[key] = rel_err_per_elem(out[key].cpu().numpy(), colmajor([b[key] for b in blocks]))
    print(name, errs, flush=True)
    for key, err in errs.items():
        assert err <= TOL, (key, err)
    # S and Y come from solves with the local block, whose condition number sigma_S can raise
    # (its entropy and shear parts vanish where u.n does): per element, forward error within
    # 1e-12 or within 64 eps cond(A) (a backward-stable solve's bound), whichever is larger
    Sg, Yg = cond["S"].cpu().numpy(), cond["Y"].cpu().numpy()
    worst = 0.0
    for e, b in enumerate(blocks):
        bound = max(TOL, 64 * np.finfo(float).eps * np.linalg.cond(b["A"]))
        for got, ref in ((Sg[e].T, b["S"]), (Yg[e].T, b["Y"])):
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            worst = max(worst, err / bound)
            assert err <= bound, (e, err, bound)
    print(name, "S, Y: worst error / bound", worst, flush=True)
    _, _, _, base = _case(name)
    assert rel_err_per_elem(np.stack([b["A"] for b in blocks]), np.stack([b["A"] for b in base])) > 1e-6


@pytest.mark.parametrize("name", ["ns2d_tri_p2", "euler3d_hex_p2"])
def test_mean_value_stabilization_across_sign_changes(torch, name):
    """sigma_MV where the wave speeds change sign between v_hat and v: the trace states carry the
    reversed velocity, so u_n (and, where |u_n| is near c, u_n -/+ c) changes sign on the path at
    most face points and the integrand has kinks there.  The GPU's split path integral against
    the oracle's (both exact to rounding): blocks and residuals to 1e-12."""
    from oracle import physics as oph
    wl = SMALL_CASES[name]()
    disc = oracle_disc(wl, sigma="mv")
    inp = ostate.oracle_inputs(wl, disc)
    rho, V, p = oph.prim_of_v(inp["vhat"].T, wl.gamma)
    inp["vhat"] = np.ascontiguousarray(oph.v_of_prim(rho, -V, p, wl.gamma).T)
    # the case exercises the kinks: count face points whose path has an inner breakpoint
    kinks = 0
    for e in range(disc.mesh.n_elem):
        x, lam, _, _ = disc.elem_inputs(e, inp["v"], inp["q"], inp["vhat"])
        G = disc.geom(e)
        LN = lam.reshape(disc.nf, disc.m, disc.Nfp)
        vN = x[:disc.m * disc.Np].reshape(disc.m, disc.Np)
        for f in range(disc.nf):
            F = G.faces[f]
            br = oph.mv_breakpoints(F["psi"] @ LN[f].T, F["phi"] @ vN.T, F["n"], wl.gamma)
            kinks += int(np.sum((br > 0) & (br < 1)))
    assert kinks > disc.mesh.n_elem * disc.nf, kinks
    blocks = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"],
                                    keep_blocks=True)
    plan = gpu_plan(wl, sigma="mv")
    d = to_dev(inp)
    out = plan.assemble(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    torch.cuda.synchronize()
    errs = {
        "R_loc": rloc_err(disc, inp, out["R_loc"].cpu().numpy(), np.stack([b["R_loc"] for b in blocks])),
        "R_tr": rel_err_per_elem(out["R_tr"].cpu().numpy(), np.stack([b["R_tr"] for b in blocks])),
    }
    for key in ("A", "B", "C", "D"):
        errs[key] = rel_err_per_elem(out[key].cpu().numpy(), colmajor([b[key] for b in blocks]))
    print(name, "kinks", kinks, errs, flush=True)
    for key, err in errs.items():
        assert err <= TOL, (key, err)


def _block_tensors(torch, blocks):
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return {"A": dev(colmajor([b["A"] for b in blocks])), "B": dev(colmajor([b["B"] for b in blocks])),
            "C": dev(colmajor([b["C"] for b in blocks])), "D": dev(colmajor([b["D"] for b in blocks])),
            "R_loc": dev(np.stack([b["R_loc"] for b in blocks])), "R_tr": dev(np.stack([b["R_tr"] for b in blocks]))}


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("name", ["euler2d_tri_p2", "ns2d_tri_p2", "ns3d_hex_p2"])
def test_condense_blocks_matches_oracle(torch, name, split):
    """hdg_condense_blocks on the oracle's own blocks: the condensation alone (S, Y, g, z) against
    the oracle's LAPACK condensation of the same blocks, for the left-looking and right-looking
    kernels."""
    wl, disc, inp, blocks = _case(name)
    plan = gpu_plan(wl, split_dense=split)
    out = plan.condense_blocks(_block_tensors(torch, blocks))
    torch.cuda.synchronize()
    assert int(out["status"].abs().max()) == 0
    for key, mat in (("S", True), ("Y", True), ("g", False), ("z", False)):
        ref = colmajor([b[key] for b in blocks]) if mat else np.stack([b[key] for b in blocks])
        err = rel_err_per_elem(out[key].cpu().numpy(), ref)
        assert err <= (1e-11 if key == "z" else TOL), (key, err)


@pytest.mark.parametrize("split", [False, True])
def test_singular_local_block_is_flagged(torch, split):
    """A local block with a zero column (built on the host from the oracle's blocks) has a zero
    pivot: HDG_ESINGULAR on that element only, every other element condensed as before."""
    wl, disc, inp, blocks = _case("ns2d_tri_p2")
    bad = 3
    blocks = [dict(b) for b in blocks]
    A = blocks[bad]["A"].copy()
    A[:, 7] = 0.0
    blocks[bad]["A"] = A
    plan = gpu_plan(wl, split_dense=split)
    out = plan.condense_blocks(_block_tensors(torch, blocks))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert st[bad] == -4 and np.count_nonzero(st) == 1, st
    assert plan.status(out["status"]) == (bad, -4)
    good = [e for e in range(len(blocks)) if e != bad]
    ref = colmajor([blocks[e]["S"] for e in good])
    assert rel_err_per_elem(out["S"].cpu().numpy()[good], ref) <= TOL


def test_non_finite_q_and_vhat_are_flagged(torch):
    """A NaN in the gradient unknowns of one element flags that element HDG_ENONPHYS; a NaN at one
    trace node flags exactly the elements whose faces hold that node."""
    wl, disc, inp, _ = _case("ns2d_tri_p2")
    plan = gpu_plan(wl)
    d = to_dev(inp)
    bad = 9
    d["q"][2, bad * disc.Np + 1] = float("nan")
    out = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    st = out["status"].cpu().numpy()
    assert st[bad] == -3 and np.count_nonzero(st) == 1, st
    d = to_dev(inp)
    node = int(wl.tmap[4, 1, 0])
    d["vhat"][0, node] = float("nan")
    out = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    st = out["status"].cpu().numpy()
    holders = sorted({e for e in range(wl.mesh.n_elem) if np.any(wl.tmap[e] == node)})
    assert sorted(np.nonzero(st)[0].tolist()) == holders and np.all(st[holders] == -3), (st, holders)
