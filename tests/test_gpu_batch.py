"""Mixed batches: tetrahedra of orders 1..4 next to p = 2 hexahedra.

* every group (one element type and order) condensed on the GPU matches the
  oracle on sampled elements (S, Y, g relative <= 1e-12; z backward error
  <= 1e-12 in the summation scale of R_loc);
* the batched launches (one workgroup per item, largest blocks first and
  plan order; a persistent grid) produce the same outputs as the per-plan
  launches, bit for bit (same arithmetic in the same order), and so does the
  stream mode (every plan's own condensation on concurrent streams);
* a captured hipGraph of the whole batch, replayed several times with eager
  work and synchronizations in between, reproduces the eager outputs every
  time;
* the tuning knobs (contraction workgroup size, condensation block width,
  one or two condensation launches) change nothing but the launch shape.
"""
import numpy as np
import pytest

from oracle import hdg as ohdg
from workloads import configs as C

from cases import colmajor, gpu_plan, oracle_case, rel_err_per_elem, to_dev, z_backward_err

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def groups(torch):
    out = []
    for wl in C.mixed_batch(n_tet=3, n_hex=2):
        disc, inp = oracle_case(wl)
        plan = gpu_plan(wl)
        d = to_dev(inp)
        out.append(dict(wl=wl, disc=disc, inp=inp, plan=plan, d=d))
    return out


def _outputs(g, torch):
    res = g["plan"].alloc_outputs()
    return res


@pytest.mark.parametrize("gi", range(5))
def test_group_matches_oracle(torch, groups, gi):
    g = groups[gi]
    wl, disc, inp, plan, d = g["wl"], g["disc"], g["inp"], g["plan"], g["d"]
    print("group", wl.name, "elements", wl.mesh.n_elem, "n", plan.n, "k", plan.k, flush=True)
    out = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    torch.cuda.synchronize()
    assert int(out["status"].abs().max()) == 0
    E = wl.mesh.n_elem
    sample = sorted({0, E // 2, E - 1})
    ref = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"], elems=sample,
                                 keep_blocks=True)
    errs = {
        "S": rel_err_per_elem(out["S"].cpu().numpy()[sample], colmajor([r["S"] for r in ref])),
        "Y": rel_err_per_elem(out["Y"].cpu().numpy()[sample], colmajor([r["Y"] for r in ref])),
        "g": rel_err_per_elem(out["g"].cpu().numpy()[sample], np.stack([r["g"] for r in ref])),
        "z_backward": max(z_backward_err(disc, inp, e, r["A"], r["R_loc"], out["z"][e].cpu().numpy())
                          for e, r in zip(sample, ref)),
    }
    print(wl.name, errs)
    for key, err in errs.items():
        assert err <= TOL, (key, err)


def _io(groups, torch):
    io = []
    for g in groups:
        o = g["plan"].alloc_outputs()
        io.append(dict(v=g["d"]["v"], q=g["d"]["q"], vhat=g["d"]["vhat"], ustar=g["d"]["ustar"], vbc=g["d"]["vbc"],
                       **o))
    return io


@pytest.mark.parametrize("order,grid", [("lpt", 0), ("plan", 0), ("lpt", 256)])
def test_batch_equals_per_plan(torch, groups, order, grid):
    """Bit for bit against per-plan launches of the same arithmetic (the LU with its working
    block in LDS, which the batch runs), with one workgroup per item (grid 0) and with a
    persistent grid; the per-plan default (the register-resident LU for the small tetrahedra)
    agrees to rounding."""
    from paper_1808_05066_amd.hdg import Batch
    saved = [g["plan"].tuning()["lu_waves"] for g in groups]
    dflt = [g["plan"].assemble_condense(g["d"]["v"], g["d"]["q"], g["d"]["vhat"], g["d"]["ustar"], g["d"]["vbc"])
            for g in groups]
    for g in groups:
        g["plan"].set_tuning(lu_waves=1)
    ref = [g["plan"].assemble_condense(g["d"]["v"], g["d"]["q"], g["d"]["vhat"], g["d"]["ustar"], g["d"]["vbc"])
           for g in groups]
    for g, lw in zip(groups, saved):
        g["plan"].set_tuning(lu_waves=lw)
    b = Batch([g["plan"] for g in groups], order=order)
    b.set_groups(grid)
    print(b.info())
    io = _io(groups, torch)
    b.set_io(io)
    b.run()
    torch.cuda.synchronize()
    for r, dl, o in zip(ref, dflt, io):
        assert int(o["status"].abs().max()) == 0
        for key in ("S", "Y", "g", "z"):
            assert torch.equal(r[key], o[key]), key
        for key in ("S", "Y", "g"):
            err = float(torch.linalg.norm(dl[key] - o[key]) / torch.linalg.norm(o[key]))
            assert err <= 1e-13, (key, err)


@pytest.mark.parametrize("nstreams", [1, 4])
def test_stream_batch_equals_per_plan(torch, groups, nstreams):
    """Stream mode runs every plan's own condensation (its own tuning) concurrently: bit for bit
    the plans' own outputs."""
    from paper_1808_05066_amd.hdg import Batch
    ref = [g["plan"].assemble_condense(g["d"]["v"], g["d"]["q"], g["d"]["vhat"], g["d"]["ustar"], g["d"]["vbc"])
           for g in groups]
    b = Batch([g["plan"] for g in groups])
    b.set_streams(nstreams)
    io = _io(groups, torch)
    b.set_io(io)
    b.run()
    torch.cuda.synchronize()
    for r, o in zip(ref, io):
        assert int(o["status"].abs().max()) == 0
        for key in ("S", "Y", "g", "z"):
            assert torch.equal(r[key], o[key]), key


@pytest.mark.parametrize("nstreams", [0, 4])
def test_graph_replay_reproduces_eager(torch, groups, nstreams):
    from paper_1808_05066_amd.hdg import Batch
    b = Batch([g["plan"] for g in groups])
    b.set_streams(nstreams)
    io = _io(groups, torch)
    b.set_io(io)
    b.run()
    torch.cuda.synchronize()
    eager = [{k: o[k].clone() for k in ("S", "Y", "g", "z")} for o in io]
    b.capture()
    for rep in range(3):
        for o in io:
            for k in ("S", "Y", "g", "z"):
                o[k].fill_(float("nan"))
        junk = torch.randn(1000, device="cuda").sum()      # eager work between replays
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        for e, o in zip(eager, io):
            for k in ("S", "Y", "g", "z"):
                assert torch.equal(e[k], o[k]), (rep, k)
        del junk


def test_tuning_changes_only_the_launch_shape(torch, groups):
    g = groups[4]   # p = 2 hexes: every knob applies
    plan, d = g["plan"], g["d"]
    args = (d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    base = plan.assemble_condense(*args)
    torch.cuda.synchronize()
    t0 = plan.tuning()
    for ct, cw, nl in ((256, 32, 2), (512, 16, 2), (1024, 32, 1), (1024, 32, 2)):
        plan.set_tuning(contract_threads=ct, condense_width=cw, condense_launches=nl)
        out = plan.assemble_condense(*args)
        torch.cuda.synchronize()
        for key in ("S", "Y", "g"):
            err = float(torch.linalg.norm(out[key] - base[key]) / torch.linalg.norm(base[key]))
            assert err <= 1e-13, (ct, cw, nl, key, err)
    # the split and the fused condensation do the same arithmetic in the same order
    lp = {}
    for nl in (1, 2):
        plan.set_tuning(condense_launches=nl)
        f64 = plan.assemble_condense(*args)
        lp[nl] = plan.assemble_condense_lp(*args)
        torch.cuda.synchronize()
        lp[nl]["f64"] = f64
    for key in ("S", "Y", "g", "z"):
        assert torch.equal(lp[1][key], lp[2][key]), ("fp32", key)
        assert torch.equal(lp[1]["f64"][key], lp[2]["f64"][key]), ("fp64", key)
    plan.set_tuning(**t0)


def test_batch_mode_arguments_are_checked(torch, groups):
    """hdg_batch_set_streams takes 0..8 and hdg_batch_set_groups a non-negative grid: anything else is
    HDG_EINVAL, and the batch still runs afterwards."""
    from paper_1808_05066_amd.hdg import Batch
    b = Batch([g["plan"] for g in groups])
    for bad in (-1, 9):
        with pytest.raises(RuntimeError):
            b.set_streams(bad)
    with pytest.raises(RuntimeError):
        b.set_groups(-1)
    b.set_streams(2)
    b.set_streams(0)
    b.set_groups(0)
    io = _io(groups, torch)
    b.set_io(io)
    b.run()
    torch.cuda.synchronize()
    assert all(int(o["status"].abs().max()) == 0 for o in io)
