#!/usr/bin/env python
"""Throughput of the entropy-variable hybridized DG hot path on one MI355X.

A step is one pass of the hot path over the whole mesh:
  hdg_assemble_condense  (pointwise physics + Jacobians, block assembly,
                          LU, triangular solves, Schur complement)
  hdg_trace_rhs          (condensed right-hand side)
  hdg_trace_matvec       (one application of the condensed trace operator)
  hdg_backsolve          (local back-solve with the right-hand side as the
                          trace update; the global solve is not part of a step)
Inputs are resident in HBM before the timed region.  The value is elements per
second of whole steps.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from workloads import configs as C  # noqa: E402

METRIC = "elem/s local Jacobian+static condensation; FP64 vs mixed-prec at 1e-10 resid"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    "ns3d_hex_p2_16": ("3D Navier-Stokes, 16^3 periodic trilinear hexes on [0,2pi]^3 (jitter 5%), p=2, "
                       "Re=1600, Pr=0.72, Mach 0.1 Taylor-Green + 2% noise, DIRK(3,3) stage mass term",
                       lambda: C.ns3d_hex(n=16, p=2)),
    "euler2d_tri_p2_8": ("2D Euler, unit square 8x8 split into 128 triangles (jitter 10%), p=2, Shu vortex "
                         "+ 1% noise, Dirichlet-trace boundary", lambda: C.euler2d_tri_p2()),
}


def flops_per_elem(n, k, Np, Nq, m, d, viscous):
    """Algorithmic flops of each phase for one element (dense formulas)."""
    slots = m * m + m * d * m + (m * d * m * d + d * d + 1 if viscous else 0)
    return {
        "contract": 2.0 * Nq * Np * Np * slots,
        "lu": 2.0 * n ** 3 / 3.0,
        "solve": 2.0 * n * n * (k + 1),
        "schur": 2.0 * k * n * (k + 1),
    }


def prepare_inputs(plan, wl, torch):
    from paper_1808_05066_amd.inputs import device_inputs
    return device_inputs(plan, wl)


_ORACLE = {}


def _oracle_setup(wl):
    from oracle import hdg as ohdg
    from oracle import state as ostate
    disc = ohdg.Discretization(wl.mesh, wl.p, ohdg.Phys(wl.gamma, wl.mu, wl.Pr, wl.alpha, wl.viscous),
                               wl.tmap, wl.n_trace, wl.face_bc)
    _ORACLE.update(disc=disc, inp=ostate.oracle_inputs_fast(wl, disc))


def _oracle_element(e):
    """One element through the oracle (worker side; one BLAS thread)."""
    from threadpoolctl import threadpool_limits

    from oracle import hdg as ohdg
    disc, inp = _ORACLE["disc"], _ORACLE["inp"]
    with threadpool_limits(limits=1):
        ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"], elems=[int(e)])
    return int(e)


def _host_cores():
    """Host cores this process may use (its affinity set), at most the 16 a one-GPU share holds."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, seconds_budget=20.0):
    """Time the FP64 oracle on bounded element samples of the same workload: on one core (one BLAS
    thread), then on all host cores with one worker process per core (elements are independent)."""
    import multiprocessing as mp
    _oracle_setup(wl)
    rng = np.random.default_rng(0)
    order = rng.permutation(wl.mesh.n_elem)
    # one core
    done, t_used = 0, 0.0
    while t_used < 0.4 * seconds_budget and done < wl.mesh.n_elem:
        t0 = time.perf_counter()
        _oracle_element(order[done])
        t_used += time.perf_counter() - t0
        done += 1
    one = done / t_used
    # all cores: enough elements for about 0.6 of the budget at the one-core rate times the cores
    cores = _host_cores()
    count = int(min(wl.mesh.n_elem, max(cores, round(0.6 * seconds_budget * one * cores))))
    sample = order[:count]
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_element, sample[:cores])          # workers warm
        t0 = time.perf_counter()
        pool.map(_oracle_element, sample, chunksize=1)
        wall = time.perf_counter() - t0
    return {"value": count / wall, "unit": "elem/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "one_core": {"value": one, "unit": "elem/s", "cores": 1,
                         "sample": "%d elements, %.1f s" % (done, t_used)},
            "sample": "%d seeded-random elements of the same mesh on %d worker processes (one BLAS thread "
                      "each), residual + complex-step Jacobian + LAPACK condensation, %.1f s wall"
                      % (count, cores, wall)}


def _timed(fn, reps, torch):
    """Median milliseconds of fn() over reps runs, HIP events on the current stream."""
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def bench_mixed(plan, inp, out64, E, fp64_cond_ms, torch):
    """Low-precision condensation + FP64 refinement of the full Newton system to 1e-10, with FP32
    operands on the matrix cores (the main figures) and with BF16 operands (`bf16`).

    Mixed elem/s = E / (t_factor_lp + n_ref * t_refine_local): t_factor_lp the
    low-precision assemble + condense, t_refine_local the per-step local work
    of the refinement (low-precision local solves, matrix-free FP64 Jacobian actions,
    back-solve, norms; host wall time of the loop minus its GMRES time), n_ref
    the refinement steps to reach the tolerance.  GMRES time is reported apart.
    """
    lp = plan.alloc_outputs_lp()
    args = (inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"])

    def rel(a, b):
        a = a.double()
        return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))

    def run(ops, max_outer):
        plan.set_tuning(lp_operands=ops)
        plan.assemble_condense_lp(*args, out=lp)
        torch.cuda.synchronize()
        if int((lp["status"] != 0).sum()):
            return {"error": "non-OK element status in the low-precision path"}
        t_lp = _timed(lambda: plan.assemble_condense_lp(*args, out=lp), 5, torch)
        plan.assemble_condense(*args, out=out64)
        plan.assemble_condense_lp(*args, out=lp)
        torch.cuda.synchronize()
        dx, dlam, info = plan.refine_solve(*args[:3], lp, ustar=inp["ustar"], vbc=inp["vbc"], tol=1e-10,
                                           max_outer=max_outer, reuse_points=True, gmres_restart=50,
                                           gmres_tol=1e-8)
        n_ref = max(1, info["outer_iterations"])
        t_local = (info["total_ms"] - info["gmres_ms"]) / n_ref
        value = E / ((t_lp + n_ref * t_local) / 1e3)
        errs = {"S": rel(lp["S"], out64["S"]), "Y": rel(lp["Y"], out64["Y"]), "g": rel(lp["g"], out64["g"]),
                "z": rel(lp["z"], out64["z"])}
        return {"value": value, "unit": "elem/s",
                "dtype": "%s operands (FP32 condensation) + f64 refinement" % ("bf16" if ops == 2 else "f32"),
                "speedup_vs_fp64": value / (E / (fp64_cond_ms / 1e3)),
                "t_factor_lp_ms": t_lp, "refine_steps": info["outer_iterations"], "t_refine_local_ms": t_local,
                "refine_rel_residual": info["rel_residual"],
                "refine_history": info["history"][:max(1, info["outer_iterations"])],
                "gmres_iterations": info["gmres_iterations"], "gmres_ms": info["gmres_ms"],
                "converged": info["converged"], "rel_err_vs_fp64_gpu": errs}

    res = run(1, 10)
    res["bf16"] = run(2, 16)
    plan.set_tuning(lp_operands=1)
    return res


def bench_eliminate_q(wl, inp, out_ref, full_ms, steps, torch):
    """The same step on a plan that eliminates the gradient unknowns element by element before
    the dense condensation (identical S, g, Y, z up to rounding), timed the same way."""
    from paper_1808_05066_amd.hdg import Plan
    plan = Plan(wl.mesh.etype, wl.p, wl.mesh.elem_xyz, wl.tmap, wl.n_trace, wl.face_bc, viscous=wl.viscous,
                gamma=wl.gamma, mu=wl.mu, Pr=wl.Pr, alpha=wl.alpha, eliminate_q=True)
    out = plan.alloc_outputs()
    r = torch.empty(plan.m, plan.n_trace, dtype=torch.float64, device="cuda")
    y = torch.empty_like(r)
    dv = torch.empty(plan.m, plan.n_nodes, dtype=torch.float64, device="cuda")
    dq = torch.empty(plan.m * plan.dim, plan.n_nodes, dtype=torch.float64, device="cuda")

    def step():
        plan.assemble_condense(inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"], out=out)
        plan.trace_rhs(out["g"], r)
        plan.trace_matvec(out["S"], r, y)
        plan.backsolve(out["Y"], out["z"], r, dv, dq)

    step()
    torch.cuda.synchronize()
    if int((out["status"] != 0).sum()):
        raise RuntimeError("q-eliminating condensation reported a non-OK element status")
    ms = _timed(step, steps, torch)
    plan.set_timing(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    avg = {name: (t / c if c else 0.0) for name, (t, c) in plan.phase_times().items()}
    plan.set_timing(False)

    def rel(a, b):
        return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))

    E = plan.n_elem
    res = {"value": E / (ms / 1e3), "unit": "elem/s", "ms_per_step": ms, "vs_full_block": full_ms / ms,
           "reduced_n": plan.m * plan.Np, "phase_ms": {p: round(v, 4) for p, v in avg.items()},
           "rel_diff_vs_full_block": {key: rel(out[key], out_ref[key]) for key in ("S", "g", "Y", "z")}}
    del plan, out
    torch.cuda.empty_cache()
    return res


def bench_newton(plan, inp, torch, maxit=8, tol=1e-10):
    """Newton iterations of one implicit stage (hdg_newton_solve) from the benchmark's
    perturbed state: assemble + condense, GMRES(50) with block Jacobi on the condensed
    system, back-solve and update per iteration."""
    v, vh = inp["v"].clone(), inp["vhat"].clone()
    q = None if inp["q"] is None else inp["q"].clone()
    info = plan.newton_solve(v, q, vh, inp["ustar"], inp["vbc"], maxit=maxit, tol=tol, lin_tol=1e-10)
    its = max(info["iterations"], 1)
    return {"iterations": info["iterations"], "converged": info["converged"], "residuals": info["res"],
            "gmres_iterations": info["lin_iterations"], "ms": info["ms"], "ms_per_iteration": info["ms"] / its,
            "tol_rel": tol}


def bench_dirk(plan, inp, dt, torch):
    """One DIRK(3,3) step (hdg_dirk_step, three Newton-solved stages) from the benchmark's state."""
    v, vh = inp["v"].clone(), inp["vhat"].clone()
    q = None if inp["q"] is None else inp["q"].clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stages = plan.dirk_step(v, q, vh, dt, vbc=inp["vbc"], tol=1e-10, lin_tol=1e-10)
    ms = (time.perf_counter() - t0) * 1e3
    return {"dt": dt, "ms": ms, "newton_iterations": [st["iterations"] for st in stages],
            "gmres_iterations": [st["lin_iterations"] for st in stages],
            "converged": all(st["converged"] for st in stages),
            "final_residuals": [st["res"][-1] for st in stages]}


def bench_batch(torch, tune=True):
    """Mixed batch: 20,250 Kuhn tetrahedra with orders drawn from {1,2,3,4} plus 4,096 p = 2 hexes (NS).

    Times the per-plan launches one after another, the batched launches with one workgroup
    per item (largest blocks first, and plan order), with a persistent grid of one workgroup
    per CU, the hipGraph replay of the first, and the stream mode (every plan's own
    condensation on 2 or 4 concurrent streams; graph replay with 4).
    """
    from paper_1808_05066_amd import autotune
    from paper_1808_05066_amd.hdg import Batch
    from paper_1808_05066_amd.inputs import device_inputs, plan_for
    groups = C.mixed_batch()
    plans, io, flops = [], [], 0.0
    for wl in groups:
        pl = plan_for(wl)
        inp = device_inputs(pl, wl)
        if tune:
            autotune.apply(pl)
        o = pl.alloc_outputs()
        plans.append(pl)
        io.append(dict(v=inp["v"], q=inp["q"], vhat=inp["vhat"], ustar=inp["ustar"], vbc=inp["vbc"], **o))
        fl = flops_per_elem(pl.n, pl.k, pl.Np, pl.Nq, pl.m, pl.dim, True)
        flops += (fl["lu"] + fl["solve"] + fl["schur"]) * pl.n_elem
    E = sum(pl.n_elem for pl in plans)

    def sequential():
        for pl, d in zip(plans, io):
            pl.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"], out=d)

    res = {"elements": E, "groups": [{"name": wl.name, "elements": pl.n_elem, "n": pl.n, "k": pl.k,
                                      "tuning": pl.tuning()} for wl, pl in zip(groups, plans)],
           "dense_flop": flops}
    res["sequential_ms"] = _timed(sequential, 3, torch)
    for order in ("lpt", "plan"):
        b = Batch(plans, order=order)
        b.set_io(io)
        res["batch_%s_ms" % order] = _timed(b.run, 3, torch)
        if order == "lpt":
            b.capture()
            res["graph_replay_ms"] = _timed(b.replay, 3, torch)
            bad = sum(int((d["status"] != 0).sum()) for d in io)
            res["bad_elements"] = bad
        del b
    b = Batch(plans, order="lpt")
    b.set_groups(torch.cuda.get_device_properties(0).multi_processor_count)
    b.set_io(io)
    res["batch_persistent_ms"] = _timed(b.run, 3, torch)
    del b
    for ns in (2, 4):
        b = Batch(plans, order="lpt")
        b.set_streams(ns)
        b.set_io(io)
        res["batch_streams%d_ms" % ns] = _timed(b.run, 3, torch)
        if ns == 4:
            b.capture()
            res["graph_replay_streams4_ms"] = _timed(b.replay, 3, torch)
            res["bad_elements_streams4"] = sum(int((d["status"] != 0).sum()) for d in io)
        del b
    best = min(res["batch_lpt_ms"], res["graph_replay_ms"], res["batch_streams4_ms"],
               res["graph_replay_streams4_ms"])
    res["value"] = E / (best / 1e3)
    res["unit"] = "elem/s"
    res["dense_tflops"] = flops / (best / 1e3) / 1e12
    return res


def c4_slabs(nslab=8):
    """The 32^3 mesh of p = 3 hexahedra (32,768 elements, n = 1280, k = 480; Taylor-Green at Re 1600,
    Mach 0.1, 5% noise, jitter 5%) cut into nslab slabs of whole cell layers along z: per-element
    work (assembly, Jacobian, condensation) does not depend on the neighbours, so the slabs
    together are the whole mesh's step; faces between slabs are trace faces of one element."""
    import dataclasses

    from workloads import meshes as M
    full = C.ns3d_hex(n=32, p=3, eps=0.05, jitter=0.05, config_id=4)
    zc = full.mesh.elem_lat[:, :, 2].min(axis=1)
    per = 32 // nslab
    out = []
    for sl in range(nslab):
        idx = np.nonzero((zc >= sl * per) & (zc < (sl + 1) * per))[0]
        sub = M.subset_mesh(full.mesh, idx)
        out.append(dataclasses.replace(full, name="%s_slab%d" % (full.name, sl), mesh=sub,
                                       face_bc=np.zeros((len(idx), 6), dtype=np.int32), tmap=None, n_trace=0))
    return out


def bench_c4(torch, nslab=8, process=None, chunk=2048, tol=1e-10):
    """FP64 against mixed precision on the 32^3 p = 3 mesh (all 32,768 elements, slab by slab).

    FP64: hdg_assemble_condense (the right-looking kernels: the 1280-row block does not fit the
    left-looking kernels' LDS).  Mixed: hdg_assemble_condense_lp (FP32 condensation on the matrix
    cores after power-of-two scaling), then the element-level FP64 refinement hdg_refine_local of
    A dx = -(R_loc + B P dvhat) for a seeded trace update dvhat to a per-element relative residual
    <= tol.  Mixed elem/s = E / (t_factor_lp + t_refine_local).  Errors: FP32 outputs against the
    FP64 GPU outputs (S, Y, g, z) and the refined dx against the FP64 back-solve -z - Y P dvhat.
    `bf16`: the same with BF16 operands on the matrix cores (FP32 data and accumulation), up to 16
    refinement steps (elements that stagnate fall back to FP64 and are counted)."""
    from paper_1808_05066_amd.inputs import device_inputs, plan_for
    tot = {"fp64_ms": 0.0, "lp_ms": 0.0, "refine_ms": 0.0, "bf_ms": 0.0, "bf_refine_ms": 0.0}
    E = 0
    worst = {"S": 0.0, "Y": 0.0, "g": 0.0, "z": 0.0, "dx": 0.0}
    worst_bf = dict(worst)
    refine = {"steps_max": 0, "rel_residual_max": 0.0, "converged": True}
    refine_bf = {"steps_max": 0, "rel_residual_max": 0.0, "converged": True, "fallback_elements": 0}
    rng = np.random.default_rng([4, 9])

    def rel(a, b):
        return float(torch.linalg.norm(a.double() - b) / torch.linalg.norm(b))

    slabs = c4_slabs(nslab)[:process]
    for i, wl in enumerate(slabs):
        print("[bench] c4 slab %d/%d: %d elements" % (i + 1, len(slabs), wl.mesh.n_elem), file=sys.stderr, flush=True)
        plan = plan_for(wl, chunk_elems=chunk)
        inp = device_inputs(plan, wl)
        args = (inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"])
        out = plan.alloc_outputs()
        plan.assemble_condense(*args, out=out)
        torch.cuda.synchronize()
        if int((out["status"] != 0).sum()):
            return {"error": "non-OK element status in the FP64 condensation (slab %d)" % i}
        tot["fp64_ms"] += _timed(lambda: plan.assemble_condense(*args, out=out), 1, torch)
        lp = plan.alloc_outputs_lp()
        plan.assemble_condense_lp(*args, out=lp)
        torch.cuda.synchronize()
        if int((lp["status"] != 0).sum()):
            return {"error": "non-OK element status in the FP32 condensation (slab %d)" % i}
        tot["lp_ms"] += _timed(lambda: plan.assemble_condense_lp(*args, out=lp), 1, torch)
        dl = torch.from_numpy(1e-3 * rng.standard_normal((plan.m, plan.n_trace))).cuda() * inp["vhat"].abs()
        dx, info = plan.refine_local(*args[:3], lp, dl, ustar=inp["ustar"], vbc=inp["vbc"], tol=tol)
        dx64 = plan.backsolve_elements(out["Y"], out["z"], dl)
        torch.cuda.synchronize()
        tot["refine_ms"] += info["total_ms"]
        refine["steps_max"] = max(refine["steps_max"], info["outer_iterations"])
        refine["rel_residual_max"] = max(refine["rel_residual_max"], info["rel_residual"])
        refine["converged"] = refine["converged"] and bool(info["converged"])
        for key in ("S", "Y", "g", "z"):
            worst[key] = max(worst[key], rel(lp[key], out[key]))
        worst["dx"] = max(worst["dx"], rel(dx, dx64))
        # the same with BF16 operands on the matrix cores
        plan.set_tuning(lp_operands=2)
        plan.assemble_condense_lp(*args, out=lp)
        torch.cuda.synchronize()
        if int((lp["status"] != 0).sum()):
            return {"error": "non-OK element status in the BF16-operand condensation (slab %d)" % i}
        tot["bf_ms"] += _timed(lambda: plan.assemble_condense_lp(*args, out=lp), 1, torch)
        dxb, ib = plan.refine_local(*args[:3], lp, dl, ustar=inp["ustar"], vbc=inp["vbc"], tol=tol, max_iter=16)
        torch.cuda.synchronize()
        tot["bf_refine_ms"] += ib["total_ms"]
        refine_bf["steps_max"] = max(refine_bf["steps_max"], ib["outer_iterations"])
        refine_bf["rel_residual_max"] = max(refine_bf["rel_residual_max"], ib["rel_residual"])
        refine_bf["converged"] = refine_bf["converged"] and bool(ib["converged"])
        refine_bf["fallback_elements"] += ib["fallback_elements"]
        for key in ("S", "Y", "g", "z"):
            worst_bf[key] = max(worst_bf[key], rel(lp[key], out[key]))
        worst_bf["dx"] = max(worst_bf["dx"], rel(dxb, dx64))
        del dxb
        E += plan.n_elem
        n, k = plan.n, plan.k
        del plan, inp, out, lp, dx, dx64, dl
        torch.cuda.empty_cache()
    fl = flops_per_elem(n, k, 64, 125, 5, 3, True)
    dense = fl["lu"] + fl["solve"] + fl["schur"]
    v64 = E / (tot["fp64_ms"] / 1e3)
    vmix = E / ((tot["lp_ms"] + tot["refine_ms"]) / 1e3)
    vbf = E / ((tot["bf_ms"] + tot["bf_refine_ms"]) / 1e3)
    return {"workload": "ns3d_hex_p3_32: 32^3 periodic trilinear hexes, p = 3 (n = 1280, k = 480), Taylor-Green "
                        "Re 1600 Mach 0.1, 5%% noise, jitter 5%%; %d of its %d slabs of %d elements" % (len(slabs), nslab, E // len(slabs)),
            "elements": E, "n": n, "k": k,
            "fp64": {"value": v64, "unit": "elem/s", "ms": tot["fp64_ms"],
                     "dense_tflops": dense * E / (tot["fp64_ms"] / 1e3) / 1e12},
            "mixed": {"value": vmix, "unit": "elem/s", "dtype": "f32 condensation + f64 element refinement",
                      "t_factor_lp_ms": tot["lp_ms"], "t_refine_local_ms": tot["refine_ms"],
                      "refine_tol": tol, **refine},
            "speedup_mixed_vs_fp64": vmix / v64,
            "rel_err_fp32_vs_fp64_gpu": worst,
            "bf16": {"value": vbf, "unit": "elem/s",
                     "dtype": "bf16 operands (FP32 condensation) + f64 element refinement",
                     "t_factor_lp_ms": tot["bf_ms"], "t_refine_local_ms": tot["bf_refine_ms"],
                     "refine_tol": tol, **refine_bf, "speedup_vs_fp64": vbf / v64,
                     "rel_err_vs_fp64_gpu": worst_bf}}


def bench_learned(torch):
    """Held-out 24^3 p = 2 system: GMRES(50) to 1e-10 with plain and learned block Jacobi."""
    ck = os.path.join(ROOT, "paper_1808_05066_amd", "data", "learned_bj.npz")
    if not os.path.exists(ck):
        return {"error": "no trained checkpoint"}
    from paper_1808_05066_amd import learn
    z = np.load(ck, allow_pickle=False)
    rows = learn.evaluate(z["theta"], n=24, seeds=(learn.HELDOUT_SEED0 + 50,),
                          log=lambda s: print(s, file=sys.stderr, flush=True))
    return {"checkpoint": "paper_1808_05066_amd/data/learned_bj.npz", "heldout": rows}


def bench_solve(plan, out, rhs, torch):
    """GMRES(50) + block Jacobi to 1e-10 on the FP64 condensed system (outside the timed step)."""
    from paper_1808_05066_amd.hdg import TraceSolver
    ts = TraceSolver(plan, restart=50, maxit=2000, tol=1e-10, precond="block_jacobi")
    ts.setup(out["S"])
    plan.trace_rhs(out["g"], rhs)
    t_setup = _timed(lambda: ts.setup(out["S"]), 3, torch)
    x, info = ts.solve(out["S"], rhs)
    torch.cuda.synchronize()
    return {"restart": 50, "precond": "block_jacobi", "tol": 1e-10, "iterations": info["iterations"],
            "rel_residual": info["rel_residual"], "converged": info["converged"], "solve_ms": info["solve_ms"],
            "setup_ms": t_setup, "unknowns": plan.m * plan.n_trace}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "condense_ns3d_hex_p2_16_traffic.md")


def kernel_source_hash():
    """Hash of the condensation kernel source: HBM counters taken on another version do not apply."""
    import hashlib
    src = os.path.join(ROOT, "paper_1808_05066_amd", "csrc", "hdg_condense.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# timing phase -> kernel of the FP64 condensation (32-column blocks)
PHASE_KERNEL = {"condense": "k_condense_f64_w32", "condense_lu": "k_lu_f64_w32", "condense_rhs": "k_rhs_f64_w32"}


def measured_traffic(kernel):
    """HBM bytes per launch of one condensation kernel from the committed counter summary, or None.

    The summary holds a line `traffic-json: {...}` with the source hash the
    counters were taken on; a different current hash means the kernel changed.
    """
    if not os.path.exists(TRAFFIC_FILE):
        return None
    for line in open(TRAFFIC_FILE):
        if line.startswith("traffic-json:"):
            d = json.loads(line.split(":", 1)[1])
            if d.get("source_hash") != kernel_source_hash():
                return None
            k = d.get("kernels", {}).get(kernel)
            if k is None:
                return None
            return dict(k, elements_per_launch=d["elements_per_launch"])
    return None


def copy_calibration(torch, nbytes=1 << 30):
    """A plain device copy of known size, run under rocprofv3 --pmc to scale FETCH_SIZE / WRITE_SIZE."""
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ns3d_hex_p2_16", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision measurement")
    ap.add_argument("--no-solve", action="store_true", help="skip the GMRES measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the mixed-batch measurement")
    ap.add_argument("--no-newton", action="store_true", help="skip the Newton-iteration measurement")
    ap.add_argument("--no-eliminate-q", action="store_true",
                    help="skip the measurement of the condensation that eliminates q first")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner comparison")
    ap.add_argument("--no-c4", action="store_true", help="skip the 32^3 p = 3 FP64 / mixed comparison")
    ap.add_argument("--c4-slabs", type=int, default=8, help="slabs of the 32^3 p = 3 mesh to process (of 8)")
    ap.add_argument("--only-c4", action="store_true", help="run only the 32^3 p = 3 comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the per-element work shards by element partition; see the design notes).", file=sys.stderr)
        sys.exit(2)
    # the CPU oracle runs first, in worker processes forked before this process touches the GPU
    cpu_res = None
    if not args.no_cpu_baseline and not args.copy_calibration and not args.only_c4:
        print("[bench] timing the CPU oracle samples", file=sys.stderr, flush=True)
        cpu_res = cpu_baseline(WORKLOADS[args.workload][1](), args.cpu_seconds)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    if args.only_c4:
        print(json.dumps({"c4": bench_c4(torch, nslab=8, process=args.c4_slabs)}))
        return
    from paper_1808_05066_amd.hdg import Plan

    desc, make = WORKLOADS[args.workload]
    wl = make()
    print("[bench] workload %s: %d elements, building plan" % (args.workload, wl.mesh.n_elem),
          file=sys.stderr, flush=True)
    plan = Plan(wl.mesh.etype, wl.p, wl.mesh.elem_xyz, wl.tmap, wl.n_trace, wl.face_bc, viscous=wl.viscous,
                gamma=wl.gamma, mu=wl.mu, Pr=wl.Pr, alpha=wl.alpha)
    inp = prepare_inputs(plan, wl, torch)
    out = plan.alloc_outputs()
    E, n, k = plan.n_elem, plan.n, plan.k
    r = torch.empty(plan.m, plan.n_trace, dtype=torch.float64, device="cuda")
    y = torch.empty_like(r)
    dv = torch.empty(plan.m, plan.n_nodes, dtype=torch.float64, device="cuda")
    dq = torch.empty(plan.m * plan.dim, plan.n_nodes, dtype=torch.float64, device="cuda") if wl.viscous else None

    def step():
        plan.assemble_condense(inp["v"], inp["q"], inp["vhat"], inp["ustar"], inp["vbc"], out=out)
        plan.trace_rhs(out["g"], r)
        plan.trace_matvec(out["S"], r, y)
        plan.backsolve(out["Y"], out["z"], r, dv, dq)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    bad = int((out["status"] != 0).sum())
    if bad:
        print("[bench] %d elements reported a non-OK status" % bad, file=sys.stderr)
        sys.exit(1)
    print("[bench] warmup done, timing %d steps" % args.steps, file=sys.stderr, flush=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    value = E / (ms / 1e3)

    # per-kernel durations from HIP events recorded by the library on the launch stream
    plan.set_timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ph = plan.phase_times()
    plan.set_timing(False)
    avg = {name: (t / c if c else 0.0) for name, (t, c) in ph.items()}
    fl = flops_per_elem(n, k, plan.Np, plan.Nq, plan.m, plan.dim, wl.viscous)
    fl["condense"] = fl["lu"] + fl["solve"] + fl["schur"]
    fl["condense_lu"] = fl["lu"]
    fl["condense_rhs"] = fl["solve"] + fl["schur"]
    # the dominant kernel: with the condensation in two launches, "condense" is their sum, not a kernel
    kernels = [p for p in avg if not (p == "condense" and avg.get("condense_lu", 0.0) > 0.0)]
    dom = max(kernels, key=avg.get)
    if dom in fl and dom != "contract":
        achieved = fl[dom] * E / (avg[dom] / 1e3) / 1e12
        roof = {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                "flops_per_elem": fl[dom], "elems_per_launch": E, "avg_ms": avg[dom]}
    else:
        achieved = fl.get(dom, 0.0) * E / (avg[dom] / 1e3) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                "flops_per_elem": fl.get(dom), "elems_per_launch": E, "avg_ms": avg[dom]}
    roof["kernel_name"] = PHASE_KERNEL.get(dom, dom)
    tr = measured_traffic(PHASE_KERNEL[dom]) if dom in PHASE_KERNEL else None
    if tr is not None:
        roof["traffic"] = tr["bytes_per_launch"] * E / tr["elements_per_launch"]
        roof["traffic_unit"] = "bytes"
        roof["traffic_source"] = os.path.relpath(TRAFFIC_FILE, ROOT)
    dense = fl["condense"]
    dense_ms = sum(avg[p] for p in ("lu", "solve", "schur", "condense"))
    cond_ms = avg["points"] + avg["contract"] + dense_ms
    res = {
        "metric": METRIC, "value": value, "unit": "elem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "elements": E, "n": n, "k": k,
                   "p": wl.p, "precision": "fp64"},
        "roofline": roof,
        "phase_ms": {p: round(v, 4) for p, v in avg.items()},
        "condense_elem_per_s": E / (cond_ms / 1e3),
        "dense_tflops": dense * E / (dense_ms / 1e3) / 1e12,
        "condensed_GBps": E * (k * k + k) * 8 / (cond_ms / 1e3) / 1e9,
        "wall_s_timed": wall,
    }
    if wl.viscous and not args.no_eliminate_q:
        print("[bench] condensation with the gradient unknowns eliminated first", file=sys.stderr, flush=True)
        res["eliminate_q"] = bench_eliminate_q(wl, inp, out, ms, args.steps, torch)
    if not args.no_newton:
        print("[bench] Newton iterations of one implicit stage", file=sys.stderr, flush=True)
        res["newton"] = bench_newton(plan, inp, torch)
    if not args.no_newton and wl.viscous and wl.alpha > 0:
        print("[bench] one DIRK(3,3) step", file=sys.stderr, flush=True)
        res["dirk_step"] = bench_dirk(plan, inp, 1.0 / (wl.alpha * C.DIRK33_AII), torch)
    if not args.no_mixed:
        print("[bench] mixed-precision path", file=sys.stderr, flush=True)
        res["mixed"] = bench_mixed(plan, inp, out, E, cond_ms, torch)
    if not args.no_solve:
        print("[bench] global trace solve", file=sys.stderr, flush=True)
        res["trace_solve"] = bench_solve(plan, out, r, torch)
    if not args.no_learned:
        print("[bench] learned preconditioner on a held-out system", file=sys.stderr, flush=True)
        res["learned_precond"] = bench_learned(torch)
    out = inp = plan = None   # release the measured mesh before the larger legs
    torch.cuda.empty_cache()
    if not args.no_batch:
        print("[bench] mixed tetrahedron/hexahedron batch", file=sys.stderr, flush=True)
        res["batch"] = bench_batch(torch)
    if not args.no_c4:
        print("[bench] 32^3 p = 3 mesh: FP64 against mixed precision", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        res["c4"] = bench_c4(torch, nslab=8, process=args.c4_slabs)
    if cpu_res is not None:
        res["cpu_baseline"] = cpu_res
    print(json.dumps(res))


if __name__ == "__main__":
    main()
