"""Autotuner of the launch shapes, cached per (architecture, dtype, n, k).

For a plan it times hdg_assemble_condense (FP64) or hdg_assemble_condense_lp
(FP32) with every admissible combination of
  contract_threads  in (256, 512, 1024)  block-contraction workgroup size
  condense_width    in (16, 32)          condensation column-block width
  condense_launches in (1, 2)            one workgroup per element, or the LU and then
                                         one workgroup per right-hand-side block
  lu_waves          in (1, 2, 4, 8)      FP64 two-launch LU with 32-column blocks: in LDS (one
                                         element per CU) or in the registers of 2 waves (four
                                         elements per CU), 4 waves (two) or 8 waves
(median of HIP-event timings after a warm-up), keeps the fastest, and stores
it in a JSON cache; apply() sets a cached choice on a new plan.  Batches are
tuned over their mode: item lists with one workgroup per item or a persistent
grid, or the plans' own condensations on concurrent streams.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import hdg as H

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "autotune_cache.json")


def _arch():
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def key(plan, dtype):
    return "%s/%s/n%d/k%d" % (_arch(), dtype, plan.n, plan.k)


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def _admissible(plan, **kw):
    base = plan.tuning()
    try:
        plan.set_tuning(**kw)
        return True
    except H._lib.HdgError:
        return False
    finally:
        plan.set_tuning(**base)


def candidates(plan, dtype):
    """Admissible (contract_threads, width, launches, lu_waves) tuples; lu_waves 1 = LDS block."""
    shapes = []
    for w in (32, 16):
        if dtype == "fp64":
            if not _admissible(plan, condense_width=w):
                continue
            shapes += [(w, 1, 1), (w, 2, 1)]
            if w == 32:
                shapes += [(32, 2, lw) for lw in (2, 4, 8)
                           if _admissible(plan, condense_width=32, condense_launches=2, lu_waves=lw)]
        elif _admissible(plan, condense_width_lp=w):
            shapes += [(w, nl, 1) for nl in (1, 2)]
    return [(ct, w, nl, lw) for ct in (256, 512, 1024) for (w, nl, lw) in shapes]


def _set(plan, dtype, ct, w, nl, lw):
    if dtype == "fp64":
        plan.set_tuning(contract_threads=ct, condense_width=w, condense_launches=nl, lu_waves=lw)
    else:
        plan.set_tuning(contract_threads=ct, condense_width_lp=w, condense_launches=nl)


def tune_plan(plan, inputs, dtype="fp64", reps=3, cache=DEFAULT_CACHE, log=print):
    """Time every candidate on `inputs` (dict v, q, vhat, ustar, vbc); store and set the best."""
    args = (inputs["v"], inputs["q"], inputs["vhat"], inputs.get("ustar"), inputs.get("vbc"))
    out = plan.alloc_outputs() if dtype == "fp64" else plan.alloc_outputs_lp(residuals=False)
    run = (lambda: plan.assemble_condense(*args, out=out)) if dtype == "fp64" else \
        (lambda: plan.assemble_condense_lp(*args, out=out))
    results = []
    for ct, w, nl, lw in candidates(plan, dtype):
        _set(plan, dtype, ct, w, nl, lw)
        ms = _time(run, reps)
        results.append({"contract_threads": ct, "condense_width": w, "condense_launches": nl, "lu_waves": lw,
                        "ms": ms})
        log("[autotune] %s ct=%d w=%d launches=%d lu_waves=%d: %.2f ms" % (key(plan, dtype), ct, w, nl, lw, ms))
    best = min(results, key=lambda r: r["ms"])
    _set(plan, dtype, best["contract_threads"], best["condense_width"], best.get("condense_launches", 1),
         best.get("lu_waves", 1))
    entry = {"best": best, "all": results, "elements": plan.n_elem}
    if cache:
        store(cache, key(plan, dtype), entry)
    return entry


def tune_batch(batch, reps=3, log=print):
    """Mode of a batch whose io is set: item lists with one workgroup per item (groups 0) or a
    persistent grid of one or two workgroups per CU, or every plan's own condensation on 2 or 4
    concurrent streams (returns the timings)."""
    import torch
    res = []
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for streams, groups in [(0, 0), (0, cus), (0, 2 * cus), (2, 0), (4, 0)]:
        batch.set_streams(streams)
        batch.set_groups(groups)
        ms = _time(batch.run, reps)
        res.append({"streams": streams, "groups": groups, "ms": ms})
        log("[autotune] batch streams=%d groups=%d: %.2f ms" % (streams, groups, ms))
    best = min(res, key=lambda r: r["ms"])
    batch.set_streams(best["streams"])
    batch.set_groups(best["groups"])
    return {"best": best, "all": res}


def load(cache=DEFAULT_CACHE):
    if not os.path.exists(cache):
        return {}
    with open(cache) as f:
        return json.load(f)


def store(cache, k, entry):
    data = load(cache)
    data[k] = entry
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    with open(cache, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def apply(plan, dtype="fp64", cache=DEFAULT_CACHE):
    """Set the cached choice for this plan's bucket; returns it (None if absent)."""
    e = load(cache).get(key(plan, dtype))
    if not e:
        return None
    b = e["best"]
    try:
        # entries written before the launch count and LU variant were swept carry neither:
        # they leave the plan's defaults
        nl, lw = b.get("condense_launches", 0), b.get("lu_waves", 0)
        if dtype == "fp64":
            plan.set_tuning(contract_threads=b["contract_threads"], condense_width=b["condense_width"],
                            condense_launches=nl, lu_waves=lw)
        else:
            plan.set_tuning(contract_threads=b["contract_threads"], condense_width_lp=b["condense_width"],
                            condense_launches=nl)
    except H._lib.HdgError:
        return None
    return b


def main():
    """Tune the measured workloads: the 4096-element p = 2 hex mesh (FP64 and FP32)
    and every group of the mixed tetrahedron / hexahedron batch (FP64)."""
    import argparse
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from workloads import configs as C
    from .inputs import device_inputs, plan_for
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    log = lambda s: print(s, file=sys.stderr, flush=True)
    wl = C.ns3d_hex(n=16, p=2)
    pl = plan_for(wl)
    inp = device_inputs(pl, wl)
    tune_plan(pl, inp, "fp64", a.reps, a.out, log)
    tune_plan(pl, inp, "fp32", a.reps, a.out, log)
    del pl, inp
    for wl in C.mixed_batch():
        pl = plan_for(wl)
        inp = device_inputs(pl, wl)
        tune_plan(pl, inp, "fp64", a.reps, a.out, log)
        del pl, inp
    print(json.dumps(load(a.out), indent=1))


if __name__ == "__main__":
    main()
