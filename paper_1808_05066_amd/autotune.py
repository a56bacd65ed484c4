"""Autotuner of the launch shapes, cached per (architecture, dtype, n, k).

For a plan it times hdg_assemble_condense (FP64) or hdg_assemble_condense_lp
(FP32) with every admissible combination of
  contract_threads in (256, 512, 1024)   block-contraction workgroup size
  condense_width   in (16, 32)           condensation column-block width
(median of HIP-event timings after a warm-up), keeps the fastest, and stores
it in a JSON cache; apply() sets a cached choice on a new plan.  Batches are
tuned over the queue order (largest first or plan order) and the persistent
grid size.
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


def candidates(plan, dtype):
    base = plan.tuning()
    widths = []
    for w in (32, 16):
        try:
            if dtype == "fp64":
                plan.set_tuning(condense_width=w)
            else:
                plan.set_tuning(condense_width_lp=w)
            widths.append(w)
        except H._lib.HdgError:
            pass
    plan.set_tuning(**base)
    return [(ct, w) for ct in (256, 512, 1024) for w in widths]


def tune_plan(plan, inputs, dtype="fp64", reps=3, cache=DEFAULT_CACHE, log=print):
    """Time every candidate on `inputs` (dict v, q, vhat, ustar, vbc); store and set the best."""
    args = (inputs["v"], inputs["q"], inputs["vhat"], inputs.get("ustar"), inputs.get("vbc"))
    out = plan.alloc_outputs() if dtype == "fp64" else plan.alloc_outputs_lp(residuals=False)
    run = (lambda: plan.assemble_condense(*args, out=out)) if dtype == "fp64" else \
        (lambda: plan.assemble_condense_lp(*args, out=out))
    results = []
    for ct, w in candidates(plan, dtype):
        if dtype == "fp64":
            plan.set_tuning(contract_threads=ct, condense_width=w)
        else:
            plan.set_tuning(contract_threads=ct, condense_width_lp=w)
        ms = _time(run, reps)
        results.append({"contract_threads": ct, "condense_width": w, "ms": ms})
        log("[autotune] %s ct=%d w=%d: %.2f ms" % (key(plan, dtype), ct, w, ms))
    best = min(results, key=lambda r: r["ms"])
    if dtype == "fp64":
        plan.set_tuning(contract_threads=best["contract_threads"], condense_width=best["condense_width"])
    else:
        plan.set_tuning(contract_threads=best["contract_threads"], condense_width_lp=best["condense_width"])
    entry = {"best": best, "all": results, "elements": plan.n_elem}
    if cache:
        store(cache, key(plan, dtype), entry)
    return entry


def tune_batch(batch, reps=3, log=print):
    """Queue order and persistent grid size of a batch whose io is set (returns the timings)."""
    import torch
    res = []
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for groups in (cus, 2 * cus):
        batch.set_groups(groups)
        ms = _time(batch.run, reps)
        res.append({"groups": groups, "ms": ms})
        log("[autotune] batch groups=%d: %.2f ms" % (groups, ms))
    best = min(res, key=lambda r: r["ms"])
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
        if dtype == "fp64":
            plan.set_tuning(contract_threads=b["contract_threads"], condense_width=b["condense_width"])
        else:
            plan.set_tuning(contract_threads=b["contract_threads"], condense_width_lp=b["condense_width"])
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
