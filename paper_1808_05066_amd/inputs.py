"""Device-resident inputs of a workload: node coordinates from the plan, the
seeded synthetic state sampled there, converted to entropy variables by the
library (hdg_prepare_state)."""
from __future__ import annotations

import numpy as np


def device_inputs(plan, wl):
    import torch
    x, xt = plan.node_coords()
    s = wl.sample(x.cpu().numpy(), xt.cpu().numpy())
    dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()
    v, q, _ = plan.prepare_state(dev(s["prim"]), dev(s["grad"]) if wl.viscous else None)
    vhat, _, _ = plan.prepare_state(dev(s["prim_hat"]))
    _, _, ustar = plan.prepare_state(dev(s["prim_star"]), want_u=True)
    vbc = None
    if np.any(wl.face_bc):
        vbc, _, _ = plan.prepare_state(dev(s["prim_bc"]))
    torch.cuda.synchronize()
    return dict(v=v, q=q, vhat=vhat, ustar=ustar, vbc=vbc)


def plan_for(wl, chunk_elems=0):
    from .hdg import Plan
    return Plan(wl.mesh.etype, wl.p, wl.mesh.elem_xyz, wl.tmap, wl.n_trace, wl.face_bc, viscous=wl.viscous,
                gamma=wl.gamma, mu=wl.mu, Pr=wl.Pr, alpha=wl.alpha, chunk_elems=chunk_elems)
