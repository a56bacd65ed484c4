"""DIRK(3,3) steps on the GPU (hdg_dirk_step): a smooth periodic Navier-Stokes flow on a
small triangle mesh.

* Two steps of dt = 0.1 against the oracle's dirk33_step: every stage's Newton iteration
  stops below 1e-11 absolute residual on both sides (the GPU at 1e-13 of its start); the end
  states agree to 1e-9 relative (the residual tolerance times the stage Jacobian's inverse).
* Self-convergence in time on the GPU (T = 0.2 in 2, 4, 8 steps): rate >= 2.5 (third order
  pre-asymptotic, as in the oracle's own check)."""
import numpy as np
import pytest

from oracle import newton

from cases import smooth_periodic_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def gpu_plan_of(md):
    from paper_1808_05066_amd.hdg import Plan
    mesh = md["mesh"]
    return Plan(mesh.etype, md["p"], mesh.elem_xyz, md["tmap"], md["n_trace"], md["face_bc"], viscous=True,
                gamma=md["gamma"], mu=md["mu"], Pr=md["Pr"], alpha=md["alpha"])


def gpu_steps(torch, dt, nsteps, n=2):
    md, _, v0, q0, vh0 = smooth_periodic_case(dt, n=n)
    plan = gpu_plan_of(md)
    v, q, vh = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (v0, q0, vh0))
    infos = []
    for _ in range(nsteps):
        infos.append(plan.dirk_step(v, q, vh, dt, tol=1e-13, atol=1e-12, lin_tol=1e-13))
    torch.cuda.synchronize()
    return v.cpu().numpy(), q.cpu().numpy(), vh.cpu().numpy(), infos


def test_dirk_step_matches_oracle(torch):
    dt = 0.1
    _, disc, v, q, vh = smooth_periodic_case(dt)
    for _ in range(2):
        v, q, vh, hists = newton.dirk33_step(disc, v, q, vh, dt)
    gv, gq, gvh, infos = gpu_steps(torch, dt, 2)
    for step in infos:
        for st in step:
            print(st, flush=True)
            assert st["converged"] == 1 and st["lin_converged"] == 1
            assert st["res"][-1] < 1e-11
    errs = [np.linalg.norm(g - o) / np.linalg.norm(o) for g, o in ((gv, v), (gq, q), (gvh, vh))]
    print("relative differences v, q, vhat", errs, flush=True)
    assert max(errs) <= 1e-9


def test_dirk_temporal_order(torch):
    out = {ns: gpu_steps(torch, 0.2 / ns, ns)[0] for ns in (2, 4, 8)}
    e1 = np.linalg.norm(out[2] - out[4])
    e2 = np.linalg.norm(out[4] - out[8])
    print("self-convergence", e1, e2, np.log2(e1 / e2), flush=True)
    assert np.log2(e1 / e2) >= 2.5
