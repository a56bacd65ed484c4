"""Ringleb flow (the steady Euler convergence example of Section 5) on the GPU path.

* Parity: the GPU Newton iteration (hdg_newton_solve) on a 4 x 4 mesh, p = 2, for HDG, IEDG
  and EDG traces ends within 1e-9 (relative) of the oracle's newton_steady; with EDG the trace
  nodes of the Dirichlet faces are shared with interior faces, so this covers the dropped
  flux rows (blocks, residuals and the Newton system).
* Convergence against Tables 3-5 (tests/golden/paper_tables_3_5_ringleb.json): p = 1, 2 on
  1/h = 2, 4, 8 for the three traces; no error above 1.5x (p = 1) or 2x (p = 2) the printed one
  (the diagonal of the split is not stated) nor below a quarter of it (the p = 2 HDG errors
  here are up to 2.4x below the printed ones, at rate 2.96 where Table 3 has 2.71), and the
  rate on the finest pair at least k + 1 - 0.35."""
import json
import os

import numpy as np
import pytest

from oracle import hdg as ohdg, newton, physics as ph

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def ringleb_mesh(n):
    from workloads import meshes as M
    mesh = M.tri_square(n, 0.0, 0, periodic=False, lo=0.0, length=4.0)
    mesh.elem_xyz[..., 0] -= 5.0
    mesh.elem_xyz[..., 1] += 1.0
    return mesh


@pytest.mark.parametrize("scheme", ["hdg", "iedg", "edg"])
def test_ringleb_newton_matches_oracle(torch, scheme):
    from paper_1808_05066_amd.hdg import Plan
    from workloads import meshes as M
    from workloads.fields import Ringleb
    f, p = Ringleb(), 2
    mesh = ringleb_mesh(4)
    tmap, nt = M.trace_map(mesh, p, scheme)
    fbc = mesh.boundary.astype(np.int32)
    disc = ohdg.Discretization(mesh, p, ohdg.Phys(f.gamma, 0.0, 0.72, 0.0, False), tmap, nt, fbc)

    def v_of(x):
        pr = f.prim(x)
        return ph.v_of_prim(pr[0], pr[1:3].T, pr[3], f.gamma).T.copy()

    v0, vh0 = v_of(disc.node_coords()), v_of(disc.trace_coords())
    ov, _, ovh, hist = newton.newton_steady(disc, v0, None, vh0, vbc=vh0.copy(), tol=1e-13)
    plan = Plan("tri", p, mesh.elem_xyz, tmap, nt, fbc, viscous=False, gamma=f.gamma)
    v, vh = torch.from_numpy(v0).cuda(), torch.from_numpy(vh0).cuda()
    vbc = vh.clone()
    info = plan.newton_solve(v, None, vh, None, vbc, maxit=12, tol=1e-13, atol=1e-14, lin_tol=1e-14)
    print(scheme, "oracle", hist, "gpu", info["res"], flush=True)
    assert info["converged"] == 1
    ev = np.linalg.norm(v.cpu().numpy() - ov) / np.linalg.norm(ov)
    eh = np.linalg.norm(vh.cpu().numpy() - ovh) / np.linalg.norm(ovh)
    print("relative differences v, vhat", ev, eh, flush=True)
    assert max(ev, eh) <= 1e-9
    if scheme == "edg":
        # the Dirichlet nodes carry the boundary data exactly
        dn = disc.dir_node
        assert np.abs(vh.cpu().numpy()[:, dn] - vh0[:, dn]).max() < 1e-12


def test_ringleb_convergence_against_tables(torch):
    from paper_1808_05066_amd.convergence import ringleb_table
    tab = json.load(open(os.path.join(HERE, "golden", "paper_tables_3_5_ringleb.json")))
    rows = ringleb_table(ns=(8, 16, 32), ps=(1, 2))
    for r in rows:
        print(r, flush=True)
        assert r["converged"] == 1
        ref = tab["error"][r["scheme"]][r["p"] - 1][tab["inv_h"].index(int(r["inv_h"]))]
        fac = 1.5 if r["p"] == 1 else 2.0
        assert ref / 4.0 < r["error"] < ref * fac, (r, ref)
        if r["n"] == 32:
            assert r["rate"] >= r["p"] + 1 - 0.35, r
