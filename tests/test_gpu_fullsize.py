"""Full-size parity: the 4096-element 3D Navier-Stokes p=2 mesh, in the launch
configuration bench.py times (one chunk of all elements), checked against the
oracle on sampled elements (first, last and seeded random ones).

S, Y, g, R_tr: relative Frobenius error <= 1e-12.  z: backward error
||A z_gpu - R_loc|| <= 1e-12 times the summation scale of R_loc, and forward
relative error <= 1e-11 (see cases.z_backward_err)."""
import numpy as np
import pytest

from oracle import hdg as ohdg
from oracle import state as ostate
from workloads import configs as C

from cases import gpu_plan, oracle_disc, z_backward_err

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def test_ns3d_hex_p2_16_sampled(torch):
    wl = C.ns3d_hex(n=16, p=2)
    disc = oracle_disc(wl)
    inp = ostate.oracle_inputs_fast(wl, disc)
    plan = gpu_plan(wl)
    dev = {k: (None if inp[k] is None else torch.from_numpy(np.ascontiguousarray(inp[k])).cuda())
           for k in ("v", "q", "vhat", "ustar")}
    print("full-size run: %d elements" % wl.mesh.n_elem, flush=True)
    out = plan.assemble_condense(dev["v"], dev["q"], dev["vhat"], dev["ustar"], None, residuals=True)
    torch.cuda.synchronize()
    assert int((out["status"] != 0).sum()) == 0
    E = wl.mesh.n_elem
    rng = np.random.default_rng(2024)
    sample = [0, E - 1] + list(rng.choice(np.arange(1, E - 1), 2, replace=False))
    ref = ohdg.assemble_condense(disc, inp["v"], inp["q"], inp["vhat"], inp["ustar"], None, elems=sample,
                                 keep_blocks=True)
    for e, r in zip(sample, ref):
        errs = {}
        zg = out["z"][e].cpu().numpy()
        zf = np.linalg.norm(zg - r["z"]) / np.linalg.norm(r["z"])
        assert zf <= 1e-11, (e, zf)
        errs["z_backward"] = z_backward_err(disc, inp, e, r["A"], r["R_loc"], zg)
        for key, mat in (("S", True), ("Y", True), ("g", False)):
            got = out[key][e].cpu().numpy()
            got = got.T if mat else got
            errs[key] = np.linalg.norm(got - r[key]) / np.linalg.norm(r[key])
        errs["R_tr"] = np.linalg.norm(out["R_tr"][e].cpu().numpy() - r["R_tr"]) / np.linalg.norm(r["R_tr"])
        print("element", e, errs, flush=True)
        for key, err in errs.items():
            assert err <= TOL, (e, key, err)
