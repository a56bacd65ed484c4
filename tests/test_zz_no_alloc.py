"""hdg_learn_backward_noalloc (partial gradients in the library's static device array) against
hdg_learn_backward (caller's scratch): same gradient, bit for bit, on two calls in a row, the
second on a smaller plan; a plan with more rows than the static array holds is refused."""
import ctypes

import numpy as np
import pytest

from cases import SMALL_CASES, gpu_plan, oracle_case, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _learned(torch, wl):
    from paper_1808_05066_amd.hdg import LearnedPrecond, TraceSolver
    disc, inp = oracle_case(wl)
    plan = gpu_plan(wl)
    d = to_dev(inp)
    out = plan.assemble_condense(d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"])
    lp = LearnedPrecond(TraceSolver(plan, restart=10, precond="block_jacobi"))
    lp.setup(out["S"], d["vhat"])
    return plan, lp


def test_noalloc_backward_equals_backward(torch):
    from workloads import configs as C
    rng = np.random.default_rng(31)
    cases = [SMALL_CASES["ns3d_hex_p1"](), SMALL_CASES["ns2d_tri_p2"]()]
    sizes = []
    for wl in cases:                       # larger plan first, then a smaller one
        plan, lp = _learned(torch, wl)
        theta = torch.from_numpy(rng.normal(scale=0.3, size=lp.nparams).astype(np.float32)).cuda()
        dO = torch.from_numpy(rng.normal(size=(lp.N, lp.no)).astype(np.float32)).cuda()
        ref = lp.backward(theta, dO).clone()
        got = torch.full_like(ref, float("nan"))
        lp.backward_noalloc(theta, dO, got)
        torch.cuda.synchronize()
        print("rows", lp.N, "max |diff|", float((got - ref).abs().max()), flush=True)
        assert torch.equal(got, ref)
        sizes.append(lp.N)
    assert sizes[1] < sizes[0]


def test_noalloc_backward_refuses_too_many_rows(torch):
    from paper_1808_05066_amd import _lib
    from workloads import configs as C
    plan = gpu_plan(C.euler2d_tri_p2(n=120, p=1))
    assert plan.m * plan.n_trace > 278144
    buf = torch.zeros(16, dtype=torch.float32, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    rc = plan.lib.hdg_learn_backward_noalloc(plan.h, p, p, p, p, None)
    assert rc == _lib.HDG_EINVAL
    assert b"exceed" in plan.lib.hdg_last_error()
