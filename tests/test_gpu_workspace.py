"""The plan's workspace between calls.

With all elements in one chunk the plan keeps the structural zeros of its
coupling blocks (B, C, D) in the workspace and clears them only on the first
call after a bind.  Checked bit for bit against a fresh plan: a second call on
new inputs, a call after rebinding a workspace filled with NaN, and (clearing
on every call) a plan processed in several chunks.
"""
import ctypes

import pytest

from cases import SMALL_CASES, gpu_plan, oracle_case, to_dev

pytestmark = pytest.mark.gpu
KEYS = ("S", "Y", "g", "z")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _args(d):
    return d["v"], d["q"], d["vhat"], d["ustar"], d["vbc"]


def _perturbed(d, torch, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    out = dict(d)
    for key in ("v", "vhat"):
        out[key] = d[key] * (1.0 + 1e-3 * torch.randn(d[key].shape, generator=g, device="cuda", dtype=d[key].dtype))
    return out


@pytest.mark.parametrize("name", ["euler2d_tri_p2", "ns2d_tri_p2", "ns3d_hex_p1"])
def test_workspace_reuse_matches_fresh_plan(torch, name):
    from paper_1808_05066_amd.hdg import _stream
    wl = SMALL_CASES[name]()
    _, inp = oracle_case(wl)
    d1 = to_dev(inp)
    d2 = _perturbed(d1, torch, 7)
    print("case", name, flush=True)
    ref = gpu_plan(wl).assemble_condense(*_args(d2))
    torch.cuda.synchronize()

    plan = gpu_plan(wl)
    plan.assemble_condense(*_args(d1))
    second = plan.assemble_condense(*_args(d2))
    torch.cuda.synchronize()
    for key in KEYS:
        assert torch.equal(second[key], ref[key]), ("second call", key)

    # a new workspace full of NaN: the first call after the bind clears it
    ws = torch.full_like(plan.workspace, 255)
    off = (-ws.data_ptr()) % 256
    nbytes = plan.workspace.numel() - 256
    rc = plan.lib.hdg_plan_bind_workspace(plan.h, ctypes.c_void_p(ws.data_ptr() + off), ctypes.c_size_t(nbytes),
                                          _stream())
    assert rc == 0
    plan.workspace = ws
    rebound = plan.assemble_condense(*_args(d2))
    torch.cuda.synchronize()
    for key in KEYS:
        assert torch.equal(rebound[key], ref[key]), ("after rebind", key)

    chunked = gpu_plan(wl, chunk_elems=max(1, wl.mesh.n_elem // 3))
    chunked.assemble_condense(*_args(d1))
    again = chunked.assemble_condense(*_args(d2))
    torch.cuda.synchronize()
    for key in KEYS:
        assert torch.equal(again[key], ref[key]), ("chunked", key)
