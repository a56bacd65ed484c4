"""C ABI checks that need no GPU: symbols, host-side plan logic, error paths."""
import ctypes
import subprocess

import numpy as np
import pytest

from paper_1808_05066_amd import _lib
from workloads import configs as C
from workloads import meshes as M


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_library_exports_every_header_symbol(lib):
    syms = _lib.header_symbols()
    assert len(syms) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for s in syms:
        assert s in exported, s
        assert s in _lib.SIGNATURES, s
        getattr(lib, s)


def _create(lib, wl, **kw):
    xyz = np.ascontiguousarray(wl.mesh.elem_xyz)
    tm = np.ascontiguousarray(wl.tmap, dtype=np.int32)
    fbc = np.ascontiguousarray(wl.face_bc, dtype=np.int32)
    mesh = _lib.hdg_mesh(kw.get("etype", _lib.ETYPES[wl.mesh.etype]), kw.get("order", wl.p),
                         kw.get("n_elem", wl.mesh.n_elem), xyz.ctypes.data, fbc.ctypes.data, tm.ctypes.data,
                         kw.get("n_trace", wl.n_trace))
    phys = _lib.hdg_phys(int(wl.viscous), kw.get("gamma", wl.gamma), wl.mu, wl.Pr, wl.alpha)
    opts = _lib.hdg_opts(kw.get("chunk", 0), kw.get("precision", 0), 0)
    h = ctypes.c_void_p()
    rc = lib.hdg_plan_create(ctypes.byref(h), ctypes.byref(mesh), ctypes.byref(phys), ctypes.byref(opts))
    return rc, h, (xyz, tm, fbc)


@pytest.mark.parametrize("name,n,k", [("c1", 24, 36), ("c2", 540, 270), ("ns2d", 72, 36)])
def test_plan_dims_host_only(lib, name, n, k):
    wl = {"c1": lambda: C.euler2d_tri_p2(), "c2": lambda: C.ns3d_hex(n=2, p=2),
          "ns2d": lambda: C.ns2d_tri(n=3, p=2)}[name]()
    rc, h, keep = _create(lib, wl)
    assert rc == 0, lib.hdg_last_error()
    d = _lib.hdg_dims()
    assert lib.hdg_plan_dims(h, ctypes.byref(d)) == 0
    assert (d.n, d.k) == (n, k)
    assert d.n_pad % 16 == 0 and d.k_pad % 16 == 0 and d.n_pad >= n and d.k_pad >= k
    nb = ctypes.c_size_t()
    assert lib.hdg_plan_workspace_bytes(h, ctypes.byref(nb)) == 0 and nb.value > 0
    lib.hdg_plan_destroy(h)


def test_plan_create_rejects_bad_input(lib):
    wl = C.euler2d_tri_p2(n=2)
    rc, _, _ = _create(lib, wl, order=7)
    assert rc == _lib.HDG_EUNSUPPORTED
    rc, _, _ = _create(lib, wl, gamma=0.9)
    assert rc == _lib.HDG_EINVAL
    rc, _, _ = _create(lib, wl, n_trace=3)           # map entries out of range
    assert rc == _lib.HDG_EINVAL
    rc, _, _ = _create(lib, wl, precision=2)
    assert rc == _lib.HDG_EUNSUPPORTED
    # a collapsed (inverted) element is caught at plan time
    bad = C.euler2d_tri_p2(n=2)
    bad.mesh.elem_xyz[0] = bad.mesh.elem_xyz[0][[0, 2, 1]]
    rc, _, _ = _create(lib, bad)
    assert rc == _lib.HDG_EINVAL
    assert b"Jacobian" in lib.hdg_last_error()


def test_calls_without_workspace_fail_cleanly(lib):
    wl = C.euler2d_tri_p2(n=2)
    rc, h, keep = _create(lib, wl)
    assert rc == 0
    assert lib.hdg_assemble_condense(h, *([None] * 12), None) == _lib.HDG_EINVAL
    assert lib.hdg_trace_matvec(h, None, None, None, None) == _lib.HDG_EINVAL
    lib.hdg_plan_destroy(h)
