"""The C ABI library loads and exports every entry point of include/nm.h; its
host-side argument checks reject bad input before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2411_11725_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "nm.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nm_[a-z_0-9]+)\s*\(", text)))


needs_lib = pytest.mark.skipif(not os.path.exists(binding.LIB_PATH),
                               reason="libnm.so not built (run __graft_entry__.build())")


def test_header_and_binding_agree():
    assert _declared() == sorted(binding.EXPORTS)


@needs_lib
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(binding.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


@needs_lib
def test_footprint_is_host_only_and_validates():
    fp = binding.nm_mesh_footprint_bytes((128, 128, 32), (2e-9,) * 3)
    # at least the spectrum workspace 3 N3 P2 (P1/2+1) complex64
    assert fp > 3 * 32 * 256 * 129 * 8
    assert binding.nm_mesh_footprint_bytes((1, 128, 32), (2e-9,) * 3) == 0
    assert binding.nm_mesh_footprint_bytes((2000, 4, 4), (2e-9,) * 3) == 0
    # the longest padded axis is 1024 points: 512 cells fit on every axis, 513 do not
    for ax in range(3):
        n = [4, 4, 4]
        n[ax] = 512
        assert binding.nm_mesh_footprint_bytes(tuple(n), (2e-9,) * 3) > 0, n
        n[ax] = 513
        assert binding.nm_mesh_footprint_bytes(tuple(n), (2e-9,) * 3) == 0, n
    # x and y need two cells, z one; the film basis one cell layer
    for n in [(4, 1, 4), (4, 4, 0), (-3, 4, 4)]:
        assert binding.nm_mesh_footprint_bytes(n, (2e-9,) * 3) == 0, n
    assert binding.nm_mesh_footprint_bytes((2, 2, 1), (2e-9,) * 3) > 0
    assert binding.nm_mesh_footprint_bytes((4, 4, 1), (2e-9,) * 3, basis=binding.NM_BASIS_FILM) > 0
    assert binding.nm_mesh_footprint_bytes((4, 4, 2), (2e-9,) * 3, basis=binding.NM_BASIS_FILM) == 0
    assert binding.nm_mesh_footprint_bytes((4, 4, 4), (2e-9,) * 3, basis=7) == 0


@needs_lib
def test_null_arguments_are_rejected_before_any_gpu_work():
    L = binding.lib()
    out = ctypes.c_void_p()
    assert L.nm_mesh_create(None, None, ctypes.byref(out)) == binding.NM_EINVAL
    assert b"NULL" in L.nm_last_error()
    desc = binding.nm_mesh_desc((ctypes.c_int * 3)(0, 4, 4), (ctypes.c_double * 3)(1e-9, 1e-9, 1e-9),
                                2.211e5, None)
    mat = binding.nm_material()
    assert L.nm_mesh_create(ctypes.byref(desc), ctypes.byref(mat), ctypes.byref(out)) == binding.NM_EINVAL
    desc.n[0] = 4
    desc.h[1] = -1.0
    assert L.nm_mesh_create(ctypes.byref(desc), ctypes.byref(mat), ctypes.byref(out)) == binding.NM_EINVAL
    desc.h[1] = 1e-9
    # Ms, A and alpha are required
    assert L.nm_mesh_create(ctypes.byref(desc), ctypes.byref(mat), ctypes.byref(out)) == binding.NM_EINVAL
    assert L.nm_heff(None, None, None, 15, 0.0) == binding.NM_EINVAL
    clk = binding.nm_clock()
    integ = binding.nm_integrator()
    assert L.nm_llg_step(None, None, ctypes.byref(clk), ctypes.byref(integ), 0.0, 1) == binding.NM_EINVAL
    assert L.nm_mesh_destroy(None) == binding.NM_OK
    n = (ctypes.c_int * 3)(0, 1, 1)
    h = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    assert L.nm_newell_octant(n, h, ctypes.c_void_p(1), None) == binding.NM_EINVAL


@needs_lib
def test_adjoint_and_server_reject_bad_arguments_on_the_host():
    L = binding.lib()
    P = ctypes.c_void_p
    assert L.nm_adjoint_step(None, None, 0.0, 1e-14, 1, 15, None, 1, None, None, None) == binding.NM_EINVAL
    assert L.nm_adjoint_workspace_bytes(None, 4) == 0
    assert L.nm_adjoint_continuous(None, None, 0.0, 1e-14, 1, 15, None, None) == binding.NM_EINVAL
    out = ctypes.c_void_p()
    for bad in [(0, 0, 1, 4), (0, 2, 0, 4), (0, 2, 17, 4), (0, 2, 4, 0), (0, 2, 4, 65)]:
        d = binding.nm_server_desc(*bad)
        assert L.nm_server_create(ctypes.byref(d), ctypes.byref(out)) == binding.NM_EINVAL
    assert L.nm_server_create(None, ctypes.byref(out)) == binding.NM_EINVAL
    assert L.nm_serve_submit(None, None, None) == binding.NM_EINVAL
    res = binding.nm_solve_result()
    assert L.nm_serve_poll(None, ctypes.c_uint64(1), ctypes.byref(res), None, 0) == binding.NM_EINVAL
    assert L.nm_server_destroy(None) == binding.NM_OK
    assert L.nm_profile_enable(None, 1) == binding.NM_EINVAL
    y, z = ctypes.c_int(0), ctypes.c_int(0)
    assert L.nm_mesh_tuning(None, 0, ctypes.byref(y), ctypes.byref(z)) == binding.NM_EINVAL


def test_missing_library_raises_and_the_package_never_imports_the_oracle(monkeypatch, tmp_path):
    """Without the HIP library every entry point raises (there is no fallback
    path); no module of the package imports the oracle."""
    import ast
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "libnm.so"))
    with pytest.raises(RuntimeError, match="not built"):
        binding.lib()
    with pytest.raises(RuntimeError, match="not built"):
        binding.nm_mesh_footprint_bytes((4, 4, 4), (2e-9,) * 3)
    pkg = os.path.dirname(binding.__file__)
    for name in sorted(os.listdir(pkg)):
        if not name.endswith(".py"):
            continue
        tree = ast.parse(open(os.path.join(pkg, name)).read())
        for node in ast.walk(tree):
            mods = []
            if isinstance(node, ast.Import):
                mods = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                mods = [node.module or ""]
            assert not any(m == "oracle" or m.startswith("oracle.") for m in mods), (name, mods)
