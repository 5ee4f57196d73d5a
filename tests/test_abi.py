"""The C-ABI library loads, exports every function include/etac.h declares,
and validates arguments on the host (no GPU needed for any of these)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2604_20295_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "etac.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(etac_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = _native.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_native.EXPORTED)


def test_status_strings():
    lib = _native.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        s = lib.etac_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.etac_status_string(12345).decode() == "unknown status"


def _mesh(K=2, n=4, bad=None):
    off = np.arange(K + 1, dtype=np.int32) * n
    N = K * n
    pos = np.zeros((3, N), np.float32)
    pos[0] = np.arange(N)
    nrm = np.zeros((3, N), np.float32)
    nrm[2] = 1
    origin = np.zeros((K, 3), np.float32)
    if bad == "offset":
        off[1] = off[2] + 1
    if bad == "nan":
        pos[1, 3] = np.nan
    if bad == "end":
        off[-1] = N - 1
    keep = (off, pos, nrm, origin)
    m = _native.etac_mesh(K, N, off.ctypes.data, pos.ctypes.data, nrm.ctypes.data, origin.ctypes.data)
    return m, keep


def _create(m, E=1, O=1, flags=0):
    h = C.c_void_p()
    rc = _native.lib().etac_plan_create(C.byref(m), E, O, flags, C.byref(h))
    return rc, h


def test_plan_create_validation_without_gpu():
    lib = _native.lib()
    h = C.c_void_p()
    assert lib.etac_plan_create(None, 1, 1, 0, C.byref(h)) == -1
    m, keep = _mesh()
    assert lib.etac_plan_create(C.byref(m), 1, 1, 0, None) == -1
    for bad, code in (("offset", -2), ("nan", -3), ("end", -2)):
        mb, kb = _mesh(bad=bad)
        assert _create(mb)[0] == code, bad
    assert _create(m, E=0)[0] == -2
    assert _create(m, O=0)[0] == -2
    assert _create(m, O=9)[0] == -2
    assert _create(m, flags=0x10)[0] == -3
    m0, k0 = _mesh(K=1, n=70000)
    assert _create(m0)[0] == -2          # patch larger than ETAC_MAX_PATCH_NODES
    mz = _native.etac_mesh(0, 0, None, None, None, None)
    assert _create(mz)[0] == -1


def test_calls_reject_null_plan():
    lib = _native.lib()
    sc = _native.etac_scene()
    md = _native.etac_model()
    assert lib.etac_contact(None, C.byref(sc), None, None, None, None) == -1
    assert lib.etac_propagate(None, C.byref(md), 1, None, None, None, None, None) == -1
    assert lib.etac_step(None, C.byref(sc), C.byref(md), None, None, None, None, None) == -1
    assert lib.etac_contact_backward(None, C.byref(sc), None, None, None, None) == -1
    assert lib.etac_propagate_backward(None, C.byref(md), 1, None, None, None, None, None, None, None, None) == -1
    assert lib.etac_step_backward(None, C.byref(sc), C.byref(md), None, None, None, None, None, None, None) == -1
    assert lib.etac_contact_mesh(None, None, C.byref(sc), None, None, None, None, None) == -1
    assert lib.etac_contact_mesh_backward(None, None, C.byref(sc), None, None, None, None, None, None) == -1
    assert lib.etac_meshset_destroy(None) == 0
    assert lib.etac_plan_destroy(None) == 0
    assert lib.etac_plan_info(None, None, None, None) == -1
    assert lib.etac_plan_set_occupancy(None, 1) == -1
    assert lib.etac_plan_set_timing(None, 1) == -1
    assert lib.etac_plan_set_batch(None, 4) == -1
    assert lib.etac_plan_set_launch(None, 0, 0, 0, 0, 0) == -1
    assert lib.etac_plan_get_launch(None, None) == -1
    assert lib.etac_plan_autotune(None, None, None, None, None, None, None, None, None, None, None, None, 1,
                                  None, None) == -1
    n, ms = C.c_int32(), C.c_double()
    assert lib.etac_plan_kernel_time(None, 0, C.byref(n), C.byref(ms)) == -1
    assert lib.etac_regress(None, None, 0, None, None, None, None) == -1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_native, "_lib", None)
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "libetac.so"))
    with pytest.raises(ImportError):
        _native.lib()


def test_meshset_validation_without_gpu():
    """Mesh-set arguments are checked on the host before any device call."""
    from scenes import trimeshes as tm
    lib = _native.lib()
    ms = tm.merge([tm.cube_mesh(half=4.0, n=1)], ("cube",))
    v, t, off = ms.verts.copy(), ms.tris.copy(), ms.tri_offset.copy()

    def create(v, t, off, M=None):
        h = C.c_void_p()
        M = off.size - 1 if M is None else M
        return lib.etac_meshset_create(M, off.ctypes.data, v.shape[0], v.ctypes.data, t.ctypes.data, C.byref(h))

    assert lib.etac_meshset_create(1, None, 3, None, None, None) == -1
    assert create(v, t, off, M=0) == -2
    assert create(v, t, off, M=4097) == -2                                     # more meshes than the grids allow
    assert create(v, t, np.array([1, 12], np.int32)) == -2                    # offsets must start at 0
    assert create(v, t[:3], np.array([0, 3], np.int32)) == -2                 # fewer than 4 triangles
    bad = t.copy(); bad[0, 0] = v.shape[0]
    assert create(v, bad, off) == -3                                          # vertex index out of range
    vn = v.copy(); vn[0, 0] = np.nan
    assert create(vn, t, off) == -3                                           # non-finite vertex
    assert create(v, np.ascontiguousarray(t[1:]), np.array([0, 11], np.int32)) == -3   # open mesh
    flip = t.copy(); flip[0] = flip[0, [0, 2, 1]]
    assert create(v, flip, off) == -3                                         # inconsistent orientation
    deg = t.copy(); deg[0, 2] = deg[0, 1]
    assert create(v, deg, off) == -3                                          # repeated vertex


def test_regressor_constants_match_the_layer_table():
    """The C ABI's regressor sizes and the benchmark's flop accounting follow
    the packed layer table the oracle and the input generator use."""
    import bench
    import scenes
    sizes = {name: o * i for name, o, i in scenes.REG_LAYERS}
    assert _native.ETAC_REG_SIZE == scenes.REG_SIZE == sum(sizes.values())
    assert _native.ETAC_TAXELS == dict((n, o) for n, o, _ in scenes.REG_LAYERS)["d2"]
    assert bench.REG_NODE_MAC == sizes["E1"] + sizes["E2"] + sizes["E3"] + sizes["A1"]
    assert bench.REG_HEAD_MAC == sizes["D1"] + sizes["D2"]
