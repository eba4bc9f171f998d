"""C-ABI checks that need no GPU: the library loads, exports every function
include/lod.h declares, and rejects bad arguments before enqueueing work."""
import ctypes as C
import os
import re

import pytest

from paper_0811_2055_amd import lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lod.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:lod_status|const char \*)\s*(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    L = lib.load()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(lib.EXPORTS)


def test_status_strings():
    for code in range(0, -7, -1):
        assert lib.status_string(code) not in ("", "unknown status")
    assert lib.status_string(-99) == "unknown status"


def _plan(N, **kw):
    return lib.build_plan(N, lib.BuildParams(**kw))


def test_plan_bounds():
    ws, nc, pc = _plan(262144, n=4096, max_depth=4)
    per = 262144 // 4097
    assert nc == 1 + 8 * 4 * per and pc == 262144 + 4096 * 4 * per and ws > 40 * 262144
    ws0, nc0, pc0 = _plan(0, n=4, max_depth=3)
    assert nc0 >= 1 and pc0 >= 1
    # batch: bounds count every snapshot's root
    ws, nc, pc = lib.build_plan(1000, lib.BuildParams(n=10, max_depth=3), n_snapshots=5)
    assert nc == 5 + 8 * 3 * (1000 // 11)


@pytest.mark.parametrize("kw,code", [
    (dict(n=0, max_depth=3), lib.LOD_EINVAL),
    (dict(n=4, max_depth=11), lib.LOD_EINVAL),
    (dict(n=4, max_depth=3, density_level=4), lib.LOD_EINVAL),
    (dict(n=4, max_depth=3, alpha=2), lib.LOD_EINVAL),
    (dict(n=4, max_depth=3, mode=7), lib.LOD_EINVAL),
    (dict(n=4, max_depth=3, select_threads=100), lib.LOD_EINVAL),
])
def test_plan_rejects_bad_parameters(kw, code):
    with pytest.raises(lib.LodError) as e:
        _plan(100, **kw)
    assert e.value.code == code


def test_plan_rejects_oversized_keys_and_counts():
    with pytest.raises(lib.LodError) as e:
        lib.build_plan(1000, lib.BuildParams(n=4, max_depth=10), n_snapshots=8)   # 30 + 3 bits
    assert e.value.code == lib.LOD_EUNSUPPORTED
    with pytest.raises(lib.LodError) as e:
        _plan(1 << 31, n=4, max_depth=3)
    assert e.value.code == lib.LOD_EUNSUPPORTED


def test_build_rejects_null_arrays_without_device_work():
    L = lib.load()
    p = lib.BuildParams(n=4, max_depth=3).c()
    inp = lib.Input(None, None, None, None, 10, None, 1)
    tree = lib.TreeC()
    ws = C.create_string_buffer(1 << 12)
    code = L.lod_build(C.byref(inp), C.byref(p), C.cast(ws, C.c_void_p), 1 << 12, C.byref(tree), None)
    assert code == lib.LOD_EINVAL


def test_splat_plan_validation():
    cam = lib.Camera.ortho(256, 256)
    assert lib.splat_workspace_bytes(1000, cam) > 0
    with pytest.raises(lib.LodError):
        lib.splat_workspace_bytes(1000, cam, sigma=0.0)
    with pytest.raises(lib.LodError):
        lib.splat_workspace_bytes(1000, cam, radius_sigmas=7.0)
    with pytest.raises(lib.LodError) as e:
        lib.splat_workspace_bytes(1000, lib.Camera.ortho(4096, 4096))    # too many tiles
    assert e.value.code == lib.LOD_EUNSUPPORTED
    bad = lib.Camera(1, 64, 64, F=-1.0)
    with pytest.raises(lib.LodError):
        lib.splat_workspace_bytes(10, bad)
