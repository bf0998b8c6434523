"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol include/dp.h declares, and rejects bad arguments in the host
validation that runs before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2410_22867_amd import dpse, inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "dp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = dpse.lib()
    names = _header_functions()
    assert len(names) >= 16
    assert set(names) == set(dpse.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_n_params_matches_layout():
    assert dpse.n_params(I.WATER) == I.WATER.n_params
    assert dpse.n_params(I.COPPER) == I.COPPER.n_params


def _create(desc, params):
    c = dpse.make_desc(desc)
    h = ctypes.c_void_p()
    p = np.ascontiguousarray(params, dtype=np.float64)
    rc = dpse.lib().dp_model_create(ctypes.byref(c), p.ctypes.data, p.size, ctypes.byref(h))
    return rc, dpse.lib().dp_last_error().decode()


def test_model_create_validation_before_gpu():
    import dataclasses
    p = I.init_params(I.WATER, 1)
    rc, msg = _create(dataclasses.replace(I.WATER, ntypes=0, sel=()), p)
    assert rc == -1 and "ntypes" in msg
    rc, msg = _create(dataclasses.replace(I.WATER, emb=(20, 40, 80)), p)
    assert rc == -2 and "embedding" in msg
    rc, msg = _create(dataclasses.replace(I.WATER, fit=(240, 120, 240)), p)
    assert rc == -2
    rc, msg = _create(dataclasses.replace(I.WATER, rcut_smth=7.0), p)
    assert rc == -1 and "rcut" in msg
    rc, msg = _create(I.WATER, p[:-1])
    assert rc == -1 and "params" in msg
    q = p.copy()
    q[5] = np.nan
    rc, msg = _create(I.WATER, q)
    assert rc == -1 and "finite" in msg


def test_null_arguments_rejected():
    L = dpse.lib()
    h = ctypes.c_void_p()
    assert L.dp_ctx_create(None, 10, 1, 0, ctypes.byref(h)) == -1
    assert L.dp_compute(None, None, None, None, 0, None, 0, None, None, None, None, None) == -1
    assert L.dp_build_nlist(None, None, None, None, -1, None, None, None) == -1
    f = ctypes.c_int32(0)
    assert L.dp_ctx_status(None, ctypes.byref(f)) == -1
    cap, used = ctypes.c_int64(0), ctypes.c_int32(0)
    assert L.dp_ctx_store_info(None, ctypes.byref(cap), ctypes.byref(used)) == -1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library every entry point raises: there is no CPU
    fallback behind the binding."""
    monkeypatch.setattr(dpse, "LIB_PATH", str(tmp_path / "libdpse.so"))
    monkeypatch.setattr(dpse, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        dpse.lib()
    fr, desc, p, dt = I.workload("water192")
    with pytest.raises(RuntimeError, match="not built"):
        dpse.Model(desc, p)


def _body(src, name):
    i = src.index(name + "(")
    i = src.index("{", i)
    depth, j = 0, i
    while True:
        if src[j] == "{":
            depth += 1
        elif src[j] == "}":
            depth -= 1
            if depth == 0:
                return src[i:j + 1]
        j += 1


def test_parameter_updates_allocate_nothing():
    """Both parameter-update entry points, and the gathers they run, call no
    allocator and do not wait for the whole device (static check of the
    source: the calls need a GPU to run)."""
    src = open(os.path.join(ROOT, "paper_2410_22867_amd", "csrc", "dp_api.cpp")).read()
    for fn in ("int dp_model_set_params", "int dp_model_set_params_device", "void gather_all"):
        body = _body(src, fn)
        for bad in ("hipMalloc", "hipFree", "hipDeviceSynchronize", "dev_alloc", "build_maps", "new ", "malloc"):
            assert bad not in body, (fn, bad)
