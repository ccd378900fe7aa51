"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/mgr.h declares, and rejects bad arguments before touching a
device."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2105_12764_amd import mgr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mgr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mgr_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert {"mgr_decompose", "mgr_recompose", "mgr_workspace_size", "mgr_max_levels"} <= set(names)
    L = mgr.lib()
    for n in names:
        assert hasattr(L, n), n


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(mgr, "_lib", None)
    monkeypatch.setattr(mgr, "LIB_PATH", "/nonexistent/libmgr.so")
    with pytest.raises(RuntimeError):
        mgr.lib()


@pytest.mark.parametrize("shape", [(513, 513, 513), (65, 65, 65), (400, 300, 250), (2, 2, 2),
                                   (3,), (1000,), (129, 70), (5, 2, 9), (2, 1025),
                                   (16, 65, 65, 65), (65, 9, 9, 5), (2, 2, 2, 2), (3, 2, 2, 2)])
def test_max_levels_matches_oracle(shape):
    assert mgr.max_levels(shape) == oracle.max_levels(shape)


def test_workspace_size():
    assert mgr.workspace_size((513, 513, 513), np.float64, 0) == 0
    n1, n2 = 257 ** 3, 129 ** 3
    al = lambda b: (b + 255) // 256 * 256
    # three FP64 level-1 grids (level grids and load vector; FP64 for FP32
    # fields too) and (two or more levels) an FP64 level-2 grid
    assert mgr.workspace_size((513, 513, 513), np.float64, 9) == 3 * al(8 * n1) + al(8 * n2)
    assert mgr.workspace_size((513, 513, 513), np.float32, 9) == 3 * al(8 * n1) + al(8 * n2)
    assert mgr.workspace_size((513, 513, 513), np.float32, 1) == 3 * al(8 * n1)
    with pytest.raises(mgr.MgrError):
        mgr.workspace_size((513, 513, 513), np.float64, 10)
    # 4-D: two FP64 coarse 4-D level grids, the FP64 coarse grid and the FP64
    # load vectors of every time slice
    cs, ct = 201 ** 3, 9
    assert mgr.workspace_size((16, 401, 401, 401), np.float32, 8) == \
        3 * al(8 * ct * cs) + al(8 * 16 * cs)
    assert mgr.workspace_size((16, 401, 401, 401), np.float32, 0) == 0
    with pytest.raises(mgr.MgrError):
        mgr.workspace_size((16, 401, 401, 401), np.float32, 10)


def _call(shape=(5, 5, 5), coords=None, dtype=mgr.MGR_FLOAT64, nlev=2, inp=4096,
          out=1 << 20, ws=1 << 24, wsb=1 << 24, fn="mgr_decompose"):
    L = mgr.lib()
    carr = None
    keep = []
    if coords is not None:
        dp = ctypes.POINTER(ctypes.c_double)
        carr = (dp * len(coords))()
        for k, c in enumerate(coords):
            c = np.ascontiguousarray(c, dtype=np.float64)
            keep.append(c)
            carr[k] = c.ctypes.data_as(dp)
    nd = len(shape) if shape is not None else 3
    sh = mgr._shape(shape) if shape is not None else None
    return getattr(L, fn)(nd, sh, carr, dtype, nlev, ctypes.c_void_p(inp), ctypes.c_void_p(out),
                          ctypes.c_void_p(ws), ctypes.c_size_t(wsb), None)


@pytest.mark.parametrize("fn", ["mgr_decompose", "mgr_recompose"])
def test_invalid_arguments_are_rejected_before_any_device_call(fn):
    E = mgr.MGR_ERR_INVALID_ARG
    assert _call(shape=(5, 5, 5, 5, 5), fn=fn) == E
    assert _call(shape=(5, 1, 5), fn=fn) == E
    # 4-D (time, then space): rejected shapes and level counts, all before any device call
    assert _call(shape=(1, 5, 5, 5), fn=fn) == E
    assert _call(shape=(5, 5, 1, 5), fn=fn) == E
    assert _call(shape=(5, 5, 5, 5), nlev=3, fn=fn) == E
    assert _call(shape=(5, 5, 5, 5), nlev=2, ws=0, fn=fn) == mgr.MGR_ERR_WORKSPACE
    assert _call(nlev=3, fn=fn) == E
    assert _call(nlev=-1, fn=fn) == E
    assert _call(dtype=7, fn=fn) == E
    assert _call(inp=0, fn=fn) == E
    assert _call(out=0, fn=fn) == E
    assert _call(out=4096 + 8, fn=fn) == E  # overlaps in
    bad = [np.arange(5.0), np.array([0, 1, 1, 2, 3.0]), np.arange(5.0)]
    assert _call(coords=bad, fn=fn) == E
    nan = [np.arange(5.0), np.array([0, 1, np.nan, 2, 3.0]), np.arange(5.0)]
    assert _call(coords=nan, fn=fn) == E
    assert _call(ws=0, fn=fn) == mgr.MGR_ERR_WORKSPACE
    assert _call(wsb=16, fn=fn) == mgr.MGR_ERR_WORKSPACE
    assert _call(ws=(1 << 24) + 8, fn=fn) == E  # misaligned workspace
    assert _call(ws=4096, fn=fn) == E          # workspace overlaps in
    assert mgr.last_error() != ""


def test_status_strings():
    for s in range(6):
        assert mgr.status_string(s)
    assert mgr.status_string(0) == "ok"


def _fields(specs):
    """ctypes mgr_field array from (shape, dtype code, nlevels, in address, out address)."""
    arr = (mgr.MgrField * len(specs))()
    for i, (shape, dt, nl, inp, out) in enumerate(specs):
        arr[i].ndim = len(shape)
        for k, v in enumerate(shape):
            arr[i].shape[k] = v
        arr[i].coords = None
        arr[i].dtype = dt
        arr[i].nlevels = nl
        arr[i].in_ = inp
        arr[i].out = out
    return arr


def test_batch_workspace_is_the_aligned_sum_of_the_fields():
    specs = [((33, 33, 33), mgr.MGR_FLOAT64, 4, 1 << 30, 2 << 30),
             ((300, 41), mgr.MGR_FLOAT32, 3, 3 << 30, 4 << 30),
             ((9, 9, 9), mgr.MGR_FLOAT64, 0, 5 << 30, 6 << 30)]
    al = lambda b: (b + 255) // 256 * 256
    want = sum(al(mgr.workspace_size(s, np.float64 if d == mgr.MGR_FLOAT64 else np.float32, n))
               for s, d, n, _, _ in specs)
    out = ctypes.c_size_t(0)
    assert mgr.lib().mgr_batch_workspace_size(3, _fields(specs), ctypes.byref(out)) == mgr.MGR_OK
    assert out.value == want


@pytest.mark.parametrize("fn", ["mgr_decompose_batch", "mgr_recompose_batch"])
def test_batch_rejects_bad_fields_before_any_device_call(fn):
    L = mgr.lib()
    E = mgr.MGR_ERR_INVALID_ARG
    ok = ((9, 9, 9), mgr.MGR_FLOAT64, 2, 1 << 30, 2 << 30)
    call = lambda specs, ws=1 << 34, wsb=1 << 30: getattr(L, fn)(
        len(specs), _fields(specs), ctypes.c_void_p(ws), ctypes.c_size_t(wsb), None)
    assert getattr(L, fn)(0, _fields([ok]), ctypes.c_void_p(1 << 34), ctypes.c_size_t(1 << 30), None) == E
    assert getattr(L, fn)(1, None, ctypes.c_void_p(1 << 34), ctypes.c_size_t(1 << 30), None) == E
    # the detail names the failing field
    bad_shape = ((9, 1, 9), mgr.MGR_FLOAT64, 1, 3 << 30, 4 << 30)
    assert call([ok, ok[:3] + (5 << 30, 6 << 30), bad_shape]) == E
    assert mgr.last_error().startswith("field 2:")
    bad_levels = ((9, 9, 9), mgr.MGR_FLOAT64, 9, 3 << 30, 4 << 30)
    assert call([ok, bad_levels]) == E and mgr.last_error().startswith("field 1:")
    # one field's out overlapping another field's in or out
    clash = ((9, 9, 9), mgr.MGR_FLOAT64, 2, 3 << 30, (2 << 30) + 64)
    assert call([ok, clash]) == E and "overlaps" in mgr.last_error()
    clash_in = ((9, 9, 9), mgr.MGR_FLOAT64, 2, 3 << 30, (1 << 30) + 8)  # its out over field 1's in
    assert call([clash_in, ok]) == E and "overlaps" in mgr.last_error()
    # workspace too small, or overlapping a field
    assert call([ok], wsb=16) == mgr.MGR_ERR_WORKSPACE
    assert call([ok], ws=(1 << 30)) == E


def test_partial_recompose_rejects_nkeep_out_of_range():
    L = mgr.lib()
    sh = mgr._shape((9, 9, 9))
    for nkeep in (-1, 3):
        s = L.mgr_recompose_partial(3, sh, None, mgr.MGR_FLOAT64, 2, nkeep, ctypes.c_void_p(1 << 30),
                                    ctypes.c_void_p(2 << 30), ctypes.c_void_p(1 << 34),
                                    ctypes.c_size_t(1 << 30), None)
        assert s == mgr.MGR_ERR_INVALID_ARG
        assert "nkeep" in mgr.last_error()


@pytest.mark.parametrize("shape", [(513, 513, 513), (66, 70, 45), (300, 41), (1000,), (2, 2, 2), (5, 2, 9)])
def test_class_sizes_follow_the_level_grids(shape):
    nlev = mgr.max_levels(shape)
    sizes = mgr.class_sizes(shape, nlev)
    assert sum(sizes) == int(np.prod(shape))
    # level grids from the coarsening rule written out here: even positions and the last
    dims = [list(range(n)) for n in shape]
    grids = []
    for _ in range(nlev + 1):
        grids.append(int(np.prod([len(d) for d in dims])))
        dims = [[p for i, p in enumerate(d) if i % 2 == 0 or i == len(d) - 1] if len(d) >= 3 else d
                for d in dims]
    assert sizes[0] == grids[nlev]
    assert sizes[1:] == [grids[s] - grids[s + 1] for s in range(nlev - 1, -1, -1)]
    with pytest.raises(mgr.MgrError):
        mgr.class_sizes(shape, nlev + 1)


def test_class_export_rejects_bad_arguments_without_a_device():
    L = mgr.lib()
    sh = mgr._shape((9, 9, 9))
    E = mgr.MGR_ERR_INVALID_ARG
    for fn in (L.mgr_export_classes, L.mgr_import_classes):
        assert fn(3, sh, mgr.MGR_FLOAT64, 4, ctypes.c_void_p(1 << 30), ctypes.c_void_p(2 << 30), None) == E
        assert fn(3, sh, 5, 2, ctypes.c_void_p(1 << 30), ctypes.c_void_p(2 << 30), None) == E
        assert fn(3, sh, mgr.MGR_FLOAT64, 2, ctypes.c_void_p(1 << 30), ctypes.c_void_p((1 << 30) + 8), None) == E
        assert fn(3, sh, mgr.MGR_FLOAT64, 2, None, ctypes.c_void_p(2 << 30), None) == E


def test_service_rejects_bad_arguments_without_a_device():
    L = mgr.lib()
    h = ctypes.c_void_p()
    E = mgr.MGR_ERR_INVALID_ARG
    assert L.mgr_service_create(ctypes.c_size_t(16), 2, ctypes.byref(h)) == E
    assert L.mgr_service_create(ctypes.c_size_t(1 << 30), 0, ctypes.byref(h)) == E
    assert L.mgr_service_create(ctypes.c_size_t(1 << 30), 17, ctypes.byref(h)) == E
    assert L.mgr_service_create(ctypes.c_size_t(1 << 30), 2, None) == E
    t = ctypes.c_uint64()
    assert L.mgr_service_submit(None, 0, 3, mgr._shape((9, 9, 9)), None, mgr.MGR_FLOAT64, 2,
                                ctypes.c_void_p(1), ctypes.c_void_p(2), ctypes.byref(t)) == E
    assert L.mgr_service_wait_all(None) == E
    assert L.mgr_service_destroy(None) == mgr.MGR_OK


def test_binding_rejects_mismatched_outputs_before_the_library():
    """The C ABI takes raw pointers, so the binding checks that `out` can hold
    what the library writes (no device needed: CPU tensors are rejected
    first, and a mismatched `out` is rejected before any pointer is passed)."""
    import torch

    x = torch.zeros((5, 5, 5), dtype=torch.float64)
    with pytest.raises(ValueError):
        mgr.decompose(x)
    with pytest.raises(ValueError):
        mgr._check_pair(x, torch.zeros((5, 5, 5), dtype=torch.float64))


def _noalloc(shape, nlev, dtype=mgr.MGR_FLOAT64):
    L = mgr.lib()
    return L.mgr_decompose_noalloc(len(shape), mgr._shape(shape), None, dtype, nlev, ctypes.c_void_p(4096),
                                   ctypes.c_void_p(1 << 30), None)


def test_noalloc_limits_are_checked_before_any_device_call():
    # 513^3 FP64 needs 425 MB of workspace, beyond the static scratch: rejected
    # with the size in the message, before the library touches a device
    need = mgr.workspace_size((513, 513, 513), np.float64, 9)
    assert need > mgr.MGR_NOALLOC_SCRATCH_BYTES - mgr.MGR_NOALLOC_TABLE_BYTES
    assert _noalloc((513, 513, 513), 9) == mgr.MGR_ERR_WORKSPACE
    assert str(need) in mgr.last_error()
    # a single level of 513^3 needs three FP64 257^3 grids (408 MB): also too large
    assert _noalloc((513, 513, 513), 1, mgr.MGR_FLOAT32) == mgr.MGR_ERR_WORKSPACE
    assert _noalloc((9, 9, 9, 9), 1) == mgr.MGR_ERR_UNSUPPORTED
    assert _noalloc((9, 9, 9), 5) == mgr.MGR_ERR_INVALID_ARG
    assert _noalloc((1, 9, 9), 1) == mgr.MGR_ERR_INVALID_ARG
    # the largest cube that fits with all levels, FP64
    assert mgr.workspace_size((257, 257, 257), np.float64, 8) <= \
        mgr.MGR_NOALLOC_SCRATCH_BYTES - mgr.MGR_NOALLOC_TABLE_BYTES


def test_noalloc_limits_match_the_header():
    txt = open(os.path.join(ROOT, "include", "mgr.h")).read()
    assert re.search(r"#define MGR_NOALLOC_SCRATCH_BYTES \(64u << 20\)", txt)
    assert re.search(r"#define MGR_NOALLOC_TABLE_BYTES \(4u << 20\)", txt)
    assert mgr.MGR_NOALLOC_SCRATCH_BYTES == 64 << 20 and mgr.MGR_NOALLOC_TABLE_BYTES == 4 << 20


@pytest.mark.parametrize("fn", ["mgr_decompose_batch_ex", "mgr_recompose_batch_ex"])
def test_batch_ex_rejects_unknown_flags_before_any_device_call(fn):
    L = mgr.lib()
    ok = ((9, 9, 9), mgr.MGR_FLOAT64, 2, 1 << 30, 2 << 30)
    for flags in (2, 4, -1, 1 << 30):
        assert getattr(L, fn)(1, _fields([ok]), ctypes.c_void_p(1 << 34), ctypes.c_size_t(1 << 30), None,
                              flags) == mgr.MGR_ERR_INVALID_ARG
        assert "flags" in mgr.last_error()
    # valid flags still validate the fields first
    bad = ((9, 1, 9), mgr.MGR_FLOAT64, 1, 3 << 30, 4 << 30)
    for flags in (0, mgr.MGR_BATCH_PER_FIELD):
        assert getattr(L, fn)(1, _fields([bad]), ctypes.c_void_p(1 << 34), ctypes.c_size_t(1 << 30), None,
                              flags) == mgr.MGR_ERR_INVALID_ARG
