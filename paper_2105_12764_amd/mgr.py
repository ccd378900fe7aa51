"""Python binding of libmgr (include/mgr.h): argument marshalling only.

Every step of the refactoring runs in the HIP library; this module turns
PyTorch tensors into device pointers, passes the current HIP stream and maps
status codes to exceptions.  PyTorch provides device memory and streams only.
The library must be built (``paper_2105_12764_amd.build``); there is no CPU
fallback and a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmgr.so")

MGR_OK = 0
MGR_ERR_INVALID_ARG = 1
MGR_ERR_UNSUPPORTED = 2
MGR_ERR_WORKSPACE = 3
MGR_ERR_OUT_OF_MEMORY = 4
MGR_ERR_DEVICE = 5

MGR_FLOAT32 = 0
MGR_FLOAT64 = 1

MGR_BATCH_STREAMS = 4
MGR_BATCH_PER_FIELD = 1
# static device scratch of mgr_decompose_noalloc (include/mgr.h)
MGR_NOALLOC_SCRATCH_BYTES = 64 << 20
MGR_NOALLOC_TABLE_BYTES = 4 << 20

_lib = None


class MgrField(ctypes.Structure):
    """Mirror of ``mgr_field`` (include/mgr.h)."""
    _fields_ = [("ndim", ctypes.c_int),
                ("shape", ctypes.c_int64 * 3),
                ("coords", ctypes.c_void_p),
                ("dtype", ctypes.c_int),
                ("nlevels", ctypes.c_int),
                ("in_", ctypes.c_void_p),
                ("out", ctypes.c_void_p)]


class MgrError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{status_string(status)} ({status}): {detail}")


def lib() -> ctypes.CDLL:
    """The loaded libmgr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_2105_12764_amd.build.build() "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dpp = ctypes.POINTER(ctypes.POINTER(ctypes.c_double))
        L.mgr_max_levels.argtypes = [ctypes.c_int, i64p]
        L.mgr_max_levels.restype = ctypes.c_int
        L.mgr_workspace_size.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_size_t)]
        L.mgr_workspace_size.restype = ctypes.c_int
        for fn in (L.mgr_decompose, L.mgr_recompose):
            fn.argtypes = [ctypes.c_int, i64p, dpp, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
            fn.restype = ctypes.c_int
        L.mgr_decompose_noalloc.argtypes = [ctypes.c_int, i64p, dpp, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.mgr_decompose_noalloc.restype = ctypes.c_int
        L.mgr_status_string.argtypes = [ctypes.c_int]
        L.mgr_status_string.restype = ctypes.c_char_p
        L.mgr_last_error.argtypes = []
        L.mgr_last_error.restype = ctypes.c_char_p
        L.mgr_release_caches.argtypes = []
        L.mgr_release_caches.restype = None
        vp = ctypes.c_void_p
        L.mgr_service_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(vp)]
        L.mgr_service_create.restype = ctypes.c_int
        L.mgr_service_submit.argtypes = [vp, ctypes.c_int, ctypes.c_int, i64p, dpp, ctypes.c_int, ctypes.c_int,
                                         vp, vp, ctypes.POINTER(ctypes.c_uint64)]
        L.mgr_service_submit.restype = ctypes.c_int
        L.mgr_service_wait_all.argtypes = [vp]
        L.mgr_service_wait_all.restype = ctypes.c_int
        L.mgr_service_result.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
        L.mgr_service_result.restype = ctypes.c_int
        L.mgr_service_destroy.argtypes = [vp]
        L.mgr_service_destroy.restype = ctypes.c_int
        L.mgr_service_last_error.argtypes = []
        L.mgr_service_last_error.restype = ctypes.c_char_p
        L.mgr_recompose_partial.argtypes = [ctypes.c_int, i64p, dpp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.c_void_p]
        L.mgr_recompose_partial.restype = ctypes.c_int
        L.mgr_class_sizes.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i64p]
        L.mgr_class_sizes.restype = ctypes.c_int
        for fn in (L.mgr_export_classes, L.mgr_import_classes):
            fn.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_void_p]
            fn.restype = ctypes.c_int
        L.mgr_autotune.argtypes = [ctypes.c_int, i64p, dpp, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.mgr_autotune.restype = ctypes.c_int
        L.mgr_autotune_report.argtypes = []
        L.mgr_autotune_report.restype = ctypes.c_char_p
        fp = ctypes.POINTER(MgrField)
        L.mgr_batch_workspace_size.argtypes = [ctypes.c_int, fp, ctypes.POINTER(ctypes.c_size_t)]
        L.mgr_batch_workspace_size.restype = ctypes.c_int
        for fn in (L.mgr_decompose_batch, L.mgr_recompose_batch):
            fn.argtypes = [ctypes.c_int, fp, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
            fn.restype = ctypes.c_int
        for fn in (L.mgr_decompose_batch_ex, L.mgr_recompose_batch_ex):
            fn.argtypes = [ctypes.c_int, fp, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int]
            fn.restype = ctypes.c_int
        L.mgr_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p]
        L.mgr_probe_copy.restype = ctypes.c_int
        L.mgr_timing_enable.argtypes = [ctypes.c_int]
        L.mgr_timing_enable.restype = ctypes.c_int
        L.mgr_timing_reset.argtypes = []
        L.mgr_timing_reset.restype = None
        L.mgr_timing_count.argtypes = []
        L.mgr_timing_count.restype = ctypes.c_int
        L.mgr_timing_get.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
        L.mgr_timing_get.restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().mgr_status_string(int(s)).decode()


def last_error() -> str:
    return lib().mgr_last_error().decode()


def _shape(shape: Sequence[int]):
    return (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])


def max_levels(shape: Sequence[int]) -> int:
    r = lib().mgr_max_levels(len(shape), _shape(shape))
    if r < 0:
        raise MgrError(-r, last_error())
    return r


def _dtype_code(dtype) -> int:
    import torch
    if dtype in (torch.float64, np.float64):
        return MGR_FLOAT64
    if dtype in (torch.float32, np.float32):
        return MGR_FLOAT32
    raise ValueError(f"unsupported dtype {dtype}")


def workspace_size(shape: Sequence[int], dtype, nlevels: int) -> int:
    out = ctypes.c_size_t(0)
    s = lib().mgr_workspace_size(len(shape), _shape(shape), _dtype_code(dtype), int(nlevels),
                                 ctypes.byref(out))
    if s != MGR_OK:
        raise MgrError(s, last_error())
    return int(out.value)


def _coords_arg(shape, coords):
    if coords is None:
        return None, []
    if len(coords) != len(shape):
        raise ValueError("coords needs one entry per dimension")
    dp = ctypes.POINTER(ctypes.c_double)
    arr = (dp * len(shape))()
    keep = []
    for k, c in enumerate(coords):
        if c is None:
            arr[k] = dp()
            continue
        c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        if c.shape != (shape[k],):
            raise ValueError(f"coords[{k}] must have shape ({shape[k]},)")
        keep.append(c)
        arr[k] = c.ctypes.data_as(dp)
    return arr, keep


def _check_pair(x, out):
    """The library takes raw pointers: make sure `out` can hold what it writes."""
    if not (x.is_cuda and x.is_contiguous()):
        raise ValueError("input must be a contiguous (C order) HIP device tensor")
    if not (out.is_cuda and out.is_contiguous()):
        raise ValueError("out must be a contiguous (C order) HIP device tensor")
    if out.shape != x.shape or out.dtype != x.dtype or out.device != x.device:
        raise ValueError("out must match the input in shape, dtype and device")


def _workspace_bytes(ws, device) -> int:
    if not (ws.is_cuda and ws.is_contiguous() and ws.device == device):
        raise ValueError("workspace must be a contiguous HIP tensor on the input's device")
    return ws.numel() * ws.element_size()


def alloc_workspace(shape, dtype, nlevels, device=None):
    import torch
    nb = workspace_size(shape, dtype, nlevels)
    return torch.empty(max(nb, 1), dtype=torch.uint8, device=device or "cuda")


def _on_stream(made, stream, device) -> None:
    """Tensors the binding allocated come from the current stream's pool of
    PyTorch's caching allocator.  When the library's work runs on another
    stream, record that stream on them, so that their blocks are not handed
    out again before that work is done."""
    import torch
    if not made:
        return
    if not isinstance(stream, torch.cuda.Stream):  # a raw handle wrapper (any object with .cuda_stream)
        stream = torch.cuda.ExternalStream(stream.cuda_stream, device=device)
    if stream != torch.cuda.current_stream(device):
        for t in made:
            t.record_stream(stream)


def _call(fn, x, coords, nlevels, out, workspace, stream):
    import torch
    if not (x.is_cuda and x.is_contiguous()):
        raise ValueError("input must be a contiguous (C order) HIP device tensor")
    shape = tuple(x.shape)
    if nlevels is None:
        nlevels = max_levels(shape)
    made = []
    if out is None:
        out = torch.empty_like(x)
        made.append(out)
    _check_pair(x, out)
    if workspace is None:
        workspace = alloc_workspace(shape, x.dtype, nlevels, device=x.device)
        made.append(workspace)
    wsb = _workspace_bytes(workspace, x.device)
    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    carr, keep = _coords_arg(shape, coords)
    with torch.cuda.device(x.device):
        s = fn(len(shape), _shape(shape), carr, _dtype_code(x.dtype), int(nlevels),
               ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
               ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(wsb),
               ctypes.c_void_p(stream.cuda_stream))
    del keep
    if s != MGR_OK:
        raise MgrError(s, last_error())
    _on_stream(made, stream, x.device)
    return out


def decompose(x, coords=None, nlevels: Optional[int] = None, out=None, workspace=None, stream=None):
    """mgr_decompose on a contiguous float32/float64 HIP tensor; returns ``out``."""
    return _call(lib().mgr_decompose, x, coords, nlevels, out, workspace, stream)


def recompose(x, coords=None, nlevels: Optional[int] = None, out=None, workspace=None, stream=None):
    """mgr_recompose (inverse of :func:`decompose`); returns ``out``."""
    return _call(lib().mgr_recompose, x, coords, nlevels, out, workspace, stream)


def decompose_noalloc(x, coords=None, nlevels: Optional[int] = None, out=None, stream=None):
    """mgr_decompose_noalloc: the decomposition with its workspace and plan
    tables in the library's static device scratch (no device allocation in
    the library; `out` is allocated here only when not given)."""
    import torch
    if not (x.is_cuda and x.is_contiguous()):
        raise ValueError("input must be a contiguous (C order) HIP device tensor")
    shape = tuple(x.shape)
    if nlevels is None:
        nlevels = max_levels(shape)
    made = []
    if out is None:
        out = torch.empty_like(x)
        made.append(out)
    _check_pair(x, out)
    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    carr, keep = _coords_arg(shape, coords)
    with torch.cuda.device(x.device):
        s = lib().mgr_decompose_noalloc(len(shape), _shape(shape), carr, _dtype_code(x.dtype), int(nlevels),
                                        ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(stream.cuda_stream))
    del keep
    if s != MGR_OK:
        raise MgrError(s, last_error())
    _on_stream(made, stream, x.device)
    return out


class Batch:
    """Descriptors of a batch of independent fields for the batched entry points.

    ``items`` is a sequence of ``(in_tensor, out_tensor, coords, nlevels)``;
    coords may be None (uniform) and nlevels None (all levels).  The object
    keeps the coordinate arrays alive for the calls.
    """

    def __init__(self, items):
        n = len(items)
        self.fields = (MgrField * n)()
        self._keep = []
        self.tensors = []
        for i, (x, y, coords, nlevels) in enumerate(items):
            if not (x.is_cuda and y.is_cuda and x.is_contiguous() and y.is_contiguous()):
                raise ValueError(f"field {i}: in and out must be contiguous HIP tensors")
            if x.shape != y.shape or x.dtype != y.dtype or x.device != y.device:
                raise ValueError(f"field {i}: in and out must match in shape, dtype and device")
            shape = tuple(x.shape)
            f = self.fields[i]
            f.ndim = len(shape)
            for k, v in enumerate(shape):
                f.shape[k] = int(v)
            carr, keep = _coords_arg(shape, coords)
            self._keep.append((carr, keep))
            f.coords = ctypes.cast(carr, ctypes.c_void_p) if carr is not None else None
            f.dtype = _dtype_code(x.dtype)
            f.nlevels = int(max_levels(shape) if nlevels is None else nlevels)
            f.in_ = x.data_ptr()
            f.out = y.data_ptr()
            self.tensors.append((x, y))

    def __len__(self):
        return len(self.fields)

    def swapped(self):
        """The same fields with in and out exchanged (recompose what was decomposed)."""
        b = Batch.__new__(Batch)
        n = len(self.fields)
        b.fields = (MgrField * n)()
        ctypes.memmove(b.fields, self.fields, ctypes.sizeof(self.fields))
        for i in range(n):
            b.fields[i].in_, b.fields[i].out = self.fields[i].out, self.fields[i].in_
        b._keep = self._keep
        b.tensors = [(y, x) for (x, y) in self.tensors]
        return b

    def workspace_size(self) -> int:
        out = ctypes.c_size_t(0)
        s = lib().mgr_batch_workspace_size(len(self.fields), self.fields, ctypes.byref(out))
        if s != MGR_OK:
            raise MgrError(s, last_error())
        return int(out.value)

    def alloc_workspace(self, device=None):
        import torch
        return torch.empty(max(self.workspace_size(), 1), dtype=torch.uint8, device=device or "cuda")


def _call_batch(fn, batch: Batch, workspace, stream, flags: int = 0):
    import torch
    dev = batch.tensors[0][0].device
    made = []
    if workspace is None:
        workspace = batch.alloc_workspace(dev)
        made.append(workspace)
    wsb = _workspace_bytes(workspace, dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        s = fn(len(batch.fields), batch.fields, ctypes.c_void_p(workspace.data_ptr()),
               ctypes.c_size_t(wsb), ctypes.c_void_p(stream.cuda_stream), int(flags))
    if s != MGR_OK:
        raise MgrError(s, last_error())
    _on_stream(made, stream, dev)


def decompose_batch(batch: Batch, workspace=None, stream=None, per_field: bool = False) -> None:
    """mgr_decompose_batch_ex: every field's in decomposed into its out, with
    grouped launches (default) or each field's own launch chain on internal
    streams (per_field=True, MGR_BATCH_PER_FIELD)."""
    _call_batch(lib().mgr_decompose_batch_ex, batch, workspace, stream,
                MGR_BATCH_PER_FIELD if per_field else 0)


def recompose_batch(batch: Batch, workspace=None, stream=None, per_field: bool = False) -> None:
    """mgr_recompose_batch_ex: every field's in (a representation) recomposed
    into its out; launch modes as for :func:`decompose_batch`."""
    _call_batch(lib().mgr_recompose_batch_ex, batch, workspace, stream,
                MGR_BATCH_PER_FIELD if per_field else 0)


def recompose_partial(x, nkeep: int, coords=None, nlevels: Optional[int] = None, out=None, workspace=None,
                      stream=None):
    """mgr_recompose_partial: recompose from the coarsest values and the ``nkeep``
    coarsest coefficient classes (finer classes taken as zero)."""
    import torch
    if nlevels is None:
        nlevels = max_levels(tuple(x.shape))
    L = lib()

    def fn(nd, sh, carr, dt, nl, a, b, w, wb, st):
        return L.mgr_recompose_partial(nd, sh, carr, dt, nl, int(nkeep), a, b, w, wb, st)
    return _call(fn, x, coords, nlevels, out, workspace, stream)


def _classes(fn, x, nlevels, out, stream):
    import torch
    if not (x.is_cuda and x.is_contiguous()):
        raise ValueError("input must be a contiguous HIP tensor")
    shape = tuple(x.shape)
    if nlevels is None:
        nlevels = max_levels(shape)
    made = []
    if out is None:
        out = torch.empty_like(x)
        made.append(out)
    _check_pair(x, out)
    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    with torch.cuda.device(x.device):
        s = fn(len(shape), _shape(shape), _dtype_code(x.dtype), int(nlevels), ctypes.c_void_p(x.data_ptr()),
               ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    if s != MGR_OK:
        raise MgrError(s, last_error())
    _on_stream(made, stream, x.device)
    return out


def export_classes(rep, nlevels: Optional[int] = None, out=None, stream=None):
    """mgr_export_classes: nodal representation -> class-contiguous order."""
    return _classes(lib().mgr_export_classes, rep, nlevels, out, stream)


def import_classes(buf, nlevels: Optional[int] = None, out=None, stream=None):
    """mgr_import_classes: class-contiguous order -> nodal representation."""
    return _classes(lib().mgr_import_classes, buf, nlevels, out, stream)


def class_sizes(shape, nlevels: Optional[int] = None):
    """mgr_class_sizes: element counts of the class-contiguous layout's parts,
    the coarsest grid first, then the classes from the coarsest level to the
    finest."""
    if nlevels is None:
        nlevels = max_levels(shape)
    out = (ctypes.c_int64 * (int(nlevels) + 1))()
    s = lib().mgr_class_sizes(len(shape), _shape(shape), int(nlevels), out)
    if s != MGR_OK:
        raise MgrError(s, last_error())
    return [int(v) for v in out]


def autotune(x, coords=None, nlevels: Optional[int] = None, out=None, workspace=None, stream=None) -> str:
    """mgr_autotune for the field shape of ``x`` (values unused; ``out`` and the
    workspace are overwritten).  Returns the library's report of its choices."""
    _call(lib().mgr_autotune, x, coords, nlevels, out, workspace, stream)
    return lib().mgr_autotune_report().decode()


class Service:
    """mgr_service: requests admitted by HBM footprint, run on internal streams."""

    def __init__(self, budget_bytes: int, nstreams: int = 4):
        self._h = ctypes.c_void_p()
        s = lib().mgr_service_create(ctypes.c_size_t(int(budget_bytes)), int(nstreams), ctypes.byref(self._h))
        if s != MGR_OK:
            raise MgrError(s, lib().mgr_service_last_error().decode())
        self._keep = {}

    def submit(self, recompose: bool, x, out, coords=None, nlevels: Optional[int] = None) -> int:
        """Queue one request; ``x`` and ``out`` must stay alive and untouched
        until it is done (:meth:`result` or :meth:`wait_all`)."""
        _check_pair(x, out)
        shape = tuple(x.shape)
        if nlevels is None:
            nlevels = max_levels(shape)
        carr, keep = _coords_arg(shape, coords)
        t = ctypes.c_uint64(0)
        s = lib().mgr_service_submit(self._h, 1 if recompose else 0, len(shape), _shape(shape), carr,
                                     _dtype_code(x.dtype), int(nlevels), ctypes.c_void_p(x.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), ctypes.byref(t))
        if s != MGR_OK:
            raise MgrError(s, lib().mgr_service_last_error().decode())
        return int(t.value)

    def wait_all(self) -> None:
        lib().mgr_service_wait_all(self._h)

    def result(self, ticket: int):
        """(done, status, queue_ms, latency_ms) of a request."""
        d, st = ctypes.c_int(), ctypes.c_int()
        q, lat = ctypes.c_double(), ctypes.c_double()
        s = lib().mgr_service_result(self._h, ctypes.c_uint64(ticket), ctypes.byref(d), ctypes.byref(st),
                                     ctypes.byref(q), ctypes.byref(lat))
        if s != MGR_OK:
            raise MgrError(s, lib().mgr_service_last_error().decode())
        return bool(d.value), int(st.value), float(q.value), float(lat.value)

    def close(self) -> None:
        if self._h:
            lib().mgr_service_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def release_caches() -> None:
    lib().mgr_release_caches()


def timing_enable(on: bool = True) -> None:
    """Bracket every later kernel launch with HIP events on its stream."""
    lib().mgr_timing_enable(1 if on else 0)


def timing_reset() -> None:
    lib().mgr_timing_reset()


def timing_totals():
    """{kernel name: (launches, total ms, algorithmic bytes)} of the recorded launches."""
    L = lib()
    out = {}
    for i in range(L.mgr_timing_count()):
        name = ctypes.c_char_p()
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        b = ctypes.c_double()
        if L.mgr_timing_get(i, ctypes.byref(name), ctypes.byref(n), ctypes.byref(ms),
                            ctypes.byref(b)) == MGR_OK:
            out[name.value.decode()] = (int(n.value), float(ms.value), float(b.value))
    return out


def probe_copy(src, dst, stream=None) -> None:
    """Streaming copy of src into dst (same byte size): the single-pass bandwidth probe."""
    import torch
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst must have the same byte size")
    if stream is None:
        stream = torch.cuda.current_stream(src.device)
    s = lib().mgr_probe_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                             ctypes.c_size_t(nbytes), ctypes.c_void_p(stream.cuda_stream))
    if s != MGR_OK:
        raise MgrError(s, last_error())
