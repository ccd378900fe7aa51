"""FP64 CPU oracle for multigrid hierarchical decomposition / recomposition.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The HIP library never imports, links
or runs anything here, and this package imports nothing from it.

The arithmetic lives in ``mgr_oracle.c`` (plain C, FP64); this module only
builds it with gcc and marshals NumPy arrays through ctypes.  The method is
Chen et al., arXiv 2105.12764, Sec. II-A (Eq. 1, Eq. 2 and the variational
problem for the correction) with the Thomas solve of Sec. III-A.3; the
readings taken where the paper is silent are listed in the C file's header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mgr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _compile(path: str, native: bool) -> None:
    tmp = path + ".tmp"
    cmd = ["gcc", "-O2", *(["-march=native"] if native else []), "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, path)


def build(force: bool = True) -> str:
    """Compile mgr_oracle.c into liboracle.so with gcc (-O2, OpenMP, no
    fast-math; ISO C, so no floating-point contraction either)."""
    if force or not os.path.exists(_LIB_PATH):
        _compile(_LIB_PATH, native=False)
    return _LIB_PATH


def _bind(lib):
    i64p = ctypes.POINTER(ctypes.c_int64)
    dpp = ctypes.POINTER(ctypes.POINTER(ctypes.c_double))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_max_levels.argtypes = [ctypes.c_int, i64p]
    lib.oracle_max_levels.restype = ctypes.c_int
    for fn in (lib.oracle_decompose, lib.oracle_recompose):
        fn.argtypes = [ctypes.c_int, i64p, dpp, ctypes.c_int, dp, dp]
        fn.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


class Native:
    """The same C source built for the host it runs on (-O2 -march=native,
    still ISO C without fast-math or contraction, so the same arithmetic),
    in a temporary directory: used to time the oracle as a CPU baseline.
    ``threads(n)`` sets the OpenMP thread count of later calls made from
    this thread."""

    def __init__(self):
        import tempfile
        self._dir = tempfile.mkdtemp(prefix="mgr_oracle_")
        path = os.path.join(self._dir, "liboracle_native.so")
        _compile(path, native=True)
        self._lib = _bind(ctypes.CDLL(path))
        self._omp = ctypes.CDLL("libgomp.so.1")
        self._omp.omp_set_num_threads.argtypes = [ctypes.c_int]
        self._omp.omp_get_max_threads.restype = ctypes.c_int
        self.flags = "gcc -O2 -march=native -fopenmp -std=c11"

    def threads(self, n: int) -> None:
        self._omp.omp_set_num_threads(int(n))

    def max_threads(self) -> int:
        return int(self._omp.omp_get_max_threads())

    def decompose(self, u, coords=None, nlevels=None) -> np.ndarray:
        return _run(self._lib.oracle_decompose, u, coords, nlevels)

    def recompose(self, v, coords=None, nlevels=None) -> np.ndarray:
        return _run(self._lib.oracle_recompose, v, coords, nlevels)


def _shape_arg(shape):
    return (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])


def max_levels(shape) -> int:
    """Deepest level count for ``shape`` (each dim coarsens while it has >= 3 nodes)."""
    r = _load().oracle_max_levels(len(shape), _shape_arg(shape))
    if r < 0:
        raise ValueError(f"invalid shape {tuple(shape)}")
    return r


def _coords_arg(shape, coords):
    if coords is None:
        return None, []
    keep = []
    arr = (ctypes.POINTER(ctypes.c_double) * len(shape))()
    for k, n in enumerate(shape):
        c = coords[k]
        if c is None:
            arr[k] = ctypes.POINTER(ctypes.c_double)()
            continue
        c = np.ascontiguousarray(c, dtype=np.float64)
        if c.shape != (n,):
            raise ValueError(f"coords[{k}] must have shape ({n},)")
        keep.append(c)
        arr[k] = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return arr, keep


def _run(fn, u, coords, nlevels):
    u = np.ascontiguousarray(u, dtype=np.float64)
    shape = u.shape
    if nlevels is None:
        nlevels = max_levels(shape)
    out = np.empty_like(u)
    carr, keep = _coords_arg(shape, coords)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = fn(len(shape), _shape_arg(shape), carr, int(nlevels),
            u.ctypes.data_as(dp), out.ctypes.data_as(dp))
    del keep
    if rc != 0:
        raise ValueError("oracle rejected the arguments (shape, coords or nlevels)")
    return out


def decompose(u, coords=None, nlevels=None) -> np.ndarray:
    """Nodal multilevel decomposition of ``u`` (FP64 copy of the input)."""
    return _run(_load().oracle_decompose, u, coords, nlevels)


def recompose(v, coords=None, nlevels=None) -> np.ndarray:
    """Inverse of :func:`decompose`."""
    return _run(_load().oracle_recompose, v, coords, nlevels)
