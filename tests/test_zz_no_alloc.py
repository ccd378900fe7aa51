"""mgr_decompose_noalloc (workspace and plan tables in the library's static
device scratch) against mgr_decompose, the entry point it is a variant of:
bit for bit, on consecutive calls of different sizes through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2105_12764_amd import mgr
from paper_2105_12764_amd.synth import make_input

pytestmark = pytest.mark.gpu


def _direct(x, coords, nlev):
    """mgr_decompose with a workspace of its own."""
    return mgr.decompose(x, coords, nlev)


def _noalloc_raw(x, out, coords, nlev, stream):
    shape = tuple(x.shape)
    carr, keep = mgr._coords_arg(shape, coords)
    s = mgr.lib().mgr_decompose_noalloc(len(shape), mgr._shape(shape), carr, mgr._dtype_code(x.dtype),
                                        nlev, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(stream.cuda_stream))
    del keep
    return s


# (shape, nlevels, nonuniform coords, dtype, seed): the first two make the
# second call smaller than the first; then the first request again (its tables
# copied in once more) and once more (nothing copied)
CASES = [((129, 200, 97), 6, True, np.float64, 71),
         ((33, 20, 41), 3, False, np.float32, 72),
         ((129, 200, 97), 6, True, np.float64, 71),
         ((129, 200, 97), 6, True, np.float64, 73)]


def test_noalloc_equals_decompose_on_consecutive_calls():
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    outs = []
    for shape, nlev, nonuni, dt, seed in CASES:
        print(f"noalloc {shape} nlev={nlev} {np.dtype(dt).name} seed={seed}", flush=True)
        u, coords = make_input(shape, seed, nonuniform=nonuni, dtype=dt)
        x = torch.from_numpy(u).to(dev)
        out = torch.full_like(x, float("nan"))
        assert _noalloc_raw(x, out, coords, nlev, stream) == mgr.MGR_OK, mgr.last_error()
        outs.append((x, out, coords, nlev))
    torch.cuda.synchronize()
    for (x, out, coords, nlev), case in zip(outs, CASES):
        ref = _direct(x, coords, nlev)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"noalloc differs from mgr_decompose for {case}"


def test_noalloc_largest_fitting_cube_and_binding():
    dev = torch.device("cuda:0")
    shape = (257, 257, 257)
    nlev = mgr.max_levels(shape)
    u, coords = make_input(shape, 74, nonuniform=False, dtype=np.float64)
    x = torch.from_numpy(u).to(dev)
    print(f"noalloc {shape} nlev={nlev} float64 via the binding", flush=True)
    got = mgr.decompose_noalloc(x, coords, nlev)
    ref = mgr.decompose(x, coords, nlev)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    # a request beyond the scratch is refused and leaves `out` untouched
    big = torch.zeros((300, 300, 300), dtype=torch.float64, device=dev)
    sentinel = torch.full_like(big, 7.0)
    with pytest.raises(mgr.MgrError) as ei:
        mgr.decompose_noalloc(big, None, None, out=sentinel)
    assert ei.value.status == mgr.MGR_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((sentinel == 7.0).all())
