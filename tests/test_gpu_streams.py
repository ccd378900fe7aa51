"""GPU: stream semantics of the single-field calls.

A recomposition with two or more levels runs its finest level's load vector
and first solves on a library-owned helper stream forked from the caller's
stream.  It must stay ordered on the caller's stream (it sees the writes
before it, the work after it sees its result), give the same bits as the
serial order (the batched path runs it serially), replay correctly from a
HIP graph, and fall back to the serial order once the library holds helper
streams for 64 caller streams.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_12764_amd import mgr
from paper_2105_12764_amd.synth import make_input

pytestmark = pytest.mark.gpu

CASES = [((129, 100, 77), True, np.float64), ((65, 65, 65), False, np.float32), ((300, 41), True, np.float64),
         ((40, 150, 2), True, np.float64)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mgr.lib()


@pytest.mark.parametrize("shape,nonuni,dtype", CASES)
def test_recompose_is_ordered_on_a_side_stream(shape, nonuni, dtype):
    print(f"\n[case] recompose ordering {shape} {np.dtype(dtype).name}", flush=True)
    u, coords = make_input(shape, 91, nonuniform=nonuni, dtype=dtype)
    nlev = oracle.max_levels(shape)
    x = torch.from_numpy(u).cuda()
    d = mgr.decompose(x, coords, nlev)
    ref = mgr.recompose(d, coords, nlev)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    src = torch.zeros_like(d)
    out = torch.empty_like(d)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        src.copy_(d)                      # the call must see this write
        mgr.recompose(src, coords, nlev, out=out, stream=side)
        after = out.clone()               # and this must see its result
    torch.cuda.synchronize()
    assert torch.equal(after, ref)


@pytest.mark.parametrize("shape,nonuni,dtype", CASES)
def test_recompose_equals_the_serial_order_bitwise(shape, nonuni, dtype):
    """The batched entry point runs a field's recomposition in the serial
    order on one stream; the single call forks part of it."""
    print(f"\n[case] forked vs serial recompose {shape} {np.dtype(dtype).name}", flush=True)
    u, coords = make_input(shape, 92, nonuniform=nonuni, dtype=dtype)
    nlev = oracle.max_levels(shape)
    x = torch.from_numpy(u).cuda()
    d = mgr.decompose(x, coords, nlev)
    single = mgr.recompose(d, coords, nlev)
    out = torch.empty_like(d)
    b = mgr.Batch([(d, out, coords, nlev)])
    mgr.recompose_batch(b, b.alloc_workspace())
    torch.cuda.synchronize()
    assert torch.equal(single, out)


def test_recompose_replays_from_a_graph():
    print("\n[case] recompose captured in a HIP graph, three replays", flush=True)
    shape, nlev = (97, 65, 80), 5
    u, coords = make_input(shape, 93, nonuniform=True)
    x = torch.from_numpy(u).cuda()
    d = mgr.decompose(x, coords, nlev)
    ws = mgr.alloc_workspace(shape, x.dtype, nlev)
    out = torch.empty_like(x)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        mgr.recompose(d, coords, nlev, out=out, workspace=ws, stream=side)  # creates the helper stream
    torch.cuda.synchronize()
    ref = out.clone()
    g = torch.cuda.CUDAGraph()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            mgr.recompose(d, coords, nlev, out=out, workspace=ws, stream=side)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep}"
    e = float((out - x).abs().max() / x.abs().max())
    assert e <= 1e-12


class _RawStream:
    """A caller stream created through the HIP runtime (not torch's pool)."""

    def __init__(self, handle):
        self.cuda_stream = handle


def test_recompose_from_more_caller_streams_than_helpers():
    """The library keeps helper streams for at most 64 (device, caller stream)
    pairs; recompositions from further caller streams run serially on the
    caller's stream and give the same bits as the forked ones."""
    import ctypes

    hip = ctypes.CDLL("libamdhip64.so.7")  # the runtime the library is linked against
    shape, nlev = (65, 65, 65), 5
    print(f"\n[case] recompose {shape} from 72 caller streams", flush=True)
    u, coords = make_input(shape, 94, nonuniform=True)
    x = torch.from_numpy(u).cuda()
    d = mgr.decompose(x, coords, nlev)
    ws = mgr.alloc_workspace(shape, x.dtype, nlev)
    ref = mgr.recompose(d, coords, nlev, workspace=ws)
    out = torch.empty_like(x)
    torch.cuda.synchronize()
    streams = []
    try:
        for i in range(72):
            h = ctypes.c_void_p()
            assert hip.hipStreamCreateWithFlags(ctypes.byref(h), ctypes.c_uint(1)) == 0
            streams.append(h)
            out.fill_(-1.0)
            torch.cuda.synchronize()
            mgr.recompose(d, coords, nlev, out=out, workspace=ws, stream=_RawStream(h.value))
            assert hip.hipStreamSynchronize(h) == 0
            assert torch.equal(out, ref), f"caller stream {i}"
    finally:
        torch.cuda.synchronize()
        for h in streams:
            hip.hipStreamDestroy(h)


def test_captured_graph_outlives_the_plan_cache():
    """A captured graph keeps the plans whose tables its kernels read: after
    the cache is emptied and refilled with other plans, replays still give
    the eager results bitwise.  Capturing a call whose plan is not cached is
    refused (building it would allocate device memory) and leaves the capture
    usable."""
    print("\n[case] graph replay after the plan cache dropped its plans", flush=True)
    u, ca = make_input((97, 65, 80), 95, nonuniform=True)
    v, cb = make_input((300, 41), 96, nonuniform=True, dtype=np.float32)
    w, cc = make_input((33, 47, 20), 97, nonuniform=False)
    xa, xb, xc = (torch.from_numpy(t).cuda() for t in (u, v, w))
    da, db, dc = (torch.empty_like(t) for t in (xa, xb, xc))
    ra = torch.empty_like(xa)
    wsa = mgr.alloc_workspace(tuple(xa.shape), xa.dtype, mgr.max_levels(tuple(xa.shape)))
    batch = mgr.Batch([(xb, db, cb, None), (xc, dc, None, None)])
    wsb = batch.alloc_workspace()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())

    def work():
        mgr.decompose(xa, ca, None, out=da, workspace=wsa, stream=side)
        mgr.recompose(da, ca, None, out=ra, workspace=wsa, stream=side)
        mgr.decompose_batch(batch, wsb, stream=side)

    with torch.cuda.stream(side):
        work()  # builds the plans and the helper stream outside the capture
    torch.cuda.synchronize()
    refs = [t.clone() for t in (da, ra, db, dc)]
    fresh = torch.from_numpy(make_input((21, 22, 23), 98)[0]).cuda()
    g = torch.cuda.CUDAGraph()
    refused = None
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            try:
                mgr.decompose(fresh, None, None, stream=side)
            except mgr.MgrError as e:
                refused = e
            work()
    torch.cuda.synchronize()
    assert refused is not None and refused.status == mgr.MGR_ERR_UNSUPPORTED, refused
    mgr.release_caches()
    for i in range(1030):  # more plans than the cache keeps (1024)
        t = torch.zeros((5 + i, 3), dtype=torch.float64, device="cuda")
        mgr.decompose(t)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in (da, ra, db, dc):
            t.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, ref in zip((da, ra, db, dc), refs):
            assert torch.equal(got, ref), f"replay {rep}"
    del g
    torch.cuda.synchronize()
    mgr.decompose(fresh)  # an ordinary call after the graph is gone
    torch.cuda.synchronize()


def test_binding_workspace_survives_a_call_on_another_stream():
    """A workspace (and output) that the binding allocates comes from the
    current stream's allocator pool; when the call runs on another stream,
    the block must not be handed out again before that stream's work is done.
    The side stream is held back by a bounded spin kernel, so its work is
    still pending when a same-sized tensor is allocated and filled on the
    current stream."""
    print("\n[case] binding-allocated workspace on a side stream", flush=True)
    shape, nlev = (129, 129, 129), 7
    u, coords = make_input(shape, 99, nonuniform=True)
    x = torch.from_numpy(u).cuda()
    ref = mgr.decompose(x, coords, nlev)
    torch.cuda.synchronize()
    seen = {}
    real_alloc = mgr.alloc_workspace

    def spy(*a, **k):
        t = real_alloc(*a, **k)
        seen["ws"] = (t.data_ptr(), t.numel())
        return t

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        torch.cuda._sleep(50_000_000)  # bounded spin: keeps the side stream busy for a while
    mgr.alloc_workspace = spy
    try:
        d = mgr.decompose(x, coords, nlev, stream=side)  # workspace and out from the current stream's pool
    finally:
        mgr.alloc_workspace = real_alloc
    busy = not side.query()
    other = torch.empty(seen["ws"][1], dtype=torch.uint8, device="cuda")
    other.fill_(255)
    if busy:
        assert other.data_ptr() != seen["ws"][0], "workspace handed out while its stream still uses it"
    side.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(d, ref)
