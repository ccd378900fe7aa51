"""GPU: the batched entry points (mgr_decompose_batch / mgr_recompose_batch and
their _ex forms), in both launch modes: grouped launches (one grid per kernel
and level step across the fields) and per-field chains on internal streams.

Each field of a batch must come out bitwise equal to the single-field call on
the same input (the same kernel bodies run), agree with the oracle to the
usual tolerances, stay stream-ordered, and give the same result on every
replay of a HIP graph that captured the batch.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_12764_amd import mgr
from paper_2105_12764_amd.synth import make_input

pytestmark = pytest.mark.gpu

# (shape, nlevels or None for all, non-uniform coordinates, dtype)
FIELDS = [
    ((33, 33, 33), None, True, np.float64),
    ((65, 40, 23), 4, False, np.float32),
    ((129, 70), None, False, np.float64),
    ((300, 41), 3, True, np.float32),
    ((17, 17, 17), 2, False, np.float64),
    ((1000,), None, True, np.float64),
    ((2, 2, 2), 0, False, np.float64),
    ((40, 150, 2), 2, True, np.float32),
    ((2100, 5), None, True, np.float64),   # lines of 1051 unknowns: the long-line solver
    ((4100, 3), 2, False, np.float32),     # lines of 2051: the long-line solver, 33 partitions
    ((16500, 3), 2, True, np.float64),     # lines of 8251: the sequential solver (launched alone)
]
MODES = [False, True]  # per_field


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mgr.lib()


def _inputs(seed0=300):
    out = []
    for i, (shape, nlev, nonuni, dtype) in enumerate(FIELDS):
        u, coords = make_input(shape, seed0 + i, nonuniform=nonuni, dtype=dtype)
        if nlev is None:
            nlev = oracle.max_levels(shape)
        out.append((u, coords, nlev, torch.from_numpy(u).cuda()))
    return out


def _err(got, ref, dtype):
    got = got.astype(np.float64)
    if dtype == np.float64:
        return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


@pytest.mark.parametrize("per_field", MODES)
def test_batch_equals_single_calls_bitwise(per_field):
    print(f"\n[case] batch of {len(FIELDS)} mixed fields vs single calls, per_field={per_field}", flush=True)
    ins = _inputs()
    singles = [mgr.decompose(x, coords, nlev) for (_, coords, nlev, x) in ins]
    outs = [torch.empty_like(x) for (_, _, _, x) in ins]
    batch = mgr.Batch([(x, y, coords, nlev) for (_, coords, nlev, x), y in zip(ins, outs)])
    ws = batch.alloc_workspace()
    mgr.decompose_batch(batch, ws, per_field=per_field)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(singles, outs)):
        assert torch.equal(a, b), f"field {i} {FIELDS[i][0]}: decompose batch differs from single call"
    # recompose: outs -> fields, against single recompositions
    back = [torch.empty_like(x) for (_, _, _, x) in ins]
    rb = mgr.Batch([(y, z, coords, nlev) for (_, coords, nlev, _), y, z in zip(ins, outs, back)])
    mgr.recompose_batch(rb, ws, per_field=per_field)
    rsingles = [mgr.recompose(y, coords, nlev) for (_, coords, nlev, _), y in zip(ins, outs)]
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(rsingles, back)):
        assert torch.equal(a, b), f"field {i} {FIELDS[i][0]}: recompose batch differs from single call"


@pytest.mark.parametrize("per_field", MODES)
def test_batch_matches_oracle(per_field):
    print(f"\n[case] batch of {len(FIELDS)} mixed fields vs the oracle, per_field={per_field}", flush=True)
    ins = _inputs(seed0=400)
    outs = [torch.empty_like(x) for (_, _, _, x) in ins]
    back = [torch.empty_like(x) for (_, _, _, x) in ins]
    batch = mgr.Batch([(x, y, coords, nlev) for (_, coords, nlev, x), y in zip(ins, outs)])
    ws = batch.alloc_workspace()
    mgr.decompose_batch(batch, ws, per_field=per_field)
    rb = mgr.Batch([(y, z, coords, nlev) for (_, coords, nlev, _), y, z in zip(ins, outs, back)])
    mgr.recompose_batch(rb, ws, per_field=per_field)
    torch.cuda.synchronize()
    for i, ((u, coords, nlev, _), y, z) in enumerate(zip(ins, outs, back)):
        dtype = FIELDS[i][3]
        tol = 1e-12 if dtype == np.float64 else 1e-5
        ref = oracle.decompose(u.astype(np.float64), coords, nlev)
        e_dec = _err(y.cpu().numpy(), ref, dtype)
        e_rt = _err(z.cpu().numpy(), u.astype(np.float64), dtype)
        print(f"  field {i} {FIELDS[i][0]} {np.dtype(dtype).name}: dec {e_dec:.2e} round trip {e_rt:.2e}")
        assert e_dec <= tol, (i, e_dec)
        assert e_rt <= tol, (i, e_rt)


@pytest.mark.parametrize("per_field", MODES)
def test_batch_graph_replays_match_eager(per_field):
    print(f"\n[case] batch captured in a HIP graph, three replays, per_field={per_field}", flush=True)
    ins = _inputs(seed0=500)
    outs = [torch.empty_like(x) for (_, _, _, x) in ins]
    back = [torch.empty_like(x) for (_, _, _, x) in ins]
    batch = mgr.Batch([(x, y, coords, nlev) for (_, coords, nlev, x), y in zip(ins, outs)])
    rb = mgr.Batch([(y, z, coords, nlev) for (_, coords, nlev, _), y, z in zip(ins, outs, back)])
    ws = batch.alloc_workspace()
    ws2 = rb.alloc_workspace()
    # eager reference (also builds every plan before the capture)
    mgr.decompose_batch(batch, ws, per_field=per_field)
    mgr.recompose_batch(rb, ws2, per_field=per_field)
    torch.cuda.synchronize()
    ref_d = [y.clone() for y in outs]
    ref_r = [z.clone() for z in back]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            mgr.decompose_batch(batch, ws, stream=side, per_field=per_field)
            mgr.recompose_batch(rb, ws2, stream=side, per_field=per_field)
    torch.cuda.synchronize()
    for rep in range(3):
        for y, z in zip(outs, back):  # eager work between replays
            y.fill_(7.0)
            z.fill_(-3.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(FIELDS)):
            assert torch.equal(outs[i], ref_d[i]), f"replay {rep}: field {i} decomposition differs"
            assert torch.equal(back[i], ref_r[i]), f"replay {rep}: field {i} recomposition differs"


def test_batch_is_stream_ordered():
    print("\n[case] batch on a side stream after and before dependent work", flush=True)
    ins = _inputs(seed0=600)
    side = torch.cuda.Stream()
    srcs = [x.clone() for (_, _, _, x) in ins]
    xs = [torch.zeros_like(x) for (_, _, _, x) in ins]
    outs = [torch.empty_like(x) for (_, _, _, x) in ins]
    batch = mgr.Batch([(x, y, coords, nlev) for (_, coords, nlev, _), x, y in zip(ins, xs, outs)])
    ws = batch.alloc_workspace()
    singles = [mgr.decompose(x, coords, nlev) for (_, coords, nlev, x) in ins]
    torch.cuda.synchronize()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for x, s in zip(xs, srcs):  # the batch must see these writes
            x.copy_(s)
        mgr.decompose_batch(batch, ws, stream=side)
        copies = [y.clone() for y in outs]  # and this must see the batch's results
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(singles, copies)):
        assert torch.equal(a, b), f"field {i}: stream order broken"


def test_grouped_batch_of_many_fields_equals_single_calls():
    """More jobs of one kernel in a step than one grouped launch takes (the
    launch is split), fields of different depths, both dtypes, 2-D and 3-D."""
    print("\n[case] grouped batch of 70 fields vs single calls", flush=True)
    specs = [((17 + (i % 5), 19, 21 + (i % 3)), np.float64) for i in range(40)] + \
            [((65 + 2 * (i % 7), 33 + (i % 4)), np.float32) for i in range(30)]
    ins = []
    for i, (shape, dt) in enumerate(specs):
        u, coords = make_input(shape, 900 + i, nonuniform=(i % 2 == 0), dtype=dt)
        ins.append((torch.from_numpy(u).cuda(), coords, oracle.max_levels(shape)))
    singles = [mgr.decompose(x, c, n) for (x, c, n) in ins]
    outs = [torch.empty_like(x) for (x, _, _) in ins]
    back = [torch.empty_like(x) for (x, _, _) in ins]
    batch = mgr.Batch([(x, y, c, n) for (x, c, n), y in zip(ins, outs)])
    ws = batch.alloc_workspace()
    mgr.decompose_batch(batch, ws)
    rb = mgr.Batch([(y, z, c, n) for (_, c, n), y, z in zip(ins, outs, back)])
    mgr.recompose_batch(rb, ws)
    rsingles = [mgr.recompose(y, c, n) for (_, c, n), y in zip(ins, singles)]
    torch.cuda.synchronize()
    for i in range(len(specs)):
        assert torch.equal(singles[i], outs[i]), f"field {i} {specs[i]}: decomposition differs"
        assert torch.equal(rsingles[i], back[i]), f"field {i} {specs[i]}: recomposition differs"
    u0 = ins[0][0].double()
    assert float((back[0].double() - u0).abs().max() / u0.abs().max()) <= 1e-12


@pytest.mark.parametrize("shape,nonuni,dtype", [((129, 100, 77), True, np.float64),
                                                ((97, 65, 80), False, np.float32),
                                                ((600, 130), True, np.float64)])
def test_autotuned_shapes_leave_results_bitwise_unchanged(shape, nonuni, dtype):
    print(f"\n[case] autotune {shape} {np.dtype(dtype).name}", flush=True)
    mgr.release_caches()
    u, coords = make_input(shape, 77, nonuniform=nonuni, dtype=dtype)
    nlev = oracle.max_levels(shape)
    x = torch.from_numpy(u).cuda()
    d0 = mgr.decompose(x, coords, nlev)
    r0 = mgr.recompose(d0, coords, nlev)
    torch.cuda.synchronize()
    scratch = torch.empty_like(x)
    report = mgr.autotune(x, coords, nlev, out=scratch)
    print(report, flush=True)
    assert "level 0" in report
    d1 = mgr.decompose(x, coords, nlev)
    r1 = mgr.recompose(d1, coords, nlev)
    torch.cuda.synchronize()
    assert torch.equal(d0, d1)
    assert torch.equal(r0, r1)
    ref = oracle.decompose(u.astype(np.float64), coords, nlev)
    tol = 1e-12 if dtype == np.float64 else 1e-5
    assert _err(d1.cpu().numpy(), ref, dtype) <= tol
