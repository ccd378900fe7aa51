"""GPU: the refactoring service (mgr_service_*).

Requests admitted by HBM footprint must produce what the FP64 CPU oracle
produces (FP64: max|served - oracle| / max|oracle| <= 1e-12; FP32: relative
L2 <= 1e-5 against the oracle run on the FP32 values), exactly what the
direct calls produce, also when the budget admits only one request at a time,
and report consistent queue and completion times.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_12764_amd import mgr
from paper_2105_12764_amd.synth import make_input

pytestmark = pytest.mark.gpu

REQS = [((33, 33, 33), np.float64, False), ((65, 40, 23), np.float32, True),
        ((129, 70), np.float64, True), ((60, 61, 62), np.float32, False),
        ((300, 41), np.float64, False), ((17, 17, 17), np.float64, False),
        ((97, 65, 80), np.float64, False), ((1000,), np.float32, True)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mgr.lib()


def _oracle_err(got, ref, dtype):
    got = got.cpu().numpy().astype(np.float64)
    if dtype == np.float64:
        return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _footprint(x):
    return 2 * x.numel() * x.element_size() + mgr.workspace_size(tuple(x.shape), x.dtype,
                                                                 mgr.max_levels(tuple(x.shape)))


@pytest.mark.parametrize("tight", [False, True])
def test_service_results_equal_direct_calls(tight):
    print(f"\n[case] service, tight budget={tight}", flush=True)
    xs, coords_l = [], []
    for i, (shape, dtype, nonuni) in enumerate(REQS):
        u, coords = make_input(shape, 900 + i, nonuniform=nonuni, dtype=dtype)
        xs.append(torch.from_numpy(u).cuda())
        coords_l.append(coords)
    # references: decompose each, and recompose its decomposition
    dref = [mgr.decompose(x, c) for x, c in zip(xs, coords_l)]
    rref = [mgr.recompose(d, c) for d, c in zip(dref, coords_l)]
    torch.cuda.synchronize()
    budget = max(_footprint(x) for x in xs) + 4096 if tight else 1 << 31
    svc = mgr.Service(budget, nstreams=3)
    douts = [torch.empty_like(x) for x in xs]
    routs = [torch.empty_like(x) for x in xs]
    tickets = []
    for x, c, y in zip(xs, coords_l, douts):
        tickets.append(svc.submit(False, x, y, c))
    for d, c, z in zip(dref, coords_l, routs):  # recompose the reference decompositions
        tickets.append(svc.submit(True, d, z, c))
    svc.wait_all()
    for t in tickets:
        done, status, q, lat = svc.result(t)
        assert done and status == mgr.MGR_OK, (t, status)
        assert 0.0 <= q <= lat, (t, q, lat)
    svc.close()
    torch.cuda.synchronize()
    for i, (shape, dtype, _) in enumerate(REQS):
        assert torch.equal(douts[i], dref[i]), f"request {i}: decomposition differs"
        assert torch.equal(routs[i], rref[i]), f"request {i}: recomposition differs"
        # against the oracle: the served decomposition, and the served
        # recomposition of the representation it was given
        u = xs[i].cpu().numpy().astype(np.float64)
        o_dec = oracle.decompose(u, coords_l[i])
        o_rec = oracle.recompose(dref[i].cpu().numpy().astype(np.float64), coords_l[i])
        tol = 1e-12 if dtype == np.float64 else 1e-5
        e_dec, e_rec = _oracle_err(douts[i], o_dec, dtype), _oracle_err(routs[i], o_rec, dtype)
        print(f"  request {i} {shape} {np.dtype(dtype).name}: decompose {e_dec:.2e}, recompose {e_rec:.2e}",
              flush=True)
        assert e_dec <= tol and e_rec <= tol, (i, e_dec, e_rec)


def test_service_rejects_oversized_requests():
    print("\n[case] service budget smaller than a request", flush=True)
    x = torch.zeros((65, 65, 65), dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    svc = mgr.Service(1 << 20, nstreams=1)
    with pytest.raises(mgr.MgrError):
        svc.submit(False, x, y)
    svc.close()


def test_service_reports_a_failing_request_and_serves_the_rest():
    """A request that the library rejects when it is enqueued (in and out
    overlap) is retired with its error status; the others complete."""
    print("\n[case] service with one invalid request", flush=True)
    u, coords = make_input((33, 33, 33), 5, nonuniform=True)
    x = torch.from_numpy(u).cuda()
    ref = mgr.decompose(x, coords)
    torch.cuda.synchronize()
    svc = mgr.Service(1 << 30, nstreams=2)
    y0, y1 = torch.empty_like(x), torch.empty_like(x)
    t0 = svc.submit(False, x, y0, coords)
    tbad = svc.submit(False, x, x, coords)  # out overlaps in
    t1 = svc.submit(False, x, y1, coords)
    svc.wait_all()
    d0, s0, _, _ = svc.result(t0)
    dbad, sbad, _, _ = svc.result(tbad)
    d1, s1, _, _ = svc.result(t1)
    svc.close()
    assert d0 and d1 and dbad
    assert s0 == mgr.MGR_OK and s1 == mgr.MGR_OK
    assert sbad == mgr.MGR_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.equal(y0, ref) and torch.equal(y1, ref)


def test_service_serves_4d_requests():
    print("\n[case] service with 4-D requests", flush=True)
    shapes = [(5, 17, 9, 12), (9, 9, 9, 9), (16, 5, 6, 7)]
    svc = mgr.Service(1 << 30, nstreams=3)
    jobs = []
    for i, sh in enumerate(shapes):
        u, coords = make_input(sh, 60 + i, nonuniform=True)
        x = torch.from_numpy(u).cuda()
        y = torch.empty_like(x)
        jobs.append((x, y, coords, svc.submit(False, x, y, coords)))
    svc.wait_all()
    for x, y, coords, t in jobs:
        done, st, _, _ = svc.result(t)
        assert done and st == mgr.MGR_OK
    svc.close()
    for x, y, coords, _ in jobs:
        assert torch.equal(y, mgr.decompose(x, coords))


@pytest.mark.parametrize("shape", [(2_000_000,), (200_000, 2), (100_001, 2, 2, 2)])
def test_service_admits_a_request_whose_footprint_is_the_whole_budget(shape):
    """Workspace-heavy FP32 shapes (one coarsened dimension: the workspace is
    about two thirds of the footprint, large enough that the arena's fixed
    1 MiB margin does not cover it): a budget equal to the request's
    footprint admits it, and the result matches the oracle."""
    print(f"\n[case] service budget = footprint of {shape} float32", flush=True)
    u, coords = make_input(shape, 77, nonuniform=True, dtype=np.float32)
    x = torch.from_numpy(u).cuda()
    y = torch.empty_like(x)
    svc = mgr.Service(_footprint(x), nstreams=1)
    t = svc.submit(False, x, y, coords)
    svc.wait_all()
    done, st, _, _ = svc.result(t)
    svc.close()
    assert done and st == mgr.MGR_OK, st
    ref = oracle.decompose(u.astype(np.float64), coords)
    assert _oracle_err(y, ref, np.float32) <= 1e-5
