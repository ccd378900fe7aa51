"""GPU: the refactoring service (mgr_service_*).

Requests admitted by HBM footprint must produce exactly what the direct calls
produce, also when the budget admits only one request at a time, and report
consistent queue and completion times.
"""
import numpy as np
import pytest
import torch

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
    for i in range(len(xs)):
        assert torch.equal(douts[i], dref[i]), f"request {i}: decomposition differs"
        assert torch.equal(routs[i], rref[i]), f"request {i}: recomposition differs"


def test_service_rejects_oversized_requests():
    print("\n[case] service budget smaller than a request", flush=True)
    x = torch.zeros((65, 65, 65), dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    svc = mgr.Service(1 << 20, nstreams=1)
    with pytest.raises(mgr.MgrError):
        svc.submit(False, x, y)
    svc.close()
