"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Tolerances (stated per result, the bar of the target):
  FP64:  max|gpu - oracle| / max|oracle| <= 1e-12 over the whole nodal array,
         and for the decomposition also per coefficient class (the nodes
         that leave the hierarchy at one level, and the coarsest grid): the
         class's max error over the class's own max |oracle| <= 1e-12, so
         that small fine-level coefficients are held to the same relative
         bar as the field's scale
  FP32:  ||gpu - oracle||_2 / ||oracle||_2 <= 1e-5, oracle run in FP64 on the
         FP32 input (so only the FP32 storage rounding is measured)
Both directions are checked: decompose against the oracle's decomposition,
recompose against the oracle's recomposition of the same representation, and
the round trip.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_12764_amd import mgr
from paper_2105_12764_amd.synth import WORKLOADS, make_input

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mgr.lib()


def _err(got, ref, dtype):
    got = got.astype(np.float64)
    if dtype == np.float64:
        return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _tol(dtype):
    return TOL64 if dtype == np.float64 else TOL32


def _class_map(shape, nlev):
    """Coefficient class of every node: the level at which it leaves the
    hierarchy (nlev for the coarsest grid), from the coarsening rule."""
    cls = None
    for k, n in enumerate(shape):
        lv = _drop_level(n, nlev).astype(np.int8)
        sh = [1] * len(shape)
        sh[k] = n
        lv = lv.reshape(sh)
        cls = lv if cls is None else np.minimum(cls, lv)
    return np.broadcast_to(cls, shape)


def _per_class_fp64(got, ref, shape, nlev):
    """Max error of each coefficient class over that class's max |oracle|."""
    cls = _class_map(shape, nlev)
    diff = np.abs(got.astype(np.float64) - ref)
    aref = np.abs(ref)
    out = []
    for c in range(nlev + 1):
        m = cls == c
        if not m.any():
            continue
        e, r = float(diff[m].max()), float(aref[m].max())
        out.append((c, int(m.sum()), e / r if r > 0 else e, r))
    return out


def _case(shape, nlev, nonuni, dtype, seed=7):
    print(f"\n[case] shape={shape} nlev={nlev} nonuniform={nonuni} dtype={np.dtype(dtype).name}",
          flush=True)
    u, coords = make_input(shape, seed, nonuniform=nonuni, dtype=dtype)
    if nlev is None:
        nlev = oracle.max_levels(shape)
    x = torch.from_numpy(u).cuda()
    d = mgr.decompose(x, coords, nlev)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    ref = oracle.decompose(u.astype(np.float64), coords, nlev)
    e_dec = _err(got, ref, dtype)
    # recompose: GPU recomposition of the oracle's representation (rounded to dtype)
    rep = torch.from_numpy(ref.astype(dtype)).cuda()
    r = mgr.recompose(rep, coords, nlev)
    torch.cuda.synchronize()
    ref_r = oracle.recompose(ref.astype(dtype).astype(np.float64), coords, nlev)
    e_rec = _err(r.cpu().numpy(), ref_r, dtype)
    # round trip of the GPU's own output
    rt = mgr.recompose(d, coords, nlev)
    torch.cuda.synchronize()
    e_rt = _err(rt.cpu().numpy(), u.astype(np.float64), dtype)
    print(f"[case] dec {e_dec:.2e} rec {e_rec:.2e} roundtrip {e_rt:.2e}", flush=True)
    if dtype == np.float64 and nlev > 0:
        for c, cnt, e, r in _per_class_fp64(got, ref, shape, nlev):
            print(f"[case]   class {c} ({cnt} nodes, max |oracle| {r:.2e}): {e:.2e}", flush=True)
            assert e <= TOL64, ("decompose class", c, e)
    tol = _tol(dtype)
    assert e_dec <= tol, ("decompose", e_dec)
    assert e_rec <= tol, ("recompose", e_rec)
    assert e_rt <= tol, ("round trip", e_rt)


SMALL = [
    ((65, 65, 65), 5, False, np.float64),       # 65^3, 5 levels (to 3^3)
    ((65, 65, 65), 6, False, np.float64),       # full depth to 2^3
    ((33, 33, 33), 5, True, np.float64),
    ((17, 40, 23), None, True, np.float64),     # ragged, even sizes
    ((66, 70, 130), 4, True, np.float64),       # several tiles, ragged tails
    ((9, 130, 70), 3, False, np.float64),
    ((200, 3, 2), None, True, np.float64),      # tiny and never-coarsened dims
    ((129, 150, 2), 3, True, np.float64),       # last coarsened dim strided: subtracting epilogue
    ((40, 150, 2), 2, True, np.float32),
    ((3, 3, 3), 1, False, np.float64),
    ((2, 2, 2), 0, False, np.float64),          # nlevels = 0: copy
    ((129, 257), None, False, np.float64),      # 2-D
    ((300, 41), None, True, np.float64),
    ((1000,), None, True, np.float64),          # 1-D
    ((65,), 3, False, np.float64),
    ((5000,), 4, True, np.float64),             # line of 2501 unknowns: long-line solver, 40 partitions
    ((17000,), 2, True, np.float64),            # line > 8192 unknowns: sequential solver
    ((9000, 20), 2, True, np.float32),          # strided lines of 4501: long-line solver, 71 partitions
    ((20, 6000), 2, True, np.float64),          # rows of 3001: long-line solver, 47 partitions
    ((3000, 40), 2, True, np.float64),          # strided line of 1501: long-line solver
    ((40, 3000), 2, True, np.float64),          # row of 1501: long-line solver
    ((2049, 9), 1, False, np.float64),          # 1025 unknowns: 17 partitions of 64
    ((2100,), 2, True, np.float32),             # 1-D long line, FP32
    ((2500, 3, 4), 2, True, np.float64),        # long dim-0 lines in 3-D
    ((1500, 30), 2, True, np.float64),          # 64-partition strided lines: long-line solver
    ((9, 1100, 20), 2, True, np.float32),       # the same along dim 1, FP32
    ((1030, 6, 40), 3, False, np.float64),      # dim 0 of 515: nine partitions of 64
    ((30, 1500), 2, True, np.float64),          # 64-partition row solve
    ((129, 129, 129), None, True, np.float64),
    ((65, 65, 65), 5, False, np.float32),
    ((20, 17, 26), 3, True, np.float32),
    ((129, 100, 77), None, True, np.float32),
]


@pytest.mark.parametrize("shape,nlev,nonuni,dtype", SMALL)
def test_parity_small(shape, nlev, nonuni, dtype):
    _case(shape, nlev, nonuni, dtype)


def test_deterministic_and_stream_ordered():
    u, coords = make_input((70, 66, 90), 3, nonuniform=True)
    x = torch.from_numpy(u).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = mgr.decompose(x, coords, 4)
        b = mgr.decompose(x, coords, 4)
    s.synchronize()
    assert torch.equal(a, b)
    c = mgr.decompose(x, coords, 4)
    torch.cuda.synchronize()
    assert torch.equal(a, c)


def test_workspace_reuse_between_shapes():
    """A workspace sized for a big request serves a smaller one; contents on entry are ignored."""
    ws = mgr.alloc_workspace((129, 129, 129), torch.float64, 7)
    ws.fill_(255)  # NaN bit patterns in the scratch must not leak into results
    for shape, nlev in (((129, 129, 129), 7), ((40, 33, 65), 4)):
        u, coords = make_input(shape, 9, nonuniform=True)
        d = mgr.decompose(torch.from_numpy(u).cuda(), coords, nlev, workspace=ws)
        torch.cuda.synchronize()
        ref = oracle.decompose(u, coords, nlev)
        assert _err(d.cpu().numpy(), ref, np.float64) <= TOL64


def test_multilinear_field_gives_zero_coefficients_on_gpu():
    """Property that holds at any size: a field multilinear on the final coarse
    grid has zero coefficients and keeps its coarse values."""
    shape, nlev = (97, 65, 80), 5
    _, coords = make_input(shape, 4, nonuniform=True)
    from dense_l2 import coarse_positions, level_coords
    xs = [level_coords(coords[k], nlev) for k in range(3)]
    q = np.random.default_rng(5).standard_normal([len(xs[k][nlev]) for k in range(3)])
    f = q
    for k in range(3):
        f = np.apply_along_axis(lambda v: np.interp(xs[k][0], xs[k][nlev], v), k, f)
    d = mgr.decompose(torch.from_numpy(np.ascontiguousarray(f)).cuda(), coords, nlev)
    got = d.cpu().numpy()
    idx = []
    for n in shape:
        lev = np.arange(n)
        for _ in range(nlev):
            lev = lev[coarse_positions(len(lev))]
        idx.append(lev)
    mask = np.ones(shape, bool)
    mask[np.ix_(*idx)] = False
    assert np.max(np.abs(got[mask])) < 1e-12 * np.max(np.abs(q))
    assert np.max(np.abs(got[np.ix_(*idx)] - q)) < 1e-12 * np.max(np.abs(q))


@pytest.mark.parametrize("name", ["cube65_f64", "box400x300x250_f32", "cube513_f64", "cube513_f32"])
def test_parity_benchmark_workloads(name):
    """The benchmark's workloads at full size, in the launch configuration it times."""
    shape, seed, nonuni, dtype, nlev = WORKLOADS[name]
    _case(shape, nlev, nonuni, dtype, seed=seed)


def _drop_level(n, nlev):
    """Level at which each finest position of a dim of n nodes leaves the
    hierarchy (nlev for positions on the coarsest grid)."""
    from dense_l2 import coarse_positions
    out = np.full(n, nlev)
    pos = np.arange(n)
    for s in range(nlev):
        keep = pos[coarse_positions(len(pos))]
        out[np.setdiff1d(pos, keep)] = s
        pos = keep
    return out


def test_beyond_2pow31_elements_against_the_oracle():
    """Maximum sizes: 1300^3 FP64 (2.2e9 nodes, offsets past 2^31), all 11
    levels.  The field repeats a 2-D pattern g along dim 0, so by the tensor
    structure its decomposition is the oracle's 2-D decomposition of g at
    every node that leaves the hierarchy no earlier along dim 0 than in
    (dims 1, 2), and zero elsewhere; sampled planes, including planes past the
    2^31-element offset, are checked against that, and the round trip
    everywhere."""
    n = 1300
    shape = (n, n, n)
    nlev = mgr.max_levels(shape)
    print(f"\n[case] {shape} float64 nlev={nlev}: u = 1 (x) g", flush=True)
    g, cyz = make_input((n, n), 31, nonuniform=True)
    cx = np.cumsum(np.random.default_rng(32).uniform(0.5, 1.5, n))
    coords = [cx, cyz[0], cyz[1]]
    ref2 = oracle.decompose(g, cyz, nlev)
    gd = torch.from_numpy(g).cuda()
    u = gd.unsqueeze(0).expand(n, n, n).contiguous()
    d = mgr.decompose(u, coords, nlev)
    torch.cuda.synchronize()
    s_i = _drop_level(n, nlev)
    s_jk = np.minimum.outer(_drop_level(n, nlev), _drop_level(n, nlev))
    scale = np.max(np.abs(ref2))
    planes = sorted({0, 1, 2, 3, 4, 8, 640, 1024, 1270, 1271, 1272, 1280, 1296, 1298, n - 1})
    assert (n - 1) * n * n > 2 ** 31 and 1272 * n * n > 2 ** 31
    for i in planes:
        want = np.where(s_jk <= s_i[i], ref2, 0.0)
        err = float(np.max(np.abs(d[i].cpu().numpy() - want))) / scale
        assert err <= TOL64, (i, err)
    r = mgr.recompose(d, coords, nlev)
    torch.cuda.synchronize()
    e_rt = float((r - u).abs().max() / u.abs().max())
    print(f"[case] sampled planes ok, round trip {e_rt:.2e}", flush=True)
    assert e_rt <= TOL64
    del u, d, r
    torch.cuda.empty_cache()


def test_binding_checks_out_and_workspace():
    """The C ABI takes raw pointers: the binding refuses an `out` that cannot
    hold the result and counts the workspace in bytes whatever its dtype."""
    print("\n[case] binding checks of out and workspace", flush=True)
    u, coords = make_input((33, 20, 17), 3, nonuniform=True)
    x = torch.from_numpy(u).cuda()
    for bad in (torch.empty((33, 20, 17), dtype=torch.float32, device="cuda"),
                torch.empty((33, 20, 16), dtype=torch.float64, device="cuda"),
                torch.empty((33, 20, 17), dtype=torch.float64)):
        with pytest.raises(ValueError):
            mgr.decompose(x, coords, out=bad)
    nlev = mgr.max_levels(tuple(x.shape))
    nb = mgr.workspace_size(tuple(x.shape), x.dtype, nlev)
    ws64 = torch.empty((nb + 7) // 8, dtype=torch.float64, device="cuda")  # the same bytes as uint8
    d = mgr.decompose(x, coords, nlev, workspace=ws64)
    ref = mgr.decompose(x, coords, nlev)
    torch.cuda.synchronize()
    assert torch.equal(d, ref)


@pytest.mark.parametrize("name", ["box400x300x250_f32", "cube513_f32"])
def test_fp32_errors_per_coefficient_class(name):
    """FP32 mode against the FP64 oracle, stated per result: max and L2 error
    of the whole representation, and of every coefficient class (the nodes
    that leave the hierarchy at one level; the last class is the coarsest
    grid).  Overall: relative L2 <= 1e-5.  Per class: max error over the
    field's scale (max |oracle|) <= 1e-5."""
    shape, seed, nonuni, dtype, nlev = WORKLOADS[name]
    print(f"\n[case] {name}: FP32 errors per class", flush=True)
    u, coords = make_input(shape, seed, nonuniform=nonuni, dtype=dtype)
    d = mgr.decompose(torch.from_numpy(u).cuda(), coords, nlev)
    torch.cuda.synchronize()
    got = d.cpu().numpy().astype(np.float64)
    ref = oracle.decompose(u.astype(np.float64), coords, nlev)
    scale = float(np.max(np.abs(ref)))
    diff = got - ref
    l2 = float(np.linalg.norm(diff) / np.linalg.norm(ref))
    mx = float(np.max(np.abs(diff)) / scale)
    print(f"  all: max {mx:.2e}  L2 {l2:.2e}", flush=True)
    assert l2 <= TOL32
    lv = [_drop_level(n, nlev) for n in shape]
    cls = np.minimum.outer(np.minimum.outer(lv[0], lv[1]), lv[2])
    for c in range(nlev + 1):
        m = cls == c
        e_max = float(np.max(np.abs(diff[m])))
        e_l2 = float(np.linalg.norm(diff[m]) / max(np.linalg.norm(ref[m]), 1e-300))
        print(f"  class {c} ({int(m.sum())} nodes): max {e_max / scale:.2e} of the field scale, "
              f"L2 {e_l2:.2e} of the class", flush=True)
        assert e_max <= TOL32 * scale, (c, e_max / scale)


def test_fp32_smooth_field_within_tolerance():
    """FP32 mode on a smooth field with no noise, where a coefficient is the
    small difference of nearly equal values: relative L2 against the FP64
    oracle within 1e-5, overall and in every coefficient class (so neither
    the coefficient arithmetic nor the coarser level grids may round at the
    field's scale)."""
    n = 257
    shape, nlev = (n, n, n), mgr.max_levels((n, n, n))
    print(f"\n[case] smooth field {shape} float32, {nlev} levels", flush=True)
    x = np.linspace(0.0, 1.0, n)
    u = (np.sin(2 * np.pi * x)[:, None, None] * np.cos(2 * np.pi * x)[None, :, None]
         * np.sin(np.pi * x)[None, None, :] + 2.0).astype(np.float32)
    d = mgr.decompose(torch.from_numpy(u).cuda(), None, nlev)
    torch.cuda.synchronize()
    got = d.cpu().numpy().astype(np.float64)
    ref = oracle.decompose(u.astype(np.float64), None, nlev)
    diff = got - ref
    l2 = float(np.linalg.norm(diff) / np.linalg.norm(ref))
    print(f"  all: L2 {l2:.2e}", flush=True)
    assert l2 <= TOL32
    lv = _drop_level(n, nlev)
    cls = np.minimum.outer(np.minimum.outer(lv, lv), lv)
    for c in range(nlev + 1):
        m = cls == c
        e = float(np.linalg.norm(diff[m]) / np.linalg.norm(ref[m]))
        print(f"  class {c}: L2 {e:.2e} of the class", flush=True)
        assert e <= TOL32, (c, e)
