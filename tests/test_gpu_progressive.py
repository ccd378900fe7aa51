"""GPU: progressive (partial) recomposition, mgr_recompose_partial.

Keeping the nkeep coarsest coefficient classes must equal the oracle's full
recomposition of the representation with the finer classes set to zero; all
classes must be bitwise the full recomposition; and the error against the
field must not grow as classes are added (nested L2 projections).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_12764_amd import mgr
from paper_2105_12764_amd.synth import make_input

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mgr.lib()


def _level_positions(n, steps):
    """Indices of the level grid after `steps` coarsenings of 0..n-1: even
    positions and the last, while a dimension has at least 3 nodes."""
    pos = np.arange(n)
    for _ in range(steps):
        if len(pos) < 3:
            break
        keep = [i for i in range(len(pos)) if i % 2 == 0 or i == len(pos) - 1]
        pos = pos[keep]
    return pos


def _zero_finer_classes(rep, nlev, nkeep):
    """The representation with every coefficient finer than the kept classes
    set to zero: only the nodes of the level-(nlev - nkeep) grid survive."""
    steps = nlev - nkeep
    mask = np.zeros(rep.shape, dtype=bool)
    idx = np.ix_(*[_level_positions(n, steps) for n in rep.shape])
    mask[idx] = True
    return np.where(mask, rep, 0.0)


@pytest.mark.parametrize("shape,nonuni,dtype", [((65, 65, 65), False, np.float64),
                                                ((66, 70, 45), True, np.float64),
                                                ((300, 41), True, np.float64),
                                                ((97, 65, 80), False, np.float32)])
def test_partial_recompose_matches_oracle_with_dropped_classes(shape, nonuni, dtype):
    print(f"\n[case] partial recompose {shape} {np.dtype(dtype).name}", flush=True)
    u, coords = make_input(shape, 11, nonuniform=nonuni, dtype=dtype)
    nlev = oracle.max_levels(shape)
    x = torch.from_numpy(u).cuda()
    d = mgr.decompose(x, coords, nlev)
    full = mgr.recompose(d, coords, nlev)
    torch.cuda.synchronize()
    assert torch.equal(mgr.recompose_partial(d, nlev, coords, nlev), full)
    rep = d.cpu().numpy().astype(np.float64)
    errs = []
    for nkeep in sorted({0, 1, nlev // 2, nlev - 1, nlev}):
        got = mgr.recompose_partial(d, nkeep, coords, nlev).cpu().numpy().astype(np.float64)
        ref = oracle.recompose(_zero_finer_classes(rep, nlev, nkeep), coords, nlev)
        if dtype == np.float64:
            e = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            assert e <= 1e-12, (nkeep, e)
        else:
            e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            assert e <= 1e-5, (nkeep, e)
        err_u = np.linalg.norm(got - u.astype(np.float64)) / np.linalg.norm(u.astype(np.float64))
        errs.append(err_u)
        print(f"  nkeep {nkeep}: vs oracle {e:.2e}, relative L2 error to the field {err_u:.3e}")
    for a, b in zip(errs, errs[1:]):
        assert b <= a * (1 + 1e-9) + 1e-12, errs


def _classes_reference(rep, nlev):
    """Class-contiguous order written out from its definition: the coarsest
    grid's values, then per level (coarsest first) the nodes of its grid that
    are not in the next coarser grid, in C order of the level grid."""
    parts = []
    grids = [tuple(_level_positions(n, s) for n in rep.shape) for s in range(nlev + 1)]
    parts.append(rep[np.ix_(*grids[nlev])].ravel())
    for s in range(nlev - 1, -1, -1):
        g, c = grids[s], grids[s + 1]
        vals = rep[np.ix_(*g)]
        inside = np.ones(vals.shape, dtype=bool)
        for k, (gk, ck) in enumerate(zip(g, c)):
            sh = [1] * rep.ndim
            sh[k] = len(gk)
            inside &= np.isin(gk, ck).reshape(sh)
        parts.append(vals[~inside])
    return np.concatenate(parts)


@pytest.mark.parametrize("shape,nlev,dtype", [((65, 65, 65), None, np.float64),
                                              ((66, 70, 45), 5, np.float32),
                                              ((300, 41), None, np.float64),
                                              ((1000,), 4, np.float64),
                                              ((5, 2, 9), None, np.float64),
                                              ((9, 9, 9), 0, np.float32)])
def test_class_export_layout_and_import(shape, nlev, dtype):
    print(f"\n[case] class export {shape} nlev={nlev} {np.dtype(dtype).name}", flush=True)
    if nlev is None:
        nlev = oracle.max_levels(shape)
    rng = np.random.default_rng(5)
    rep = rng.standard_normal(shape).astype(dtype)
    x = torch.from_numpy(rep).cuda()
    buf = mgr.export_classes(x, nlev)
    back = mgr.import_classes(buf, nlev)
    torch.cuda.synchronize()
    ref = _classes_reference(rep, nlev)
    assert np.array_equal(buf.cpu().numpy().ravel(), ref)
    assert torch.equal(back, x)
    sizes = mgr.class_sizes(shape, nlev)
    assert sum(sizes) == x.numel()


@pytest.mark.parametrize("shape,nonuni", [((65, 65, 65), False), ((66, 70, 45), True)])
def test_class_prefix_recomposes_like_partial_recompose(shape, nonuni):
    print(f"\n[case] class prefix vs partial recompose {shape}", flush=True)
    u, coords = make_input(shape, 21, nonuniform=nonuni, dtype=np.float64)
    nlev = oracle.max_levels(shape)
    x = torch.from_numpy(u).cuda()
    d = mgr.decompose(x, coords, nlev)
    buf = mgr.export_classes(d, nlev)
    sizes = mgr.class_sizes(shape, nlev)
    for nkeep in range(nlev + 1):
        prefix = sum(sizes[:1 + nkeep])
        cut = torch.zeros_like(buf)
        cut.view(-1)[:prefix] = buf.view(-1)[:prefix]
        rep = mgr.import_classes(cut, nlev)
        full = mgr.recompose(rep, coords, nlev)
        part = mgr.recompose_partial(d, nkeep, coords, nlev)
        torch.cuda.synchronize()
        assert torch.equal(full, part), nkeep
