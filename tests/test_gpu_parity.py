"""GPU parity of every hot-path step against the FP64 oracle (through the C ABI).

Tolerances: integer outputs bit-exact; FP64 results within 1e-12 relative
(normwise over the covered cells or markers); FP32 results within 1e-5
relative of the oracle run on the same FP64 inputs; per-particle sums within
tol * sum |summands| (they cancel around a sphere).
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import Case, announce, gpu_device, rel, resid_bounds, small_workload

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def _cases():
    return [
        ("small32_P4", lambda: small_workload(32, 16, 4, 3, 1)),
        ("small32_P3", lambda: small_workload(32, 16, 3, 2, 2)),
        ("small64_partial_P4", lambda: small_workload(64, 16, 4, 3, 3, cover_all=False, k=5)),
        ("sphere1_64", lambda: W.config(1, 0)),
    ]


CASES = _cases()


def _odd_tiles():
    """A 40^3 grid of 8^3 boxes: five tiles per axis, so with 16-wide
    interpolation work tiles the last tile of every row is an item on its
    own; one sphere reaches into those tiles across the periodic seam."""
    h = 1.0 / 40
    return [("odd_tiles40_P4",
             lambda: W.make_workload("odd40", 40, 8, 2, 4, 3, np.array([9.0, 7.5]),
                                     centres=[[37.3 * h, 20.4 * h, 11.8 * h],
                                              [14.6 * h, 9.9 * h, 30.2 * h]],
                                     nmodes=8, K=4, cover_all=True))]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_build_markers(dev, name, mk):
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce(f"build_markers {name}")
    wl = mk()
    c = Case(wl, dev)
    m = ibx.build_markers(c.dl, c.parts)
    torch.cuda.synchronize()
    assert np.array_equal(m.offs.cpu().numpy(), c.m.offs)
    assert np.array_equal(m.pid.cpu().numpy(), c.m.pid)
    assert rel(m.dv.cpu().numpy(), c.m.dv) <= 1e-15
    X = m.xyz().cpu().numpy()
    assert np.max(np.abs(X - c.m.xyz())) <= 4e-16 * 4
    assert ibx.count_markers(wl.d, wl.level.h).tolist() == O.count_markers(wl.d, wl.level.h).tolist()


def _bucket_extra():
    """Grids that take the other branches of the source-list construction: two
    bounded axes (stencils within a few cells of both ends, and wrapping on
    the periodic one), and a 16^3 grid with only two tiles per axis (the
    sort-based construction)."""
    h48 = 1.0 / 48
    bounded = [[6.3 * h48, 2.1 * h48, 40.2 * h48], [24.5 * h48, 24.2 * h48, 7.0 * h48],
               [41.0 * h48, 46.7 * h48, 24.3 * h48]]
    h16 = 1.0 / 16
    return [
        ("bounded48_P4", lambda: W.make_workload("bounded48", 48, 16, 2, 4, 2,
                                                 np.full(3, 8.0), centres=bounded, nmodes=8,
                                                 K=4, cover_all=True, periodic=(0, 1, 0))),
        ("bounded48_P3", lambda: W.make_workload("bounded48", 48, 16, 2, 3, 2,
                                                 np.full(3, 8.0), centres=bounded, nmodes=8,
                                                 K=4, cover_all=True, periodic=(0, 1, 0))),
        ("two_tiles16_P4", lambda: W.make_workload("two16", 16, 16, 2, 4, 2, np.full(2, 5.0),
                                                   centres=[[4 * h16, 4.2 * h16, 3.9 * h16],
                                                            [12.1 * h16, 11 * h16, 10.3 * h16]],
                                                   nmodes=8, K=4, cover_all=True)),
    ]


@pytest.mark.parametrize("name,mk", CASES + _bucket_extra(),
                         ids=[c[0] for c in CASES + _bucket_extra()])
def test_bucket_bit_exact(dev, name, mk):
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce(f"bucket {name}")
    wl = mk()
    c = Case(wl, dev)
    ref = O.bucket(c.lev, wl.delta, c.m)
    b = ibx.bucket(c.dl, c.dm, wl.delta)
    torch.cuda.synchronize()
    assert ref["flagged"] == 0 and int(b.flag[0].item()) == 0 and int(b.flag[1].item()) == 0
    for k in ("cell", "base", "perm", "tile_offs", "src_offs"):
        got = getattr(b, k if k != "tile" else "tileid").cpu().numpy()
        assert np.array_equal(got, ref[k]), k
    assert np.array_equal(b.tileid.cpu().numpy(), ref["tile"])
    ns = int(ref["src_offs"][-1])
    assert np.array_equal(b.src_idx[:ns].cpu().numpy(), ref["src_idx"])


def test_bucket_flags_uncovered_support(dev):
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce("bucket flag")
    n, box = 32, 16
    cov = np.ones((2, 2, 2), bool)
    cov[0, 0, 1] = False
    lev = W.make_level((n, n, n), 1.0 / n, box=box, ngrow=2, covered=cov)
    m = O.build_markers([[0.45, 0.25, 0.25], [0.25, 0.25, 0.75]], [6 / n, 5 / n], 1 / n)
    ref = O.bucket(lev, 4, m)
    dl = ibx.device_level(lev, dev)
    dm = ibx.markers_from(m.x, m.y, m.z, m.pid, m.dv, m.offs, dev)
    b = ibx.bucket(dl, dm, 4)
    torch.cuda.synchronize()
    assert ref["flagged"] > 0
    assert int(b.flag[0].item()) == ref["flagged"]
    assert np.array_equal(b.perm.cpu().numpy(), ref["perm"])


def _valid_cells(dl, t):
    g = dl.ngrow
    return t[:, :, g:g + dl.box, g:g + dl.box, g:g + dl.box]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_flagged_buckets_poison_outputs(dev, dtype):
    """A marker stencil reaching an uncovered box: every call that uses the
    flagged bucket set writes NaN into all its outputs (no host read of the
    flag is needed), interpolation gives NaN exactly on the markers whose
    stencil leaves the coverage, and the per-particle sums are NaN for the
    particle whose cells do."""
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce(f"flagged buckets poison outputs {dtype}")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    n, box = 32, 16
    cov = np.ones((2, 2, 2), bool)
    cov[0, 0, 1] = False
    lev = W.make_level((n, n, n), 1.0 / n, box=box, ngrow=2, covered=cov)
    xc = np.array([[0.45, 0.25, 0.25], [0.25, 0.25, 0.75]])
    d = np.array([6 / n, 5 / n])
    rng = np.random.default_rng(21)
    up, om = rng.normal(0, 0.1, (2, 3)), rng.normal(0, 1, (2, 3))
    m = O.build_markers(xc, d, 1 / n)
    ref = O.bucket(lev, 4, m)
    dl = ibx.device_level(lev, dev)
    parts = ibx.particles(xc, d, up, om, dev)
    dm = ibx.markers_from(m.x, m.y, m.z, m.pid, m.dv, m.offs, dev)
    b = ibx.bucket(dl, dm, 4)
    u0 = torch.as_tensor(rng.normal(size=dl.field_shape()), device=dev).to(tdt)
    ns, dt = 3, 0.5 / n
    for path in (ibx.IB_PATH_PLAIN, ibx.IB_PATH_BATCHED):
        plan = ibx.Plan(4, tdt, path)
        r = torch.zeros(ns + 1, dtype=torch.float64, device=dev)
        Fh = torch.zeros((ns, m.nl, 3), dtype=tdt, device=dev)
        ustar, f, F = plan.multidirect_force(dl, parts, dm, b, ns, dt, u0, resid=r, Fhist=Fh)
        bw = plan.backward(dl, parts, dm, b, ns, dt, u0, Fh, g_f=torch.ones_like(u0),
                           g_F=torch.ones_like(F))
        torch.cuda.synchronize()
        for t in (_valid_cells(dl, ustar), _valid_cells(dl, f), F, r, Fh,
                  _valid_cells(dl, bw[0]), bw[1], bw[2], bw[3]):
            assert bool(torch.isnan(t).all()), path
    f = ibx.spread(dl, dm, b, 4, torch.ones((m.nl, 3), dtype=tdt, device=dev))
    torch.cuda.synchronize()
    assert bool(torch.isnan(_valid_cells(dl, f)).all())
    # the loop in particle order buckets each level itself
    plan = ibx.Plan(4, tdt, ibx.IB_PATH_BATCHED)
    flag = torch.zeros(2, dtype=torch.int32, device=dev)
    ustar, f, F = plan.multidirect_sequential(dl, parts, dm, ns, dt, u0, flag=flag)
    torch.cuda.synchronize()
    assert int(flag[0].item()) > 0
    for t in (_valid_cells(dl, ustar), _valid_cells(dl, f), F):
        assert bool(torch.isnan(t).all())
    # interpolation: NaN exactly on the markers the bucketing counted
    U = ibx.interp(dl, dm, 4, u0)
    torch.cuda.synchronize()
    bad = torch.isnan(U).any(dim=1)
    assert bool((torch.isnan(U).all(dim=1) == bad).all())
    assert int(bad.sum().item()) == ref["flagged"] == int(b.flag[0].item())
    # reductions: particle 0's body crosses x = 1/2 into the uncovered box
    # (boxes are indexed z, y, x), particle 1 lies in covered boxes
    rflag = torch.zeros(1, dtype=torch.int32, device=dev)
    out = ibx.particle_reductions(dl, parts, dm, torch.ones((m.nl, 3), dtype=tdt, device=dev),
                                  u0, flag=rflag)
    torch.cuda.synchronize()
    assert int(rflag.item()) == 1
    assert bool(torch.isnan(out[0]).all()) and bool(torch.isfinite(out[1]).all())


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_interp_and_spread(dev, name, mk, dtype):
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce(f"interp/spread {name} {dtype}")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    tol = TOL64 if dtype == "f64" else TOL32
    wl = mk()
    c = Case(wl, dev)
    rng = np.random.default_rng(7)
    F = rng.normal(size=(c.m.nl, 3))
    Uref = O.interp(c.g, wl.delta, c.m, wl.u0)
    fref = O.spread(c.g, wl.delta, c.m, F)
    b = ibx.bucket(c.dl, c.dm, wl.delta)
    U = ibx.interp(c.dl, c.dm, wl.delta, c.u0_boxes(tdt))
    f = ibx.spread(c.dl, c.dm, b, wl.delta, torch.as_tensor(F, device=dev).to(tdt))
    torch.cuda.synchronize()
    assert rel(U.cpu().numpy(), Uref) <= tol
    assert c.field_rel(f, fref) <= tol


def _run(c, dtype, path, resid=True, inplace=False, ns=None, fhist=False, **kw):
    import torch

    import paper_2408_14140_amd as ibx
    wl = c.wl
    ns = wl.ns if ns is None else ns
    tdt = torch.float64 if dtype == "f64" else torch.float32
    b = ibx.bucket(c.dl, c.dm, wl.delta)
    plan = ibx.Plan(wl.delta, tdt, path, **kw)
    u0 = c.u0_boxes(tdt)
    r = torch.zeros(ns + 1, dtype=torch.float64, device=c.dev) if resid else None
    Fh = torch.zeros((max(ns, 1), c.m.nl, 3), dtype=tdt, device=c.dev) if fhist else None
    ustar, f, F = plan.multidirect_force(c.dl, c.parts, c.dm, b, ns, wl.dt, u0,
                                         ustar=u0 if inplace else None, resid=r, Fhist=Fh)
    torch.cuda.synchronize()
    return ustar, f, F, r, Fh, b


PATHS = [("f64", 1), ("f64", 2), ("f32", 2), ("f32", 1)]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("dtype,path", PATHS, ids=[f"{d}-{'plain' if p == 1 else 'batched'}" for d, p in PATHS])
def test_multidirect_matches_oracle(dev, name, mk, dtype, path):
    import oracle as O
    announce(f"multidirect {name} {dtype} path={path}")
    wl = mk()
    c = Case(wl, dev)
    ref = O.multidirect(c.g, wl.delta, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0,
                        history=True)
    ustar, f, F, r, Fh, _ = _run(c, dtype, path, fhist=True)
    tol = TOL64 if dtype == "f64" else TOL32
    assert rel(F.cpu().numpy(), ref["F"]) <= tol
    assert c.field_rel(f, ref["f"]) <= tol
    assert c.field_rel(ustar, ref["ustar"]) <= tol
    assert rel(Fh.cpu().numpy(), ref["Fhist"]) <= tol
    bound = resid_bounds(c.g, wl.delta, c.m, wl.xc, wl.up, wl.om, wl.u0, ref["resid"], tol)
    assert np.all(np.abs(r.cpu().numpy() - ref["resid"]) <= bound)


def _two_tiles_p3():
    h16 = 1.0 / 16
    return W.make_workload("two16_P3", 16, 16, 2, 3, 2, np.full(2, 5.0),
                           centres=[[3.6 * h16, 12.2 * h16, 7.7 * h16],
                                    [12.1 * h16, 4.4 * h16, 15.2 * h16]],
                           nmodes=8, K=4, cover_all=True)


_SMALL_GRIDS = _bucket_extra() + [("two_tiles16_P3", _two_tiles_p3)]


@pytest.mark.parametrize("name,mk", _SMALL_GRIDS, ids=[c[0] for c in _SMALL_GRIDS])
@pytest.mark.parametrize("dtype,path", PATHS, ids=[f"{d}-{'plain' if p == 1 else 'batched'}" for d, p in PATHS])
def test_bounded_and_small_grids_match_oracle(dev, name, mk, dtype, path):
    """Walls on x and z (y periodic), particles a few cells from them: tiles
    beyond a wall have no neighbour (their halo reads zero) in every kernel;
    and a 16^3 grid of two tiles per axis (source lists built by sorting,
    both neighbours of a tile the same tile across the periodic seam)."""
    import oracle as O
    announce(f"bounded or small grid {name} {dtype} path={path}")
    wl = mk()
    c = Case(wl, dev)
    ref = O.multidirect(c.g, wl.delta, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0)
    ustar, f, F, _, _, b = _run(c, dtype, path, resid=False)
    assert int(b.flag[0].item()) == 0
    tol = TOL64 if dtype == "f64" else TOL32
    assert rel(F.cpu().numpy(), ref["F"]) <= tol
    assert c.field_rel(f, ref["f"]) <= tol
    assert c.field_rel(ustar, ref["ustar"]) <= tol


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_row_masks_match_oracle_and_unmasked(dev, name, mk, dtype):
    """The batched loop with the slot row masks (zero rows of G neither stored
    nor loaded): against the oracle, and the same values as without them,
    with residuals, force history and in place."""
    import torch

    import oracle as O
    announce(f"row masks {name} {dtype}")
    wl = mk()
    c = Case(wl, dev)
    ref = O.multidirect(c.g, wl.delta, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0,
                        history=True)
    a = _run(c, dtype, 2, fhist=True)
    mk_ = _run(c, dtype, 2, fhist=True, row_masks=True)
    tol = TOL64 if dtype == "f64" else TOL32
    ustar, f, F, r, Fh, _ = mk_
    assert rel(F.cpu().numpy(), ref["F"]) <= tol
    assert c.field_rel(f, ref["f"]) <= tol
    assert c.field_rel(ustar, ref["ustar"]) <= tol
    assert rel(Fh.cpu().numpy(), ref["Fhist"]) <= tol
    bound = resid_bounds(c.g, wl.delta, c.m, wl.xc, wl.up, wl.om, wl.u0, ref["resid"], tol)
    assert np.all(np.abs(r.cpu().numpy() - ref["resid"]) <= bound)
    m = np.broadcast_to(c.mask, (3,) + c.mask.shape)
    for x, y in zip(a[:2], mk_[:2]):
        assert np.array_equal(c.to_global(x)[m], c.to_global(y)[m])
    for x, y in zip(a[2:5], mk_[2:5]):
        assert torch.equal(x, y)
    ip = _run(c, dtype, 2, inplace=True, resid=False, row_masks=True)
    assert np.array_equal(c.to_global(ip[0])[m], c.to_global(a[0])[m])
    assert torch.equal(ip[2], a[2])


@pytest.mark.parametrize("name,mk", CASES + _odd_tiles(), ids=[c[0] for c in CASES + _odd_tiles()])
@pytest.mark.parametrize("masks", [False, True], ids=["", "masks"])
def test_interp_tile_16_matches_oracle_and_8(dev, name, mk, masks):
    """FP32 loop with interpolation work tiles of two x neighbours (16 x 8 x 8,
    one shared halo): against the oracle, and against the 8^3 work tiles to
    rounding (1e-6; an item's marker count decides over how many lanes each
    marker's stencil is summed), with residuals, force history and in
    place."""
    import torch

    import oracle as O
    announce(f"interp tile 16 {name} masks={masks}")
    wl = mk()
    c = Case(wl, dev)
    ref = O.multidirect(c.g, wl.delta, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0,
                        history=True)
    a = _run(c, "f32", 2, fhist=True, row_masks=masks)
    w = _run(c, "f32", 2, fhist=True, row_masks=masks, interp_tile=16)
    ustar, f, F, r, Fh, _ = w
    assert rel(F.cpu().numpy(), ref["F"]) <= TOL32
    assert c.field_rel(f, ref["f"]) <= TOL32
    assert c.field_rel(ustar, ref["ustar"]) <= TOL32
    m = np.broadcast_to(c.mask, (3,) + c.mask.shape)
    for x, y in zip(a[:2], w[:2]):
        assert rel(c.to_global(y)[m], c.to_global(x)[m]) <= 1e-6
    for x, y in zip(a[2:5], w[2:5]):
        assert rel(y.double().cpu().numpy(), x.double().cpu().numpy()) <= 1e-6
    ip = _run(c, "f32", 2, inplace=True, resid=False, row_masks=masks, interp_tile=16)
    assert np.array_equal(c.to_global(ip[0])[m], c.to_global(w[0])[m])
    assert torch.equal(ip[2], w[2])
    # and reproducible: a second run gives the same bits
    w2 = _run(c, "f32", 2, fhist=True, row_masks=masks, interp_tile=16)
    for x, y in zip(w[2:5], w2[2:5]):
        assert torch.equal(x, y)


def test_interp_tile_16_is_fp32_only(dev):
    import torch

    import paper_2408_14140_amd as ibx
    announce("interp tile 16 refused in FP64")
    with pytest.raises(ibx.IbxError) as e:
        ibx.Plan(4, torch.float64, ibx.IB_PATH_BATCHED, interp_tile=16)
    assert e.value.status == ibx.IB_EUNSUPPORTED
    with pytest.raises(ibx.IbxError):
        ibx.Plan(4, torch.float32, ibx.IB_PATH_BATCHED, interp_tile=12)


@pytest.mark.parametrize("ns", [1, 2])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_row_masks_short_loops(dev, ns, dtype):
    """One and two iterations with the slot row masks: the last spreading
    writes the masks that the finalize step and the residual read."""
    import torch
    announce(f"row masks ns={ns} {dtype}")
    wl = small_workload(32, 16, 4, 3, 1)
    c = Case(wl, dev)
    a = _run(c, dtype, 2, ns=ns)
    b = _run(c, dtype, 2, ns=ns, row_masks=True)
    m = np.broadcast_to(c.mask, (3,) + c.mask.shape)
    for x, y in zip(a[:2], b[:2]):
        assert np.array_equal(c.to_global(x)[m], c.to_global(y)[m])
    for x, y in zip(a[2:4], b[2:4]):
        assert torch.equal(x, y)


def test_batched_in_place_and_deterministic(dev):
    import torch
    announce("in-place + determinism")
    wl = small_workload(64, 16, 4, 3, 3, cover_all=False, k=5)
    c = Case(wl, dev)
    a = _run(c, "f32", 2)
    b = _run(c, "f32", 2)
    # fields: valid cells of covered boxes only (ghost cells are never written)
    m = np.broadcast_to(c.mask, (3,) + c.mask.shape)
    for x, y in zip(a[:2], b[:2]):
        assert np.array_equal(c.to_global(x)[m], c.to_global(y)[m])
    for x, y in zip(a[2:4], b[2:4]):
        assert torch.equal(x, y)
    ip = _run(c, "f32", 2, inplace=True)
    assert np.array_equal(c.to_global(ip[0])[m], c.to_global(a[0])[m])
    assert torch.equal(ip[2], a[2])


@pytest.mark.parametrize("ns", [0, 1])
@pytest.mark.parametrize("dtype,path", PATHS, ids=[f"{d}-{p}" for d, p in PATHS])
def test_short_loops(dev, ns, dtype, path):
    import oracle as O
    announce(f"short loop ns={ns} {dtype} {path}")
    wl = small_workload(32, 16, 4, 3, 1)
    c = Case(wl, dev)
    ref = O.multidirect(c.g, wl.delta, ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0)
    ustar, f, F, r, _, _ = _run(c, dtype, path, ns=ns)
    tol = TOL64 if dtype == "f64" else TOL32
    assert rel(F.cpu().numpy(), ref["F"]) <= tol
    assert c.field_rel(ustar, ref["ustar"]) <= tol
    got_f = c.to_global(f)
    m = np.broadcast_to(c.mask, got_f.shape)
    assert np.max(np.abs(got_f[m] - ref["f"][m])) <= tol * max(1.0, np.abs(ref["f"]).max())
    bound = resid_bounds(c.g, wl.delta, c.m, wl.xc, wl.up, wl.om, wl.u0, ref["resid"], tol)
    assert abs(r.cpu().numpy()[0] - ref["resid"][0]) <= bound[0]


def test_no_markers(dev):
    import torch

    import paper_2408_14140_amd as ibx
    announce("no particles")
    wl = small_workload(32, 16, 4, 3, 1)
    lev = wl.level
    dl = ibx.device_level(lev, dev)
    parts = ibx.particles(np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)), dev)
    dm = ibx.markers_from(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0, np.int32),
                          np.zeros(0), np.zeros(1, np.int64), dev)
    b = ibx.bucket(dl, dm, 4)
    for dtype, path in PATHS:
        tdt = torch.float64 if dtype == "f64" else torch.float32
        plan = ibx.Plan(4, tdt, path)
        u0 = torch.as_tensor(W.to_boxes(wl.u0, lev, fill=np.nan), device=dev).to(tdt)
        r = torch.full((4,), -1.0, dtype=torch.float64, device=dev)
        ustar, f, F = plan.multidirect_force(dl, parts, dm, b, 3, wl.dt, u0, resid=r)
        torch.cuda.synchronize()
        us = W.from_boxes(ustar.double().cpu().numpy(), lev)
        assert np.array_equal(us, W.from_boxes(u0.double().cpu().numpy(), lev))
        assert float(np.nanmax(np.abs(W.from_boxes(f.double().cpu().numpy(), lev)))) == 0.0
        assert torch.all(r == 0)


def test_box_tiling_invariance(dev):
    """32^3 boxes and one 64^3 box hold the same grid: results agree."""
    import torch
    announce("box tiling invariance")
    wl = small_workload(64, 16, 4, 3, 5, cover_all=True, k=4)
    outs = []
    for box in (64, 32, 16):
        lev = W.make_level(wl.level.n, wl.level.h, box=box, ngrow=2 if box < 64 else 0)
        w2 = W.Workload(wl.name, lev, wl.delta, wl.ns, wl.dt, wl.xc, wl.d, wl.up, wl.om, wl.u0)
        c = Case(w2, dev)
        ustar, f, F, _, _, _ = _run(c, "f64", 2, resid=False)
        outs.append((c.to_global(ustar), F.cpu().numpy()))
    for u, F in outs[1:]:
        assert rel(u, outs[0][0]) <= 1e-14
        assert rel(F, outs[0][1]) <= 1e-14


@pytest.mark.parametrize("delta", [3, 4])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_odd_ghost_width(dev, dtype, delta):
    """Ghost widths 1 and 3 (the halo staged cell by cell) against the oracle,
    and against ghost width 2 (staged in x pairs) bit for bit: the same
    values reach every kernel, only from other addresses."""
    import oracle as O
    announce(f"odd ghost width {dtype} P{delta}")
    wl = small_workload(32, 16, delta, 3, 6)
    c0 = Case(wl, dev)
    ref = O.multidirect(c0.g, wl.delta, wl.ns, wl.dt, c0.m, wl.xc, wl.up, wl.om, wl.u0)
    tol = TOL64 if dtype == "f64" else TOL32
    outs = []
    for ng in (2, 1, 3):
        lev = W.make_level(wl.level.n, wl.level.h, box=16, ngrow=ng)
        w2 = W.Workload(wl.name, lev, wl.delta, wl.ns, wl.dt, wl.xc, wl.d, wl.up, wl.om, wl.u0)
        c = Case(w2, dev)
        ustar, f, F, _, _, _ = _run(c, dtype, 2, resid=False)
        outs.append((c.to_global(ustar), c.to_global(f), F.cpu().numpy()))
        assert rel(outs[-1][2], ref["F"]) <= tol
        assert rel(outs[-1][0], ref["ustar"]) <= tol
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def _dense_clump(delta):
    """40 spheres of 6-10 cells packed around one point of a 64^3 grid (each
    centre within 2 cells of it): a few tiles receive thousands of sources,
    so every spreading batch cuts the heavier rows or blocks into pieces."""
    rng = np.random.default_rng(31 + delta)
    n = 64
    xc = 0.5 + rng.normal(0.0, 1.0 / n, size=(40, 3))
    return W.make_workload(f"dense_clump_P{delta}", n, 16, 2, delta, 3,
                           rng.uniform(6.0, 10.0, 40), centres=xc, nmodes=8, K=4,
                           cover_all=True)


@pytest.mark.parametrize("delta", [3, 4])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dense_clump_matches_oracle(dev, dtype, delta):
    """Heavy tiles (the pieces of the spreading's second phase) with and
    without the slot row masks, against the oracle; the masks change no bit."""
    import torch

    import oracle as O
    announce(f"dense clump {dtype} P{delta}")
    wl = _dense_clump(delta)
    c = Case(wl, dev)
    ref = O.multidirect(c.g, wl.delta, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0)
    counts = np.diff(O.bucket(c.lev, wl.delta, c.m)["src_offs"])
    assert counts.max() > 2000                    # heavy tiles, as intended
    tol = TOL64 if dtype == "f64" else TOL32
    outs = []
    for masks in (False, True):
        ustar, f, F, _, _, _ = _run(c, dtype, 2, resid=False, row_masks=masks)
        assert rel(F.cpu().numpy(), ref["F"]) <= tol
        assert c.field_rel(f, ref["f"]) <= tol
        assert c.field_rel(ustar, ref["ustar"]) <= tol
        outs.append((c.to_global(ustar), c.to_global(f), F.cpu().numpy()))
    for x, y in zip(*outs):                       # valid cells only
        assert np.array_equal(x, y)


def _big_spheres():
    """Two spheres far larger than the others here (bounding boxes of 64 and
    75 cells per axis, thousands of near-surface cells per workgroup, so the
    per-wavefront queues fill and drain many times), both wrapping across the
    periodic boundaries."""
    h = 1.0 / 96
    xc = np.array([[48.9 * h] * 3, [10.3 * h, 88.6 * h, 47.2 * h]])
    return W.make_workload("big_spheres96", 96, 32, 2, 4, 2, np.array([60.4, 72.0]),
                           centres=xc, nmodes=8, K=4, cover_all=True)


def _exact_edges():
    """Spheres whose extents end exactly on nodes: centred on a node (one at a
    box corner, one on node 0, wrapping x and z) with R = 8 h, and centred in a
    cell with R = 7.5 h, so s - e and s + e are integers and the surface passes
    through nodes (phi = 0 there), the edge of the cells the volume sums visit."""
    h = 1.0 / 64
    xc = np.array([[32 * h, 32 * h, 32 * h], [0.0, 16 * h, 63 * h],
                   [20.5 * h, 50.5 * h, 10.5 * h]])
    return W.make_workload("exact_edges64", 64, 32, 2, 4, 2, np.array([16.0, 16.0, 15.0]),
                           centres=xc, nmodes=8, K=4, cover_all=True)


RED_CASES = CASES + [("big_spheres96", _big_spheres), ("exact_edges64", _exact_edges)]


@pytest.mark.parametrize("name,mk", RED_CASES, ids=[c[0] for c in RED_CASES])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_particle_reductions(dev, name, mk, dtype):
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce(f"reductions {name} {dtype}")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    wl = mk()
    c = Case(wl, dev)
    rng = np.random.default_rng(9)
    F = rng.normal(size=(c.m.nl, 3))
    if dtype == "f32":
        F = F.astype(np.float32).astype(np.float64)
        u_in = wl.u0.astype(np.float32).astype(np.float64)
    else:
        u_in = wl.u0
    ref = O.particle_reductions(c.g, c.m, wl.xc, wl.d, F, u_in)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    u = torch.as_tensor(W.to_boxes(u_in, c.lev, fill=np.nan), device=dev).to(tdt)
    out = ibx.particle_reductions(c.dl, c.parts, c.dm, torch.as_tensor(F, device=dev).to(tdt),
                                  u, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    got = out.cpu().numpy()
    # scale: a bound on sum |summands| per particle and quantity
    absref = O.particle_reductions(c.g, c.m, wl.xc, wl.d, np.abs(F), np.abs(u_in))
    Rmax = 0.5 * wl.d.max() + 3 * c.lev.h
    scale = np.empty_like(absref)
    scale[:, 0:3] = absref[:, 0:3]
    scale[:, 3:6] = absref[:, 0:3].sum(axis=1, keepdims=True) * Rmax
    scale[:, 6:9] = absref[:, 6:9]
    scale[:, 9:12] = absref[:, 6:9].sum(axis=1, keepdims=True) * Rmax
    assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-300)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_autotune_keeps_parity(dev, dtype):
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce(f"autotune {dtype}")
    wl = small_workload(64, 16, 4, 3, 3, cover_all=False, k=5)
    c = Case(wl, dev)
    ref = O.multidirect(c.g, wl.delta, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    b = ibx.bucket(c.dl, c.dm, wl.delta)
    plan = ibx.Plan(wl.delta, tdt, ibx.IB_PATH_BATCHED)
    u0 = c.u0_boxes(tdt)
    u0_before = u0.clone()
    outs = (torch.full_like(u0, float("nan")), torch.full_like(u0, float("nan")),
            torch.full((c.m.nl, 3), float("nan"), dtype=tdt, device=dev))
    choice = plan.autotune(c.dl, c.parts, c.dm, b, wl.ns, wl.dt, u0, outputs=outs)
    # the timing runs leave u0 as it was, and the outputs hold one whole run
    # at the chosen tuning (the timed runs write ustar only where G != 0)
    assert torch.allclose(u0, u0_before, rtol=0.0, atol=0.0, equal_nan=True)   # NaN ghosts
    assert choice["bucket_width"] in (64, 128, 256)
    assert choice["spread_wgs_per_cu"] in (4, 8, 16, 32)
    assert choice["loop_ms"] > 0.0
    assert plan.query() == {k: v for k, v in choice.items() if k != "loop_ms"}
    ustar, f, F = plan.multidirect_force(c.dl, c.parts, c.dm, b, wl.ns, wl.dt, u0)
    torch.cuda.synchronize()
    for x, y in zip(outs[:2], (ustar, f)):       # valid cells (NaN where uncovered)
        assert np.array_equal(c.to_global(x), c.to_global(y), equal_nan=True)
    assert torch.equal(outs[2], F)
    tol = TOL64 if dtype == "f64" else TOL32
    assert rel(F.cpu().numpy(), ref["F"]) <= tol
    assert c.field_rel(f, ref["f"]) <= tol
    assert c.field_rel(ustar, ref["ustar"]) <= tol
    with pytest.raises(ibx.IbxError):
        ibx.Plan(wl.delta, tdt, ibx.IB_PATH_PLAIN).autotune(c.dl, c.parts, c.dm, b, wl.ns,
                                                             wl.dt, u0)


def test_batched_rejects_unsupported_levels(dev):
    """The batched path needs at least 16 cells per axis and a stencil base
    that fits its 21-bit packed field (n <= 2^21 - 5 per axis); beyond either
    it returns IB_EUNSUPPORTED before any kernel runs."""
    import torch

    import paper_2408_14140_amd as ibx
    announce("batched path rejects unsupported levels")
    for n, box in (((32, 32, 8), 8), ((1 << 21, 16, 16), 16)):
        h = 1.0 / 16
        nb = [v // box for v in n]
        cov = np.zeros((nb[2], nb[1], nb[0]), dtype=bool)
        cov[0, 0, 0] = True
        lev = W.make_level(n, h, box=box, ngrow=2, covered=cov)
        dl = ibx.device_level(lev, dev)
        xc = np.array([[0.5 * box * h + 0.01 * h, 0.5 * box * h, 0.5 * box * h - 0.02 * h]])
        d = np.array([0.3 * box * h])
        parts = ibx.particles(xc, d, np.zeros((1, 3)), np.zeros((1, 3)), dev)
        m = ibx.build_markers(dl, parts)
        b = ibx.bucket(dl, m, 4)
        plan = ibx.Plan(4, torch.float32, ibx.IB_PATH_BATCHED)
        u0 = torch.zeros((lev.nbox, 3) + (box + 4,) * 3, dtype=torch.float32, device=dev)
        with pytest.raises(ibx.IbxError) as e:
            plan.multidirect_force(dl, parts, m, b, 2, 0.5 * h, u0)
        assert e.value.status == ibx.IB_EUNSUPPORTED


@pytest.mark.parametrize("delta", [3, 4])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_misaligned_fields(dev, dtype, delta):
    """Fields that start one element past a two-element boundary take the
    single-cell halo staging and finalize instead of the pair ones: the
    results are the same bit for bit."""
    import torch

    import paper_2408_14140_amd as ibx
    announce(f"batched path, misaligned field pointers {dtype} P{delta}")
    wl = small_workload(32, 16, delta, 3, 2)
    c = Case(wl, dev)
    b = ibx.bucket(c.dl, c.dm, wl.delta)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    plan = ibx.Plan(wl.delta, tdt, ibx.IB_PATH_BATCHED)
    u0 = c.u0_boxes(tdt)

    def shifted(t):
        base = torch.full((t.numel() + 1,), float("nan"), dtype=t.dtype, device=dev)
        v = base[1:].view(t.shape)
        v.copy_(t)
        assert v.data_ptr() % (2 * t.element_size()) == t.element_size()
        return v

    outs = []
    for mis in (False, True):
        src = shifted(u0) if mis else u0.clone()
        ustar = shifted(torch.zeros_like(u0)) if mis else torch.zeros_like(u0)
        f = shifted(torch.zeros_like(u0)) if mis else torch.zeros_like(u0)
        _, _, F = plan.multidirect_force(c.dl, c.parts, c.dm, b, wl.ns, wl.dt, src, ustar=ustar,
                                         f=f)
        torch.cuda.synchronize()
        outs.append((ustar.cpu().numpy(), f.cpu().numpy(), F.cpu().numpy()))
    for a, bb in zip(outs[0], outs[1]):
        assert np.array_equal(a, bb, equal_nan=True)


@pytest.mark.parametrize("name,mk", [CASES[0], _bucket_extra()[2]],
                         ids=[CASES[0][0], _bucket_extra()[2][0]])
def test_bucket_source_list_overflow(dev, name, mk):
    """A source-list capacity below the pair count raises flag[1]; the list
    bounds stay within the capacity and non-decreasing, so consumers never
    read past it."""
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce(f"bucket overflow {name}")
    wl = mk()
    c = Case(wl, dev)
    ref = O.bucket(c.lev, wl.delta, c.m)
    need = int(ref["src_offs"][-1])
    cap = need // 2
    # the by-direction case has tiles that no stencil reaches, placed past the
    # capacity: their bounds must be clamped too, although they have no runs
    if name == CASES[0][0]:
        ro = np.asarray(ref["src_offs"])
        assert np.any((np.diff(ro) == 0) & (ro[:-1] > cap))
    b = ibx.bucket(c.dl, c.dm, wl.delta, src_cap=cap)
    torch.cuda.synchronize()
    assert int(b.flag[1].item()) == 1
    so = b.src_offs.cpu().numpy()
    assert so[0] == 0 and so[-1] == cap and np.all(np.diff(so) >= 0)
    assert np.array_equal(b.tile_offs.cpu().numpy(), ref["tile_offs"])
