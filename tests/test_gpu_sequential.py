"""GPU parity of the particle-by-particle order of the loop (Sec. 3.1, the
remarks after Algorithm 1): conflict levels bit-exact against their
definition, and the level-by-level loop against the oracle's index-order
sweep -- whole on small grids, and per interacting cluster (on a window
around it) at the 1000-sphere 256^3 size."""
import numpy as np
import pytest

import workloads as W
from gpu_common import Case, announce, gpu_device, rel
from seq_ref import chain_workload, ref_levels

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def _L(lev):
    return [lev.n[a] * lev.h if lev.periodic[a] else 0.0 for a in range(3)]


@pytest.mark.parametrize("which", ["chain4", "chain3", "spheres1000_256", "spheres20000_512"])
def test_levels_bit_exact(dev, which):
    import paper_2408_14140_amd as ibx
    announce(f"particle levels {which}")
    if which.startswith("chain"):
        wl = chain_workload(delta=4 if which == "chain4" else 3)
    else:
        wl = W.config(W.CONFIG_NAMES.index(which) + 1, 0, with_field=False)
    lev = wl.level
    ref = ref_levels(wl.xc, wl.d, lev.h, wl.delta, _L(lev))
    dl = ibx.device_level(lev, dev)
    parts = ibx.particles(wl.xc, wl.d, wl.up, wl.om, dev)
    lvl, n = ibx.particle_levels(dl, parts, wl.delta)
    assert np.array_equal(lvl.cpu().numpy(), ref)
    assert n == int(ref.max()) + 1


@pytest.mark.parametrize("masks", [False, True], ids=["", "masks"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("P", [4, 3])
def test_sequential_matches_oracle(dev, dtype, P, masks):
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce(f"sequential chain P={P} {dtype} masks={masks}")
    wl = chain_workload(delta=P, seed=0)
    c = Case(wl, dev)
    ref = O.multidirect(c.g, P, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0,
                        order="sequential")
    jac = O.multidirect(c.g, P, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    tol = TOL64 if dtype == "f64" else TOL32
    assert rel(jac["F"], ref["F"]) > 100 * tol      # the order matters here
    plan = ibx.Plan(P, tdt, ibx.IB_PATH_BATCHED, row_masks=masks)
    levels = ibx.particle_levels(c.dl, c.parts, P)
    assert levels[1] >= 3
    flag = torch.ones(2, dtype=torch.int32, device=dev)
    ustar, f, F = plan.multidirect_sequential(c.dl, c.parts, c.dm, wl.ns, wl.dt,
                                              c.u0_boxes(tdt), levels=levels, flag=flag)
    torch.cuda.synchronize()
    assert flag.cpu().tolist() == [0, 0]
    assert rel(F.cpu().numpy(), ref["F"]) <= tol
    assert c.field_rel(f, ref["f"]) <= tol
    assert c.field_rel(ustar, ref["ustar"]) <= tol


def test_sequential_in_place_without_f(dev):
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce("sequential in place")
    wl = chain_workload(delta=4, seed=2)
    c = Case(wl, dev)
    ref = O.multidirect(c.g, 4, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0,
                        order="sequential")
    plan = ibx.Plan(4, torch.float32, ibx.IB_PATH_BATCHED)
    u = c.u0_boxes(torch.float32)
    ustar, f, F = plan.multidirect_sequential(c.dl, c.parts, c.dm, wl.ns, wl.dt, u, ustar=u,
                                              want_f=False)
    torch.cuda.synchronize()
    assert f is None
    assert rel(F.cpu().numpy(), ref["F"]) <= TOL32
    assert c.field_rel(u, ref["ustar"]) <= TOL32


def test_sequential_rejects_bad_levels(dev):
    import torch

    import paper_2408_14140_amd as ibx
    announce("sequential bad levels")
    wl = chain_workload(delta=4, seed=0)
    c = Case(wl, dev)
    plan = ibx.Plan(4, torch.float32, ibx.IB_PATH_BATCHED)
    u = c.u0_boxes(torch.float32)
    lvl, n = ibx.particle_levels(c.dl, c.parts, 4)
    bad = lvl.clone()
    bad[3] = n                                  # outside [0, n)
    with pytest.raises(ibx.IbxError):
        plan.multidirect_sequential(c.dl, c.parts, c.dm, wl.ns, wl.dt, u, levels=(bad, n))
    with pytest.raises(ibx.IbxError):
        plan.multidirect_sequential(c.dl, c.parts, c.dm, wl.ns, wl.dt, u, levels=(lvl, 0))
    plain = ibx.Plan(4, torch.float32, ibx.IB_PATH_PLAIN)
    with pytest.raises(ibx.IbxError):
        plain.multidirect_sequential(c.dl, c.parts, c.dm, wl.ns, wl.dt, u, levels=(lvl, n))


def _components(xc, d, h, P, L):
    """Connected components of the conservative conflict graph."""
    n = d.shape[0]
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    reach = 2.0 * P * h
    for j in range(n):
        dx = xc[:j] - xc[j]
        dx -= np.array(L) * np.floor(dx / np.array(L) + 0.5)
        hit = np.nonzero((dx * dx).sum(axis=1) < (0.5 * (d[:j] + d[j]) + reach) ** 2)[0]
        for i in hit:
            parent[find(int(i))] = find(j)
    comp = {}
    for p in range(n):
        comp.setdefault(find(p), []).append(p)
    return list(comp.values())


def test_sequential_spheres1000_256_clusters(dev):
    """Full size: every interacting cluster's markers against the oracle's
    index-order sweep of that cluster alone on a window around it (other
    particles never share a cell with it), and force conservation over the
    whole grid."""
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce("sequential spheres1000_256")
    wl = W.config(3, 0)
    lev = wl.level
    h, n, P = lev.h, lev.n[0], wl.delta
    mo = O.build_markers(wl.xc, wl.d, h)
    dl = ibx.device_level(lev, dev)
    parts = ibx.particles(wl.xc, wl.d, wl.up, wl.om, dev)
    dm = ibx.markers_from(mo.x, mo.y, mo.z, mo.pid, mo.dv, mo.offs, dev)
    u = torch.as_tensor(W.to_boxes(wl.u0, lev, fill=np.nan, dtype=np.float32), device=dev)
    plan = ibx.Plan(P, torch.float32, ibx.IB_PATH_BATCHED)
    levels = ibx.particle_levels(dl, parts, P)
    assert levels[1] >= 2
    flag = torch.ones(2, dtype=torch.int32, device=dev)
    ustar, f, F = plan.multidirect_sequential(dl, parts, dm, wl.ns, wl.dt, u, levels=levels,
                                              flag=flag)
    torch.cuda.synchronize()
    assert flag.cpu().tolist() == [0, 0]
    Fh = F.double().cpu().numpy()
    g = lev.ngrow
    fv = f[:, :, g:g + lev.box, g:g + lev.box, g:g + lev.box]
    lhs = fv.double().sum(dim=(0, 2, 3, 4)).cpu().numpy() * h ** 3
    wdv = mo.dv[mo.pid][:, None]
    assert np.all(np.abs(lhs - (Fh * wdv).sum(axis=0)) <= TOL32 * (np.abs(Fh) * wdv).sum(axis=0))
    comps = [cp for cp in _components(wl.xc, wl.d, h, P, _L(lev)) if len(cp) >= 2]
    span = lambda cp: np.ptp(wl.xc[cp], axis=0).max()
    comps = sorted([cp for cp in comps if span(cp) < 0.4], key=len, reverse=True)[:4]
    assert comps and len(comps[0]) >= 2
    for cp in comps:
        cp = sorted(cp)
        lo = np.floor((wl.xc[cp] - 0.5 * wl.d[cp, None]).min(axis=0) / h).astype(int) - (P + 2)
        hi = np.ceil((wl.xc[cp] + 0.5 * wl.d[cp, None]).max(axis=0) / h).astype(int) + (P + 2)
        idx = [np.arange(lo[a], hi[a]) % n for a in range(3)]
        uw = np.ascontiguousarray(wl.u0[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]])
        gw = O.grid(tuple(int(v) for v in hi - lo), h, tuple(float(v) for v in lo * h),
                    periodic=(0, 0, 0))
        sub = O.build_markers(wl.xc[cp], wl.d[cp], h)
        ref = O.multidirect(gw, P, wl.ns, wl.dt, sub, wl.xc[cp], wl.up[cp], wl.om[cp], uw,
                            order="sequential")
        got = np.concatenate([Fh[mo.offs[p]:mo.offs[p + 1]] for p in cp])
        assert rel(got, ref["F"]) <= TOL32, cp
