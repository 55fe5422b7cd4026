"""GPU parity of the particle side of a time step (Sec. 3.2): the rigid-body
update and the rigid marker advection against the FP64 oracle, alone and
chained after the multidirect loop and the per-particle sums."""
import numpy as np
import pytest

import workloads as W
from gpu_common import Case, announce, gpu_device, rel, small_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def test_rigid_update_matches_oracle(dev):
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce("rigid update")
    rng = np.random.default_rng(11)
    n = 300
    xc = rng.uniform(0, 1, (n, 3))
    d = rng.uniform(0.02, 0.1, n)
    up = rng.normal(0, 0.1, (n, 3))
    om = rng.normal(0, 1, (n, 3))
    rho_p = rng.uniform(1.2, 10.0, n)
    s0, s1 = rng.normal(size=(n, 12)), rng.normal(size=(n, 12))
    Fc, Tc = rng.normal(size=(n, 3)), rng.normal(size=(n, 3))
    pr = (rng.uniform(size=n) < 0.2).astype(np.int32)
    g, rho_f, dt = [0.0, -9.81, 0.0], 1.1, 1.5e-3
    ref = O.rigid_update(xc, d, up, om, rho_p, s0, s1, rho_f, g, dt, Fc=Fc, Tc=Tc, prescribed=pr)
    parts = ibx.particles(xc, d, up, om, dev)
    t = lambda a: torch.as_tensor(a, device=dev)
    got = ibx.rigid_update(parts, t(rho_p), t(s0), t(s1), rho_f, g, dt, Fc=t(Fc), Tc=t(Tc),
                           prescribed=t(pr))
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert rel(a.cpu().numpy(), b) <= 1e-14
    # without the optional terms
    ref = O.rigid_update(xc, d, up, om, rho_p, s0, s1, rho_f, g, dt)
    got = ibx.rigid_update(parts, t(rho_p), t(s0), t(s1), rho_f, g, dt)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert rel(a.cpu().numpy(), b) <= 1e-14


def test_marker_advection_full_size(dev):
    """The 1000-sphere workload's 922,600 markers, out of place and in place."""
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce("advect markers spheres1000_256")
    wl = W.config(3, 0)
    rng = np.random.default_rng(12)
    xc1 = wl.xc + rng.normal(0, 1e-3, wl.xc.shape)
    om1 = wl.om + rng.normal(0, 0.5, wl.om.shape)
    dt = wl.dt
    mo = O.build_markers(wl.xc, wl.d, wl.level.h)
    ref = O.advect_markers(mo, wl.xc, xc1, wl.om, om1, dt)
    dm = ibx.markers_from(mo.x, mo.y, mo.z, mo.pid, mo.dv, mo.offs, dev)
    t = lambda a: torch.as_tensor(a, device=dev)
    out = ibx.advect_markers(dm, t(wl.xc), t(xc1), t(wl.om), t(om1), dt)
    torch.cuda.synchronize()
    assert np.max(np.abs(out.xyz().cpu().numpy() - ref.xyz())) <= 1e-15
    ibx.advect_markers(dm, t(wl.xc), t(xc1), t(wl.om), t(om1), dt, out=dm)
    torch.cuda.synchronize()
    assert torch.equal(dm.xyz(), out.xyz())


@pytest.mark.parametrize("dtype,path", [("f64", 1), ("f64", 2)])
def test_coupled_particle_step(dev, dtype, path):
    """Multidirect loop -> per-particle sums at u^n and u^{n+1} -> rigid
    update -> marker advection, each stage against the oracle's own chain."""
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce(f"coupled step {dtype} path={path}")
    wl = small_workload(32, 16, 4, 3, 5)
    c = Case(wl, dev)
    rng = np.random.default_rng(13)
    rho_p = rng.uniform(1.5, 3.0, wl.npart)
    g, rho_f = [0.0, 0.0, -1.0], 1.0
    res = O.multidirect(c.g, wl.delta, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0)
    s0 = O.particle_reductions(c.g, c.m, wl.xc, wl.d, res["F"], wl.u0)
    s1 = O.particle_reductions(c.g, c.m, wl.xc, wl.d, res["F"], res["ustar"])
    up1, om1, xc1 = O.rigid_update(wl.xc, wl.d, wl.up, wl.om, rho_p, s0, s1, rho_f, g, wl.dt)
    m1 = O.advect_markers(c.m, wl.xc, xc1, wl.om, om1, wl.dt)

    b = ibx.bucket(c.dl, c.dm, wl.delta)
    plan = ibx.Plan(wl.delta, torch.float64, path)
    u0 = c.u0_boxes(torch.float64)
    ustar, f, F = plan.multidirect_force(c.dl, c.parts, c.dm, b, wl.ns, wl.dt, u0)
    g0 = ibx.particle_reductions(c.dl, c.parts, c.dm, F, u0)
    g1 = ibx.particle_reductions(c.dl, c.parts, c.dm, F, ustar)
    t = lambda a: torch.as_tensor(a, device=dev)
    gu, gw, gx = ibx.rigid_update(c.parts, t(rho_p), g0, g1, rho_f, g, wl.dt)
    gm = ibx.advect_markers(c.dm, c.parts.xc, gx, c.parts.om, gw, wl.dt)
    torch.cuda.synchronize()
    scale = lambda a: np.abs(a).max()
    assert np.max(np.abs(g0.cpu().numpy() - s0)) <= 1e-12 * scale(s0)
    assert np.max(np.abs(g1.cpu().numpy() - s1)) <= 1e-12 * scale(s1)
    assert rel(gu.cpu().numpy(), up1) <= 1e-11
    assert rel(gw.cpu().numpy(), om1) <= 1e-11
    assert rel(gx.cpu().numpy(), xc1) <= 1e-14
    assert np.max(np.abs(gm.xyz().cpu().numpy() - m1.xyz())) <= 1e-14


@pytest.mark.parametrize("cfg", [3, 4], ids=["spheres1000_256", "spheres20000_512"])
def test_collision_forces_match_oracle(dev, cfg):
    """Every particle's collision force at full size (the clumped 20000-sphere
    workload overlaps heavily), periodic minimum image, against the oracle."""
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce(f"collision forces config {cfg}")
    wl = W.config(cfg, 0, with_field=False)
    rng = np.random.default_rng(14)
    rho = rng.uniform(1000.0, 3000.0, wl.npart)
    lev = wl.level
    L = [lev.n[a] * lev.h if lev.periodic[a] else 0.0 for a in range(3)]
    ref = O.collision_forces(wl.xc, wl.d, rho, 9.81, lev.h, 1e-4, L)
    dl = ibx.device_level(lev, dev)
    parts = ibx.particles(wl.xc, wl.d, wl.up, wl.om, dev)
    got = ibx.collision_forces(dl, parts, torch.as_tensor(rho, device=dev), 9.81, 1e-4)
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    assert np.abs(ref).max() > 0
    assert rel(g, ref) <= 1e-13
    assert np.abs(g.sum(axis=0)).max() <= 1e-12 * np.abs(g).sum()



@pytest.mark.parametrize("npart", [400, 9000], ids=["np400", "np9000"])
@pytest.mark.parametrize("n,periodic,dmax", [
    ((16, 24, 40), (1, 0, 1), 6.0),
    ((16, 48, 32), (0, 1, 1), 10.0),
    ((8, 8, 8), (1, 1, 0), 3.0),
], ids=["bins2x3x5", "bins1x3x2", "onebin"])
def test_collision_forces_few_bins(dev, n, periodic, dmax, npart):
    """Small domains where an axis has one, two or three bins, bounded and
    periodic, with centroids beyond both ends of every axis (clamped or
    wrapped): every force against the oracle's all-pairs sum.  400 particles
    are put in bin order by counting, 9000 by the device-wide radix sort."""
    import torch

    import oracle as O
    import paper_2408_14140_amd as ibx
    announce(f"collision forces few bins n={n} periodic={periodic}")
    h = 1.0 / 32
    lev = W.make_level(n, h, periodic=periodic, box=8)
    rng = np.random.default_rng(sum(n) + npart)
    ext = np.array(n) * h
    xc = rng.uniform(0, 1, (npart, 3)) * (ext + 4 * h) - 2 * h
    d = rng.uniform(1.0, dmax, npart) * h
    rho = rng.uniform(1000.0, 3000.0, npart)
    L = [n[a] * h if periodic[a] else 0.0 for a in range(3)]
    ref = O.collision_forces(xc, d, rho, 9.81, h, 1e-4, L)
    dl = ibx.device_level(lev, dev)
    parts = ibx.particles(xc, d, np.zeros((npart, 3)), np.zeros((npart, 3)), dev)
    got = ibx.collision_forces(dl, parts, torch.as_tensor(rho, device=dev), 9.81, 1e-4)
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    assert (np.abs(ref).sum(axis=1) > 0).mean() > 0.5
    assert rel(g, ref) <= 1e-13
