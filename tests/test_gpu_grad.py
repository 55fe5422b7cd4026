"""GPU adjoint (a11): against the FP64 oracle's reverse sweep, and against
central finite differences of the GPU forward (FP64).

Loss (differentiation workload): L = sum over valid cells |f^ns|^2 +
sum_p w_p . (sum_l F_l dV_l), w ~ N(0, 1), marker positions independent."""
import numpy as np
import pytest

import workloads as W
from fd_common import fd_bound
from gpu_common import Case, announce, gpu_device, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def _valid(lev, t):
    g, b = lev.ngrow, lev.box
    return t[:, :, g:g + b, g:g + b, g:g + b]


def _loss(c, f, F, wts_t):
    import torch
    dvl = c.dm.dv[c.dm.pid.long()][:, None]
    return (_valid(c.lev, f) ** 2).sum() + (wts_t[c.dm.pid.long()] * F * dvl).sum()


def _grads(c, dtype, path, wts, with_ustar=None, **plan_kw):
    import torch

    import paper_2408_14140_amd as ibx
    from paper_2408_14140_amd.autograd import multidirect
    wl = c.wl
    tdt = torch.float64 if dtype == "f64" else torch.float32
    plan = ibx.Plan(wl.delta, tdt, path, **plan_kw)
    b = ibx.bucket(c.dl, c.dm, wl.delta)
    u0 = torch.as_tensor(W.to_boxes(wl.u0, c.lev, fill=0.0), device=c.dev).to(tdt).requires_grad_()
    up = c.parts.up.clone().requires_grad_()
    om = c.parts.om.clone().requires_grad_()
    X = c.dm.xyz().clone().requires_grad_()
    ustar, f, F = multidirect(plan, c.dl, c.parts, c.dm, b, wl.ns, wl.dt, u0, up, om, X)
    wts_t = torch.as_tensor(wts, device=c.dev).to(tdt)
    L = _loss(c, f, F, wts_t)
    if with_ustar is not None:
        L = L + (_valid(c.lev, ustar) * torch.as_tensor(with_ustar, device=c.dev).to(tdt)).sum()
    L.backward()
    torch.cuda.synchronize()
    return L, u0.grad, up.grad, om.grad, X.grad


def _oracle_grads(c, wts, gus_valid=None):
    import oracle as O
    wl = c.wl
    res = O.multidirect(c.g, wl.delta, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0,
                        history=True)
    gus = None
    if gus_valid is not None:
        gus = W.from_boxes(_pad(gus_valid, c.lev), c.lev)
    return O.reverse(c.g, wl.delta, wl.ns, wl.dt, c.m, wl.xc, wl.up, wl.om, wl.u0,
                     res["Fhist"], g_ustar=gus, g_f=2 * res["f"],
                     g_F=wts[c.m.pid] * c.m.dv[c.m.pid][:, None])


def _pad(valid, lev):
    g, b = lev.ngrow, lev.box
    e = b + 2 * g
    out = np.zeros((valid.shape[0], 3, e, e, e))
    out[:, :, g:g + b, g:g + b, g:g + b] = valid
    return out


def _small():
    return W.make_workload("grad_small", 32, 16, 2, 4, 3, np.array([6.3, 7.7]), seed=11,
                           nmodes=8, K=4, cover_all=True)


def _small_p3():
    return W.make_workload("grad_small_P3", 32, 16, 2, 3, 3, np.array([6.9, 8.4]), seed=12,
                           nmodes=8, K=4, cover_all=True)


CASES = [("grad_small", _small), ("grad_small_P3", _small_p3),
         ("spheres64_128", lambda: W.config(5, 0))]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("dtype,path", [("f64", 1), ("f64", 2), ("f32", 2)])
def test_adjoint_matches_oracle(dev, name, mk, dtype, path):
    announce(f"adjoint {name} {dtype} path={path}")
    wl = mk()
    c = Case(wl, dev)
    rng = np.random.default_rng(5)
    wts = rng.normal(size=(wl.npart, 3))
    gus = rng.normal(size=(c.lev.nbox, 3, c.lev.box, c.lev.box, c.lev.box))
    L, gu0, gup, gom, gX = _grads(c, dtype, path, wts, with_ustar=gus)
    ref = _oracle_grads(c, wts, gus_valid=gus)
    tol = 1e-11 if dtype == "f64" else 1e-4
    assert c.field_rel(gu0, ref["u0"]) <= tol
    assert rel(gup.cpu().numpy(), ref["up"]) <= tol
    assert rel(gom.cpu().numpy(), ref["om"]) <= tol
    assert rel(gX.cpu().numpy(), ref["X"]) <= tol


@pytest.mark.parametrize("name,mk,dtype", [("grad_small", _small, "f64"),
                                           ("grad_small_P3", _small_p3, "f32"),
                                           ("spheres64_128", lambda: W.config(5, 0), "f32")],
                         ids=["grad_small-f64", "grad_small_P3-f32", "spheres64_128-f32"])
def test_adjoint_with_row_masks(dev, name, mk, dtype):
    """The adjoint's spreads through the slot row masks give the same
    gradients as without them (and, in FP32, its interpolation on 16 x 8 x 8
    work tiles the same to rounding)."""
    import torch
    announce(f"adjoint row masks {name} {dtype}")
    wl = mk()
    c = Case(wl, dev)
    rng = np.random.default_rng(8)
    wts = rng.normal(size=(wl.npart, 3))
    gus = rng.normal(size=(c.lev.nbox, 3, c.lev.box, c.lev.box, c.lev.box))
    a = _grads(c, dtype, 2, wts, with_ustar=gus)
    b = _grads(c, dtype, 2, wts, with_ustar=gus, row_masks=True)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    if dtype == "f32":      # and with work tiles of two x neighbours, to rounding
        t = _grads(c, dtype, 2, wts, with_ustar=gus, row_masks=True, interp_tile=16)
        for x, y in zip(a, t):
            x = x.detach().double().cpu().numpy()
            y = y.detach().double().cpu().numpy()
            assert np.linalg.norm(y - x) <= 1e-5 * np.linalg.norm(x)


def test_adjoint_matches_central_differences_on_gpu(dev):
    """20 random directions, eps = 1e-6, FP64 forward on the GPU."""
    import torch

    import paper_2408_14140_amd as ibx
    announce("adjoint FD")
    wl = _small()
    c = Case(wl, dev)
    rng = np.random.default_rng(6)
    torch.manual_seed(6)
    wts = rng.normal(size=(wl.npart, 3))
    L0, gu0, gup, gom, gX = _grads(c, "f64", 2, wts)
    plan = ibx.Plan(wl.delta, torch.float64, 2)
    u0 = torch.as_tensor(W.to_boxes(wl.u0, c.lev, fill=0.0), device=dev)
    wts_t = torch.as_tensor(wts, device=dev)
    X0 = c.dm.xyz().clone()
    g_all = {"u0": gu0, "up": gup, "om": gom, "X": gX}
    mask = torch.zeros_like(u0)
    _valid(c.lev, mask)[...] = 1.0

    def L_at(du, dup, dom, dX):
        X = X0 + dX
        m = ibx.Markers(c.dm.offs, X[:, 0].contiguous(), X[:, 1].contiguous(),
                        X[:, 2].contiguous(), c.dm.pid, c.dm.dv)
        parts = ibx.Particles(c.parts.xc, c.parts.d, (c.parts.up + dup).contiguous(),
                              (c.parts.om + dom).contiguous())
        b = ibx.bucket(c.dl, m, wl.delta)
        _, f, F = plan.multidirect_force(c.dl, parts, m, b, wl.ns, wl.dt, (u0 + du).contiguous())
        dvl = m.dv[m.pid.long()][:, None]
        t1 = _valid(c.lev, f) ** 2
        t2 = wts_t[m.pid.long()] * F * dvl
        return (float((t1.sum() + t2.sum()).item()),
                float((t1.abs().sum() + t2.abs().sum()).item()))

    eps = 1e-6
    # phi is C^1 with jumps of phi'' where a marker coordinate sits on a cell
    # centre (4-point) or face (3-point); central differences are only second
    # order where no step crosses such a join, so markers within 10 steps of
    # one are held fixed (the quotients step up to 20 eps away).
    s = c.m.xyz() / c.lev.h - (0.5 if wl.delta == 4 else 0.0)
    dist = np.abs(s - np.round(s)).min(axis=1)
    keep = torch.as_tensor((dist > 10 * 4 * eps / c.lev.h).astype(np.float64), device=dev)
    for _ in range(20):
        v = {"u0": torch.randn_like(u0) * mask, "up": torch.randn_like(gup),
             "om": torch.randn_like(gom), "X": torch.randn_like(X0).clamp(-4, 4)}
        for k in v:
            v[k] = v[k] / torch.sqrt((v[k] ** 2).sum() / (mask.sum() if k == "u0" else v[k].numel()))
        v["X"] = v["X"].clamp(-4, 4) * keep[:, None]
        fd, bound = fd_bound(lambda t: L_at(t * v["u0"], t * v["up"], t * v["om"], t * v["X"]),
                             eps)
        an = sum(float((g_all[k] * v[k]).sum().item()) for k in v)
        assert abs(fd - an) <= bound, (fd, an, bound)
