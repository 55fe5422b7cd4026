"""Pins of the oracle's per-particle reductions (a10) and reverse sweep (a11)."""
import math
import os

import numpy as np
import pytest

import workloads as W
from fd_common import fd_bound

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pvf_tables.txt")


def _golden_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            shape, q, vol, err, order = line.split()
            rows.append((shape, int(q), float(vol), float(err), float(order)))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: f"{r[0]}{r[1]}")
def test_pvf_volume_reproduces_tables_1_and_2(oracle_mod, row):
    shape, q, vol, err, _ = row
    h = 0.8 / q
    n = int(round(2.0 / h))
    g = oracle_mod.grid(n, h, periodic=(0, 0, 0))
    axes = [0.4, 0.4, 0.4] if shape == "sphere" else [0.4, 0.6, 0.4]
    v = oracle_mod.pvf_volume(g, [1.0, 1.0, 1.0], axes)
    assert abs(v - vol) <= 1e-10
    exact = 4.0 * math.pi * axes[0] * axes[1] * axes[2] / 3.0
    assert abs(abs(v - exact) / exact * 100 - err) <= 0.0006 * err


def test_pvf_orders_match_tables(oracle_mod):
    rows = _golden_rows()
    for shape in ("sphere", "ellipsoid"):
        errs = [r[3] for r in rows if r[0] == shape]
        orders = [r[4] for r in rows if r[0] == shape][1:]
        for i, o in enumerate(orders):
            assert abs(math.log(errs[i] / errs[i + 1], 2) - o) < 2e-3


def _one_sphere(oracle_mod, q, centre=(0.5, 0.5, 0.5)):
    n = 4 * q
    h = 1.0 / n
    g = oracle_mod.grid(n, h)
    xc = np.array([centre])
    d = np.array([q * h])
    m = oracle_mod.build_markers(xc, d, h)
    cen = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(cen, cen, cen, indexing="ij")
    return g, xc, d, m, (x, y, z)


def test_volume_integral_of_uniform_field_is_pvf_volume(oracle_mod):
    g, xc, d, m, (x, y, z) = _one_sphere(oracle_mod, 16)
    u = np.stack([np.ones_like(x), np.zeros_like(x), np.zeros_like(x)])
    out = oracle_mod.particle_reductions(g, m, xc, d, np.zeros((m.nl, 3)), u)
    vol = oracle_mod.pvf_volume(g, xc[0], [d[0] / 2] * 3)
    assert abs(out[0, 6] - vol) < 1e-15
    assert np.all(out[0, :6] == 0) and abs(out[0, 7]) == 0 and abs(out[0, 8]) == 0


def test_angular_momentum_of_rigid_rotation_converges(oracle_mod):
    """For u = w x r, int r x u dV = (8 pi / 15) R^5 w.

    The alpha-weighted sum is a second-order quadrature whose error oscillates
    with the sphere's position against the grid, so the check is over an
    eightfold refinement: the error must drop by at least 2^5."""
    w = np.array([0.3, -1.1, 0.7])
    errs = []
    for q in (8, 64):
        g, xc, d, m, (x, y, z) = _one_sphere(oracle_mod, q, (0.5123, 0.4871, 0.5037))
        r = np.stack([x - xc[0, 0], y - xc[0, 1], z - xc[0, 2]])
        u = np.stack([w[1] * r[2] - w[2] * r[1], w[2] * r[0] - w[0] * r[2],
                      w[0] * r[1] - w[1] * r[0]])
        out = oracle_mod.particle_reductions(g, m, xc, d, np.zeros((m.nl, 3)), u)
        exact = 8 * math.pi / 15 * (d[0] / 2) ** 5 * w
        errs.append(np.linalg.norm(out[0, 9:12] - exact) / np.linalg.norm(exact))
    assert errs[0] < 3e-3
    assert errs[0] / errs[1] > 2 ** 5


def test_lagrangian_sums(oracle_mod):
    g, xc, d, m, _ = _one_sphere(oracle_mod, 16)
    rng = np.random.default_rng(8)
    c = rng.normal(size=3)
    u = np.zeros((3,) + tuple(g.n)[::-1])
    out = oracle_mod.particle_reductions(g, m, xc, d, np.tile(c, (m.nl, 1)), u)
    assert np.allclose(out[0, :3], m.nl * m.dv[0] * c, rtol=1e-13, atol=0)
    # F = w x R gives sum R x (w x R) dV = dV (sum |R|^2 w - sum R (R.w));
    R = m.xyz() - xc[0]
    w = rng.normal(size=3)
    F = np.cross(w, R)
    out = oracle_mod.particle_reductions(g, m, xc, d, F, u)
    expect = m.dv[0] * ((R * R).sum() * w - R.T @ (R @ w))
    assert np.allclose(out[0, 3:6], expect, rtol=1e-12, atol=1e-18)
    # equal-area markers make sum R R^T close to (N R^2 / 3) I
    iso = m.dv[0] * (2.0 / 3.0) * m.nl * (d[0] / 2) ** 2 * w
    assert np.linalg.norm(out[0, 3:6] - iso) < 1e-2 * np.linalg.norm(iso)


def _loss_and_grads(oracle_mod, g, P, ns, dt, m, xc, up, om, u0, wts, gus=None):
    res = oracle_mod.multidirect(g, P, ns, dt, m, xc, up, om, u0, history=True)
    L = (res["f"] ** 2).sum() + (wts[m.pid] * res["F"] * m.dv[m.pid][:, None]).sum()
    if gus is not None:
        L += (gus * res["ustar"]).sum()
    grads = oracle_mod.reverse(g, P, ns, dt, m, xc, up, om, u0, res["Fhist"],
                               g_ustar=gus, g_f=2 * res["f"],
                               g_F=wts[m.pid] * m.dv[m.pid][:, None])
    return L, grads


def _loss_terms(oracle_mod, g, P, ns, dt, m, xc, up, om, u0, wts, gus=None):
    """The loss and the sum of the magnitudes of its terms."""
    res = oracle_mod.multidirect(g, P, ns, dt, m, xc, up, om, u0, residuals=False)
    t = [res["f"] ** 2, wts[m.pid] * res["F"] * m.dv[m.pid][:, None]]
    if gus is not None:
        t.append(gus * res["ustar"])
    return sum(a.sum() for a in t), sum(np.abs(a).sum() for a in t)


@pytest.mark.parametrize("P,with_ustar", [(4, False), (3, True)])
def test_reverse_sweep_matches_central_differences(oracle_mod, P, with_ustar):
    n = 16
    h = 1.0 / n
    g = oracle_mod.grid(n, h)
    rng = np.random.default_rng(30 + P)
    # generic centres: a marker exactly on a cell face (3-point) or centre
    # (4-point) sits on a jump of phi'' and central differences lose an order
    xc = np.array([[0.3071, 0.3529, 0.4113], [0.6937, 0.6518, 0.6042]])
    m0 = oracle_mod.build_markers(xc, [5 * h, 4 * h], h)
    s = m0.xyz() / h - (0.0 if P == 3 else 0.5)
    assert np.abs(s - np.round(s)).min() > 1e-4
    up = rng.normal(0, 0.1, (2, 3))
    om = rng.normal(0, 1, (2, 3))
    u0 = rng.normal(size=(3, n, n, n))
    wts = rng.normal(size=(2, 3))
    gus = rng.normal(size=u0.shape) if with_ustar else None
    ns, dt = 3, 0.5 * h
    L0, G = _loss_and_grads(oracle_mod, g, P, ns, dt, m0, xc, up, om, u0, wts, gus)
    X0 = m0.xyz()
    eps = 1e-6

    def mk(X):
        return oracle_mod.Markers(X[:, 0], X[:, 1], X[:, 2], m0.pid, m0.dv, m0.offs)

    # markers within 10 steps of a kernel join (a jump of the second
    # derivative of phi) are held fixed: the quotients step up to 20 eps away
    keep = (np.abs(s - np.round(s)).min(axis=1) > 10 * 4 * eps / h).astype(float)
    for _ in range(20):
        v = {k: rng.normal(size=s) for k, s in
             (("u0", u0.shape), ("up", up.shape), ("om", om.shape), ("X", X0.shape))}
        for k in v:
            v[k] /= np.sqrt((v[k] ** 2).mean())
        v["X"] = np.clip(v["X"], -4, 4) * keep[:, None]

        def L_at(t):
            return _loss_terms(oracle_mod, g, P, ns, dt, mk(X0 + t * v["X"]), xc,
                               up + t * v["up"], om + t * v["om"], u0 + t * v["u0"], wts, gus)

        fd, bound = fd_bound(L_at, eps)
        an = sum((G[k] * v[k]).sum() for k in v)
        assert abs(fd - an) <= bound, (fd, an, bound)
