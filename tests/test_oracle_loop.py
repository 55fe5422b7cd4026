"""Pins of the oracle's interpolation, spreading and Algorithm 1 loop."""
import numpy as np
import pytest

import workloads as W
from dense_ref import dense_multidirect, dense_weights


def _markers(oracle_mod, n, rng, k=3, dmin=4, dmax=8):
    h = 1.0 / n
    return oracle_mod.build_markers(rng.uniform(0, 1, (k, 3)), rng.uniform(dmin, dmax, k) * h, h)


@pytest.mark.parametrize("P", [3, 4])
def test_interp_exact_for_constant_and_linear_fields(oracle_mod, P):
    n = 24
    h = 1.0 / n
    g = oracle_mod.grid(n, h, periodic=(0, 0, 0))
    m = oracle_mod.build_markers([[0.5, 0.45, 0.55]], [8 * h], h)
    cen = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(cen, cen, cen, indexing="ij")
    const = np.stack([np.full_like(x, 1.5), np.full_like(x, -2.0), np.full_like(x, 0.25)])
    U = oracle_mod.interp(g, P, m, const)
    assert np.max(np.abs(U - [1.5, -2.0, 0.25])) < 1e-14
    A = np.array([[0.3, 1.0, -2.0, 0.5], [-1.0, 0.2, 0.7, 3.0], [2.0, -0.4, 0.1, -1.0]])
    lin = np.stack([A[c, 0] + A[c, 1] * x + A[c, 2] * y + A[c, 3] * z for c in range(3)])
    U = oracle_mod.interp(g, P, m, lin)
    X = m.xyz()
    expect = A[:, :1].T + X @ A[:, 1:].T
    assert np.max(np.abs(U - expect)) < 1e-13


@pytest.mark.parametrize("P", [3, 4])
def test_adjoint_identity(oracle_mod, P):
    """<u, S F>_h = <J u, F>_dV (Sec. 2: spreading and interpolation are adjoint)."""
    rng = np.random.default_rng(11)
    n = 32
    h = 1.0 / n
    g = oracle_mod.grid(n, h)
    m = _markers(oracle_mod, n, rng)
    u = rng.normal(size=(3, n, n, n))
    F = rng.normal(size=(m.nl, 3))
    lhs = (u * oracle_mod.spread(g, P, m, F)).sum() * h ** 3
    rhs = (oracle_mod.interp(g, P, m, u) * F * m.dv[m.pid][:, None]).sum()
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs) + 1e-15


@pytest.mark.parametrize("P", [3, 4])
def test_force_and_torque_conservation(oracle_mod, P):
    rng = np.random.default_rng(12)
    n = 32
    h = 1.0 / n
    g = oracle_mod.grid(n, h, periodic=(0, 0, 0))
    xc = np.array([0.51, 0.47, 0.5])
    m = oracle_mod.build_markers([xc], [10 * h], h)
    F = rng.normal(size=(m.nl, 3))
    f = oracle_mod.spread(g, P, m, F)
    dv = m.dv[0]
    tot_l = (F * dv).sum(axis=0)
    tot_e = f.reshape(3, -1).sum(axis=1) * h ** 3
    assert np.max(np.abs(tot_l - tot_e)) < 1e-12 * np.abs(F * dv).sum()
    R = m.xyz() - xc
    tq_l = np.cross(R, F).sum(axis=0) * dv
    cen = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(cen, cen, cen, indexing="ij")
    r = np.stack([x - xc[0], y - xc[1], z - xc[2]]).reshape(3, -1)
    tq_e = np.cross(r.T, f.reshape(3, -1).T).sum(axis=0) * h ** 3
    assert np.max(np.abs(tq_l - tq_e)) < 1e-12 * np.abs(np.cross(R, F) * dv).sum()


@pytest.mark.parametrize("P", [3, 4])
def test_dense_brute_force_agrees(oracle_mod, P):
    rng = np.random.default_rng(13 + P)
    for n in (8, 12):
        h = 1.0 / n
        g = oracle_mod.grid(n, h)
        xc = rng.uniform(0, 1, (2, 3))
        m = oracle_mod.build_markers(xc, [2.2 * h, 1.9 * h], h)
        assert m.nl <= 50
        up = rng.normal(0, 0.1, (2, 3))
        om = rng.normal(0, 1, (2, 3))
        u0 = rng.normal(size=(3, n, n, n))
        dt = 0.5 * h
        res = oracle_mod.multidirect(g, P, 3, dt, m, xc, up, om, u0)
        Wd = dense_weights(n, h, m.xyz(), lambda r: oracle_mod.phi(P, r))
        # desired velocity written out from Eq. (pr1)
        R = m.xyz() - xc[m.pid]
        Ud = up[m.pid] + np.cross(om[m.pid], R)
        u, f, F, resid = dense_multidirect(Wd, m.dv[m.pid], h, 3, dt, Ud, u0.reshape(3, -1))
        scale = np.abs(res["F"]).max()
        assert np.max(np.abs(res["F"] - F)) < 1e-13 * scale
        assert np.max(np.abs(res["f"].reshape(3, -1) - f)) < 1e-13 * np.abs(f).max()
        assert np.max(np.abs(res["ustar"].reshape(3, -1) - u)) < 1e-13 * np.abs(u).max()
        assert np.max(np.abs(res["resid"] - resid)) < 1e-12 * resid.max()


def test_residual_decays_when_coupling_bound_below_two(oracle_mod):
    """e_(m+1) = (I - J S) e_m with J S self-adjoint, PSD in <.,.>_dV.

    Its spectral radius is at most max_x sum_l delta_h(x - X_l) dV_l; below 2 the
    residual norm cannot grow."""
    wl = W.make_workload("t", 32, 16, 2, 4, 6, np.array([8.0, 6.0, 7.0]), seed=3,
                         cover_all=True)
    g = oracle_mod.grid_of(wl.level)
    m = oracle_mod.build_markers(wl.xc, wl.d, wl.level.h)
    ones = np.ones((m.nl, 3))
    bound = oracle_mod.spread(g, 4, m, ones)[0].max()
    assert bound < 2.0
    res = oracle_mod.multidirect(g, 4, 6, wl.dt, m, wl.xc, wl.up, wl.om, wl.u0)
    r = res["resid"]
    assert np.all(np.diff(r) <= 1e-12 * r[0])
    assert r[-1] < 0.5 * r[0]


@pytest.mark.parametrize("P", [3, 4])
def test_single_marker_closed_form(oracle_mod, P):
    """One marker: e_m = (1-a)^m e_0 with a = (dV/h^3) prod_d sum_i phi_i^2."""
    n = 16
    h = 1.0 / n
    g = oracle_mod.grid(n, h)
    X = np.array([0.4132, 0.5771, 0.3019])
    M = oracle_mod.Markers([X[0]], [X[1]], [X[2]], [0], [0.7 * h ** 3], [0, 1])
    rng = np.random.default_rng(21)
    u0 = rng.normal(size=(3, n, n, n))
    up = np.array([[0.05, -0.02, 0.1]])
    om = np.zeros((1, 3))
    dt = 0.5 * h
    ns = 4
    res = oracle_mod.multidirect(g, P, ns, dt, M, X[None], up, om, u0)
    a = 0.7
    for d in range(3):
        s = X[d] / h
        base = (np.floor(s) - 1) if P == 3 else (np.floor(s - 0.5) - 1)
        r = s - (base + np.arange(P)) - 0.5
        a *= (oracle_mod.phi(P, r) ** 2).sum()
    e0 = up[0] - oracle_mod.interp(g, P, M, u0)[0]
    Fm = e0 * (1 - (1 - a) ** ns) / (a * dt)
    assert np.max(np.abs(res["F"][0] - Fm)) < 1e-12 * np.abs(Fm).max()
    assert np.allclose(res["resid"], np.linalg.norm(e0) * np.sqrt(0.7 * h ** 3)
                       * np.abs(1 - a) ** np.arange(ns + 1), rtol=1e-11, atol=0)


def test_sequential_equals_jacobi_for_disjoint_supports(oracle_mod):
    n = 48
    h = 1.0 / n
    g = oracle_mod.grid(n, h)
    xc = np.array([[0.2, 0.25, 0.3], [0.7, 0.72, 0.68]])
    m = oracle_mod.build_markers(xc, [8 * h, 9 * h], h)
    rng = np.random.default_rng(4)
    u0 = rng.normal(size=(3, n, n, n))
    up = rng.normal(0, 0.1, (2, 3))
    om = rng.normal(0, 1, (2, 3))
    a = oracle_mod.multidirect(g, 4, 3, 0.5 * h, m, xc, up, om, u0)
    b = oracle_mod.multidirect(g, 4, 3, 0.5 * h, m, xc, up, om, u0, order="sequential")
    assert np.max(np.abs(a["F"] - b["F"])) <= 1e-14 * np.abs(a["F"]).max()
    assert np.max(np.abs(a["ustar"] - b["ustar"])) <= 1e-14 * np.abs(a["ustar"]).max()


def _sub(oracle_mod, m, p):
    """Markers of particle p alone (pid 0)."""
    a, z = int(m.offs[p]), int(m.offs[p + 1])
    return oracle_mod.Markers(m.x[a:z], m.y[a:z], m.z[a:z], np.zeros(z - a, np.int32),
                              m.dv[p:p + 1], np.array([0, z - a], np.int64))


def test_sequential_order_composes_single_particle_loops(oracle_mod):
    """Sec. 3.1: with several particles each runs the N_s loop in turn.  For
    two particles whose supports overlap, the sequential order equals particle
    0's loop from u0 followed by particle 1's loop from the field particle 0
    left, with f the sum of the two; it differs from the Jacobi order and from
    the other particle order."""
    n = 40
    h = 1.0 / n
    g = oracle_mod.grid(n, h)
    xc = np.array([[0.4, 0.5, 0.5], [0.4 + 10.5 * h, 0.52, 0.49]])
    d = np.array([9.0 * h, 10.0 * h])
    m = oracle_mod.build_markers(xc, d, h)
    rng = np.random.default_rng(21)
    u0 = rng.normal(size=(3, n, n, n))
    up = rng.normal(0, 0.1, (2, 3))
    om = rng.normal(0, 1, (2, 3))
    dt, ns, P = 0.5 * h, 3, 4
    seq = oracle_mod.multidirect(g, P, ns, dt, m, xc, up, om, u0, order="sequential")
    r0 = oracle_mod.multidirect(g, P, ns, dt, _sub(oracle_mod, m, 0), xc[:1], up[:1], om[:1], u0)
    r1 = oracle_mod.multidirect(g, P, ns, dt, _sub(oracle_mod, m, 1), xc[1:], up[1:], om[1:],
                                r0["ustar"])
    k = int(m.offs[1])
    scale = np.abs(seq["F"]).max()
    assert np.max(np.abs(seq["F"][:k] - r0["F"])) <= 1e-14 * scale
    assert np.max(np.abs(seq["F"][k:] - r1["F"])) <= 1e-14 * scale
    assert np.max(np.abs(seq["ustar"] - r1["ustar"])) <= 1e-14 * np.abs(u0).max()
    assert np.max(np.abs(seq["f"] - (r0["f"] + r1["f"]))) <= 1e-14 * np.abs(seq["f"]).max()
    jac = oracle_mod.multidirect(g, P, ns, dt, m, xc, up, om, u0)
    assert np.max(np.abs(jac["F"] - seq["F"])) > 1e-6 * scale
    # particle 1 first
    rb = oracle_mod.multidirect(g, P, ns, dt, _sub(oracle_mod, m, 1), xc[1:], up[1:], om[1:], u0)
    assert np.max(np.abs(seq["F"][k:] - rb["F"])) > 1e-6 * scale
