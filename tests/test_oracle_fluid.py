"""Pins of the oracle's single-level periodic fluid steps (Sec. 3.1, Step 1 =
Eq. (31), Step 3 = Eqs. (ns_lp1)-(ns_lp3)) against identities of the discrete
operators, closed forms of single Fourier modes and convergence to the
analytic derivatives."""
import numpy as np
import pytest

from oracle import fluid as FL


def _centres(n):
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return x, y, z, h


def _nodes(n):
    h = 1.0 / n
    c = np.arange(n) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return x, y, z, h


def test_div_is_minus_grad_transpose():
    rng = np.random.default_rng(1)
    n, h = 12, 1.0 / 12
    p = rng.normal(size=(n, n, n))
    V = rng.normal(size=(3, n, n, n))
    lhs = (V * FL.grad_nodes(p, h)).sum()
    rhs = -(p * FL.div_nodes(V, h)).sum()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_grad_and_div_converge_at_second_order():
    err_g, err_d = [], []
    for n in (16, 32, 64):
        xn, yn, zn, h = _nodes(n)
        p = np.sin(2 * np.pi * xn) * np.cos(2 * np.pi * yn) * np.sin(4 * np.pi * zn)
        xc, yc, zc, _ = _centres(n)
        exact = 2 * np.pi * np.stack([
            np.cos(2 * np.pi * xc) * np.cos(2 * np.pi * yc) * np.sin(4 * np.pi * zc),
            -np.sin(2 * np.pi * xc) * np.sin(2 * np.pi * yc) * np.sin(4 * np.pi * zc),
            2 * np.sin(2 * np.pi * xc) * np.cos(2 * np.pi * yc) * np.cos(4 * np.pi * zc)])
        err_g.append(np.abs(FL.grad_nodes(p, h) - exact).max())
        V = np.stack([np.sin(2 * np.pi * yc), np.cos(2 * np.pi * xc) * np.sin(2 * np.pi * zc),
                      np.sin(2 * np.pi * zc)])
        div = 2 * np.pi * np.cos(2 * np.pi * zn)        # only the z component varies along itself
        err_d.append(np.abs(FL.div_nodes(V, h) - div).max())
    for e in (err_g, err_d):
        assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5


@pytest.mark.parametrize("k", [(1, 0, 0), (2, 3, 1), (4, 4, 0), (8, 8, 8), (3, 8, 5)])
def test_symbols_match_the_real_space_operators(k):
    n, h = 16, 1.0 / 16
    idx = np.arange(n)
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    mode = np.exp(2j * np.pi * (k[0] * x + k[1] * y + k[2] * z) / n)
    lam = FL.laplacian_symbol(n, h)[k[2], k[1], k[0]]
    sig = FL.dg_symbol(n, h)[k[2], k[1], k[0]]
    for part in (mode.real, mode.imag):
        lap = FL.laplacian(np.stack([part] * 3), h)[0]
        assert np.allclose(lap, lam * part, rtol=0, atol=1e-9 * (1 + abs(lam)))
    dg = FL.div_nodes(FL.grad_nodes(mode.real, h), h) + 1j * FL.div_nodes(
        FL.grad_nodes(mode.imag, h), h)
    assert np.allclose(dg, sig * mode, rtol=0, atol=1e-9 * (1 + abs(sig)))
    if sum(v == n // 2 for v in k) >= 2:
        assert abs(sig) < 1e-20 / h ** 2               # null mode of D G


def test_projection_is_divergence_free_and_idempotent():
    rng = np.random.default_rng(2)
    n, h, rho, dt = 16, 1.0 / 16, 1.3, 0.01
    ustar = rng.normal(size=(3, n, n, n))
    p_old = rng.normal(size=(n, n, n))
    u1, p1 = FL.project(ustar, p_old, h, rho, dt)
    V = ustar / dt + FL.grad_nodes(p_old, h) / rho
    dv = FL.div_nodes(V, h)
    assert np.abs(FL.div_nodes(u1, h)).max() <= 1e-12 * dt * np.abs(dv).max()
    # the solve: (1/rho) D G p = D V
    assert np.abs(FL.div_nodes(FL.grad_nodes(p1, h), h) / rho - dv).max() <= 1e-10 * np.abs(dv).max()
    u2, p2 = FL.project(u1, np.zeros_like(p_old), h, rho, dt)
    assert np.abs(u2 - u1).max() <= 1e-12 * np.abs(u1).max()
    assert np.abs(p2).max() <= 1e-10 * np.abs(p1).max()


def test_projection_removes_a_nodal_gradient():
    rng = np.random.default_rng(3)
    n, h, rho, dt = 16, 1.0 / 16, 0.7, 0.02
    phi = rng.normal(size=(n, n, n))
    g = FL.grad_nodes(phi, h)
    u1, p1 = FL.project(dt * g / rho, np.zeros((n, n, n)), h, rho, dt)
    assert np.abs(u1).max() <= 1e-11 * dt * np.abs(g).max()
    assert np.abs(FL.grad_nodes(p1, h) - g).max() <= 1e-10 * np.abs(g).max()


def test_predict_uniform_flow_and_gravity():
    n, h = 8, 1.0 / 8
    u = np.stack([np.full((n, n, n), v) for v in (0.3, -1.2, 0.5)])
    g = (0.0, -9.81, 1.5)
    out = FL.predict(u, np.zeros((n, n, n)), h, 1.0, 0.01, 0.002, g)
    expect = u + 0.002 * np.array(g)[:, None, None, None]
    assert np.abs(out - expect).max() <= 1e-14


@pytest.mark.parametrize("m", [1, 3])
def test_predict_shear_mode_decays_by_the_crank_nicolson_factor(m):
    """u_x = a sin(2 pi m y): div(uu) = 0 exactly, so Eq. (31) reduces to
    u~* = (1 + a dt nu lam / 2) / (1 - a dt nu lam / 2) u with lam the
    7-point eigenvalue of the mode."""
    n = 16
    x, y, z, h = _centres(n)
    rho, mu, dt = 2.0, 0.05, 0.01
    u = np.zeros((3, n, n, n))
    u[0] = 0.7 * np.sin(2 * np.pi * m * y)
    out = FL.predict(u, np.zeros((n, n, n)), h, rho, mu, dt, (0.0, 0.0, 0.0))
    lam = (2 * np.cos(2 * np.pi * m / n) - 2) / h ** 2
    a = 0.5 * (mu / rho) * dt * lam
    assert np.abs(out[0] - (1 + a) / (1 - a) * u[0]).max() <= 1e-14
    assert np.abs(out[1:]).max() <= 1e-15


def test_predict_convection_converges_at_second_order():
    err = []
    for n in (16, 32, 64):
        x, y, z, h = _centres(n)
        u = np.stack([np.sin(2 * np.pi * y), np.sin(2 * np.pi * z), np.sin(2 * np.pi * x)])
        exact = 2 * np.pi * np.stack([np.sin(2 * np.pi * z) * np.cos(2 * np.pi * y),
                                      np.sin(2 * np.pi * x) * np.cos(2 * np.pi * z),
                                      np.sin(2 * np.pi * y) * np.cos(2 * np.pi * x)])
        err.append(np.abs(FL.convection(u, h) - exact).max())
    assert 3.5 < err[0] / err[1] < 4.5 and 3.5 < err[1] / err[2] < 4.5


def test_predict_pressure_term():
    """u = 0, mu = 0: u~* = -(dt/rho) G p."""
    rng = np.random.default_rng(4)
    n, h, rho, dt = 8, 1.0 / 8, 1.7, 0.03
    p = rng.normal(size=(n, n, n))
    out = FL.predict(np.zeros((3, n, n, n)), p, h, rho, 0.0, dt, (0.0, 0.0, 0.0))
    assert np.abs(out + dt / rho * FL.grad_nodes(p, h)).max() <= 1e-14 * np.abs(p).max() / h
