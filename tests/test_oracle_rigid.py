"""Pins of the oracle's particle update (Sec. 3.2: Eqs. (particle1),
(particle2), (pr2); markers by Eq. (x)) against closed forms and a library
rotation."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation


def _setup(rng, n=5):
    xc = rng.uniform(0.2, 0.8, (n, 3))
    d = rng.uniform(0.05, 0.1, n)
    up = rng.normal(0, 0.1, (n, 3))
    om = rng.normal(0, 1.0, (n, 3))
    rho_p = rng.uniform(1.5, 10.0, n)
    return xc, d, up, om, rho_p


def test_free_fall_matches_constant_acceleration(oracle_mod):
    """No IB force and steady volume integrals: a = (1 - rho_f/rho_p) g, and
    the midpoint centroid update reproduces x0 + u0 t + a t^2/2 exactly."""
    rng = np.random.default_rng(1)
    xc, d, up, om, rho_p = _setup(rng)
    g = np.array([0.0, 0.0, -9.81])
    rho_f, dt = 1.0, 1e-3
    sums = np.zeros((5, 12))
    x, u, w = xc.copy(), up.copy(), om.copy()
    for _ in range(7):
        u, w, x = oracle_mod.rigid_update(x, d, u, w, rho_p, sums, sums, rho_f, g, dt)
    t = 7 * dt
    a = (1.0 - rho_f / rho_p)[:, None] * g[None, :]
    assert np.allclose(u, up + a * t, rtol=0, atol=1e-14)
    assert np.allclose(x, xc + up * t + 0.5 * a * t * t, rtol=0, atol=1e-14)
    assert np.array_equal(w, om)


def test_torque_and_force_terms(oracle_mod):
    """Collision torque alone: W' = W + dt T / I_p with I_p = rho_p pi D^5/60.
    IB force and the change of the volume integrals enter with -rho_f and
    +rho_f/dt divided by the particle mass."""
    rng = np.random.default_rng(2)
    xc, d, up, om, rho_p = _setup(rng)
    rho_f, dt = 1.3, 2e-3
    g = np.zeros(3)
    Tc = rng.normal(size=(5, 3))
    zero = np.zeros((5, 12))
    _, w1, _ = oracle_mod.rigid_update(xc, d, up, om, rho_p, zero, zero, rho_f, g, dt, Tc=Tc)
    Ip = rho_p * np.pi * d ** 5 / 60.0
    assert np.allclose(w1, om + dt * Tc / Ip[:, None], rtol=1e-14, atol=0)
    s0 = rng.normal(size=(5, 12))
    s1 = rng.normal(size=(5, 12))
    Fc = rng.normal(size=(5, 3))
    u1, w1, x1 = oracle_mod.rigid_update(xc, d, up, om, rho_p, s0, s1, rho_f, g, dt, Fc=Fc)
    m = rho_p * np.pi * d ** 3 / 6.0
    fu = -rho_f * s0[:, 0:3] + rho_f * (s1[:, 6:9] - s0[:, 6:9]) / dt + Fc
    ft = -rho_f * s0[:, 3:6] + rho_f * (s1[:, 9:12] - s0[:, 9:12]) / dt
    assert np.allclose(u1, up + dt * fu / m[:, None], rtol=1e-13, atol=1e-15)
    assert np.allclose(w1, om + dt * ft / (m * d * d / 10.0)[:, None], rtol=1e-13, atol=1e-15)
    assert np.allclose(x1, xc + 0.5 * dt * (up + u1), rtol=0, atol=1e-16)


def test_prescribed_particles_keep_their_velocity(oracle_mod):
    rng = np.random.default_rng(3)
    xc, d, up, om, rho_p = _setup(rng)
    s0 = rng.normal(size=(5, 12))
    pr = np.array([1, 0, 1, 0, 1], np.int32)
    u1, w1, x1 = oracle_mod.rigid_update(xc, d, up, om, rho_p, s0, s0, 1.0, [0, 0, -1.0], 0.01,
                                         prescribed=pr)
    k = pr.astype(bool)
    assert np.array_equal(u1[k], up[k]) and np.array_equal(w1[k], om[k])
    assert np.allclose(x1[k], xc[k] + 0.01 * up[k], rtol=0, atol=1e-16)
    assert not np.allclose(u1[~k], up[~k])


def _markers(oracle_mod, xc, d, h=1 / 64):
    return oracle_mod.build_markers(xc, d, h)


def test_translation_moves_every_marker_with_its_centroid(oracle_mod):
    rng = np.random.default_rng(4)
    xc, d, up, om, rho_p = _setup(rng, 3)
    m = _markers(oracle_mod, xc, d)
    z = np.zeros((3, 3))
    xc1 = xc + rng.normal(0, 0.01, (3, 3))
    m1 = oracle_mod.advect_markers(m, xc, xc1, z, z, 0.01)
    shift = (xc1 - xc)[m.pid]
    assert np.allclose(m1.xyz() - m.xyz(), shift, rtol=0, atol=1e-15)


@pytest.mark.parametrize("axis", ["z", "random"])
def test_rotation_matches_a_library_rotation(oracle_mod, axis):
    """Midpoint angular velocity W = (W^n + W^{n+1})/2: the markers turn by
    |W| dt about W/|W| around the new centroid (Rodrigues), which a rotation
    vector in scipy reproduces; distances to the centroid are kept."""
    rng = np.random.default_rng(5)
    xc, d, up, om, rho_p = _setup(rng, 3)
    m = _markers(oracle_mod, xc, d)
    if axis == "z":
        w0 = np.zeros((3, 3))
        w0[:, 2] = [0.5, -1.0, 2.0]
        w1 = 3.0 * w0
    else:
        w0 = rng.normal(size=(3, 3))
        w1 = rng.normal(size=(3, 3))
    dt = 0.05
    xc1 = xc + 0.01
    m1 = oracle_mod.advect_markers(m, xc, xc1, w0, w1, dt)
    R0 = m.xyz() - xc[m.pid]
    R1 = m1.xyz() - xc1[m.pid]
    wm = 0.5 * (w0 + w1)
    for p in range(3):
        sel = m.pid == p
        ref = Rotation.from_rotvec(wm[p] * dt).apply(R0[sel])
        assert np.allclose(R1[sel], ref, rtol=0, atol=1e-15)
        if axis == "z":
            th = wm[p, 2] * dt
            c, s = np.cos(th), np.sin(th)
            rz = np.stack([c * R0[sel, 0] - s * R0[sel, 1], s * R0[sel, 0] + c * R0[sel, 1],
                           R0[sel, 2]], 1)
            assert np.allclose(R1[sel], rz, rtol=0, atol=1e-15)
    assert np.allclose(np.linalg.norm(R1, axis=1), np.linalg.norm(R0, axis=1), rtol=1e-14)


def test_collision_force_of_two_spheres(oracle_mod):
    """Eq. (DKT_model) by hand: D = 0.1, h = 0.01, so D_c = 0.11; at a centre
    distance 0.105 the gap term is ((0.105 - 0.11)/0.01)^2 = 1/4."""
    xc = np.array([[0.3, 0.4, 0.5], [0.3, 0.4, 0.605]])
    d = np.array([0.1, 0.1])
    rho = np.array([1140.0, 1140.0])
    F = oracle_mod.collision_forces(xc, d, rho, 9.81, 0.01)
    m = 1140.0 * np.pi * 0.1 ** 3 / 6.0
    mag = m * 9.81 / 1e-4 * 0.25
    assert np.allclose(F[0], [0.0, 0.0, -mag], rtol=1e-12, atol=0)
    assert np.allclose(F[1], [0.0, 0.0, mag], rtol=1e-12, atol=0)
    # zero beyond the contact distance, continuous at it
    far = oracle_mod.collision_forces(xc + [[0, 0, 0], [0, 0, 0.006]], d, rho, 9.81, 0.01)
    assert np.array_equal(far, np.zeros((2, 3)))
    near = oracle_mod.collision_forces(xc + [[0, 0, 0], [0, 0, 0.005 - 1e-9]], d, rho, 9.81, 0.01)
    assert np.abs(near).max() < 1e-7 * mag


def test_collision_forces_balance_and_wrap(oracle_mod):
    """Pairwise equal and opposite (total zero), and across a periodic face by
    the minimum image."""
    rng = np.random.default_rng(9)
    n = 60
    xc = rng.uniform(0, 1, (n, 3))
    d = rng.uniform(0.1, 0.2, n)
    rho = rng.uniform(1000, 3000, n)
    F = oracle_mod.collision_forces(xc, d, rho, 9.81, 1 / 64, L=(1.0, 1.0, 1.0))
    assert np.abs(F).max() > 0
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * np.abs(F).sum()
    pair = np.array([[0.01, 0.5, 0.5], [0.99, 0.5, 0.5]])
    dd = np.array([0.02, 0.02])
    rr = np.array([1000.0, 1000.0])
    Fp = oracle_mod.collision_forces(pair, dd, rr, 9.81, 0.01, L=(1.0, 1.0, 1.0))
    Fb = oracle_mod.collision_forces(pair, dd, rr, 9.81, 0.01)
    assert Fp[0, 0] > 0 and Fp[1, 0] < 0          # pushed apart across the face
    assert np.array_equal(Fb, np.zeros((2, 3)))   # bounded axes: far apart
