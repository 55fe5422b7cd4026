"""FP64 oracle of the single-level periodic fluid steps around the IB loop
(Sec. 3.1, Steps 1 and 3 of the time advancement).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and by nothing in the GPU
library.  Plain NumPy: stencils by ``numpy.roll``, the two linear solves by
``numpy.fft`` (a library primitive), nothing blocked or fused.

Grid: n^3 cells of edge h, periodic on every axis.  Velocity is
cell-centred, ``u[c][z][y][x]``; pressure is node-centred (the semi-staggered
grid of the paper's figure), ``p[z][y][x]`` with node (i, j, k) at the low
corner of cell (i, j, k).  Readings of what the paper leaves open:

* G p (cell-centred gradient of a nodal field): the difference across the
  cell along the axis, averaged over the cell's four edges parallel to it.
* D V (nodal divergence of a cell-centred field): the transpose construction
  -- differences between the two layers of cells that share the node,
  averaged over the four cells of each layer.  D = -G^T in the plain sums
  over cells and nodes.
* L (cell-centred Laplacian in Eq. (31)): the 7-point stencil.
* The convective term of Eq. (31): the paper's second-order Godunov scheme is
  cited, not given; here it is the second-order central flux form at t^n,
  div(u u) = sum_d [(u_d u)(i+1/2) - (u_d u)(i-1/2)] / h with face values the
  mean of the two cells.  Parity unpinned to the paper for this term: it is
  pinned to its own definition (second-order convergence to the analytic
  divergence of u u), not to the scheme the paper cites.
* Step 1 solve: (I - (nu dt / 2) L) u~* = u^n - dt div(uu) - (dt/rho) G p
  + (nu dt / 2) L u^n + dt g  (Eq. (31) with constant mu = rho nu), exactly by
  FFT.
* Step 3 solve: (1/rho) D G p = D V (Eq. (ns_lp2)), exactly by FFT; Fourier
  modes where the symbol of D G vanishes (the constant and the modes with two
  or more components at the Nyquist frequency) get p = 0.
"""
from __future__ import annotations

import numpy as np

# (z, y, x) array axes of the spatial directions x, y, z
_AX = (2, 1, 0)


def _fwd(a, d):
    """a shifted so that entry i holds a(i + 1) along direction d."""
    return np.roll(a, -1, axis=_AX[d] + (a.ndim - 3))


def _bwd(a, d):
    """a shifted so that entry i holds a(i - 1) along direction d."""
    return np.roll(a, 1, axis=_AX[d] + (a.ndim - 3))


def grad_nodes(p, h):
    """G p: [3][n][n][n] cell-centred gradient of nodal p."""
    out = np.empty((3,) + p.shape)
    for d in range(3):
        e1, e2 = [e for e in range(3) if e != d]
        avg = 0.25 * (p + _fwd(p, e1) + _fwd(p, e2) + _fwd(_fwd(p, e1), e2))
        out[d] = (_fwd(avg, d) - avg) / h
    return out


def div_nodes(V, h):
    """D V: nodal divergence of cell-centred V[3]."""
    out = np.zeros(V.shape[1:])
    for d in range(3):
        e1, e2 = [e for e in range(3) if e != d]
        v = V[d]
        avg = 0.25 * (v + _bwd(v, e1) + _bwd(v, e2) + _bwd(_bwd(v, e1), e2))
        out += (avg - _bwd(avg, d)) / h
    return out


def laplacian(u, h):
    """7-point Laplacian of every component of cell-centred u[3]."""
    out = np.zeros_like(u)
    for d in range(3):
        out += (_fwd(u, d) - 2.0 * u + _bwd(u, d)) / (h * h)
    return out


def convection(u, h):
    """div(u u) in central flux form: component c of sum_d d_d(u_d u_c)."""
    out = np.zeros_like(u)
    for d in range(3):
        uf = 0.5 * (u + _fwd(u, d))          # face i+1/2 along d, every component
        flux = uf[d][None] * uf              # (u_d u_c) on that face
        out += (flux - _bwd(flux, d)) / h
    return out


def _theta(n):
    k = np.arange(n)
    return 2.0 * np.pi * k / n


def laplacian_symbol(n, h):
    """Eigenvalue of the 7-point Laplacian for every Fourier mode [z][y][x]."""
    lam1 = (2.0 * np.cos(_theta(n)) - 2.0) / (h * h)
    return lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]


def dg_symbol(n, h):
    """Eigenvalue of D G for every Fourier mode [z][y][x]."""
    th = _theta(n)
    s2 = np.sin(0.5 * th) ** 2
    c2 = np.cos(0.5 * th) ** 2
    sx, sy, sz = s2[None, None, :], s2[None, :, None], s2[:, None, None]
    cx, cy, cz = c2[None, None, :], c2[None, :, None], c2[:, None, None]
    return -4.0 / (h * h) * (sx * cy * cz + sy * cx * cz + sz * cx * cy)


def predict(u, p, h, rho, mu, dt, g):
    """Step 1, Eq. (31): u~* from u^n and p^{n-1/2}."""
    n = u.shape[1]
    nu = mu / rho
    a = 0.5 * nu * dt
    rhs = (u - dt * convection(u, h) - (dt / rho) * grad_nodes(p, h) + a * laplacian(u, h)
           + dt * np.asarray(g, dtype=np.float64)[:, None, None, None])
    den = 1.0 - a * laplacian_symbol(n, h)
    out = np.empty_like(u)
    for c in range(3):
        out[c] = np.fft.ifftn(np.fft.fftn(rhs[c]) / den).real
    return out


def project(ustar, p_old, h, rho, dt):
    """Step 3, Eqs. (ns_lp1)-(ns_lp3): returns (u^{n+1}, p^{n+1/2})."""
    n = ustar.shape[1]
    V = ustar / dt + grad_nodes(p_old, h) / rho
    r = div_nodes(V, h)
    sig = dg_symbol(n, h)
    keep = np.abs(sig) > 1e-10 * np.abs(sig).max()
    rh = np.fft.fftn(r)
    ph = np.zeros_like(rh)
    ph[keep] = rho * rh[keep] / sig[keep]
    p = np.fft.ifftn(ph).real
    u = dt * (V - grad_nodes(p, h) / rho)
    return u, p
