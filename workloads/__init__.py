"""Seeded synthetic inputs for the multidirect-forcing immersed-boundary loop.

This module draws inputs and converts layouts; it performs no step of the
method (no markers, no delta kernel, no interpolation or spreading).  Both the
FP64 oracle (tests, CPU baseline) and the GPU library consume what it returns.

Recipe (all draws from ``numpy.random.default_rng(seed)``, in this order):

1. particle diameters, then centres (random sequential addition without solid
   overlap under the periodic minimum image, or Gaussian clumps);
2. rigid-body velocities: ``U_p ~ N(0, 0.1^2)`` then ``omega_p ~ N(0, 1)`` per
   component;
3. the velocity field: ``u(x) = sum_q a_q cos(2 pi k_q.x / L + theta_q)`` over
   distinct integer wave vectors ``1 <= |k_q| <= K`` (``k`` and ``-k`` counted
   once), ``a_q`` a unit vector orthogonal to ``k_q`` and
   ``theta_q ~ U[0, 2 pi)``, evaluated in FP64 at cell centres.

Grids are cell-centred on ``[lo, lo + n h)^3`` and tiled into cubic boxes of
``box`` cells; a box is covered when it lies within ``ceil(P/2) + 1`` cells of
some particle's bounding box (all boxes when ``cover_all``).  Fields are held
either as a global array ``[3][nz][ny][nx]`` (x fastest) or in the box layout
``[nbox][3][B+2g][B+2g][B+2g]`` used by the library, whose ghost cells the
library never reads (tests fill them with NaN).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Level", "Workload", "make_level", "make_workload", "config",
    "CONFIG_NAMES", "to_boxes", "from_boxes", "fourier_field",
]


@dataclasses.dataclass
class Level:
    """Finest-level grid: ``n`` cells per axis of size ``h`` from ``lo``."""
    n: tuple
    h: float
    lo: tuple
    periodic: tuple
    box: int
    ngrow: int
    box_coords: np.ndarray          # (nbox, 3) int32, box index (x, y, z)
    lut: np.ndarray                 # (nbz*nby*nbx,) int32, x fastest -> box id / -1

    @property
    def nbox(self) -> int:
        return int(self.box_coords.shape[0])

    @property
    def nb(self) -> tuple:
        return tuple(int(v) // self.box for v in self.n)

    @property
    def box_lo(self) -> np.ndarray:
        return (self.box_coords * self.box).astype(np.int32)

    @property
    def box_extent(self) -> int:
        return self.box + 2 * self.ngrow

    def covered_mask(self) -> np.ndarray:
        """Boolean global mask ``[nz][ny][nx]`` of cells inside covered boxes."""
        nbx, nby, nbz = self.nb
        m = (self.lut.reshape(nbz, nby, nbx) >= 0)
        b = self.box
        return np.repeat(np.repeat(np.repeat(m, b, 0), b, 1), b, 2)


@dataclasses.dataclass
class Workload:
    name: str
    level: Level
    delta: int                      # 3 or 4 (kernel width P)
    ns: int                         # multidirect iterations
    dt: float
    xc: np.ndarray                  # (np, 3) particle centres
    d: np.ndarray                   # (np,) diameters
    up: np.ndarray                  # (np, 3) translational velocity
    om: np.ndarray                  # (np, 3) angular velocity
    u0: np.ndarray                  # (3, nz, ny, nx) float64 velocity field
    seed: int = 0
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def npart(self) -> int:
        return int(self.d.shape[0])


def make_level(n, h, lo=(0.0, 0.0, 0.0), periodic=(1, 1, 1), box=32, ngrow=2,
               covered=None) -> Level:
    """Build a level; ``covered`` is a boolean array over boxes (z, y, x) or None (all)."""
    n = tuple(int(v) for v in (n if np.iterable(n) else (n, n, n)))
    for v in n:
        if v % box:
            raise ValueError("box size must divide the grid")
    nbx, nby, nbz = (v // box for v in n)
    if covered is None:
        covered = np.ones((nbz, nby, nbx), dtype=bool)
    covered = np.asarray(covered, dtype=bool).reshape(nbz, nby, nbx)
    lut = np.full(nbz * nby * nbx, -1, dtype=np.int32)
    coords = []
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                if covered[bz, by, bx]:
                    lut[bx + nbx * (by + nby * bz)] = len(coords)
                    coords.append((bx, by, bz))
    box_coords = np.asarray(coords, dtype=np.int32).reshape(-1, 3)
    return Level(n=n, h=float(h), lo=tuple(float(v) for v in lo),
                 periodic=tuple(int(v) for v in periodic), box=int(box),
                 ngrow=int(ngrow), box_coords=box_coords, lut=lut)


def _coverage(n, h, lo, box, xc, d, delta):
    """Boxes within ceil(P/2)+1 cells of any particle bounding box (periodic)."""
    nb = [v // box for v in n]
    cov = np.zeros((nb[2], nb[1], nb[0]), dtype=bool)
    dil = int(math.ceil(delta / 2.0)) + 1
    for p in range(xc.shape[0]):
        rng_ax = []
        for a in range(3):
            s = (xc[p, a] - lo[a]) / h
            r = 0.5 * d[p] / h
            c0 = math.floor(s - r) - dil
            c1 = math.floor(s + r) + dil
            bset = sorted({(c // box) % nb[a] for c in range(c0, c1 + 1)})
            rng_ax.append(bset)
        for bz in rng_ax[2]:
            for by in rng_ax[1]:
                for bx in rng_ax[0]:
                    cov[bz, by, bx] = True
    return cov


def _wave_vectors(K: int) -> np.ndarray:
    """All integer k with 1 <= |k| <= K, one of each +-k pair, lexicographic order."""
    out = []
    for kx in range(-K, K + 1):
        for ky in range(-K, K + 1):
            for kz in range(-K, K + 1):
                k2 = kx * kx + ky * ky + kz * kz
                if k2 == 0 or k2 > K * K:
                    continue
                first = next(v for v in (kx, ky, kz) if v != 0)
                if first > 0:
                    out.append((kx, ky, kz))
    return np.asarray(out, dtype=np.int64)


def fourier_field(rng, n, h, lo, nmodes: int, K: int) -> np.ndarray:
    """Velocity field of ``nmodes`` random divergence-free Fourier modes, FP64.

    Each mode is evaluated separably, cos(A + B + C + theta) =
    cos A cos(B + C + theta) - sin A sin(B + C + theta) with A, B, C the
    phases along x, y, z, using torch's threaded CPU kernels."""
    import torch
    ks = _wave_vectors(K)
    pick = rng.choice(ks.shape[0], size=nmodes, replace=False)
    modes = []
    for j in pick:
        k = ks[j].astype(np.float64)
        a = rng.normal(size=3)
        a -= (a @ k) / (k @ k) * k
        a /= np.linalg.norm(a)
        theta = rng.uniform(0.0, 2.0 * np.pi)
        modes.append((ks[j], a, theta))
    nx, ny, nz = n
    L = [n[i] * h for i in range(3)]
    xs = [(torch.arange(n[i], dtype=torch.float64) + 0.5) * h for i in range(3)]
    u = torch.zeros((3, nz, ny, nx), dtype=torch.float64)
    val = torch.empty((nz, ny, nx), dtype=torch.float64)
    for k, a, theta in modes:
        A = (2.0 * np.pi * float(k[0]) / L[0]) * xs[0]
        B = (2.0 * np.pi * float(k[1]) / L[1]) * xs[1]
        C = (2.0 * np.pi * float(k[2]) / L[2]) * xs[2]
        bc = B[None, :] + C[:, None] + theta
        torch.mul(torch.cos(bc)[:, :, None], torch.cos(A)[None, None, :], out=val)
        val.addcmul_(torch.sin(bc)[:, :, None], torch.sin(A)[None, None, :], value=-1.0)
        for c in range(3):
            if a[c] != 0.0:
                u[c].add_(val, alpha=float(a[c]))
    return u.numpy()


def _rsa(rng, diam, nplace, max_tries=200000):
    """Random sequential addition in the periodic unit cube, no solid overlap."""
    pos = np.zeros((nplace, 3))
    for i in range(nplace):
        for _ in range(max_tries):
            x = rng.uniform(0.0, 1.0, size=3)
            if i == 0:
                break
            dx = pos[:i] - x
            dx -= np.round(dx)
            dist = np.sqrt((dx * dx).sum(axis=1))
            if np.all(dist >= 0.5 * (diam[:i] + diam[i])):
                break
        else:
            raise RuntimeError("random sequential addition jammed")
        pos[i] = x
    return pos


def make_workload(name, n, box, ngrow, delta, ns, diam_cells, *, seed=0,
                  placement="rsa", centres=None, nmodes=32, K=8, cover_all=False,
                  periodic=(1, 1, 1), clumps=64, clump_sigma=0.05, dt_cells=0.5,
                  with_field=True):
    """Generic builder on the periodic unit cube with ``n`` cells per axis.

    ``diam_cells``: array of diameters in cells (already drawn) or a callable
    ``rng -> array``.  ``with_field=False`` skips the velocity field (u0 is
    None); every other draw is unchanged.
    """
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    lo = (0.0, 0.0, 0.0)
    dcell = diam_cells(rng) if callable(diam_cells) else np.asarray(diam_cells, float)
    d = dcell * h
    npart = d.shape[0]
    if centres is not None:
        xc = np.asarray(centres, dtype=np.float64).reshape(npart, 3)
    elif placement == "rsa":
        xc = _rsa(rng, d, npart)
    elif placement == "clumps":
        cc = rng.uniform(0.0, 1.0, size=(clumps, 3))
        which = rng.integers(0, clumps, size=npart)
        xc = np.mod(cc[which] + rng.normal(0.0, clump_sigma, size=(npart, 3)), 1.0)
    else:
        raise ValueError(placement)
    up = rng.normal(0.0, 0.1, size=(npart, 3))
    om = rng.normal(0.0, 1.0, size=(npart, 3))
    ntup = (n, n, n)
    u0 = fourier_field(rng, ntup, h, lo, nmodes, K) if with_field else None
    cov = None if cover_all else _coverage(ntup, h, lo, box, xc, d, delta)
    level = make_level(ntup, h, lo, periodic, box, ngrow, cov)
    return Workload(name=name, level=level, delta=delta, ns=ns, dt=dt_cells * h,
                    xc=xc, d=d, up=up, om=om, u0=u0, seed=seed)


CONFIG_NAMES = ("sphere1_64", "spheres8_256", "spheres1000_256",
                "spheres20000_512", "spheres64_128")


def config(k, seed=0, with_field=True) -> Workload:
    """The five reference workloads (index 1..5 or name)."""
    if isinstance(k, str):
        k = CONFIG_NAMES.index(k) + 1
    if k == 1:
        return make_workload("sphere1_64", 64, 64, 2, 3, 2, np.array([16.0]),
                             seed=seed, centres=[[0.5, 0.5, 0.5]], nmodes=8, K=4,
                             cover_all=True, with_field=with_field)
    if k == 2:
        return make_workload("spheres8_256", 256, 32, 2, 4, 5, np.full(8, 24.0),
                             seed=seed, cover_all=True, with_field=with_field)
    if k == 3:
        def lognormal(rng):
            return np.clip(np.exp(np.log(16.0) + 0.3 * rng.normal(size=1000)), 8.0, 32.0)
        return make_workload("spheres1000_256", 256, 32, 2, 4, 5, lognormal, seed=seed,
                             with_field=with_field)
    if k == 4:
        def uniform(rng):
            return rng.uniform(8.0, 24.0, size=20000)
        return make_workload("spheres20000_512", 512, 32, 2, 3, 5, uniform, seed=seed,
                             placement="clumps", with_field=with_field)
    if k == 5:
        return make_workload("spheres64_128", 128, 32, 2, 4, 3, np.full(64, 16.0),
                             seed=seed, cover_all=True, with_field=with_field)
    raise ValueError(k)


def to_boxes(u: np.ndarray, level: Level, fill=np.nan, dtype=None) -> np.ndarray:
    """Global ``[3][nz][ny][nx]`` -> box layout ``[nbox][3][E][E][E]`` (ghosts = fill)."""
    b, g = level.box, level.ngrow
    e = b + 2 * g
    out = np.full((level.nbox, u.shape[0], e, e, e), fill,
                  dtype=dtype if dtype is not None else u.dtype)
    for i, (bx, by, bz) in enumerate(level.box_coords):
        out[i, :, g:g + b, g:g + b, g:g + b] = u[:, bz * b:(bz + 1) * b,
                                                 by * b:(by + 1) * b, bx * b:(bx + 1) * b]
    return out


def from_boxes(ub: np.ndarray, level: Level, fill=np.nan) -> np.ndarray:
    """Box layout -> global array; cells of uncovered boxes get ``fill``."""
    b, g = level.box, level.ngrow
    nx, ny, nz = level.n
    out = np.full((ub.shape[1], nz, ny, nx), fill, dtype=np.float64)
    for i, (bx, by, bz) in enumerate(level.box_coords):
        out[:, bz * b:(bz + 1) * b, by * b:(by + 1) * b, bx * b:(bx + 1) * b] = \
            ub[i, :, g:g + b, g:g + b, g:g + b]
    return out
