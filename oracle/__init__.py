"""FP64 oracle of the multidirect-forcing IB loop (ctypes over liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the GPU library.
Shares no code with the GPU path.  See ``ibx_oracle.c`` for the equations and
readings each function follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, LIB_OMP, build

_lib = None
_lib_omp = None

_d = C.c_double
_i32 = C.c_int32
_i64 = C.c_int64
_p = C.c_void_p


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double), ("lo", C.c_double * 3),
                ("periodic", C.c_int32 * 3)]


def _load(threads: int = 0):
    """The single-threaded oracle, or with threads > 0 the OpenMP build of the
    same source set to that many threads (identical results)."""
    global _lib, _lib_omp
    if threads > 0:
        if _lib_omp is None:
            if not os.path.exists(LIB_OMP):
                build()
            _lib_omp = _setup(C.CDLL(LIB_OMP))
        _lib_omp.ibo_threads(int(threads))
        return _lib_omp
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _setup(C.CDLL(LIB))
    return _lib


def threads_available() -> int:
    """Threads the OpenMP build runs with by default (OMP_NUM_THREADS, else the
    host's cores)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(LIB_OMP):
            build()
        _lib_omp = _setup(C.CDLL(LIB_OMP))
    return int(_lib_omp.ibo_threads(0))


def _setup(lib):
    lib.ibo_threads.restype = C.c_int
    lib.ibo_threads.argtypes = [C.c_int]
    lib.ibo_phi.restype = _d
    lib.ibo_phi.argtypes = [C.c_int, _d]
    lib.ibo_dphi.restype = _d
    lib.ibo_dphi.argtypes = [C.c_int, _d]
    lib.ibo_count_markers.restype = _i64
    lib.ibo_count_markers.argtypes = [_i32, _p, _d, _p]
    lib.ibo_build_markers.restype = None
    lib.ibo_build_markers.argtypes = [_i32, _p, _p, _d, _p, _p, _p, _p, _p, _p]
    lib.ibo_bucket.restype = _i64
    lib.ibo_bucket.argtypes = [_p, _p, _d, _p, _i32, _p, _i32, _i32, _i64, _p, _p, _p,
                               _p, _p, _p, _p, _p, _p, _p, _i64, _p]
    lib.ibo_desired_velocity.restype = None
    lib.ibo_desired_velocity.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _p, _p]
    lib.ibo_interp.restype = C.c_int
    lib.ibo_interp.argtypes = [C.POINTER(Grid), C.c_int, _i64, _p, _p, _p, _p, _p]
    lib.ibo_spread.restype = C.c_int
    lib.ibo_spread.argtypes = [C.POINTER(Grid), C.c_int, _i64, _p, _p, _p, _p, _p, _p, _p]
    lib.ibo_multidirect.restype = C.c_int
    lib.ibo_multidirect.argtypes = [C.POINTER(Grid), C.c_int, C.c_int, _d, C.c_int, _i32,
                                    _p, _p, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _p,
                                    _p, _p, _p]
    lib.ibo_pvf_volume.restype = _d
    lib.ibo_pvf_volume.argtypes = [C.POINTER(Grid), _p, _p]
    lib.ibo_particle_reductions.restype = C.c_int
    lib.ibo_particle_reductions.argtypes = [C.POINTER(Grid), _i32, _p, _p, _p, _p, _p, _p,
                                            _p, _p, _p, _p]
    lib.ibo_reverse.restype = C.c_int
    lib.ibo_reverse.argtypes = [C.POINTER(Grid), C.c_int, C.c_int, _d, _i32, _p, _p, _p,
                                _p, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p,
                                _p, _p]
    lib.ibo_rigid_update.restype = None
    lib.ibo_rigid_update.argtypes = [_i32] + [_p] * 10 + [_d, _p, _d, _p, _p, _p]
    lib.ibo_advect_markers.restype = None
    lib.ibo_advect_markers.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _p, _p, _d, _p, _p, _p]
    lib.ibo_collision_forces.restype = None
    lib.ibo_collision_forces.argtypes = [_i32, _p, _p, _p, _d, _d, _d, _p, _p]
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def grid(n, h, lo=(0.0, 0.0, 0.0), periodic=(1, 1, 1)) -> Grid:
    n = tuple(n) if np.iterable(n) else (n, n, n)
    g = Grid()
    g.n[:] = [int(v) for v in n]
    g.h = float(h)
    g.lo[:] = [float(v) for v in lo]
    g.periodic[:] = [int(v) for v in periodic]
    return g


def grid_of(level) -> Grid:
    return grid(level.n, level.h, level.lo, level.periodic)


def phi(P: int, r):
    lib = _load()
    r = np.asarray(r, dtype=np.float64)
    return np.vectorize(lambda v: lib.ibo_phi(int(P), float(v)), otypes=[np.float64])(r)


def dphi(P: int, r):
    lib = _load()
    r = np.asarray(r, dtype=np.float64)
    return np.vectorize(lambda v: lib.ibo_dphi(int(P), float(v)), otypes=[np.float64])(r)


class Markers:
    """Markers of all particles: SoA positions, owner id, per-particle dV."""

    def __init__(self, x, y, z, pid, dv, offs):
        self.x, self.y, self.z = _f64(x), _f64(y), _f64(z)
        self.pid = np.ascontiguousarray(pid, dtype=np.int32)
        self.dv = _f64(dv)
        self.offs = np.ascontiguousarray(offs, dtype=np.int64)

    @property
    def nl(self) -> int:
        return int(self.x.shape[0])

    def xyz(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)


def count_markers(d, h) -> np.ndarray:
    lib = _load()
    d = _f64(d)
    offs = np.zeros(d.shape[0] + 1, dtype=np.int64)
    lib.ibo_count_markers(d.shape[0], _ptr(d), float(h), _ptr(offs))
    return offs


def build_markers(xc, d, h) -> Markers:
    lib = _load()
    xc, d = _f64(xc), _f64(d)
    offs = count_markers(d, h)
    nl = int(offs[-1])
    x, y, z = (np.zeros(nl) for _ in range(3))
    pid = np.zeros(nl, dtype=np.int32)
    dv = np.zeros(d.shape[0])
    lib.ibo_build_markers(d.shape[0], _ptr(xc), _ptr(d), float(h), _ptr(offs), _ptr(x),
                          _ptr(y), _ptr(z), _ptr(pid), _ptr(dv))
    return Markers(x, y, z, pid, dv, offs)


def bucket(level, P: int, m: Markers, tile: int = 8) -> dict:
    lib = _load()
    n = np.asarray(level.n, dtype=np.int32)
    lo = _f64(level.lo)
    per = np.asarray(level.periodic, dtype=np.int32)
    lut = np.ascontiguousarray(level.lut, dtype=np.int32)
    nl = m.nl
    T = int(np.prod(n // tile))
    cell = np.zeros(nl, np.int32)
    tid = np.zeros(nl, np.int32)
    base = np.zeros((nl, 3), np.int32)
    perm = np.zeros(nl, np.int32)
    toffs = np.zeros(T + 1, np.int32)
    soffs = np.zeros(T + 1, np.int32)
    cap = 8 * max(nl, 1)
    sidx = np.zeros(cap, np.int32)
    nsrc = np.zeros(1, np.int64)
    flagged = lib.ibo_bucket(_ptr(n), _ptr(lo), float(level.h), _ptr(per), int(level.box),
                             _ptr(lut), int(tile), int(P), nl, _ptr(m.x), _ptr(m.y),
                             _ptr(m.z), _ptr(cell), _ptr(tid), _ptr(base), _ptr(perm),
                             _ptr(toffs), _ptr(soffs), _ptr(sidx), cap, _ptr(nsrc))
    return dict(cell=cell, tile=tid, base=base, perm=perm, tile_offs=toffs,
                src_offs=soffs, src_idx=sidx[:int(nsrc[0])].copy(), flagged=int(flagged))


def desired_velocity(m: Markers, xc, up, om) -> np.ndarray:
    lib = _load()
    xc, up, om = _f64(xc), _f64(up), _f64(om)
    Ud = np.zeros((m.nl, 3))
    lib.ibo_desired_velocity(m.nl, _ptr(m.x), _ptr(m.y), _ptr(m.z), _ptr(m.pid), _ptr(xc),
                             _ptr(up), _ptr(om), _ptr(Ud))
    return Ud


def interp(g: Grid, P: int, m: Markers, u, threads: int = 0) -> np.ndarray:
    lib = _load(threads)
    u = _f64(u)
    U = np.zeros((m.nl, 3))
    rc = lib.ibo_interp(C.byref(g), int(P), m.nl, _ptr(m.x), _ptr(m.y), _ptr(m.z), _ptr(u),
                        _ptr(U))
    if rc:
        raise ValueError("marker stencil leaves the grid")
    return U


def spread(g: Grid, P: int, m: Markers, F, threads: int = 0) -> np.ndarray:
    lib = _load(threads)
    F = _f64(F)
    f = np.zeros((3, g.n[2], g.n[1], g.n[0]))
    rc = lib.ibo_spread(C.byref(g), int(P), m.nl, _ptr(m.x), _ptr(m.y), _ptr(m.z),
                        _ptr(m.pid), _ptr(m.dv), _ptr(F), _ptr(f))
    if rc:
        raise ValueError("marker stencil leaves the grid")
    return f


def multidirect(g: Grid, P: int, ns: int, dt: float, m: Markers, xc, up, om, u0,
                order: str = "jacobi", history: bool = False, residuals: bool = True,
                threads: int = 0) -> dict:
    """Algorithm 1; threads > 0 runs the OpenMP build (same bits)."""
    lib = _load(threads)
    xc, up, om, u0 = _f64(xc), _f64(up), _f64(om), _f64(u0)
    ustar = np.zeros_like(u0)
    f = np.zeros_like(u0)
    F = np.zeros((m.nl, 3))
    Fh = np.zeros((ns, m.nl, 3)) if history else None
    resid = np.zeros(ns + 1)
    rc = lib.ibo_multidirect(C.byref(g), int(P), int(ns), float(dt),
                             0 if order == "jacobi" else 1, xc.shape[0], _ptr(m.offs),
                             _ptr(xc), _ptr(up), _ptr(om), m.nl, _ptr(m.x), _ptr(m.y),
                             _ptr(m.z), _ptr(m.pid), _ptr(m.dv), _ptr(u0), _ptr(ustar),
                             _ptr(f), _ptr(F), _ptr(Fh),
                             _ptr(resid) if (order == "jacobi" and residuals) else None)
    if rc:
        raise ValueError("marker stencil leaves the grid")
    out = dict(ustar=ustar, f=f, F=F,
               resid=resid if (order == "jacobi" and residuals) else None)
    if history:
        out["Fhist"] = Fh
    return out


def pvf_volume(g: Grid, centre, axes) -> float:
    lib = _load()
    c, a = _f64(centre), _f64(axes)
    return float(lib.ibo_pvf_volume(C.byref(g), _ptr(c), _ptr(a)))


def particle_reductions(g: Grid, m: Markers, xc, d, F, u) -> np.ndarray:
    lib = _load()
    xc, d, F, u = _f64(xc), _f64(d), _f64(F), _f64(u)
    out = np.zeros((d.shape[0], 12))
    rc = lib.ibo_particle_reductions(C.byref(g), d.shape[0], _ptr(xc), _ptr(d), _ptr(m.offs),
                                     _ptr(m.x), _ptr(m.y), _ptr(m.z), _ptr(m.dv), _ptr(F),
                                     _ptr(u), _ptr(out))
    if rc:
        raise ValueError("particle bounding box leaves the grid")
    return out


def reverse(g: Grid, P: int, ns: int, dt: float, m: Markers, xc, up, om, u0, Fhist,
            g_ustar=None, g_f=None, g_F=None) -> dict:
    lib = _load()
    xc, up, om, u0, Fhist = (_f64(a) for a in (xc, up, om, u0, Fhist))
    gus = None if g_ustar is None else _f64(g_ustar)
    gf = None if g_f is None else _f64(g_f)
    gF = None if g_F is None else _f64(g_F)
    gu0 = np.zeros_like(u0)
    npart = xc.shape[0]
    gup = np.zeros((npart, 3))
    gom = np.zeros((npart, 3))
    gX = np.zeros((m.nl, 3))
    rc = lib.ibo_reverse(C.byref(g), int(P), int(ns), float(dt), npart, _ptr(m.offs),
                         _ptr(xc), _ptr(up), _ptr(om), m.nl, _ptr(m.x), _ptr(m.y), _ptr(m.z),
                         _ptr(m.pid), _ptr(m.dv), _ptr(u0), _ptr(Fhist), _ptr(gus), _ptr(gf),
                         _ptr(gF), _ptr(gu0), _ptr(gup), _ptr(gom), _ptr(gX))
    if rc:
        raise ValueError("marker stencil leaves the grid")
    return dict(u0=gu0, up=gup, om=gom, X=gX)


def rigid_update(xc, d, up, om, rho_p, sums_n, sums_np1, rho_f, grav, dt, Fc=None, Tc=None,
                 prescribed=None):
    """Rigid-body update of the particles (Eqs. (particle1), (particle2), (pr2));
    returns (up_new, om_new, xc_new)."""
    lib = _load()
    xc, d, up, om = _f64(xc), _f64(d), _f64(up), _f64(om)
    rho_p, sums_n, sums_np1 = _f64(rho_p), _f64(sums_n), _f64(sums_np1)
    g3 = _f64(grav)
    Fc = None if Fc is None else _f64(Fc)
    Tc = None if Tc is None else _f64(Tc)
    pr = None if prescribed is None else np.ascontiguousarray(prescribed, dtype=np.int32)
    np_ = d.shape[0]
    up1, om1, xc1 = np.zeros((np_, 3)), np.zeros((np_, 3)), np.zeros((np_, 3))
    lib.ibo_rigid_update(np_, _ptr(xc), _ptr(d), _ptr(up), _ptr(om), _ptr(rho_p),
                         _ptr(sums_n), _ptr(sums_np1), _ptr(Fc), _ptr(Tc), _ptr(pr),
                         float(rho_f), _ptr(g3), float(dt), _ptr(up1), _ptr(om1), _ptr(xc1))
    return up1, om1, xc1


def advect_markers(m: Markers, xc_n, xc_np1, om_n, om_np1, dt) -> Markers:
    """Markers moved with their particle's rigid motion (Eq. (x))."""
    lib = _load()
    xc_n, xc_np1, om_n, om_np1 = _f64(xc_n), _f64(xc_np1), _f64(om_n), _f64(om_np1)
    xn, yn, zn = (np.zeros(m.nl) for _ in range(3))
    lib.ibo_advect_markers(m.nl, _ptr(m.x), _ptr(m.y), _ptr(m.z), _ptr(m.pid), _ptr(xc_n),
                           _ptr(xc_np1), _ptr(om_n), _ptr(om_np1), float(dt), _ptr(xn),
                           _ptr(yn), _ptr(zn))
    return Markers(xn, yn, zn, m.pid, m.dv, m.offs)


def collision_forces(xc, d, rho_p, gnorm, h, eps_c=1e-4, L=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Repulsive collision force of Eq. (DKT_model) on every particle, [np][3]."""
    lib = _load()
    xc, d, rho_p, L = _f64(xc), _f64(d), _f64(rho_p), _f64(L)
    Fc = np.zeros((d.shape[0], 3))
    lib.ibo_collision_forces(d.shape[0], _ptr(xc), _ptr(d), _ptr(rho_p), float(gnorm), float(h),
                             float(eps_c), _ptr(L), _ptr(Fc))
    return Fc
