"""ctypes binding of libibx (the C ABI in ``include/ibx.h``).

Argument marshalling only: every step of the IB loop runs in the library's
HIP kernels.  Tensors are torch tensors on the current HIP device; calls are
enqueued on torch's current stream.  Importing this module fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibx.so")

IB_OK, IB_EINVAL, IB_EDOMAIN, IB_EWORKSPACE, IB_EHIP, IB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
IB_F64, IB_F32 = 0, 1
IB_PATH_AUTO, IB_PATH_PLAIN, IB_PATH_BATCHED = 0, 1, 2

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libibx.so is not built ({LIB_PATH}); run __graft_entry__.build()")
_lib = C.CDLL(LIB_PATH)

_p = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_d = C.c_double
_sz = C.c_size_t


class IbLevel(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double), ("lo", C.c_double * 3),
                ("periodic", C.c_int32 * 3), ("box", C.c_int32), ("ngrow", C.c_int32),
                ("nbox", C.c_int32), ("box_lo", _p), ("box_lut", _p)]


class IbParticles(C.Structure):
    _fields_ = [("np", C.c_int32), ("xc", _p), ("d", _p), ("up", _p), ("om", _p)]


class IbMarkers(C.Structure):
    _fields_ = [("nl", C.c_int64), ("offs", _p), ("x", _p), ("y", _p), ("z", _p),
                ("pid", _p), ("dv", _p)]


class IbBuckets(C.Structure):
    _fields_ = [("cell", _p), ("tileid", _p), ("base", _p), ("perm", _p), ("tile_offs", _p),
                ("src_offs", _p), ("src_idx", _p), ("src_cap", C.c_int64), ("flag", _p)]


_PL = C.POINTER(IbLevel)
_PP = C.POINTER(IbParticles)
_PM = C.POINTER(IbMarkers)
_PB = C.POINTER(IbBuckets)


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_count_markers = _sig("ib_count_markers", _i64, [_i32, _p, _d, _p])
_build_markers = _sig("ib_build_markers", C.c_int, [_PL, _PP, _PM, _p])
_desired_velocity = _sig("ib_desired_velocity", C.c_int, [_PP, _PM, C.c_int, _p, _p])
_bucket_ws = _sig("ib_bucket_workspace", _sz, [_PL, _i64])
_bucket = _sig("ib_bucket", C.c_int, [_PL, _PM, C.c_int, _PB, _p, _sz, _p])
_interp = _sig("ib_interp", C.c_int, [_PL, _PM, C.c_int, C.c_int, _p, _p, _p])
_spread = _sig("ib_spread", C.c_int, [_PL, _PM, _PB, C.c_int, C.c_int, _p, _p, _p])
_plan_create = _sig("ib_plan_create", C.c_int,
                    [C.POINTER(_p), C.c_int, C.c_int, C.c_int, _i32, _i32, _i32, _i32, _i32])
_plan_destroy = _sig("ib_plan_destroy", None, [_p])
_plan_query = _sig("ib_plan_query", C.c_int, [_p, _p])
_ws_bytes = _sig("ib_workspace_bytes", _sz, [_p, _PL, _i64, _i32])
_plan_profile = _sig("ib_plan_profile", C.c_int, [_p, _i32])
_plan_profile_read = _sig("ib_plan_profile_read", C.c_int, [_p, _p, _p, _i32])
PROF_CLASSES = ("prep", "lists", "interp_u0", "spread", "interp_g", "spread_final", "fill",
                "unsort", "resid")
_multidirect = _sig("ib_multidirect_force", C.c_int,
                    [_p, _PL, _PP, _PM, _PB, _i32, _d, _p, _p, _p, _p, _p, _p, _p, _sz, _p])
_autotune = _sig("ib_plan_autotune", C.c_int,
                 [_p, _PL, _PP, _PM, _PB, _i32, _d, _p, _p, _p, _p, _p, _sz, _p, _p])
_red_ws = _sig("ib_reductions_workspace", _sz, [_i32])
_reductions = _sig("ib_particle_reductions", C.c_int,
                   [_PL, _PP, _PM, C.c_int, _p, _p, _p, _p, _p, _sz, _p])
_reductions_noalloc = _sig("ib_particle_reductions_noalloc", C.c_int,
                          [_PL, _PP, _PM, C.c_int, _p, _p, _p, _p, _p])
_bwd_ws = _sig("ib_backward_workspace_bytes", _sz, [_p, _PL, _i64])
_backward = _sig("ib_multidirect_backward", C.c_int,
                 [_p, _PL, _PP, _PM, _PB, _i32, _d, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p,
                  _sz, _p])
_rigid = _sig("ib_rigid_update", C.c_int,
              [_PP, _p, _p, _p, _p, _p, _p, _d, _p, _d, _p, _p, _p, _p])
_advect = _sig("ib_advect_markers", C.c_int, [_PM, _p, _p, _p, _p, _d, _p, _p, _p, _p])
_coll_ws = _sig("ib_collision_workspace", _sz, [_PL, _i32])
_collide = _sig("ib_collision_forces", C.c_int, [_PL, _PP, _p, _d, _d, _p, _p, _sz, _p])
_lv_ws = _sig("ib_levels_workspace", _sz, [_i32])
_levels = _sig("ib_particle_levels", C.c_int, [_PL, _PP, C.c_int, _p, _p, _p, _sz, _p])
_seq_ws = _sig("ib_sequential_workspace_bytes", _sz, [_p, _PL, _i32, _i64, _i32])
_sequential = _sig("ib_multidirect_sequential", C.c_int,
                   [_p, _PL, _PP, _PM, _i32, _d, _p, _i32, _p, _p, _p, _p, _p, _p, _sz, _p])
_fl_ws = _sig("ib_fluid_workspace", _sz, [_i32, C.c_int])
_fl_predict = _sig("ib_fluid_predict", C.c_int,
                   [_i32, _d, C.c_int, _d, _d, _d, _p, _p, _p, _p, _p, _sz, _p])
_fl_project = _sig("ib_fluid_project", C.c_int,
                   [_i32, _d, C.c_int, _d, _d, _p, _p, _p, _p, _p, _sz, _p])
_to_boxes = _sig("ib_field_to_boxes", C.c_int, [_PL, C.c_int, _p, _p, _p])
_from_boxes = _sig("ib_field_from_boxes", C.c_int, [_PL, C.c_int, _p, _p, _p])
_status_string = _sig("ib_status_string", C.c_char_p, [C.c_int])
_last_hip_error = _sig("ib_last_hip_error", C.c_char_p, [])
_version = _sig("ib_version", C.c_int, [])

EXPORTED = ("ib_count_markers", "ib_build_markers", "ib_desired_velocity", "ib_bucket_workspace",
            "ib_bucket", "ib_interp", "ib_spread", "ib_plan_create", "ib_plan_destroy",
            "ib_plan_query", "ib_workspace_bytes", "ib_plan_profile", "ib_plan_profile_read",
            "ib_multidirect_force", "ib_plan_autotune",
            "ib_reductions_workspace", "ib_particle_reductions", "ib_particle_reductions_noalloc",
            "ib_backward_workspace_bytes", "ib_multidirect_backward",
            "ib_rigid_update", "ib_advect_markers", "ib_collision_workspace",
            "ib_collision_forces",
            "ib_levels_workspace", "ib_particle_levels", "ib_sequential_workspace_bytes",
            "ib_multidirect_sequential", "ib_fluid_workspace", "ib_fluid_predict",
            "ib_fluid_project", "ib_field_to_boxes", "ib_field_from_boxes", "ib_status_string", "ib_last_hip_error", "ib_version")


class IbxError(RuntimeError):
    def __init__(self, status, where):
        msg = _status_string(status).decode()
        if status == IB_EHIP:
            msg += ": " + _last_hip_error().decode()
        super().__init__(f"{where}: {msg} ({status})")
        self.status = status


def _check(rc, where):
    if rc < 0:
        raise IbxError(rc, where)
    return rc


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _prec_of(dtype):
    if dtype == torch.float64:
        return IB_F64
    if dtype == torch.float32:
        return IB_F32
    raise TypeError(f"unsupported field dtype {dtype}")


def _dev(device):
    return torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())


# ---------------------------------------------------------------- containers

@dataclasses.dataclass
class DeviceLevel:
    n: tuple
    h: float
    lo: tuple
    periodic: tuple
    box: int
    ngrow: int
    box_lo: torch.Tensor
    lut: torch.Tensor

    @property
    def nbox(self):
        return int(self.box_lo.shape[0])

    @property
    def ext(self):
        return self.box + 2 * self.ngrow

    @property
    def ntiles(self):
        return int(np.prod([v // 8 for v in self.n]))

    def field_shape(self):
        e = self.ext
        return (self.nbox, 3, e, e, e)

    @property
    def c(self):
        s = IbLevel()
        s.n[:] = list(self.n)
        s.h = self.h
        s.lo[:] = list(self.lo)
        s.periodic[:] = list(self.periodic)
        s.box, s.ngrow, s.nbox = self.box, self.ngrow, self.nbox
        s.box_lo = _ptr(self.box_lo) if self.nbox else None
        s.box_lut = _ptr(self.lut)
        return s


def device_level(level, device=None) -> DeviceLevel:
    """From a host level description (``workloads.Level`` or anything alike)."""
    dev = _dev(device)
    box_lo = torch.as_tensor(np.ascontiguousarray(level.box_lo, dtype=np.int32).reshape(-1, 3),
                             device=dev)
    lut = torch.as_tensor(np.ascontiguousarray(level.lut, dtype=np.int32), device=dev)
    return DeviceLevel(tuple(int(v) for v in level.n), float(level.h),
                       tuple(float(v) for v in level.lo), tuple(int(v) for v in level.periodic),
                       int(level.box), int(level.ngrow), box_lo, lut)


@dataclasses.dataclass
class Particles:
    xc: torch.Tensor   # (np, 3) float64
    d: torch.Tensor    # (np,)
    up: torch.Tensor   # (np, 3)
    om: torch.Tensor   # (np, 3)

    @property
    def np(self):
        return int(self.d.shape[0])

    @property
    def c(self):
        s = IbParticles()
        s.np = self.np
        s.xc, s.d, s.up, s.om = _ptr(self.xc), _ptr(self.d), _ptr(self.up), _ptr(self.om)
        return s


def particles(xc, d, up, om, device=None) -> Particles:
    dev = _dev(device)
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev) \
        if not isinstance(a, torch.Tensor) else a.to(dev, torch.float64).contiguous()
    return Particles(f(xc).reshape(-1, 3), f(d).reshape(-1), f(up).reshape(-1, 3),
                     f(om).reshape(-1, 3))


@dataclasses.dataclass
class Markers:
    offs: torch.Tensor  # (np+1,) int64
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    pid: torch.Tensor   # int32
    dv: torch.Tensor    # (np,)

    @property
    def nl(self):
        return int(self.x.shape[0])

    def xyz(self):
        return torch.stack([self.x, self.y, self.z], dim=1)

    @property
    def c(self):
        s = IbMarkers()
        s.nl = self.nl
        s.offs = _ptr(self.offs)
        s.x, s.y, s.z = _ptr(self.x), _ptr(self.y), _ptr(self.z)
        s.pid, s.dv = _ptr(self.pid), _ptr(self.dv)
        return s


def markers_from(x, y, z, pid, dv, offs, device=None) -> Markers:
    """Wrap existing marker arrays (host or device) as device tensors."""
    dev = _dev(device)
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(dt).contiguous()
    return Markers(t(offs, torch.int64), t(x, torch.float64), t(y, torch.float64),
                   t(z, torch.float64), t(pid, torch.int32), t(dv, torch.float64))


@dataclasses.dataclass
class Buckets:
    cell: torch.Tensor
    tileid: torch.Tensor
    base: torch.Tensor
    perm: torch.Tensor
    tile_offs: torch.Tensor
    src_offs: torch.Tensor
    src_idx: torch.Tensor
    flag: torch.Tensor

    @property
    def c(self):
        s = IbBuckets()
        s.cell, s.tileid, s.base, s.perm = (_ptr(self.cell), _ptr(self.tileid),
                                            _ptr(self.base), _ptr(self.perm))
        s.tile_offs, s.src_offs, s.src_idx = (_ptr(self.tile_offs), _ptr(self.src_offs),
                                              _ptr(self.src_idx))
        s.src_cap = int(self.src_idx.numel())
        s.flag = _ptr(self.flag)
        return s

    def nsrc(self):
        return int(self.src_offs[-1].item())


# ---------------------------------------------------------------- a1 / a3

def count_markers(d, h) -> np.ndarray:
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64))
    offs = np.zeros(d.shape[0] + 1, dtype=np.int64)
    _check(_count_markers(d.shape[0], d.ctypes.data, float(h), offs.ctypes.data),
           "ib_count_markers")
    return offs


def build_markers_into(level: DeviceLevel, parts: Particles, m: Markers) -> Markers:
    """Rebuild the markers of ``parts`` into existing arrays (counts unchanged)."""
    lc, pc, mc = level.c, parts.c, m.c
    _check(_build_markers(C.byref(lc), C.byref(pc), C.byref(mc), _stream()), "ib_build_markers")
    return m


def build_markers(level: DeviceLevel, parts: Particles) -> Markers:
    offs_h = count_markers(parts.d.cpu().numpy(), level.h)
    dev = parts.d.device
    nl = int(offs_h[-1])
    m = Markers(torch.as_tensor(offs_h, device=dev),
                torch.empty(nl, dtype=torch.float64, device=dev),
                torch.empty(nl, dtype=torch.float64, device=dev),
                torch.empty(nl, dtype=torch.float64, device=dev),
                torch.empty(nl, dtype=torch.int32, device=dev),
                torch.empty(parts.np, dtype=torch.float64, device=dev))
    lc, pc, mc = level.c, parts.c, m.c
    _check(_build_markers(C.byref(lc), C.byref(pc), C.byref(mc), _stream()), "ib_build_markers")
    return m


def desired_velocity(parts: Particles, m: Markers, dtype=torch.float64) -> torch.Tensor:
    Ud = torch.empty((m.nl, 3), dtype=dtype, device=m.x.device)
    pc, mc = parts.c, m.c
    _check(_desired_velocity(C.byref(pc), C.byref(mc), _prec_of(dtype), _ptr(Ud), _stream()),
           "ib_desired_velocity")
    return Ud


# ---------------------------------------------------------------- a2

def bucket_into(level: DeviceLevel, m: Markers, delta: int, b: Buckets) -> Buckets:
    """Re-bucket into existing arrays and workspace (no allocation)."""
    lc, mc, bc = level.c, m.c, b.c
    _check(_bucket(C.byref(lc), C.byref(mc), int(delta), C.byref(bc), _ptr(b._ws),
                   int(b._ws.numel()), _stream()), "ib_bucket")
    return b


def bucket(level: DeviceLevel, m: Markers, delta: int, src_cap=None) -> Buckets:
    dev = m.x.device
    nl = m.nl
    T = level.ntiles
    cap = 8 * nl if src_cap is None else int(src_cap)
    i32 = dict(dtype=torch.int32, device=dev)
    b = Buckets(torch.empty(nl, **i32), torch.empty(nl, **i32), torch.empty((nl, 3), **i32),
                torch.empty(nl, **i32), torch.empty(T + 1, **i32), torch.empty(T + 1, **i32),
                torch.empty(max(cap, 1), **i32), torch.zeros(2, **i32))
    if cap == 0:
        b.src_idx = b.src_idx[:0]
    lc, mc = level.c, m.c
    nbytes = _bucket_ws(C.byref(lc), nl)
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=dev)
    bc = b.c
    _check(_bucket(C.byref(lc), C.byref(mc), int(delta), C.byref(bc), _ptr(ws), int(nbytes),
                   _stream()), "ib_bucket")
    b._ws = ws  # keep alive until the stream has run
    return b


# ---------------------------------------------------------------- a4 / a6

def interp(level: DeviceLevel, m: Markers, delta: int, u: torch.Tensor) -> torch.Tensor:
    U = torch.empty((m.nl, 3), dtype=u.dtype, device=u.device)
    lc, mc = level.c, m.c
    _check(_interp(C.byref(lc), C.byref(mc), int(delta), _prec_of(u.dtype), _ptr(u), _ptr(U),
                   _stream()), "ib_interp")
    return U


def spread(level: DeviceLevel, m: Markers, b: Buckets, delta: int, F: torch.Tensor,
           out: torch.Tensor = None) -> torch.Tensor:
    f = out if out is not None else torch.zeros(level.field_shape(), dtype=F.dtype,
                                                device=F.device)
    lc, mc, bc = level.c, m.c, b.c
    _check(_spread(C.byref(lc), C.byref(mc), C.byref(bc), int(delta), _prec_of(F.dtype),
                   _ptr(F), _ptr(f), _stream()), "ib_spread")
    return f


# ---------------------------------------------------------------- a3-a9

class Plan:
    """Kernel width, precision and path of the multidirect loop."""

    def __init__(self, delta: int, dtype=torch.float32, path: int = IB_PATH_AUTO,
                 bucket_width: int = 0, spread_wgs_per_cu: int = 0, use_graph: bool = False,
                 row_masks: bool = False, interp_tile: int = 0):
        self.delta = int(delta)
        self.dtype = dtype
        h = _p()
        _check(_plan_create(C.byref(h), self.delta, _prec_of(dtype), int(path),
                            int(bucket_width), int(spread_wgs_per_cu), int(bool(use_graph)),
                            int(bool(row_masks)), int(interp_tile)), "ib_plan_create")
        self._h = h
        self._ws = None

    def query(self):
        out = np.zeros(6, dtype=np.int32)
        _check(_plan_query(self._h, out.ctypes.data), "ib_plan_query")
        return dict(path=int(out[0]), bucket_width=int(out[1]), spread_wgs_per_cu=int(out[2]),
                    use_graph=int(out[3]), row_masks=int(out[4]), interp_tile=int(out[5]))

    def profile(self, enable: bool = True):
        _check(_plan_profile(self._h, int(bool(enable))), "ib_plan_profile")

    def profile_read(self, reset: bool = True) -> dict:
        ms = np.zeros(len(PROF_CLASSES), dtype=np.float64)
        calls = np.zeros(len(PROF_CLASSES), dtype=np.int64)
        _check(_plan_profile_read(self._h, ms.ctypes.data, calls.ctypes.data, int(bool(reset))),
               "ib_plan_profile_read")
        return {k: (float(ms[i]), int(calls[i])) for i, k in enumerate(PROF_CLASSES)}

    def workspace_bytes(self, level: DeviceLevel, nl: int, ns: int) -> int:
        lc = level.c
        return int(_ws_bytes(self._h, C.byref(lc), int(nl), int(ns)))

    def workspace(self, level, nl, ns, device):
        nb = self.workspace_bytes(level, nl, ns)
        if self._ws is None or self._ws.numel() < nb or self._ws.device != device:
            self._ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=device)
        return self._ws

    def multidirect_force(self, level: DeviceLevel, parts: Particles, m: Markers, b: Buckets,
                          ns: int, dt: float, u0: torch.Tensor, ustar: torch.Tensor = None,
                          f: torch.Tensor = None, F: torch.Tensor = None, resid=None,
                          Fhist=None, want_f: bool = True):
        dev = u0.device
        if u0.dtype != self.dtype:
            raise TypeError("u0 dtype differs from the plan precision")
        if ustar is None:
            ustar = torch.empty_like(u0)
        if f is None and want_f:
            f = torch.empty_like(u0)
        if F is None:
            F = torch.empty((m.nl, 3), dtype=u0.dtype, device=dev)
        ws = self.workspace(level, m.nl, ns, dev)
        lc, pc, mc, bc = level.c, parts.c, m.c, b.c
        _check(_multidirect(self._h, C.byref(lc), C.byref(pc), C.byref(mc), C.byref(bc),
                            int(ns), float(dt), _ptr(u0), _ptr(ustar), _ptr(f), _ptr(F),
                            _ptr(resid), _ptr(Fhist), _ptr(ws), int(ws.numel()), _stream()),
               "ib_multidirect_force")
        return ustar, f, F

    def autotune(self, level: DeviceLevel, parts: Particles, m: Markers, b: Buckets, ns: int,
                 dt: float, u0: torch.Tensor, outputs=None) -> dict:
        """Pick the interpolation work tile, bucket width, spreading residency
        and the use of the slot row masks by timing the loop on these inputs
        (synchronizes the current stream).  Returns the choice and its loop
        time in ms.  ``outputs`` (ustar, f, F), if given, receive the loop's
        result at the chosen tuning (ustar must not be u0)."""
        dev = u0.device
        if u0.dtype != self.dtype:
            raise TypeError("u0 dtype differs from the plan precision")
        if outputs is None:
            ustar = torch.empty_like(u0)
            f = torch.empty_like(u0)
            F = torch.empty((m.nl, 3), dtype=u0.dtype, device=dev)
        else:
            ustar, f, F = outputs
            if ustar.data_ptr() == u0.data_ptr():
                raise ValueError("autotune cannot run in place")
            for t, shape in ((ustar, u0.shape), (f, u0.shape), (F, (m.nl, 3))):
                if tuple(t.shape) != tuple(shape) or t.dtype != u0.dtype or not t.is_contiguous():
                    raise ValueError("autotune outputs must match u0 and [nl][3] in shape and type")
        ws = self.workspace(level, m.nl, ns, dev)
        ms = C.c_double(0.0)
        lc, pc, mc, bc = level.c, parts.c, m.c, b.c
        _check(_autotune(self._h, C.byref(lc), C.byref(pc), C.byref(mc), C.byref(bc), int(ns),
                         float(dt), _ptr(u0), _ptr(ustar), _ptr(f), _ptr(F), _ptr(ws),
                         int(ws.numel()), _stream(), C.byref(ms)), "ib_plan_autotune")
        out = self.query()
        out["loop_ms"] = ms.value
        return out

    def multidirect_sequential(self, level: DeviceLevel, parts: Particles, m: Markers, ns: int,
                               dt: float, u0: torch.Tensor, levels=None, ustar=None, f=None,
                               F=None, flag=None, want_f: bool = True):
        """Algorithm 1 particle by particle, run as conflict levels one after
        another (batched plans only; synchronizes the current stream).
        ``levels`` = (level tensor, count) from :func:`particle_levels`, computed
        here when omitted."""
        dev = u0.device
        if u0.dtype != self.dtype:
            raise TypeError("u0 dtype differs from the plan precision")
        if levels is None:
            levels = particle_levels(level, parts, self.delta)
        lvl, nlev = levels
        if ustar is None:
            ustar = torch.empty_like(u0)
        if f is None and want_f:
            f = torch.empty_like(u0)
        if F is None:
            F = torch.empty((m.nl, 3), dtype=u0.dtype, device=dev)
        lc, pc, mc = level.c, parts.c, m.c
        nb = int(_seq_ws(self._h, C.byref(lc), parts.np, m.nl, int(ns)))
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        _check(_sequential(self._h, C.byref(lc), C.byref(pc), C.byref(mc), int(ns), float(dt),
                           _ptr(lvl), int(nlev), _ptr(u0), _ptr(ustar), _ptr(f), _ptr(F),
                           _ptr(flag), _ptr(ws), int(ws.numel()), _stream()),
               "ib_multidirect_sequential")
        return ustar, f, F

    def backward(self, level, parts, m, b, ns, dt, u0, Fhist, g_ustar=None, g_f=None,
                 g_F=None):
        dev = u0.device
        lc = level.c
        nb = int(_bwd_ws(self._h, C.byref(lc), m.nl))
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        g_u0 = torch.zeros_like(u0)
        g_up = torch.zeros((parts.np, 3), dtype=torch.float64, device=dev)
        g_om = torch.zeros((parts.np, 3), dtype=torch.float64, device=dev)
        g_X = torch.zeros((m.nl, 3), dtype=torch.float64, device=dev)
        pc, mc, bc = parts.c, m.c, b.c
        _check(_backward(self._h, C.byref(lc), C.byref(pc), C.byref(mc), C.byref(bc), int(ns),
                         float(dt), _ptr(u0), _ptr(Fhist), _ptr(g_ustar), _ptr(g_f), _ptr(g_F),
                         _ptr(g_u0), _ptr(g_up), _ptr(g_om), _ptr(g_X), _ptr(ws), nb,
                         _stream()), "ib_multidirect_backward")
        return g_u0, g_up, g_om, g_X

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                _plan_destroy(self._h)
                self._h = None
        except Exception:
            pass


# ---------------------------------------------------------------- a10

def particle_reductions(level: DeviceLevel, parts: Particles, m: Markers, F: torch.Tensor,
                        u: torch.Tensor, flag: torch.Tensor = None) -> torch.Tensor:
    out = torch.empty((parts.np, 12), dtype=torch.float64, device=u.device)
    ws = torch.empty(max(int(_red_ws(parts.np)), 1), dtype=torch.uint8, device=u.device)
    lc, pc, mc = level.c, parts.c, m.c
    _check(_reductions(C.byref(lc), C.byref(pc), C.byref(mc), _prec_of(u.dtype), _ptr(F), _ptr(u),
                       _ptr(out), _ptr(flag), _ptr(ws), int(ws.numel()), _stream()),
           "ib_particle_reductions")
    return out


REDUCTIONS_NOALLOC_MAX_NP = 32768


def particle_reductions_noalloc(level: DeviceLevel, parts: Particles, m: Markers,
                                F: torch.Tensor, u: torch.Tensor, out: torch.Tensor,
                                flag: torch.Tensor = None) -> torch.Tensor:
    """particle_reductions into a caller tensor out [np][12] (float64) with the
    library's fixed scratch: no device memory is allocated here or inside."""
    lc, pc, mc = level.c, parts.c, m.c
    _check(_reductions_noalloc(C.byref(lc), C.byref(pc), C.byref(mc), _prec_of(u.dtype),
                               _ptr(F), _ptr(u), _ptr(out), _ptr(flag), _stream()),
           "ib_particle_reductions_noalloc")
    return out


# ---------------------------------------------------------------- particle update

def rigid_update(parts: Particles, rho_p: torch.Tensor, sums_n: torch.Tensor,
                 sums_np1: torch.Tensor, rho_f: float, grav, dt: float, Fc=None, Tc=None,
                 prescribed=None):
    """Rigid-body update (Eqs. (particle1), (particle2), (pr2)); returns the new
    particle velocities, angular velocities and centroids."""
    dev = parts.xc.device
    up1 = torch.empty_like(parts.up)
    om1 = torch.empty_like(parts.om)
    xc1 = torch.empty_like(parts.xc)
    g3 = (C.c_double * 3)(*[float(v) for v in grav])
    pc = parts.c
    _check(_rigid(C.byref(pc), _ptr(rho_p), _ptr(sums_n), _ptr(sums_np1), _ptr(Fc), _ptr(Tc),
                  _ptr(prescribed), float(rho_f), C.cast(g3, C.c_void_p), float(dt), _ptr(up1),
                  _ptr(om1), _ptr(xc1), _stream()), "ib_rigid_update")
    return up1, om1, xc1


def advect_markers(m: Markers, xc_n, xc_np1, om_n, om_np1, dt: float, out: Markers = None):
    """Markers moved with their particle's rigid motion (Eq. (x)); in place when
    out is m."""
    if out is None:
        out = Markers(m.offs, torch.empty_like(m.x), torch.empty_like(m.y),
                      torch.empty_like(m.z), m.pid, m.dv)
    mc = m.c
    _check(_advect(C.byref(mc), _ptr(xc_n), _ptr(xc_np1), _ptr(om_n), _ptr(om_np1), float(dt),
                   _ptr(out.x), _ptr(out.y), _ptr(out.z), _stream()), "ib_advect_markers")
    return out


def collision_forces(level: DeviceLevel, parts: Particles, rho_p: torch.Tensor, g_norm: float,
                     eps_c: float = 1e-4) -> torch.Tensor:
    """Repulsive collision force of Eq. (DKT_model) on every particle, [np][3]."""
    Fc = torch.empty_like(parts.xc)
    lc, pc = level.c, parts.c
    ws = torch.empty(max(int(_coll_ws(C.byref(lc), parts.np)), 1), dtype=torch.uint8,
                     device=parts.xc.device)
    _check(_collide(C.byref(lc), C.byref(pc), _ptr(rho_p), float(g_norm), float(eps_c), _ptr(Fc),
                    _ptr(ws), int(ws.numel()), _stream()), "ib_collision_forces")
    return Fc


def particle_levels(level: DeviceLevel, parts: Particles, delta: int):
    """Conflict level of every particle for the particle-by-particle order of
    the loop: (int32 tensor [np], number of levels).  Synchronizes the current
    stream."""
    dev = parts.xc.device
    lvl = torch.empty(max(parts.np, 1), dtype=torch.int32, device=dev)[:parts.np]
    ws = torch.empty(max(int(_lv_ws(parts.np)), 1), dtype=torch.uint8, device=dev)
    n = C.c_int32(0)
    lc, pc = level.c, parts.c
    _check(_levels(C.byref(lc), C.byref(pc), int(delta), _ptr(lvl), C.byref(n), _ptr(ws),
                   int(ws.numel()), _stream()), "ib_particle_levels")
    return lvl, int(n.value)


# ---------------------------------------------------------------- fluid steps

class Fluid:
    """Single-level periodic fluid steps on an n^3 grid (Sec. 3.1, Steps 1 and
    3): velocity [3][n][n][n] cell-centred, pressure [n][n][n] on the nodes."""

    def __init__(self, n: int, h: float, dtype=torch.float64, device=None):
        self.n, self.h, self.dtype = int(n), float(h), dtype
        nb = int(_fl_ws(self.n, _prec_of(dtype)))
        if nb == 0:
            raise IbxError(IB_EUNSUPPORTED, "ib_fluid_workspace")
        self._ws = torch.empty(nb, dtype=torch.uint8, device=_dev(device))

    def predict(self, u, p, rho: float, mu: float, dt: float, grav, out=None):
        """Eq. (31): u~* from u^n and p^{n-1/2}."""
        out = torch.empty_like(u) if out is None else out
        g3 = (C.c_double * 3)(*[float(v) for v in grav])
        _check(_fl_predict(self.n, self.h, _prec_of(u.dtype), float(rho), float(mu), float(dt),
                           C.cast(g3, C.c_void_p), _ptr(u), _ptr(p), _ptr(out), _ptr(self._ws),
                           int(self._ws.numel()), _stream()), "ib_fluid_predict")
        return out

    def project(self, ustar, p_old, rho: float, dt: float, u_out=None, p_out=None):
        """Eqs. (ns_lp1)-(ns_lp3): (u^{n+1}, p^{n+1/2})."""
        u_out = torch.empty_like(ustar) if u_out is None else u_out
        p_out = torch.empty_like(p_old) if p_out is None else p_out
        _check(_fl_project(self.n, self.h, _prec_of(ustar.dtype), float(rho), float(dt),
                           _ptr(ustar), _ptr(p_old), _ptr(u_out), _ptr(p_out), _ptr(self._ws),
                           int(self._ws.numel()), _stream()), "ib_fluid_project")
        return u_out, p_out


def field_to_boxes(level: DeviceLevel, glob: torch.Tensor, boxed: torch.Tensor) -> torch.Tensor:
    lc = level.c
    _check(_to_boxes(C.byref(lc), _prec_of(glob.dtype), _ptr(glob), _ptr(boxed), _stream()),
           "ib_field_to_boxes")
    return boxed


def field_from_boxes(level: DeviceLevel, boxed: torch.Tensor, glob: torch.Tensor) -> torch.Tensor:
    lc = level.c
    _check(_from_boxes(C.byref(lc), _prec_of(boxed.dtype), _ptr(boxed), _ptr(glob), _stream()),
           "ib_field_from_boxes")
    return glob


def version() -> int:
    return int(_version())
