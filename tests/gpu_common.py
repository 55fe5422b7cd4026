"""Shared set-up of the GPU parity tests: the same seeded inputs go to the
FP64 oracle (host) and to the library (device); nothing flows back from the
device into the oracle."""
import functools

import numpy as np
import pytest

import workloads as W


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def resid_bounds(g, P, m, xc, up, om, u0, ref_resid, tol, threads=0):
    """Allowed |r_m(path) - r_m(oracle)| for the residuals of Algorithm 1.

    r_m is the dV-norm of e_m = U^d - J u0 - dt J G^m (G^m = S F^m), a sum of
    three marker vectors.  A path that forms each of them to relative accuracy
    tol gets r_m within tol (|U^d| + |J u0| + dt |J G^m|) by the triangle
    inequality, and dt J G^m = J u^(m) - J u0 with |J u^(m)| <= |U^d| + r_m, so
    the bound is tol (2 |U^d| + 2 |J u0| + r_m), all norms in dV.  The norms
    come from the oracle on the same inputs."""
    import oracle as O
    dv = m.dv[m.pid][:, None]
    Ud = O.desired_velocity(m, xc, up, om)
    Ju0 = O.interp(g, P, m, u0, threads=threads)
    a = float(np.sqrt((dv * Ud * Ud).sum()))
    b0 = float(np.sqrt((dv * Ju0 * Ju0).sum()))
    return tol * (2 * a + 2 * b0 + np.asarray(ref_resid))


@functools.lru_cache(maxsize=None)
def small_workload(n=32, box=16, delta=4, ns=3, seed=1, cover_all=True, k=3):
    rng = np.random.default_rng(100 + seed)
    diam = rng.uniform(5.0, 10.0, k)
    return W.make_workload(f"small{n}_{delta}_{seed}", n, box, 2, delta, ns, diam, seed=seed,
                           nmodes=8, K=4, cover_all=cover_all)


@functools.lru_cache(maxsize=None)
def config_workload(k, seed=0):
    return W.config(k, seed)


@functools.lru_cache(maxsize=None)
def oracle_markers(wl_key):
    import oracle as O
    wl = wl_key()
    return O.build_markers(wl.xc, wl.d, wl.level.h)


class Case:
    """A workload on host (oracle) and device (library)."""

    def __init__(self, wl, dev):
        import oracle as O
        import torch

        import paper_2408_14140_amd as ibx
        self.wl = wl
        self.lev = wl.level
        self.g = O.grid_of(self.lev)
        self.m = O.build_markers(wl.xc, wl.d, self.lev.h)
        self.dev = dev
        self.dl = ibx.device_level(self.lev, dev)
        self.parts = ibx.particles(wl.xc, wl.d, wl.up, wl.om, dev)
        self.dm = ibx.markers_from(self.m.x, self.m.y, self.m.z, self.m.pid, self.m.dv,
                                   self.m.offs, dev)
        self.mask = self.lev.covered_mask()

    def u0_boxes(self, dtype):
        import torch
        return torch.as_tensor(W.to_boxes(self.wl.u0, self.lev, fill=np.nan), device=self.dev).to(dtype)

    def to_global(self, t):
        return W.from_boxes(t.double().cpu().numpy(), self.lev)

    def field_rel(self, t, ref):
        got = self.to_global(t)
        m = np.broadcast_to(self.mask, got.shape)
        return rel(got[m], ref[m])


def gpu_device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)
