"""ib_particle_reductions_noalloc against ib_particle_reductions: the same
kernels with the partial sums in the library's fixed device array instead of a
workspace, so the results must agree bit for bit -- on two calls in a row, the
second with fewer particles (the array keeps the first call's contents), and
a call with more particles than the array holds is refused on the host."""
import numpy as np
import pytest

import workloads as W
from gpu_common import Case, announce, gpu_device, small_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def _inputs(wl, dev, dtype):
    import torch

    import paper_2408_14140_amd as ibx
    c = Case(wl, dev)
    m = ibx.build_markers(c.dl, c.parts)
    rng = np.random.default_rng(wl.npart)
    F = torch.as_tensor(rng.normal(size=(m.nl, 3)), device=dev).to(dtype)
    u = torch.as_tensor(W.to_boxes(wl.u0, wl.level, fill=0.0), device=dev).to(dtype)
    return c, m, F, u


def test_noalloc_reductions_match_workspace_call(dev):
    import torch

    import paper_2408_14140_amd as ibx
    cases = [(W.config(3, 0), torch.float32), (small_workload(32, 16, 4, 3, 1), torch.float64)]
    assert cases[1][0].npart < cases[0][0].npart
    for wl, dtype in cases:
        announce(f"noalloc reductions {wl.name} ({wl.npart} particles) {dtype}")
        c, m, F, u = _inputs(wl, dev, dtype)
        ref = ibx.particle_reductions(c.dl, c.parts, m, F, u)
        out = torch.full((wl.npart, 12), float("nan"), dtype=torch.float64, device=dev)
        ibx.particle_reductions_noalloc(c.dl, c.parts, m, F, u, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_noalloc_reductions_refuse_too_many_particles(dev):
    import torch

    import paper_2408_14140_amd as ibx
    announce("noalloc reductions: too many particles")
    wl = small_workload(32, 16, 4, 3, 1)
    c, m, F, u = _inputs(wl, dev, torch.float64)
    n = ibx.REDUCTIONS_NOALLOC_MAX_NP + 1
    z3 = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    big = ibx.Particles(z3, torch.ones(n, dtype=torch.float64, device=dev), z3, z3)
    out = torch.zeros((n, 12), dtype=torch.float64, device=dev)
    with pytest.raises(ibx.IbxError) as e:
        ibx.particle_reductions_noalloc(c.dl, big, m, F, u, out)
    assert e.value.status == ibx.IB_EUNSUPPORTED
    torch.cuda.synchronize()
    assert bool((out == 0).all())
