"""A whole time-step's IB work (markers, bucketing, the batched loop, the
per-particle sums) recorded into one graph by the caller and replayed: every
replay, with eager work and synchronizations in between, equals the eager
step bit for bit."""
import pytest

from gpu_common import Case, announce, gpu_device, small_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


@pytest.mark.parametrize("use_graph", [True, False])
def test_captured_step_replays_match_eager(dev, use_graph):
    import torch

    import paper_2408_14140_amd as ibx
    announce(f"captured step use_graph={use_graph}")
    wl = small_workload(32, 16, 4, 3, 5)
    c = Case(wl, dev)
    plan = ibx.Plan(wl.delta, torch.float32, ibx.IB_PATH_BATCHED, use_graph=use_graph)
    m = ibx.build_markers(c.dl, c.parts)
    b = ibx.bucket(c.dl, m, wl.delta)
    u0 = c.u0_boxes(torch.float32)
    u = u0.clone()
    f = torch.zeros_like(u0)
    F = torch.zeros((m.nl, 3), dtype=torch.float32, device=dev)
    red = torch.zeros((wl.npart, 12), dtype=torch.float64, device=dev)

    def step():
        ibx.build_markers_into(c.dl, c.parts, m)
        ibx.bucket_into(c.dl, m, wl.delta, b)
        u.copy_(u0)
        plan.multidirect_force(c.dl, c.parts, m, b, wl.ns, wl.dt, u, ustar=u, f=f, F=F)
        red.copy_(ibx.particle_reductions(c.dl, c.parts, m, F, u))

    def state():
        return [t.clone() for t in (m.x, m.y, m.z, b.perm, b.src_idx, u, f, F, red)]

    def same(a, e):                             # NaN ghost cells compare equal
        if not a.dtype.is_floating_point:
            return torch.equal(a, e)
        return torch.equal(a.isnan(), e.isnan()) and torch.equal(a.nan_to_num(0.0),
                                                                 e.nan_to_num(0.0))

    valid = ~u0.isnan()                         # the ghost cells of u0 hold NaN

    step()
    torch.cuda.synchronize()
    ref = state()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for r in range(3):
        # scramble every output (ghost cells of f are never written)
        f.masked_fill_(valid, float("nan"))
        for t in (u, F, red):
            t.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for k, (a, e) in enumerate(zip(state(), ref)):
            assert same(a, e), (r, k)
        step()                                  # eager work between the replays
        torch.cuda.synchronize()
        for k, (a, e) in enumerate(zip(state(), ref)):
            assert same(a, e), (r, k)


def test_plan_graph_keys_on_every_level_field(dev):
    """A use_graph plan called with levels that differ only in lo[1] or lo[2]
    (same buffers, same stream) must not replay the graph captured for
    another level: each call equals an eager plan's bit for bit."""
    import dataclasses

    import torch

    import paper_2408_14140_amd as ibx
    announce("graph key: levels differing only in lo")
    wl = small_workload(32, 16, 4, 3, 5)
    c = Case(wl, dev)
    h = c.lev.h
    levels = [c.dl,
              dataclasses.replace(c.dl, lo=(c.dl.lo[0], c.dl.lo[1], c.dl.lo[2] + 0.37 * h)),
              dataclasses.replace(c.dl, lo=(c.dl.lo[0], c.dl.lo[1] - 0.21 * h, c.dl.lo[2]))]
    m = ibx.build_markers(c.dl, c.parts)
    b = ibx.bucket(c.dl, m, wl.delta)
    u0 = c.u0_boxes(torch.float32)
    u, f = torch.empty_like(u0), torch.zeros_like(u0)
    F = torch.zeros((m.nl, 3), dtype=torch.float32, device=dev)
    graphed = ibx.Plan(wl.delta, torch.float32, ibx.IB_PATH_BATCHED, use_graph=True)
    eager = ibx.Plan(wl.delta, torch.float32, ibx.IB_PATH_BATCHED, use_graph=False)
    stream = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(stream):
        for rep in range(2):
            for k, lv in enumerate(levels):
                ibx.bucket_into(lv, m, wl.delta, b)
                res = []
                for plan in (graphed, eager):
                    u.copy_(u0)
                    f.zero_()
                    plan.multidirect_force(lv, c.parts, m, b, wl.ns, wl.dt, u, ustar=u, f=f, F=F)
                    stream.synchronize()
                    res.append((u.nan_to_num(0.0).clone(), f.clone(), F.clone()))
                for a, e in zip(*res):
                    assert torch.equal(a, e), (rep, k)
                outs.append(res[1][2])
    # the levels really differ
    assert not torch.equal(outs[0], outs[1]) and not torch.equal(outs[0], outs[2])
