"""Benchmark of the multidirect-forcing IB step on one MI355X.

One step is the whole forward hot path on the 1000-sphere 256^3 workload:
marker build (a1), bucketing (a2), desired velocity and the N_s = 5
multidirect iterations with finalization (a3-a9), and the per-particle
reductions (a10), FP32 fields with FP64 positions and sums, inputs resident in
HBM, no host synchronization inside the step.  Prints one JSON line.

Beside the headline value it reports the loop alone (mean of back-to-back
runs and median of single runs), the plain FP64 path and the FP64 batched path
on the same inputs, the 20000-sphere 512^3 workload's loop, a per-kernel
breakdown from the library's event profiler, the roofline of the dominant
kernel and of the whole loop, the adjoint (a11) on the 64-sphere 128^3
workload, and the FP64 oracle timed on the host (all cores, and one core).

Byte model (compulsory traffic of Algorithm 1, every cell or marker counted
once per pass, s = field bytes, C = the support cells, N = markers):
    per iteration  B_it = 3 s |C| + N b_m,  b_m = 24 + 9 s
                   (positions, F read and written, U^d);
    loop           B_model = N_s B_it + 6 s |C|  (final u* and f on C).
roofline.frac is B_it times the iterations one launch of the dominant kernel
covers, over its average launch time, over the 8 TB/s HBM peak.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Kernel sources whose hash tags the committed HBM counter summary: the traffic
# figure is reported only while these are unchanged since the counters were taken.
TRAFFIC_SOURCES = ("paper_2408_14140_amd/csrc/tiles.h", "paper_2408_14140_amd/csrc/batched.hip")
TRAFFIC_FILE = "profiles/spread_spheres1000_256_hbm_counters.txt"
TRAFFIC_FILE_CFG4 = "profiles/loop_spheres20000_512_hbm_counters.txt"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def support_cells(level, b, delta):
    """Number of distinct cells in the union of all marker stencils."""
    import torch
    n = torch.tensor(level.n, device=b.base.device, dtype=torch.int64)
    base = b.base.to(torch.int64)
    o = torch.arange(delta, device=base.device)
    cx = (base[:, 0, None] + o[None, :]) % n[0]
    cy = (base[:, 1, None] + o[None, :]) % n[1]
    cz = (base[:, 2, None] + o[None, :]) % n[2]
    lin = (cx[:, None, None, :] + n[0] * (cy[:, None, :, None] + n[1] * cz[:, :, None, None]))
    return int(torch.unique(lin.reshape(-1)).numel())


def iteration_bytes(s, N, C):
    """B_it of the byte model: u0 read on the support, 24 + 9 s bytes per marker."""
    return 3 * s * C + N * (24 + 9 * s)


def loop_bytes(s, N, C, ns):
    """B_model of the byte model: N_s iterations and the final u*, f on C."""
    return ns * iteration_bytes(s, N, C) + 6 * s * C


# iterations of Algorithm 1 covered by one launch of each kernel class
ITERATIONS_PER_LAUNCH = {"spread": 1, "interp_g": 1, "interp_u0": 1, "spread_final": 1}


def impl_bytes(kind, s, P, N, S, A, C, ncov):
    """Bytes one launch of a batched-path kernel class touches in this
    implementation (not compulsory: it counts the tile slots and the source
    records each tile gathers).

    N markers, S source-list entries, A active tiles (512 cells each), C
    support cells, ncov cells of the covered boxes, s field bytes.  Marker
    records: packed stencil base 8 B, the three offsets from the stencil's
    first cell and dV/h^3 4s (the weights are formed from the offsets);
    U^d / D / F 3s each.  The loop runs in place (u* overwrites u0)."""
    rec = 8 + 4 * s
    if kind == "interp_u0":
        return 3 * s * C + N * (rec + 3 * s + 6 * s)
    if kind in ("spread", "spread_final"):
        return N * (rec + 3 * s) + 4 * S + 3 * s * 512 * A
    if kind == "interp_g":
        return 3 * s * 512 * A + N * (rec + 3 * s + 3 * s + 3 * s)
    if kind == "fill":
        # f on every covered cell; G read, u0 read and u* written on active tiles
        return 3 * s * ncov + 9 * s * 512 * A
    return None


def sources_sha():
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel, fname=TRAFFIC_FILE, plan=None):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a copy-kernel calibration), taken for
    each tuning variant (row masks, work tile): the line of the variant that
    `plan` (a plan's query) runs, else the first line of the kernel.  None if
    the summary is absent, holds no such line, or the kernel sources changed
    since it was taken."""
    path = os.path.join(ROOT, fname)
    if not os.path.exists(path):
        return None
    sha, val = None, None
    for ln in open(path):
        f = ln.split()
        if len(f) == 2 and f[0] == "sources_sha256_16:":
            sha = f[1]
        if len(f) >= 3 and f[0] == "traffic_bytes_per_launch:" and f[1] == kernel:
            tuning = dict(kv.split("=") for kv in f[3:])
            if plan is not None and any(int(plan.get(k, -1)) != int(v)
                                        for k, v in tuning.items()):
                continue
            if val is None:
                val = float(f[2])
    return val if sha == sources_sha() else None


def copy_probe(mib, reps):
    """Plain device-to-device copy of `mib` MiB, `reps` times; returns GB/s."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    return 2 * 4 * n * reps / (s.elapsed_time(e) * 1e-3) / 1e9


def host_cpu():
    """nproc and the CPU model of this host."""
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def timed(fn, k):
    """Mean over k back-to-back runs between one pair of events (current stream)."""
    import torch
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(k):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / k


def timed_median(fn, k):
    """Median over k single runs, each between its own pair of events."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(k)]
    torch.cuda.synchronize()
    for s0, e0 in ev:
        s0.record()
        fn()
        e0.record()
    torch.cuda.synchronize()
    return float(np.median([s0.elapsed_time(e0) for s0, e0 in ev]))


def big_workload_leg(args, dev, timed, timed_median):
    """The FP32 batched loop on spheres20000_512 (seed 0): autotuned, in place,
    median of single runs, per-kernel averages and the byte-model fractions."""
    import torch

    import paper_2408_14140_amd as ibx
    import workloads as W
    t0 = time.time()
    wl = W.config(4, 0)
    lev = wl.level
    log(f"workload {wl.name}: {wl.npart} spheres, {lev.nbox} boxes, gen {time.time()-t0:.1f}s")
    dl = ibx.device_level(lev, dev)
    parts = ibx.particles(wl.xc, wl.d, wl.up, wl.om, dev)
    m = ibx.build_markers(dl, parts)
    b = ibx.bucket(dl, m, wl.delta)
    torch.cuda.synchronize()
    assert int(b.flag[0].item()) == 0 and int(b.flag[1].item()) == 0
    N, P, ns, dt = m.nl, wl.delta, wl.ns, wl.dt
    C = support_cells(dl, b, P)
    u = torch.as_tensor(W.to_boxes(wl.u0, lev, fill=0.0, dtype=np.float32), device=dev)
    f = torch.zeros_like(u)
    F = torch.zeros((N, 3), dtype=torch.float32, device=dev)
    plan = ibx.Plan(P, torch.float32, ibx.IB_PATH_BATCHED, bucket_width=args.bucket_width,
                    spread_wgs_per_cu=args.spread_wgs, use_graph=True,
                    row_masks=bool(args.row_masks), interp_tile=args.interp_tile)
    if not args.no_autotune and not args.bucket_width and not args.spread_wgs:
        tuned = plan.autotune(dl, parts, m, b, ns, dt, u)
    else:
        tuned = {"bucket_width": args.bucket_width, "spread_wgs_per_cu": args.spread_wgs,
                 "row_masks": int(bool(args.row_masks)), "interp_tile": args.interp_tile or 8,
                 "fixed": True}

    def loop():
        plan.multidirect_force(dl, parts, m, b, ns, dt, u, ustar=u, f=f, F=F)

    for _ in range(args.warmup):
        loop()
    ms = timed_median(loop, args.steps)
    plan.profile(True)
    for _ in range(max(2, args.steps // 4)):
        loop()
    prof = plan.profile_read(reset=True)
    plan.profile(False)
    kern = {k: {"avg_us": 1e3 * v[0] / v[1], "calls": v[1]} for k, v in prof.items() if v[1]}
    dom = max(kern, key=lambda k: kern[k]["avg_us"] * kern[k]["calls"])
    bit = iteration_bytes(4, N, C)
    bl = loop_bytes(4, N, C, ns)
    res = {"markers": N, "support_cells": C, "loop_ms": ms, "plan": tuned,
           "marker_iters_per_s": N * ns / (ms * 1e-3),
           "loop_model_bytes": bl, "loop_frac": bl / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "dominant_kernel": dom, "kernels": kern,
           "dominant_frac": (ITERATIONS_PER_LAUNCH.get(dom, 0) * bit /
                             (kern[dom]["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS),
           "dominant_traffic": committed_traffic(dom, TRAFFIC_FILE_CFG4, tuned),
           "dominant_model_bytes": ITERATIONS_PER_LAUNCH.get(dom, 0) * bit}
    log(f"spheres20000_512: {N} markers, C {C}, loop {ms:.3f} ms, frac {res['loop_frac']:.3f}")
    # the collision force of Eq. (DKT_model) on the clumped spheres (bin search)
    rho_p = torch.full((wl.npart,), 2.0, dtype=torch.float64, device=dev)
    ibx.collision_forces(dl, parts, rho_p, 9.81, 1e-4)
    res["collision_forces_ms"] = timed_median(
        lambda: ibx.collision_forces(dl, parts, rho_p, 9.81, 1e-4), args.steps)
    log(f"spheres20000_512: collision forces {res['collision_forces_ms']:.3f} ms")
    del u, f, F, plan
    return res


def main():
    if "--gpus" in sys.argv:
        i = sys.argv.index("--gpus")
        if i + 1 < len(sys.argv) and sys.argv[i + 1] != "1":
            print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
                  "(the measured figure is one GPU's share of the workload)", file=sys.stderr)
            sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()          # default priority; graph capture needs a real stream
    with torch.cuda.stream(stream):
        run()


def run():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0,
                    help="workload seed of every figure except the per-seed step times")
    ap.add_argument("--seeds", type=int, default=5,
                    help="the step is also timed on the workloads of seeds 0..SEEDS-1; value "
                         "and ms_per_step are the medians over them")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--bucket-width", type=int, default=0)
    ap.add_argument("--spread-wgs", type=int, default=0)
    ap.add_argument("--row-masks", type=int, default=0,
                    help="G slot row masks on (1) or off (0) when the tuning is fixed")
    ap.add_argument("--interp-tile", type=int, default=0,
                    help="x extent of the interpolation work tiles (8 or 16) when the tuning "
                         "is fixed")
    ap.add_argument("--no-fluid", action="store_true",
                    help="skip the fluid steps and the whole time step")
    ap.add_argument("--no-cfg4", action="store_true",
                    help="skip the 20000-sphere 512^3 loop")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the particle-by-particle (level by level) loop")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the plan's default bucket width and spreading residency")
    ap.add_argument("--only-cfg4", action="store_true",
                    help="only the 20000-sphere 512^3 loop (its line holds that leg alone)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only time a plain MiB-sized device copy (counter calibration)")
    args = ap.parse_args()

    if args.copy_probe:
        gbs = copy_probe(args.copy_probe, 4)
        print(json.dumps({"copy_probe_mib": args.copy_probe, "copy_gbs": gbs}), flush=True)
        return

    import torch

    import paper_2408_14140_amd as ibx
    import workloads as W

    dev = torch.device("cuda", 0)
    if args.only_cfg4:
        print(json.dumps({"spheres20000_512": big_workload_leg(args, dev, timed, timed_median)}),
              flush=True)
        return
    t0 = time.time()
    wl = W.config(3, args.seed)
    log(f"workload {wl.name}: {wl.npart} spheres, {wl.level.nbox} boxes, gen {time.time()-t0:.1f}s")
    lev = wl.level
    P, ns, dt = wl.delta, wl.ns, wl.dt
    dl = ibx.device_level(lev, dev)
    parts = ibx.particles(wl.xc, wl.d, wl.up, wl.om, dev)
    m = ibx.build_markers(dl, parts)
    b = ibx.bucket(dl, m, P)
    torch.cuda.synchronize()
    N = m.nl
    assert int(b.flag[0].item()) == 0 and int(b.flag[1].item()) == 0
    S = b.nsrc()
    act = (b.src_offs[1:] > b.src_offs[:-1])
    A = int(act.sum().item())
    C = support_cells(dl, b, P)
    log(f"markers {N}, source entries {S}, active tiles {A}, support cells {C}")

    u_host = W.to_boxes(wl.u0, lev, fill=0.0)
    u32 = torch.as_tensor(u_host, device=dev).to(torch.float32)
    f32 = torch.zeros_like(u32)
    F32 = torch.zeros((N, 3), dtype=torch.float32, device=dev)
    plan = ibx.Plan(P, torch.float32, ibx.IB_PATH_BATCHED, bucket_width=args.bucket_width,
                    spread_wgs_per_cu=args.spread_wgs, use_graph=True,
                    row_masks=bool(args.row_masks), interp_tile=args.interp_tile)
    red = torch.zeros((wl.npart, 12), dtype=torch.float64, device=dev)
    tuned = None
    if not args.no_autotune and not args.bucket_width and not args.spread_wgs:
        tuned = plan.autotune(dl, parts, m, b, ns, dt, u32)
        log(f"autotune {tuned}")

    def step():
        ibx.build_markers_into(dl, parts, m)
        ibx.bucket_into(dl, m, P, b)
        plan.multidirect_force(dl, parts, m, b, ns, dt, u32, ustar=u32, f=f32, F=F32)
        red.copy_(ibx.particle_reductions(dl, parts, m, F32, u32))

    def loop_only():
        plan.multidirect_force(dl, parts, m, b, ns, dt, u32, ustar=u32, f=f32, F=F32)

    def captured(fn):
        """fn recorded once into a graph (every call in it only enqueues work);
        returns its replay."""
        gph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(gph):
            fn()
        torch.cuda.synchronize()
        keep.append(gph)
        return gph.replay

    keep = []
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warm")
    # the step as one graph replay: no host launch cost inside the timed region
    step_g = captured(step)
    for _ in range(args.warmup):
        step_g()
    ms_step = timed(step_g, args.steps)
    ms_step_eager = timed(step, args.steps)
    ms_loop = timed(loop_only, args.steps)
    ms_loop_med = timed_median(loop_only, args.steps)
    log(f"step {ms_step:.3f} ms (eager launches {ms_step_eager:.3f} ms), loop {ms_loop:.3f} ms "
        f"(median of single runs {ms_loop_med:.3f} ms)")

    # the step's other parts, each captured alone and timed over the same repetitions
    parts_ms = {
        "build_markers": timed(captured(lambda: ibx.build_markers_into(dl, parts, m)),
                               args.steps),
        "bucket": timed(captured(lambda: ibx.bucket_into(dl, m, P, b)), args.steps),
        "reductions": timed(captured(
            lambda: red.copy_(ibx.particle_reductions(dl, parts, m, F32, u32))), args.steps),
    }
    log(f"step parts {json.dumps(parts_ms)}")

    # the particle side of a time step: rigid-body update and marker advection
    rho_p = torch.full((wl.npart,), 2.0, dtype=torch.float64, device=dev)
    red1 = red.clone()
    up1, om1, xc1 = ibx.rigid_update(parts, rho_p, red, red1, 1.0, [0.0, 0.0, -9.81], dt)
    madv = ibx.advect_markers(m, parts.xc, xc1, parts.om, om1, dt)
    particle_ms = {
        "rigid_update": timed(captured(lambda: ibx.rigid_update(
            parts, rho_p, red, red1, 1.0, [0.0, 0.0, -9.81], dt)), args.steps),
        "advect_markers": timed(captured(lambda: ibx.advect_markers(
            m, parts.xc, xc1, parts.om, om1, dt, out=madv)), args.steps),
        "collision_forces": timed(captured(
            lambda: ibx.collision_forces(dl, parts, rho_p, 9.81, 1e-4)), args.steps),
    }
    log(f"particle step {json.dumps(particle_ms)}")

    # the fluid steps around the loop on the same 256^3 grid (FP32), and one
    # whole time step: Step 1, Step 2 (markers, bucketing, loop, sums), Step 3,
    # Step 4 (rigid update, marker advection)
    fluid_ms = None
    if not args.no_fluid:
        nf = lev.n[0]
        fl = ibx.Fluid(nf, lev.h, torch.float32, dev)
        ug = torch.as_tensor(wl.u0, device=dev).float()
        pg = torch.zeros((nf, nf, nf), dtype=torch.float32, device=dev)
        usg = torch.empty_like(ug)
        ung = torch.empty_like(ug)
        png = torch.empty_like(pg)
        grav = (0.0, 0.0, -9.81)

        def whole_step():
            fl.predict(ug, pg, 1.0, 1e-3, dt, grav, out=usg)
            ibx.field_to_boxes(dl, usg, u32)
            step()
            ibx.field_from_boxes(dl, u32, usg)
            fl.project(usg, pg, 1.0, dt, u_out=ung, p_out=png)
            ibx.rigid_update(parts, rho_p, red, red1, 1.0, grav, dt)
            ibx.advect_markers(m, parts.xc, xc1, parts.om, om1, dt, out=madv)

        fluid_ms = {
            "predict": timed(captured(lambda: fl.predict(ug, pg, 1.0, 1e-3, dt, grav, out=usg)),
                             args.steps),
            "project": timed(captured(lambda: fl.project(usg, pg, 1.0, dt, u_out=ung, p_out=png)),
                             args.steps),
            "time_step": timed(captured(whole_step), args.steps),
        }
        log(f"fluid {json.dumps(fluid_ms)}")
        del fl, ug, pg, usg, ung, png

    # per-kernel breakdown over the same number of loops, events on the launch stream
    plan.profile(True)
    for _ in range(args.steps):
        loop_only()
    prof = plan.profile_read(reset=True)
    plan.profile(False)
    ncov = lev.nbox * lev.box ** 3
    kern = {}
    for k, v in prof.items():
        if v[1] > 0:
            kern[k] = {"ms_total": v[0], "calls": v[1], "avg_us": 1e3 * v[0] / v[1]}
            ib = impl_bytes(k, 4, P, N, S, A, C, ncov)
            if ib:
                kern[k]["impl_bytes"] = ib
            if k in ITERATIONS_PER_LAUNCH:
                kern[k]["model_bytes"] = ITERATIONS_PER_LAUNCH[k] * iteration_bytes(4, N, C)
                kern[k]["model_gbs"] = kern[k]["model_bytes"] / (1e-3 * v[0] / v[1]) / 1e9
    dom = max(kern, key=lambda k: kern[k]["ms_total"])
    nb = kern[dom].get("model_bytes")
    avg_s = kern[dom]["avg_us"] * 1e-6
    achieved = nb / avg_s / 1e9 if nb else None
    bmodel = loop_bytes(4, N, C, ns)
    roofline = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": committed_traffic(dom, plan=plan.query()), "bytes_per_launch": nb,
                "iterations_per_launch": ITERATIONS_PER_LAUNCH.get(dom),
                "avg_launch_us": kern[dom]["avg_us"],
                "impl_bytes_per_launch": kern[dom].get("impl_bytes"),
                "loop": {"bytes": bmodel, "ms": ms_loop,
                         "achieved": bmodel / (ms_loop * 1e-3) / 1e9,
                         "frac": bmodel / (ms_loop * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    log(f"kernels {json.dumps(kern)}")

    # cold loop: a 512 MiB write between repetitions evicts the 256 MB MALL
    flush = torch.empty(128 << 20, dtype=torch.float32, device=dev)
    cold = []
    for _ in range(5):
        flush.fill_(1.0)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        loop_only()
        e.record()
        torch.cuda.synchronize()
        cold.append(s.elapsed_time(e))
    ms_cold = float(np.median(cold))
    del flush
    copy_gbs = copy_probe(1024, 10)
    log(f"cold loop {ms_cold:.3f} ms, copy {copy_gbs:.0f} GB/s")

    # the same captured step on the workloads drawn with the other seeds (same
    # plan tuning, same repetitions); value and ms_per_step are the medians
    def seed_step(sd):
        w2 = W.config(3, sd)
        l2 = w2.level
        dl2 = ibx.device_level(l2, dev)
        p2 = ibx.particles(w2.xc, w2.d, w2.up, w2.om, dev)
        m2 = ibx.build_markers(dl2, p2)
        b2 = ibx.bucket(dl2, m2, P)
        torch.cuda.synchronize()
        assert int(b2.flag[0].item()) == 0 and int(b2.flag[1].item()) == 0
        u2 = torch.as_tensor(W.to_boxes(w2.u0, l2, fill=0.0), device=dev).to(torch.float32)
        f2 = torch.zeros_like(u2)
        F2 = torch.zeros((m2.nl, 3), dtype=torch.float32, device=dev)
        red2 = torch.zeros((w2.npart, 12), dtype=torch.float64, device=dev)
        q = plan.query()
        pl2 = ibx.Plan(P, torch.float32, ibx.IB_PATH_BATCHED, bucket_width=q["bucket_width"],
                       spread_wgs_per_cu=q["spread_wgs_per_cu"], use_graph=True,
                       row_masks=bool(q["row_masks"]), interp_tile=q["interp_tile"])

        def step2():
            ibx.build_markers_into(dl2, p2, m2)
            ibx.bucket_into(dl2, m2, P, b2)
            pl2.multidirect_force(dl2, p2, m2, b2, ns, dt, u2, ustar=u2, f=f2, F=F2)
            red2.copy_(ibx.particle_reductions(dl2, p2, m2, F2, u2))

        for _ in range(args.warmup):
            step2()
        g2 = captured(step2)
        for _ in range(args.warmup):
            g2()
        ms = timed(g2, args.steps)
        keep.pop()
        return ms, m2.nl

    by_seed = {args.seed: {"ms_per_step": ms_step, "markers": N,
                           "value": N * ns / (ms_step * 1e-3)}}
    for sd in range(args.seeds):
        if sd not in by_seed:
            ms_sd, n_sd = seed_step(sd)
            by_seed[sd] = {"ms_per_step": ms_sd, "markers": n_sd,
                           "value": n_sd * ns / (ms_sd * 1e-3)}
            log(f"seed {sd}: step {ms_sd:.3f} ms, {n_sd} markers")
    torch.cuda.empty_cache()
    value_med = float(np.median([v["value"] for v in by_seed.values()]))
    ms_step_med = float(np.median([v["ms_per_step"] for v in by_seed.values()]))

    out = {
        "metric": "marker-iters/s of the multidirect IB step (FP32 batched)",
        "value": value_med,
        "unit": "marker-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step_med,
        "ms_per_step_eager_launches": ms_step_eager,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "spheres1000_256: 1000 polydisperse spheres (D/h lognormal, "
                               "median 16, sigma 0.3, clipped [8,32]) in a periodic 256^3 grid "
                               "of 32^3 boxes, 4-point delta, N_s=5, dt=h/2",
                   "markers": N, "ns": ns, "seed": args.seed,
                   "seeds": sorted(by_seed),
                   "steps_cover": "a1 markers, a2 bucket, a3-a9 loop, a10 reductions",
                   "figures": "value and ms_per_step: medians over the seeds; every other "
                              "figure on the workload of `seed`"},
        "by_seed": {str(k): by_seed[k] for k in sorted(by_seed)},
        "loop_ms": ms_loop,
        "loop_ms_median": ms_loop_med,
        "step_parts_ms": parts_ms,
        "particle_step_ms": particle_ms,
        "fluid_256_fp32_ms": fluid_ms,
        "loop_marker_iters_per_s": N * ns / (ms_loop * 1e-3),
        "loop_model_gbs": bmodel / (ms_loop * 1e-3) / 1e9,
        "loop_model_bytes": bmodel,
        "loop_ms_cold": ms_cold,
        "copy_gbs": copy_gbs,
        "loop_model_frac_of_copy": bmodel / (ms_loop * 1e-3) / 1e9 / copy_gbs,
        "roofline": roofline,
        "plan": plan.query() | ({"autotune_loop_ms": tuned["loop_ms"]} if tuned else {}),
        "kernels": kern,
    }

    if not args.no_plain:
        u64 = torch.as_tensor(u_host, device=dev)
        us64 = torch.zeros_like(u64)
        f64 = torch.zeros_like(u64)
        F64 = torch.zeros((N, 3), dtype=torch.float64, device=dev)
        plan64 = ibx.Plan(P, torch.float64, ibx.IB_PATH_PLAIN)

        def plain64():
            plan64.multidirect_force(dl, parts, m, b, ns, dt, u64, ustar=us64, f=f64, F=F64)

        plain64()
        ms64 = timed(plain64, max(2, args.steps // 5))
        out["fp64_plain_loop_ms"] = ms64
        out["speedup_fp32_batched_vs_fp64_plain"] = ms64 / ms_loop
        log(f"fp64 plain loop {ms64:.3f} ms")
        # the batched path in FP64 on the same inputs (in place, autotuned)
        pb64 = ibx.Plan(P, torch.float64, ibx.IB_PATH_BATCHED, use_graph=True)
        tb64 = pb64.autotune(dl, parts, m, b, ns, dt, u64)

        def batched64():
            pb64.multidirect_force(dl, parts, m, b, ns, dt, u64, ustar=u64, f=f64, F=F64)

        for _ in range(args.warmup):
            batched64()
        msb64 = timed(batched64, args.steps)
        out["fp64_batched"] = {"loop_ms": msb64, "plan": tb64,
                               "loop_frac": loop_bytes(8, N, C, ns) / (msb64 * 1e-3) / 1e9
                               / HBM_PEAK_GBS}
        out["speedup_fp32_batched_vs_fp64_batched"] = msb64 / ms_loop
        log(f"fp64 batched loop {msb64:.3f} ms")
        del u64, us64, f64, F64, pb64

    if not args.no_cfg4:
        # 20000 clustered spheres, 512^3, 3-point kernel: working set beyond the MALL
        out["spheres20000_512"] = big_workload_leg(args, dev, timed, timed_median)
        torch.cuda.empty_cache()

    if not args.no_sequential:
        # the particle-by-particle order: conflict levels, then one loop per level
        q = plan.query()
        pseq = ibx.Plan(P, torch.float32, ibx.IB_PATH_BATCHED, bucket_width=q["bucket_width"],
                        spread_wgs_per_cu=q["spread_wgs_per_cu"], row_masks=bool(q["row_masks"]),
                        interp_tile=q["interp_tile"])
        useq = torch.empty_like(u32)
        fseq = torch.empty_like(u32)
        Fseq = torch.empty_like(F32)
        levels = ibx.particle_levels(dl, parts, P)
        ms_lv = timed(lambda: ibx.particle_levels(dl, parts, P), max(2, args.steps // 5))

        def seq():
            pseq.multidirect_sequential(dl, parts, m, ns, dt, u32, levels=levels, ustar=useq,
                                        f=fseq, F=Fseq)

        seq()
        ms_seq = timed(seq, max(2, args.steps // 5))
        out["sequential"] = {"levels": levels[1], "levels_ms": ms_lv, "loop_ms": ms_seq,
                             "vs_jacobi_loop": ms_seq / ms_loop}
        log(f"sequential: {levels[1]} levels in {ms_lv:.3f} ms, loop {ms_seq:.3f} ms")
        del useq, fseq, Fseq

    if not args.no_backward:
        wl5 = W.config(5, args.seed)
        dl5 = ibx.device_level(wl5.level, dev)
        p5 = ibx.particles(wl5.xc, wl5.d, wl5.up, wl5.om, dev)
        m5 = ibx.build_markers(dl5, p5)
        b5 = ibx.bucket(dl5, m5, wl5.delta)
        u5 = torch.as_tensor(W.to_boxes(wl5.u0, wl5.level, fill=0.0), device=dev).float()
        pl5 = ibx.Plan(wl5.delta, torch.float32, ibx.IB_PATH_BATCHED)
        Fh = torch.zeros((wl5.ns, m5.nl, 3), dtype=torch.float32, device=dev)
        _, f5, F5 = pl5.multidirect_force(dl5, p5, m5, b5, wl5.ns, wl5.dt, u5, Fhist=Fh)
        gF = torch.ones_like(F5)

        def bwd():
            pl5.backward(dl5, p5, m5, b5, wl5.ns, wl5.dt, u5, Fh, g_f=f5, g_F=gF)

        def fwd5():
            pl5.multidirect_force(dl5, p5, m5, b5, wl5.ns, wl5.dt, u5, Fhist=Fh)

        bwd()
        fwd5()
        ms_b = timed(bwd, max(3, args.steps // 4))
        ms_f = timed(fwd5, max(3, args.steps // 4))
        out["backward_spheres64_128_fp32_ms"] = ms_b
        out["backward_spheres64_128"] = {"backward_ms": ms_b, "forward_loop_ms": ms_f,
                                         "backward_over_forward": ms_b / ms_f,
                                         "markers": m5.nl, "ns": wl5.ns}
        log(f"backward {ms_b:.3f} ms, forward loop with history {ms_f:.3f} ms")

    if not args.no_cpu_baseline:
        import oracle as O
        mo = O.build_markers(wl.xc, wl.d, lev.h)
        go = O.grid_of(lev)
        host = host_cpu()

        def oracle_rate(threads, budget):
            reps, el = 0, 0.0
            while el < budget:
                t = time.perf_counter()
                O.multidirect(go, P, ns, dt, mo, wl.xc, wl.up, wl.om, wl.u0, residuals=False,
                              threads=threads)
                el += time.perf_counter() - t
                reps += 1
            return reps, el

        nt = O.threads_available()
        reps, el = oracle_rate(nt, 10.0)
        out["cpu_baseline"] = {"value": reps * mo.nl * ns / el, "unit": "marker-iters/s",
                               "cores": nt, "kind": "oracle",
                               "sample": f"{reps} runs of the full workload's loop (a3-a9, "
                                         f"{mo.nl} markers, N_s={ns}) in the FP64 C oracle "
                                         f"built with OpenMP (same source and bits as the "
                                         f"single-threaded build), {nt} threads, {el:.1f} s",
                               "host": host}
        log(f"oracle loop x{reps} on {nt} threads {el:.1f} s")
        reps1, el1 = oracle_rate(0, 10.0)
        out["cpu_baseline_1core"] = {"value": reps1 * mo.nl * ns / el1, "unit": "marker-iters/s",
                                     "cores": 1, "kind": "oracle",
                                     "sample": f"{reps1} runs of the same loop, single-threaded "
                                               f"build, {el1:.1f} s", "host": host}
        log(f"oracle loop x{reps1} on 1 thread {el1:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
