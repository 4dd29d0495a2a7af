#!/usr/bin/env python3
"""Benchmark of the narrow-band first-order upwind level-set update on one MI355X.

Default workload (spheres512): the 512^3 FP32 union of three spheres
(seeded), speed F = 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z), band half-width
6 dx in 8^3 tiles, rebuilt every 10 steps, 200 steps.  One bench "step" is one
window of the narrow-band algorithm (Sec. 1.1, Steps 1-2): a band rebuild (a
full scan of phi for the first window, the exact incremental rescan of the
previous band afterwards; dilation; ordered compaction) and 10 upwind steps
(Eq. 3-5) on the band, so the default 20 steps are the whole 200-step run, one
driver call.  Inputs are resident in HBM before the timed region starts; the
run restarts from the initial field after the warm-up windows.

Other workloads (--workload): spheres512_cutoff, the default run with the
cut-off of Eq. 8 in every step (speed c(phi) F, beta = 3 dx, gamma = 6 dx,
the band's); spheres512_reinit, the whole narrow-band algorithm (Steps 1-3):
the cut-off run with every window ended by 24 reinitialisation steps
(Eq. 12-13, dtau = dx/2) and the clamp of Eq. 10 (its GLUPS count time steps
only; the roofline is the reinitialisation kernel's); torus1024_f16s, the
1024^3 torus with phi stored as scaled FP16 (500 steps); batch256, 256 uneven
grids (32^3..192^3, random ellipsoids, tile shapes from the autotuner, 100
steps) captured in one HIP graph and timed on replay.

Prints one JSON line: whole-job band GLUPS (band point-updates per second
including rebuilds), the roofline of the dominant kernel (the band step,
timed per launch with HIP events on its stream) and, for the default and the
cut-off workloads, the oracle timed on the host cores on a bounded sample of
the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
BYTES_PER_POINT = {"f32": 12, "f64": 24, "f16s": 8}  # phi read, F read, phi write
REINIT_BYTES_PER_POINT = {"f32": 8, "f64": 16, "f16s": 4}  # phi read, phi write (no F)
REINIT_ITERS = 24  # reinitialisation steps per window of the spheres512_reinit workload


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed windows of 10 upwind steps (default: the whole run of the "
                         "workload: 20 for spheres512, 50 for torus1024_f16s, 10 for batch256)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed warm-up windows")
    ap.add_argument("--workload", default="spheres512",
                    choices=["spheres512", "spheres512_cutoff", "spheres512_reinit",
                             "torus1024_f16s", "torus1024_f32", "batch256", "closure128"],
                    help="spheres512: the 512^3 FP32 three-sphere run (default); "
                         "spheres512_cutoff: the same with the cut-off of Eq. 8; "
                         "spheres512_reinit: the same with Steps 1-3 (cut-off, "
                         "reinitialisation, clamp); "
                         "torus1024_f16s: the 1024^3 scaled-FP16 torus run; "
                         "torus1024_f32: the same torus and speed in FP32 (a band that "
                         "streams from HBM); "
                         "batch256: 256 uneven grids, autotuned tile shapes, one HIP graph; "
                         "closure128: the learned closure on a 128^3 coarse grid against the "
                         "plain 512^3 run (trains its network first)")
    ap.add_argument("--n", type=int, default=None, help="grid points per axis (single grids)")
    ap.add_argument("--steps-per-launch", type=int, default=0, choices=[0, 1, 2],
                    help="band step launches: 0 auto (two steps per launch on bricks in FP32, "
                         "one in FP16s and on the x-fastest layout), 1 or 2 forced (results "
                         "are the same bits)")
    ap.add_argument("--layout", default="bricks", choices=["bricks", "dense"],
                    help="single grids: bricks (default) converts phi and F to the tile-major "
                         "layout, runs the driver there and converts phi back, all inside the "
                         "timed region; dense runs the driver on the x-fastest fields")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU work budget of the oracle baseline (0 disables it)")
    ap.add_argument("--snapshot-copy-blocks", type=int, default=0,
                    help="workgroups of each snapshot's counted copy (0: the library's default)")
    ap.add_argument("--snapshot-every", type=int, default=0,
                    help="spheres512 only: time the windows as separate driver calls with an "
                         "asynchronous band snapshot (gather + copy to pinned host memory on a "
                         "side stream) after every K-th window, against the same calls without")
    ap.add_argument("--closure-seeds", type=int, default=16,
                    help="closure128: training seeds (100, 101, ...)")
    ap.add_argument("--closure-iters", type=int, default=8000,
                    help="closure128: Adam iterations of the training before the timed runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, run the plain 1 GiB dword copy kernel "
                         "(the reference for calibrating the traffic counters)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"spheres512": 20, "spheres512_cutoff": 20, "spheres512_reinit": 20,
                      "torus1024_f16s": 50, "torus1024_f32": 20, "batch256": 10,
                      "closure128": 40}[args.workload]
    return args


# the sources each kind of step kernel is compiled from (its counter
# summary in profiles/traffic.json is stamped with their digest)
BRICK_KERNEL_SOURCES = ("ls_internal.h", "ls_stencil.h", "ls_brick.hip")
DENSE_KERNEL_SOURCES = ("ls_internal.h", "ls_stencil.h", "ls_step.hip")
BATCH_KERNEL_SOURCES = ("ls_internal.h", "ls_stencil.h", "ls_step.hip", "ls_batch.hip")
STEP_KERNEL_SOURCES = BRICK_KERNEL_SOURCES
GATHER_KERNEL_SOURCES = ("ls_internal.h", "ls_snapshot.hip")


def kernel_source_digest(sources=None):
    """Digest of the sources a kernel is compiled from (default: the tile-major
    band step)."""
    here = os.path.dirname(os.path.abspath(__file__))
    csrc = os.path.join(here, "paper_1612_04040_amd", "csrc")
    h = hashlib.sha256()
    for f in (STEP_KERNEL_SOURCES if sources is None else sources):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, digest):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh).get(f"{kernel}/{workload}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_digest") != digest:
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    """The host CPU's model name (as lscpu reports it), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_windows(wl, budget_s, beta, max_windows):
    """Whole windows of the oracle (band rebuild + steps) until the budget is
    spent: (band point-updates, windows, seconds)."""
    import oracle

    phi = wl.phi.astype(np.float64)
    g32 = np.float32(wl.gamma)
    updates, windows = 0, 0
    t0 = time.perf_counter()
    while True:
        tiles = oracle.band_tiles(phi.astype(np.float32), wl.tile, g32, dilate=True)
        if beta is None:
            phi = oracle.upwind_steps(phi, wl.F, wl.dx, wl.dt, tiles, wl.window, wl.tile)
        else:
            phi = oracle.cutoff_steps(phi, wl.F, wl.dx, wl.dt, tiles, wl.window, beta,
                                      float(g32), wl.tile)
        updates += int(tiles.size) * int(np.prod(wl.tile)) * wl.window
        windows += 1
        if (time.perf_counter() - t0 >= budget_s or windows * wl.window >= wl.nsteps
                or windows >= max_windows):
            break
    return updates, windows, time.perf_counter() - t0


def cpu_baseline(wl, budget_s, beta=None):
    """The oracle (FP64, OpenMP) on whole windows of the same workload (with
    the cut-off steps when beta is given), on every host thread, then on one
    thread over its first window."""
    import oracle

    if budget_s <= 0:
        return None
    threads = oracle.max_threads()
    updates, windows, elapsed = _oracle_windows(wl, budget_s, beta, 1 << 30)
    oracle.set_threads(1)
    try:
        u1, w1, e1 = _oracle_windows(wl, budget_s, beta, 1)
    finally:
        oracle.set_threads(threads)
    what = (f"band rebuild + FP64 {'cut-off ' if beta is not None else ''}upwind steps) of the "
            f"{wl.name}{_suffix(beta, None)} workload")
    return {
        "value": updates / elapsed / 1e9,
        "unit": "GLUPS",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {windows} window(s) x {wl.window} steps ({what}, {elapsed:.1f} s",
        "cpu_model": cpu_model(),
        "single_thread": {"value": u1 / e1 / 1e9, "unit": "GLUPS", "cores": 1,
                          "sample": f"first {w1} window(s) x {wl.window} steps ({what}, "
                                    f"{e1:.1f} s"},
    }


def _suffix(beta, reinit):
    return "_reinit" if reinit is not None else ("_cutoff" if beta is not None else "")


def _single_grid(args, torch, ls, W, BandGrid, dev):
    """The band driver on one grid: (result fields, workload, precision).

    With the brick layout (default) one job is: phi and F converted to the
    tile-major layout, the driver run there, phi converted back; with the
    dense layout the driver runs on the x-fastest fields."""
    beta = reinit = None
    if args.workload.startswith("spheres512"):
        n = args.n or 512
        wl = W.three_spheres_f32(n, steps=10 * args.steps)
        prec, phi_host, scale = "f32", wl.phi, None
        if args.workload != "spheres512":
            beta = float(np.float32(3 * wl.dx))
        if args.workload == "spheres512_reinit":
            reinit = (float(np.float32(0.5 * wl.dx)), REINIT_ITERS)
    elif args.workload == "torus1024_f32":
        n = args.n or 1024
        wl = W.torus_grf(n, steps=10 * args.steps)
        prec, phi_host, scale = "f32", wl.phi, None
    else:
        n = args.n or 1024
        wl = W.torus_grf(n, steps=10 * args.steps)
        scale = float(np.float32(wl.scale))
        prec, phi_host = "f16s", W.quantize_f16s(wl.phi, scale)
    assert all(n % t == 0 for t in wl.tile), "bench grid must be a whole number of tiles"
    bricks = args.layout == "bricks"
    pts_per_tile = int(np.prod(wl.tile))
    bg = BandGrid((n, n, n), wl.tile, prec, device=dev)
    phi0 = torch.from_numpy(phi_host).to(dev)
    F = torch.from_numpy(wl.F).to(dev)
    del phi_host
    if not args.workload.startswith("spheres512"):
        wl.phi = None  # (only the three-sphere workloads have a CPU baseline)
    phi = phi0.clone()
    phi_b = torch.empty_like(phi) if bricks else None
    F_b = torch.empty_like(F) if bricks else None
    gamma = float(np.float32(wl.gamma))

    def job(nsteps, stream, tile_steps):
        if bricks:
            bg.to_bricks(phi, phi_b, stream)
            bg.to_bricks(F, F_b, stream)
            bg.run_bricks(phi_b, F_b, wl.dx, wl.dt, gamma, nsteps, wl.window, scale=scale,
                          tile_steps=tile_steps, stream=stream, beta=beta, reinit=reinit)
            bg.from_bricks(phi_b, phi, stream)
        else:
            bg.run(phi, F, wl.dx, wl.dt, gamma, nsteps, wl.window, scale=scale,
                   tile_steps=tile_steps, stream=stream, beta=beta, reinit=reinit)

    stream = torch.cuda.current_stream(dev)
    # the narrow-band driver: first window from a full scan of phi, later
    # windows from the exact incremental rebuild; tile_steps counts band
    # tiles x steps on the device
    tile_steps = torch.zeros(1, dtype=torch.int64, device=dev)
    if args.warmup > 0:
        job(args.warmup * wl.window, stream, tile_steps)
    phi.copy_(phi0)
    tile_steps.zero_()
    torch.cuda.synchronize()

    # eager pass with every step launch timed by HIP events (the roofline)
    ls.ls_stats_enable(True)
    t0 = time.perf_counter()
    job(args.steps * wl.window, stream, tile_steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ls.ls_stats_enable(False)
    eager_s = t1 - t0
    eager_tile_steps = int(tile_steps.item())
    launches, timed, upd_ms = ls.ls_stats_read(ls.LS_KERNEL_UPWIND)
    _, ftimed, flag_ms = ls.ls_stats_read(ls.LS_KERNEL_BAND_FLAG)
    nsteps = args.steps * wl.window
    # one or two steps per launch (the brick driver takes pairs of steps)
    assert launches == timed and nsteps <= 2 * launches <= 2 * nsteps
    two_step = launches < nsteps
    step_avg_us = upd_ms * 1e3 / max(timed, 1)
    updates_dominant = eager_tile_steps * pts_per_tile  # time-step point updates
    if reinit is not None:
        # the dominant kernel of this workload: the reinitialisation step
        launches, timed, upd_ms = ls.ls_stats_read(ls.LS_KERNEL_REINIT)
        assert launches == timed and args.steps * reinit[1] <= 2 * launches
        updates_dominant = updates_dominant * reinit[1] // wl.window
        two_step = launches < args.steps * reinit[1]
    # key of the dominant kernel's counter summary in profiles/traffic.json
    traffic_kind = (("brick_reinit" if reinit is not None else "brick_step")
                    + ("2" if two_step else "") if bricks else
                    "reinit" if reinit is not None else "upwind")

    # the timed run: the whole job captured in one HIP graph, replayed once to
    # warm up, then timed from the initial field
    side = torch.cuda.Stream(dev)
    torch.cuda.synchronize()
    ls.ls_graph_begin(side)
    job(args.steps * wl.window, side, tile_steps)
    graph = ls.ls_graph_end(side)
    try:
        phi.copy_(phi0)
        torch.cuda.synchronize()
        ls.ls_graph_launch(graph, side)
        torch.cuda.synchronize()
        phi.copy_(phi0)
        tile_steps.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ls.ls_graph_launch(graph, side)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    finally:
        ls.ls_graph_destroy(graph)
    assert int(tile_steps.item()) == eager_tile_steps
    updates = eager_tile_steps * pts_per_tile
    if bricks:
        dom_steps = args.steps * (reinit[1] if reinit is not None else wl.window)
        pairs = dom_steps - launches  # two-step launches of the dominant kernel
        kname = (f"ls::brick_step{'2' if two_step else ''}_kernel ({prec}, 8x8x8 tiles, "
                 f"tile-major layout, runs of 4 tiles, " +
                 (f"{pairs // args.steps} two-step and {(launches - pairs) // args.steps} one-step "
                  f"launches per window" if two_step else "one step per launch"))
    elif prec == "f32":
        kname = "ls::upwind_vec_kernel (f32, 8x8x8 tiles, 32-point rows, 16-byte accesses"
    else:
        kname = "ls::upwind_vec_kernel (f16s, 8x8x8 tiles, 64-point rows, 8-byte accesses"
    kname += (", reinitialisation step of Eq. 12-13, no F)" if reinit is not None else
              ", cut-off of Eq. 8)" if beta is not None else ")")
    fields = {
        "elapsed": t1 - t0,
        "traffic_kind": traffic_kind,
        "digest_sources": BRICK_KERNEL_SOURCES if bricks else DENSE_KERNEL_SOURCES,
        "updates": updates,
        "upd_ms": upd_ms,
        "launches": launches,
        "config": {
            "workload": wl.name + ("_f32" if args.workload == "torus1024_f32" else "")
                        + _suffix(beta, reinit),
            "grid": [n, n, n],
            "tile": list(wl.tile),
            "band_halfwidth_dx": 6,
            **({"cutoff_beta_dx": 3, "cutoff_gamma_dx": 6} if beta is not None else {}),
            **({"reinit_steps_per_window": reinit[1], "reinit_dtau_dx": 0.5}
               if reinit is not None else {}),
            "steps_per_window": wl.window,
            "upwind_steps": args.steps * wl.window,
            "storage": prec,
            "layout": ("tile-major bricks (phi and F converted in, phi converted back, inside "
                       "the timed region)" if bricks else "x-fastest"),
            "parallelism": "single GPU",
        },
        "extra": {
            "band_tiles_last_window": int(bg.ntiles.item()),
            "band_scan_avg_us": round(flag_ms * 1e3 / max(ftimed, 1), 3),
            "timed_as": "one HIP graph replay of the whole job",
            "eager_value": round(updates / eager_s / 1e9, 3),
            **({"step_avg_launch_us": round(step_avg_us, 3),
                "reinit_updates_per_step": reinit[1] / wl.window} if reinit is not None else {}),
        },
        "kernel": kname,
        "beta": beta,
        "reinit": reinit,
        "pts_per_launch": updates_dominant / max(launches, 1),  # point updates per launch
        "bytes_per_point": (REINIT_BYTES_PER_POINT if reinit is not None else BYTES_PER_POINT)[prec],
        "data": ("synthetic (seeded three-sphere signed distance, sinusoidal speed)"
                 if args.workload.startswith("spheres512") else
                 "synthetic (torus signed distance, speed 1 + 0.3 GRF)" if prec == "f32" else
                 "synthetic (torus signed distance stored as scaled FP16, speed 1 + 0.3 GRF)"),
    }
    return fields, wl, prec


def _batch(args, torch, ls, W, dev):
    """256 uneven grids, tile shapes from the autotuner, the whole run
    captured in one HIP graph and timed on replay."""
    from paper_1612_04040_amd.autotune import shape_for, tune
    from paper_1612_04040_amd.batch import Batch

    insts = W.ellipsoid_batch()
    table = tune([it.n for it in insts])
    specs = [((it.n,) * 3, shape_for(it.n, table), it.dx, it.dt, it.gamma) for it in insts]
    b = Batch(specs, device=dev)
    b.load([it.phi for it in insts], [it.F for it in insts])
    phi0 = b.phi.clone()
    nsteps, window = 10 * args.steps, 10
    point_steps = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.Stream(dev)
    # eager pass with per-launch kernel timing (roofline), then the graph
    with torch.cuda.stream(stream):
        if args.warmup > 0:
            b.run(args.warmup * window, window, stream=stream)
        ls.ls_copy_f32(b.phi, phi0, b.phi.numel(), stream)
        torch.cuda.synchronize()
        ls.ls_stats_enable(True)
        t0 = time.perf_counter()
        b.run(nsteps, window, point_steps=point_steps, stream=stream)
        torch.cuda.synchronize()
        eager_s = time.perf_counter() - t0
        ls.ls_stats_enable(False)
    launches, timed, upd_ms = ls.ls_stats_read(ls.LS_KERNEL_UPWIND)
    updates = int(point_steps.item())
    # the timed run: the whole 100-step run of all grids as one HIP graph
    ls.ls_graph_begin(stream)
    b.run(nsteps, window, point_steps=point_steps, stream=stream)
    graph = ls.ls_graph_end(stream)
    try:
        b.phi.copy_(phi0)
        torch.cuda.synchronize()
        ls.ls_graph_launch(graph, stream)  # warm replay
        torch.cuda.synchronize()
        b.phi.copy_(phi0)
        point_steps.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ls.ls_graph_launch(graph, stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    finally:
        ls.ls_graph_destroy(graph)
    assert int(point_steps.item()) == updates
    shapes = sorted({tuple(s[1]) for s in specs})
    fields = {
        "elapsed": t1 - t0,
        "traffic_kind": "upwind",
        "digest_sources": BATCH_KERNEL_SOURCES,
        "updates": updates,
        "upd_ms": upd_ms,
        "launches": launches,
        "config": {
            "workload": "ellipsoid_batch256",
            "instances": len(insts),
            "sizes": [int(min(it.n for it in insts)), int(max(it.n for it in insts))],
            "total_points": int(sum(it.n ** 3 for it in insts)),
            "tile_shapes": [list(t) for t in shapes],
            "band_halfwidth_dx": 6,
            "steps_per_window": window,
            "upwind_steps": nsteps,
            "storage": "f32",
            "parallelism": "single GPU",
        },
        "extra": {"timed_as": "one HIP graph replay of the whole run",
                  "eager_value": round(updates / eager_s / 1e9, 3)},
        "kernel": "ls::upwind_fast_kernel (f32, batched, all tile shapes)",
        "data": "synthetic (seeded random-ellipsoid signed distances, speed u + 0.2 GRF)",
    }
    return fields


CLOSURE_FLOP_PER_POINT = 17280  # 3 conv layers 3->16->16->1 on 3^3 taps, 2 flop per MAC


def _closure(args, torch, ls, W, dev):
    """The learned closure (cfg 5): its network trained on the GPU by the
    library's own kernels (16 seeds of 512^3 fine runs restricted 4x, the
    Adam iterations of --closure-iters), then on the evaluation seed 5 the
    plain 512^3 fine run (1 600 steps) against the learned 128^3 coarse run
    (400 steps) judged by the plain coarse scheme, each whole run one HIP
    graph replay; the Hausdorff distances of the fronts in fine dx."""
    from paper_1612_04040_amd import closure as C
    from paper_1612_04040_amd import closure_train as CT

    nsteps = 10 * args.steps  # coarse steps (400 by default)
    nf = 512
    t0 = time.perf_counter()
    problems = []
    for s in range(100, 100 + args.closure_seeds):
        problems.append(CT.Problem(s, nf, nsteps, dev))
        print(f"closure128: training data, seed {s} ({time.perf_counter() - t0:.0f} s)",
              file=sys.stderr, flush=True)
    cg = C.ClosureGrid((nf // 4,) * 3, dev)
    params = torch.from_numpy(C.init_params(np.random.default_rng(0)).astype(np.float32)).to(dev)
    t1 = time.perf_counter()
    CT.train(cg, problems, params, args.closure_iters, 3e-4, rollout_max=4, rollout_prob=0.5)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    del problems
    torch.cuda.empty_cache()
    print(f"closure128: trained {args.closure_iters} iterations in {train_s:.0f} s",
          file=sys.stderr, flush=True)
    ev = CT.evaluate(5, nf, nsteps, params, dev, reps=3)
    # the fused network kernel: an eager learned run window by window with its
    # launches timed, the active tiles of each window counted by a band build
    case = W.ClosureCase(5, nf)
    nc = case.n_coarse
    phi = C.restrict4(torch.from_numpy(case.phi(nf)).to(dev))
    Fc = torch.from_numpy(case.F(nc)).to(dev)
    from paper_1612_04040_amd.band import BandGrid

    counter = BandGrid((nc,) * 3, (8, 8, 8), "f32", dev)
    active_steps = 0
    ls.ls_stats_enable(True)
    for _ in range(args.steps):
        counter.build(phi, case.gamma_coarse, dilate=False)
        active_steps += int(counter.ntiles.item()) * 10
        cg.run(phi, Fc, case.dx_coarse, case.dt_coarse, case.gamma_coarse, case.fmax, params, 10,
               10, judge=0)
    torch.cuda.synchronize()
    ls.ls_stats_enable(False)
    launches, timed, ms = ls.ls_stats_read(ls.LS_KERNEL_CLOSURE)
    avg_s = ms / 1e3 / max(timed, 1)
    flop_per_launch = CLOSURE_FLOP_PER_POINT * 512 * active_steps / max(launches, 1)
    return {"ev": ev, "train_s": train_s, "avg_launch_us": avg_s * 1e6,
            "flop_per_launch": flop_per_launch, "launches": launches,
            "active_tiles_per_step": active_steps / max(10 * args.steps, 1)}


def _snapshot_run(args, torch, ls, W, BandGrid, dev):
    """The spheres512 windows as separate eager driver calls (a full band
    build each), timed without and with an asynchronous snapshot every K
    windows; the gather kernel timed by HIP events."""
    from paper_1612_04040_amd.snapshot import Snapshots

    n = args.n or 512
    wl = W.three_spheres_f32(n, steps=10 * args.steps)
    bg = BandGrid((n, n, n), wl.tile, "f32", device=dev)
    phi0 = torch.from_numpy(wl.phi).to(dev)
    F = torch.from_numpy(wl.F).to(dev)
    phi = phi0.clone()
    gamma = float(np.float32(wl.gamma))
    # the band count of phi0 (read once, untimed) as the first host-known count
    bg.build(phi0, gamma)
    snaps = Snapshots(bg, copy_blocks=args.snapshot_copy_blocks,
                      expected=int(bg.ntiles[:1].item()))
    tile_steps = torch.zeros(1, dtype=torch.int64, device=dev)
    k = args.snapshot_every

    def windows(with_snaps, count, ev):
        got, pending = 0, []
        ev[0].record()
        for w in range(count):
            bg.run(phi, F, wl.dx, wl.dt, gamma, wl.window, wl.window, tile_steps=tile_steps)
            if with_snaps and (w + 1) % k == 0:
                pending.append(snaps.take(phi))
                if len(pending) == 2:
                    pending.pop(0).wait()
                    got += 1
        ev[1].record()  # the compute stream's work done (the last copy may still run)
        for p_ in pending:
            p_.wait()
            got += 1
        return got

    times = {}
    # a warm pair (the one with snapshots also times the gather kernel with HIP
    # events), then the timed pair without kernel timing
    for i, with_snaps in enumerate((False, True, False, True)):
        phi.copy_(phi0)
        tile_steps.zero_()
        torch.cuda.synchronize()
        if i == 1:
            ls.ls_stats_enable(True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        t0 = time.perf_counter()
        taken = windows(with_snaps, args.steps, ev)
        torch.cuda.synchronize()
        times[with_snaps] = (time.perf_counter() - t0, taken, int(tile_steps.item()),
                             ev[0].elapsed_time(ev[1]) / 1e3)
        if i == 1:
            ls.ls_stats_enable(False)
    g_launches, g_timed, g_ms = ls.ls_stats_read(ls.LS_KERNEL_GATHER)
    snaps.close()  # copies done, pinned buffers and the copy stream released before exit
    t_plain, _, ts, c_plain = times[False]
    t_snap, taken, _, c_snap = times[True]
    updates = ts * int(np.prod(wl.tile))
    band_pts = updates / (args.steps * wl.window)
    return {
        "value": updates / t_snap / 1e9,
        "plain_value": updates / t_plain / 1e9,
        "ms_per_step": t_snap / args.steps * 1e3,
        "snapshots": taken,
        "overhead_frac": (t_snap - t_plain) / t_plain,
        # the compute stream alone (events around the windows): the overhead
        # without the drain of the last snapshot's copy
        "compute_overhead_frac": (c_snap - c_plain) / c_plain,
        "gather_avg_us": g_ms * 1e3 / max(g_timed, 1),
        "gather_bytes_per_launch": 8 * band_pts,  # phi read + snapshot write, FP32
        "snapshot_mb": 4 * band_pts / 1e6,
        "config": {"workload": wl.name + f"_snapshot_every_{k}", "grid": [n, n, n],
                   "tile": list(wl.tile), "band_halfwidth_dx": 6,
                   "steps_per_window": wl.window, "upwind_steps": args.steps * wl.window,
                   "storage": "f32", "snapshot_copy_blocks": args.snapshot_copy_blocks,
                   "parallelism": "single GPU"},
    }


def copy_ceiling(torch, ls, dev, reps=5):
    """GB/s of the plain 1 GiB dword copy (2 GiB moved per launch), the best of
    `reps` launches timed by events: the bandwidth a streaming kernel reaches."""
    a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    s = torch.cuda.current_stream(dev)
    best = None
    for r in range(reps + 2):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        ls.ls_copy_f32(b, a, a.numel(), stream=s)
        e1.record(s)
        e1.synchronize()
        if r >= 2:
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (1 << 30) / (best / 1e3) / 1e9


def _calibration_copies(torch, ls, dev):
    """The plain 1 GiB dword copy, three times (the traffic counters' reference)."""
    a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        ls.ls_copy_f32(b, a, a.numel(), stream=torch.cuda.current_stream(dev))
    torch.cuda.synchronize()
    del a, b


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the band update of one grid is measured on one MI355X)", file=sys.stderr)
        return 2
    import torch

    from paper_1612_04040_amd import ls
    from paper_1612_04040_amd import workloads as W
    from paper_1612_04040_amd.band import BandGrid

    rank = int(os.environ.get("RANK", "0"))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.steps_per_launch:
        ls.ls_set_tuning(0, 0, 0, 0, {1: 2, 2: 1}[args.steps_per_launch])

    if args.snapshot_every > 0:
        if args.workload != "spheres512":
            print("--snapshot-every applies to the spheres512 workload", file=sys.stderr)
            return 2
        r = _snapshot_run(args, torch, ls, W, BandGrid, dev)
        gbps = r["gather_bytes_per_launch"] / (r["gather_avg_us"] * 1e-6) / 1e9
        gdigest = kernel_source_digest(GATHER_KERNEL_SOURCES)
        if args.calibrate_copy:
            _calibration_copies(torch, ls, dev)
        if rank == 0:
            print(json.dumps({
                "metric": "band GLUPS (narrow-band first-order upwind update, incl. band "
                          "rebuilds and asynchronous band snapshots)",
                "value": round(r["value"], 3), "unit": "GLUPS", "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup,
                "ms_per_step": round(r["ms_per_step"], 4), "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                "data": "synthetic (seeded three-sphere signed distance, sinusoidal speed)",
                "config": r["config"],
                "timed_as": "eager driver calls, one per window (full band build each)",
                "without_snapshots_value": round(r["plain_value"], 3),
                "snapshots": r["snapshots"],
                "snapshot_overhead_frac": round(r["overhead_frac"], 4),
                "snapshot_compute_overhead_frac": round(r["compute_overhead_frac"], 4),
                "snapshot_mb": round(r["snapshot_mb"], 2),
                "roofline": {"bound": "hbm", "kernel": "ls::band_gather_kernel (f32 quads)",
                             "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbps / HBM_PEAK_GBS, 4),
                             "traffic": measured_traffic("gather", r["config"]["workload"],
                                                         gdigest),
                             "bytes_per_launch_alg": int(r["gather_bytes_per_launch"]),
                             "avg_launch_us": round(r["gather_avg_us"], 3)},
                "kernel_source_digest": gdigest,
                "cpu_baseline": None,
            }), flush=True)
        return 0

    if args.workload == "closure128":
        r = _closure(args, torch, ls, W, dev)
        ev = r["ev"]
        tflops = r["flop_per_launch"] / (r["avg_launch_us"] * 1e-6) / 1e12
        if rank == 0:
            print(json.dumps({
                "metric": "learned-coarse vs plain-fine wall time at equal interface error "
                          "(speed-up of the judged learned 128^3 run over the plain 512^3 run)",
                "value": round(ev["fine_ms"] / ev["judged_coarse_ms"], 3), "unit": "x",
                "n_gpus": 1, "steps": args.steps, "warmup": 0,
                "ms_per_step": round(ev["judged_coarse_ms"] / args.steps, 4),
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "bf16 network, f32 level set",
                "data": "synthetic (seeded sphere unions, sinusoidal speeds; evaluation seed 5)",
                "config": {"workload": "closure128", "coarse_grid": [128] * 3,
                           "fine_grid": [512] * 3, "coarse_steps": 10 * args.steps,
                           "fine_steps": 40 * args.steps, "training_seeds": args.closure_seeds,
                           "training_iters": args.closure_iters,
                           "judge": "plain coarse shadow, topology and front within 1 coarse dx",
                           "parallelism": "single GPU"},
                "timed_as": "one HIP graph replay of each whole run (fine: 1 600 steps with its "
                            "band rebuilds; coarse: 400 corrected steps, rebuilds, shadow, judge)",
                "fine_ms": round(ev["fine_ms"], 2),
                "plain_coarse_ms": round(ev["plain_coarse_ms"], 2),
                "learned_coarse_ms": round(ev["learned_coarse_ms"], 2),
                "judged_coarse_ms": round(ev["judged_coarse_ms"], 2),
                "hausdorff_dx_fine": {k: round(ev[f"hausdorff_{k}_dx_fine"], 3) for k in (
                    "restricted_fine", "plain_coarse", "learned_coarse",
                    "judged_topology_coarse", "judged_coarse", "judged_half_coarse")},
                "judge_resets": ev.get("judged_resets"),
                "judged_half_coarse_ms": round(ev["judged_half_coarse_ms"], 2),
                "judge_half_resets": ev.get("judged_half_resets"),
                "train_s": round(r["train_s"], 1),
                "roofline": {"bound": "mfma", "kernel": "ls::closure_fused_kernel (bf16 MFMA "
                             "16x16x32, fp32 accumulation)",
                             "achieved": round(tflops, 2), "peak": 2500.0, "unit": "TFLOP/s",
                             "frac": round(tflops / 2500.0, 5), "traffic": None,
                             "flop_per_launch_alg": int(r["flop_per_launch"]),
                             "avg_launch_us": round(r["avg_launch_us"], 3),
                             "active_tiles_per_step": round(r["active_tiles_per_step"], 1)},
                "cpu_baseline": None,
            }), flush=True)
        return 0

    wl = None
    if args.workload == "batch256":
        f = _batch(args, torch, ls, W, dev)
        prec = "f32"
    else:
        f, wl, prec = _single_grid(args, torch, ls, W, BandGrid, dev)
    value = f["updates"] / f["elapsed"] / 1e9
    avg_launch_s = f["upd_ms"] / 1e3 / max(f["launches"], 1)
    pts_per_launch = f.get("pts_per_launch", f["updates"] / max(f["launches"], 1))
    bytes_per_launch = f.get("bytes_per_point", BYTES_PER_POINT[prec]) * pts_per_launch
    achieved = bytes_per_launch / avg_launch_s / 1e9
    digest = kernel_source_digest(f["digest_sources"])
    traffic = measured_traffic(f.get("traffic_kind", "upwind"), f["config"]["workload"], digest)

    ceiling = copy_ceiling(torch, ls, dev)
    result = {
        "metric": "band GLUPS (narrow-band first-order upwind update, incl. band rebuilds)",
        "value": round(value, 3),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f["elapsed"] / max(args.steps, 1) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f16s": "f32", "f64": "f64"}.get(prec, "f32"),  # arithmetic (storage: config)
        "data": f["data"],
        "config": f["config"],
        "kernel_glups": round(pts_per_launch / avg_launch_s / 1e9, 3),
        **f["extra"],
        "roofline": {
            "bound": "hbm",
            "kernel": f["kernel"],
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch_alg": int(bytes_per_launch),
            "avg_launch_us": round(avg_launch_s * 1e6, 3),
            # the 1 GiB dword copy (2 GiB moved) on the same GPU: the streaming ceiling
            "copy_ceiling_gbs": round(ceiling, 1),
            "frac_of_copy": round(achieved / ceiling, 4),
        },
        "kernel_source_digest": digest,
    }
    if args.calibrate_copy:
        _calibration_copies(torch, ls, dev)
    if rank == 0:
        # (the oracle's reinitialisation takes minutes per window at 512^3: no
        # bounded sample of that workload exists, so it has no CPU baseline)
        result["cpu_baseline"] = (cpu_baseline(wl, args.cpu_seconds, f.get("beta"))
                                  if args.workload in ("spheres512", "spheres512_cutoff")
                                  else None)
        print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
