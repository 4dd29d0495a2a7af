#!/usr/bin/env python3
"""Benchmark of the narrow-band first-order upwind level-set update on one MI355X.

Workload: the 512^3 FP32 union of three spheres (seeded), speed
F = 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z), band half-width 6 dx in 8^3
tiles, rebuilt every 10 steps, 200 steps.  One bench "step" is one window of
the narrow-band algorithm (Sec. 1.1, Steps 1-2): a band rebuild (a full scan
of phi for the first window, the exact incremental rescan of the previous
band afterwards; dilation; ordered compaction) and 10 upwind steps (Eq. 3-5)
on the band, so --steps 20 is the whole 200-step run, one driver call.  Inputs are resident in HBM before
the timed region starts; the run restarts from the initial field after the
warm-up windows.

Prints one JSON line: whole-job band GLUPS (band point-updates per second
including rebuilds), the roofline of the dominant kernel (the band step,
timed per launch with HIP events on its stream) and the oracle timed on the
host cores on a bounded sample of the same workload.
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


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed windows (10 upwind steps each)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed warm-up windows")
    ap.add_argument("--n", type=int, default=512, help="grid points per axis")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU work budget of the oracle baseline (0 disables it)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, run the plain 1 GiB dword copy kernel "
                         "(the reference for calibrating the traffic counters)")
    return ap.parse_args()


def kernel_source_digest():
    here = os.path.dirname(os.path.abspath(__file__))
    csrc = os.path.join(here, "paper_1612_04040_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
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


def cpu_baseline(wl, budget_s):
    """The oracle (FP64, OpenMP) on whole windows of the same workload."""
    import oracle

    if budget_s <= 0:
        return None
    phi = wl.phi.astype(np.float64)
    g32 = np.float32(wl.gamma)
    updates, windows = 0, 0
    t0 = time.perf_counter()
    while True:
        tiles = oracle.band_tiles(phi.astype(np.float32), wl.tile, g32, dilate=True)
        phi = oracle.upwind_steps(phi, wl.F, wl.dx, wl.dt, tiles, wl.window, wl.tile)
        updates += int(tiles.size) * int(np.prod(wl.tile)) * wl.window
        windows += 1
        if time.perf_counter() - t0 >= budget_s or windows * wl.window >= wl.nsteps:
            break
    elapsed = time.perf_counter() - t0
    return {
        "value": updates / elapsed / 1e9,
        "unit": "GLUPS",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": f"first {windows} window(s) x {wl.window} steps (band rebuild + FP64 "
                  f"upwind steps) of the {wl.name} workload, {elapsed:.1f} s",
    }


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

    wl = W.three_spheres_f32(args.n, steps=10 * args.steps)
    n = args.n
    assert all(n % t == 0 for t in wl.tile), "bench grid must be a whole number of tiles"
    pts_per_tile = int(np.prod(wl.tile))
    bg = BandGrid((n, n, n), wl.tile, "f32", device=dev)
    phi0 = torch.from_numpy(wl.phi).to(dev)
    F = torch.from_numpy(wl.F).to(dev)
    phi = phi0.clone()
    gamma = float(np.float32(wl.gamma))
    stream = torch.cuda.current_stream(dev)

    # the narrow-band driver: first window from a full scan of phi, later
    # windows from the exact incremental rebuild; tile_steps counts band
    # tiles x steps on the device
    tile_steps = torch.zeros(1, dtype=torch.int64, device=dev)
    if args.warmup > 0:
        bg.run(phi, F, wl.dx, wl.dt, gamma, args.warmup * wl.window, wl.window,
               tile_steps=tile_steps, stream=stream)
    phi.copy_(phi0)
    tile_steps.zero_()
    torch.cuda.synchronize()

    ls.ls_stats_enable(True)
    t0 = time.perf_counter()
    bg.run(phi, F, wl.dx, wl.dt, gamma, args.steps * wl.window, wl.window,
           tile_steps=tile_steps, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ls.ls_stats_enable(False)

    elapsed = t1 - t0
    updates = int(tile_steps.item()) * pts_per_tile
    value = updates / elapsed / 1e9

    launches, timed, upd_ms = ls.ls_stats_read(ls.LS_KERNEL_UPWIND)
    flaunches, ftimed, flag_ms = ls.ls_stats_read(ls.LS_KERNEL_BAND_FLAG)
    assert launches == timed == args.steps * wl.window
    avg_launch_s = upd_ms / 1e3 / max(timed, 1)
    pts_per_launch = updates / max(launches, 1)
    bytes_per_launch = BYTES_PER_POINT["f32"] * pts_per_launch
    achieved = bytes_per_launch / avg_launch_s / 1e9
    digest = kernel_source_digest()
    traffic = measured_traffic("upwind", wl.name, digest)

    result = {
        "metric": "band GLUPS (narrow-band first-order upwind update, incl. band rebuilds)",
        "value": round(value, 3),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / max(args.steps, 1) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded three-sphere signed distance, sinusoidal speed)",
        "config": {
            "workload": wl.name,
            "grid": [n, n, n],
            "tile": list(wl.tile),
            "band_halfwidth_dx": 6,
            "steps_per_window": wl.window,
            "upwind_steps": args.steps * wl.window,
            "parallelism": "single GPU",
        },
        "kernel_glups": round(pts_per_launch / avg_launch_s / 1e9, 3),
        "band_tiles_last_window": int(bg.ntiles.item()),
        "band_scan_avg_us": round(flag_ms * 1e3 / max(ftimed, 1), 3),
        "roofline": {
            "bound": "hbm",
            "kernel": "ls::upwind_fast_kernel (f32, 8x8x8 tiles)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch_alg": int(bytes_per_launch),
            "avg_launch_us": round(avg_launch_s * 1e6, 3),
        },
        "kernel_source_digest": digest,
    }
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            ls.ls_copy_f32(b, a, a.numel(), stream=stream)
        torch.cuda.synchronize()
        del a, b
    if rank == 0:
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
        print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
