"""Tile-shape autotuner for the band update, cached per grid-size bucket.

For every size bucket it times the narrow-band driver (band build or rebuild
plus the band steps, through libls) on a representative grid of that size
with each candidate tile shape, and keeps the shape with the shortest time
per window: the time to advance the same front, which is what differs
between shapes (a bigger tile updates more points of the same band).  Results
are cached as JSON at ``$LS_AUTOTUNE_CACHE`` (default
``/tmp/ls_autotune.json``), keyed by bucket and device name.
"""
import json
import os

import numpy as np
import torch

from . import workloads as W
from .band import BandGrid

# Shapes the batched step kernel is compiled for (with the default run width).
CANDIDATES = [(8, 8, 8), (16, 4, 4), (32, 4, 4), (16, 8, 8), (4, 4, 4)]
BUCKET = 32


def cache_path():
    return os.environ.get("LS_AUTOTUNE_CACHE", "/tmp/ls_autotune.json")


def bucket_of(n):
    return int(n) // BUCKET


def _time_shape(n, tile, windows=2, window=10, seed=0):
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    a = rng.uniform(0.1, 0.3, size=3)
    phi = W.ellipsoid((n, n, n), dx, rng.uniform(0.35, 0.65, 3), a, W.random_rotation(rng),
                      dtype=np.float32)
    F = np.full((n, n, n), 0.6, dtype=np.float32)
    dt = float(np.float32(W.stable_dt(F, dx)))
    gamma = float(np.float32(6 * dx))
    bg = BandGrid((n, n, n), tile, "f32")
    p0 = torch.from_numpy(phi).cuda()
    Fd = torch.from_numpy(F).cuda()
    p = p0.clone()
    bg.run(p, Fd, dx, dt, gamma, window, window)  # warm-up
    p.copy_(p0)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    bg.run(p, Fd, dx, dt, gamma, windows * window, window)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / windows


def tune(sizes, candidates=CANDIDATES, path=None, force=False):
    """{bucket: tile} for the buckets of `sizes`, measured or from the cache."""
    path = path or cache_path()
    dev = torch.cuda.get_device_name(0)
    cache = {}
    if os.path.exists(path) and not force:
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    table = cache.setdefault(dev, {})
    out = {}
    for b in sorted({bucket_of(n) for n in sizes}):
        key = str(b)
        if key not in table:
            n = b * BUCKET + BUCKET // 2
            times = {str(list(t)): _time_shape(n, t) for t in candidates}
            best = min(times, key=times.get)
            table[key] = {"tile": json.loads(best), "ms_per_window": times, "n": n}
        out[b] = tuple(table[key]["tile"])
    try:
        with open(path, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    except OSError:
        pass
    return out


def shape_for(n, table):
    return table[bucket_of(n)]
