"""Tile-shape autotuner of the band update: a thin wrapper over the native
``ls_autotune`` (libls), which times the narrow-band driver per size bucket
of 32 points with each candidate tile shape and caches the choice per device
in a text file at ``$LS_AUTOTUNE_CACHE`` (default ``/tmp/ls_autotune.txt``).
"""
import os

from . import ls

# Shapes the batched step kernel is compiled for (with the default run width).
CANDIDATES = [(8, 8, 8), (16, 4, 4), (32, 4, 4), (16, 8, 8), (4, 4, 4)]
BUCKET = 32


def cache_path():
    return os.environ.get("LS_AUTOTUNE_CACHE", "/tmp/ls_autotune.txt")


def bucket_of(n):
    return int(n) // BUCKET


def tune(sizes, path=None, force=False):
    """{bucket: tile} for the buckets of `sizes`, measured or from the cache."""
    sizes = sorted({int(n) for n in sizes})
    shapes = ls.ls_autotune(sizes, path or cache_path(), force)
    return {bucket_of(n): t for n, t in zip(sizes, shapes)}


def shape_for(n, table):
    return table[bucket_of(n)]
