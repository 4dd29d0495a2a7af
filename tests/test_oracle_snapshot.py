"""Pins of the oracle's band snapshot (the values of the band tiles, tile by
tile): explicit loops on a tiny grid with partial tiles, and the round trip
that scatters a snapshot back."""
import numpy as np

import oracle


def test_gather_matches_explicit_loops():
    rng = np.random.default_rng(0)
    nx, ny, nz = 11, 7, 5
    tile = (4, 3, 2)
    phi = rng.standard_normal((nz, ny, nx)).astype(np.float32)
    ntx, nty = 3, 3
    tiles = np.array([0, 4, 8, 13, 26], dtype=np.int32)  # corner, inner and partial tiles
    got = oracle.gather_tiles(phi, tiles, tile)
    assert got.shape == (5, 2, 3, 4) and got.dtype == np.float32
    for p, t in enumerate(tiles):
        ti, tj, tk = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        for lz in range(2):
            for ly in range(3):
                for lx in range(4):
                    i, j, k = ti * 4 + lx, tj * 3 + ly, tk * 2 + lz
                    want = phi[k, j, i] if (i < nx and j < ny and k < nz) else 0.0
                    assert got[p, lz, ly, lx] == want


def test_scatter_round_trip():
    rng = np.random.default_rng(1)
    dims = (20, 17, 9)
    phi = rng.standard_normal((9, 17, 20))
    tiles = np.sort(rng.choice(oracle.tile_count(dims, (8, 8, 8)), 7, replace=False))
    snap = oracle.gather_tiles(phi, tiles)
    back = np.zeros_like(phi)
    ntx, nty = 3, 3
    for p, t in enumerate(tiles):
        ti, tj, tk = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        blk = back[tk * 8:(tk + 1) * 8, tj * 8:(tj + 1) * 8, ti * 8:(ti + 1) * 8]
        blk[...] = snap[p, :blk.shape[0], :blk.shape[1], :blk.shape[2]]
    m = oracle.tile_mask(dims, tiles)
    assert np.array_equal(back[m], phi[m]) and np.all(back[~m] == 0)
    # the padding of partial tiles is zero and nothing else is
    assert np.count_nonzero(snap) == m.sum()
