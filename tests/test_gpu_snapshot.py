"""Band snapshots on the GPU: the gather against the oracle's definition, bit
for bit, and the asynchronous snapshot pipeline against synchronous copies of
the same (deterministic) run."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, random_tiles, to_dev
from paper_1612_04040_amd import workloads as W
from paper_1612_04040_amd.band import BandGrid
from paper_1612_04040_amd import ls
from paper_1612_04040_amd.snapshot import Snapshots

pytestmark = pytest.mark.gpu

CASES = [
    # dims, tile, precision, tile fraction, capacity cut
    ((64, 64, 64), (8, 8, 8), "f32", 0.4, None),    # quads
    ((68, 45, 33), (8, 8, 8), "f32", 0.6, None),    # quads, partial tiles in y and z
    ((67, 45, 33), (8, 8, 8), "f32", 0.6, None),    # nx odd: single points
    ((40, 24, 16), (8, 8, 8), "f16s", 0.5, None),
    ((13, 9, 7), (4, 3, 2), "f64", 0.7, None),
    ((100, 36, 20), (16, 4, 4), "f32", 0.5, 7),     # capacity below the count
    ((37, 21, 18), (8, 8, 8), "f64", 1.0, None),
]


@pytest.mark.parametrize("dims,tile,precision,frac,cap", CASES)
def test_gather_equals_oracle(dims, tile, precision, frac, cap):
    rng = np.random.default_rng(sum(dims) + len(precision))
    nx, ny, nz = dims
    dtype = {"f32": np.float32, "f64": np.float64, "f16s": np.float16}[precision]
    phi = rng.standard_normal((nz, ny, nx)).astype(dtype)
    tiles = random_tiles(rng, oracle.tile_count(dims, tile), frac)
    bg = BandGrid(dims, tile, precision)
    bg.tiles[: tiles.size] = torch.from_numpy(tiles).to(dev())
    bg.ntiles.fill_(int(tiles.size))
    capacity = bg.capacity if cap is None else cap
    tp = int(np.prod(tile))
    out = torch.full((capacity * tp,), 7, dtype=bg.scratch.dtype, device=dev())
    ids = torch.full((capacity,), -5, dtype=torch.int32, device=dev())
    bg.gather(torch.from_numpy(phi).to(dev()), out, ids=ids, capacity=capacity)
    n = min(tiles.size, capacity)
    want = oracle.gather_tiles(phi, tiles[:n], tile)
    got = host(out)[: n * tp].reshape(want.shape)
    assert got.tobytes() == want.tobytes()
    assert host(ids)[:n].tolist() == tiles[:n].tolist()
    # nothing beyond the first n tiles is written
    assert np.all(host(out)[n * tp:] == 7) and np.all(host(ids)[n:] == -5)


def test_async_snapshots_equal_synchronous_ones():
    """Six windows of the band driver with a snapshot after each, no host
    synchronisation between them (the copies run on their own stream while the
    next windows compute), against the same (deterministic) run with a gather
    read back synchronously after every window: the pipeline moves the gather's
    bytes unchanged.  (The gather itself is checked against the oracle above.)"""
    n = 96
    wl = W.three_spheres_f32(n, 60)
    g = float(np.float32(wl.gamma))
    bg = BandGrid((n, n, n), wl.tile, "f32")
    fd = to_dev(wl.F)
    tp = 512

    ref = []
    p = to_dev(wl.phi)
    out = torch.empty(bg.capacity * tp, device=dev())
    for _ in range(6):
        bg.run(p, fd, wl.dx, wl.dt, g, 10, 10)
        bg.gather(p, out)
        band = bg.band_list().numpy()
        ref.append((band, host(out)[: band.size * tp].reshape(band.size, 8, 8, 8)))

    snaps = Snapshots(bg)
    p = to_dev(wl.phi)
    got = []
    pending = []
    for _ in range(6):
        bg.run(p, fd, wl.dx, wl.dt, g, 10, 10)
        pending.append(snaps.take(p))
        if len(pending) == 2:
            got.append(pending.pop(0).wait(copy=True))
    got += [s.wait(copy=True) for s in pending]
    assert len(got) == 6
    for k, ((ids, vals), (band, want)) in enumerate(zip(got, ref)):
        assert ids.tolist() == band.tolist(), k
        assert vals.tobytes() == want.tobytes(), k
    snaps.close()
    with pytest.raises(RuntimeError):
        snaps.take(p)
    snaps.close()  # a second close does nothing


@pytest.mark.parametrize("unit_bytes", [80, 12, 6, 3])
def test_counted_copy_moves_exactly_the_counted_units(unit_bytes):
    """ls_copy_counted: min(max(count, 0), max_units) units, the count read on
    the device, into pinned host memory and into device memory, with the count
    stored; nothing beyond is written (16-, 4-, 2- and 1-byte forms)."""
    nbytes = 4000
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device=dev())
    maxu = nbytes // unit_bytes
    for count, want in ((7, 7), (maxu + 30, maxu), (-3, 0), (0, 0)):
        cnt = torch.tensor([count], dtype=torch.int32, device=dev())
        for pinned in (True, False):
            dst = torch.full((nbytes,), 0xA5, dtype=torch.uint8)
            dst = dst.pin_memory() if pinned else dst.to(dev())
            out = torch.full((1,), -9, dtype=torch.int32)
            out = out.pin_memory() if pinned else out.to(dev())
            ls.ls_copy_counted(dst, src, cnt, unit_bytes, maxu, count_out=out, blocks=3)
            torch.cuda.synchronize()
            d, s_ = dst.cpu().numpy(), src.cpu().numpy()
            m = want * unit_bytes
            assert np.array_equal(d[:m], s_[:m]), (unit_bytes, count, pinned)
            assert np.all(d[m:] == 0xA5), (unit_bytes, count, pinned)
            assert int(out.cpu()[0]) == want


@pytest.mark.parametrize("unit_bytes,first", [(80, 0), (80, 5), (12, 3), (3, 1000), (80, 13107)])
def test_counted_copy_from_moves_the_tail(unit_bytes, first):
    """ls_copy_counted_from: units [first, n) only, n = min(max(count, 0),
    max_units) stored to count_out; units below first and beyond n are not
    written.  1 MiB with one workgroup runs the four-per-thread loop."""
    nbytes = 1 << 20
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device=dev())
    maxu = nbytes // unit_bytes
    first = min(first, maxu)
    for count in (maxu - 7, first + 1, first, first - 1, maxu + 9):
        want = max(0, min(count, maxu))
        cnt = torch.tensor([count], dtype=torch.int32, device=dev())
        dst = torch.full((nbytes,), 0xA5, dtype=torch.uint8).pin_memory()
        out = torch.full((1,), -9, dtype=torch.int32).pin_memory()
        ls.ls_copy_counted_from(dst, src, cnt, unit_bytes, first, maxu, count_out=out, blocks=1)
        torch.cuda.synchronize()
        d, s_ = dst.numpy(), src.cpu().numpy()
        lo, hi = first * unit_bytes, max(first, want) * unit_bytes
        assert np.all(d[:lo] == 0xA5), (unit_bytes, first, count)
        assert np.array_equal(d[lo:hi], s_[lo:hi]), (unit_bytes, first, count)
        assert np.all(d[hi:] == 0xA5), (unit_bytes, first, count)
        assert int(out[0]) == want


def test_snapshot_beyond_the_known_count():
    """A snapshot whose band outgrows the host-known bound (4 tiles read back,
    then 300 listed: a DMA copy of 4 + 0 + 64 tiles and the counted copy of
    the other 232) and one that shrinks (8 tiles) equal the oracle's gather."""
    dims, tile = (64, 64, 64), (8, 8, 8)
    rng = np.random.default_rng(11)
    phi = rng.standard_normal(dims[::-1]).astype(np.float32)
    p = torch.from_numpy(phi).to(dev())
    bg = BandGrid(dims, tile, "f32")
    snaps = Snapshots(bg)
    for n in (4, 300, 8):
        tiles = np.sort(rng.choice(512, size=n, replace=False)).astype(np.int32)
        bg.tiles[:n] = torch.from_numpy(tiles).to(dev())
        bg.ntiles.fill_(n)
        ids, vals = snaps.take(p).wait(copy=True)
        assert ids.tolist() == tiles.tolist(), n
        assert vals.tobytes() == oracle.gather_tiles(phi, tiles, tile).tobytes(), n
    snaps.close()


def test_snapshot_buffers_full_is_an_error():
    bg = BandGrid((32, 32, 32), (8, 8, 8), "f32")
    bg.tiles[:4] = torch.arange(4, dtype=torch.int32, device=dev())
    bg.ntiles.fill_(4)
    phi = torch.zeros((32, 32, 32), device=dev())
    snaps = Snapshots(bg)
    a = snaps.take(phi)
    snaps.take(phi)
    with pytest.raises(RuntimeError):
        snaps.take(phi)
    ids, vals = a.wait()
    assert ids.tolist() == [0, 1, 2, 3] and vals.shape == (4, 8, 8, 8)
    snaps.take(phi)
