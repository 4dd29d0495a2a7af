"""Batched uneven grids on the GPU.

Every grid of a batch (rows pitched to 128-byte lines, or dense) equals the
same grid run alone through the single-grid driver with its tile shape, bit
for bit (phi and band list); one grid is
checked against the oracle; a HIP-graph capture of the batch, replayed
several times with eager work between the replays, reproduces the eager run
every time.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, fp32_step_bound, host, to_dev
from paper_1612_04040_amd import ls
from paper_1612_04040_amd import workloads as W
from paper_1612_04040_amd.autotune import CANDIDATES
from paper_1612_04040_amd.band import BandGrid
from paper_1612_04040_amd.batch import Batch

pytestmark = pytest.mark.gpu


def _specs(seed=21, count=10, nmin=20, nmax=72):
    rng = np.random.default_rng(seed)
    insts = W.ellipsoid_batch(count=count, nmin=nmin, nmax=nmax, seed=seed, base=32)
    specs, phis, Fs = [], [], []
    for k, it in enumerate(insts):
        tile = CANDIDATES[k % len(CANDIDATES)]
        dims = (it.n, it.n, it.n)
        specs.append((dims, tile, it.dx, it.dt, it.gamma))
        phis.append(it.phi)
        Fs.append(it.F)
    return specs, phis, Fs, rng


@pytest.mark.parametrize("row_align", [32, 1])
def test_batch_equals_single_grids(row_align):
    """Pitched rows (128-byte lines, the default) and dense rows."""
    specs, phis, Fs, _ = _specs()
    b = Batch(specs, row_align=row_align)
    b.load(phis, Fs)
    # row padding: phi holds a sentinel (a read would change the results),
    # which must survive the run (no write)
    pads = []
    for i, (dims, *_r) in enumerate(specs):
        nx, ny, nz = dims
        o, px = b.offsets[i], b.pitches[i]
        pad = b.phi[o:o + px * ny * nz].view(nz, ny, px)[:, :, nx:]
        pad.fill_(-7.0)
        pads.append(pad)
    acc = torch.zeros(1, dtype=torch.int64, device=dev())
    b.run(25, 10, tile_steps=acc)
    for pad in pads:
        assert bool((pad == -7.0).all())
    lists = b.band_lists()
    expect_ts = 0
    for i, ((dims, tile, dx, dt, gamma), p, f) in enumerate(zip(specs, phis, Fs)):
        bg = BandGrid(dims, tile, "f32")
        pd = to_dev(p)
        acc1 = torch.zeros(1, dtype=torch.int64, device=dev())
        bg.run(pd, to_dev(f), dx, dt, gamma, 25, 10, tile_steps=acc1)
        expect_ts += int(acc1.item())
        got = host(b.view(b.phi, i))
        assert got.tobytes() == host(pd).tobytes(), f"grid {i} {dims} {tile}"
        assert lists[i].tolist() == bg.band_list().numpy().tolist(), f"grid {i}"
    assert int(acc.item()) == expect_ts


def test_batch_grid_matches_oracle():
    specs, phis, Fs, _ = _specs(seed=5, count=4)
    b = Batch(specs)
    b.load(phis, Fs)
    b.run(20, 10)
    for i in (0, 3):
        dims, tile, dx, dt, gamma = specs[i]
        want = oracle.run_band(phis[i], Fs[i], dx, dt, np.float32(gamma), 20, window=10,
                               tile=tile)
        got = host(b.view(b.phi, i)).astype(np.float64)
        bound = fp32_step_bound(phis[i], Fs[i], dx, dt, 20)
        assert np.max(np.abs(got - want)) <= bound


@pytest.mark.parametrize("tile", CANDIDATES)
def test_batch_every_tile_shape_matches_oracle(tile):
    """Every tile shape the autotuner can pick, batched and alone, against the
    oracle run with the same tile shape: grids of 45^3 and 38^3 (partial tiles
    at every high face for every shape, ragged x-runs), 30 steps in windows of
    10.  Band lists of every window bit-exact, phi within the FP32 bound."""
    insts = W.ellipsoid_batch(seed=31, base=32, sizes=[45, 38])
    specs = [((it.n,) * 3, tile, it.dx, it.dt, it.gamma) for it in insts]
    assert all(it.n % t for it in insts for t in tile)  # partial tiles on every axis
    b = Batch(specs)
    b.load([it.phi for it in insts], [it.F for it in insts])
    b.run(30, 10)
    lists = b.band_lists()
    for i, it in enumerate(insts):
        print(f"batch tile {tile} grid {it.n}^3", flush=True)
        want, wl = oracle.run_band(it.phi, it.F, it.dx, it.dt, np.float32(it.gamma), 30,
                                   window=10, tile=tile, record_tiles=True)
        bound = fp32_step_bound(it.phi, it.F, it.dx, it.dt, 30)
        got = host(b.view(b.phi, i)).astype(np.float64)
        assert lists[i].tolist() == wl[-1].tolist(), f"batched grid {i}: band list"
        assert np.max(np.abs(got - want)) <= bound, f"batched grid {i}"
        # the same grid through the single-grid driver with this tile shape
        bg = BandGrid((it.n,) * 3, tile, "f32")
        pd = to_dev(it.phi)
        got_lists = []
        for w in range(3):
            bg.run(pd, to_dev(it.F), it.dx, it.dt, it.gamma, 10, 10)
            got_lists.append(bg.band_list().numpy().tolist())
        assert got_lists == [x.tolist() for x in wl], f"single grid {i}: band lists"
        single = host(pd).astype(np.float64)
        assert np.max(np.abs(single - want)) <= bound, f"single grid {i}"


def test_batch_graph_replay_matches_eager():
    specs, phis, Fs, _ = _specs(seed=8, count=6)
    b = Batch(specs)
    b.load(phis, Fs)
    phi0 = b.phi.clone()
    b.run(20, 10)
    eager = host(b.phi).copy()
    s = torch.cuda.Stream()
    b.phi.copy_(phi0)
    torch.cuda.synchronize()
    ls.ls_graph_begin(s)
    b.run(20, 10, stream=s)
    graph = ls.ls_graph_end(s)
    try:
        for rep in range(3):
            b.phi.copy_(phi0)  # eager work between the replays
            torch.cuda.synchronize()
            ls.ls_graph_launch(graph, s)
            s.synchronize()
            assert host(b.phi).tobytes() == eager.tobytes(), f"replay {rep}"
    finally:
        ls.ls_graph_destroy(graph)


def test_batch_point_steps_count_in_domain_points():
    """point_steps = steps x in-domain points of every band tile (partial
    tiles at the high faces count only their points), summed over grids."""
    specs, phis, Fs, _ = _specs(seed=13, count=7)
    b = Batch(specs)
    b.load(phis, Fs)
    ps = torch.zeros(1, dtype=torch.int64, device=dev())
    b.run(10, 10, point_steps=ps)  # one window: the band of the initial field
    want = 0
    for (dims, tile, dx, dt, gamma), p in zip(specs, phis):
        nx, ny, nz = dims
        tx, ty, tz = tile
        ntx, nty = -(-nx // tx), -(-ny // ty)
        for t in oracle.band_tiles(p, tile, np.float32(gamma), True):
            ti, tj, tk = t % ntx, (t // ntx) % nty, t // (ntx * nty)
            want += (min(tx, nx - ti * tx) * min(ty, ny - tj * ty) * min(tz, nz - tk * tz))
    assert int(ps.item()) == 10 * want


def test_native_autotuner_and_cache(tmp_path):
    """ls_autotune picks one of the compiled shapes per size bucket, writes its
    cache, and a second call answers from the cache."""
    from paper_1612_04040_amd import autotune

    path = str(tmp_path / "tune.txt")
    table = autotune.tune([40, 50, 72], path=path)
    assert set(table) == {1, 2}  # buckets of 32 points
    assert all(tuple(t) in CANDIDATES for t in table.values())
    with open(path) as fh:
        lines = [ln for ln in fh.read().splitlines() if ln.strip()]
    assert len(lines) == 2
    assert autotune.tune([40, 72], path=path) == table
    # an entry planted for this device is returned as it is, unmeasured: the
    # key read back matches the key written (architecture and CU count)
    key = lines[0].split("|")[0]
    prop = torch.cuda.get_device_properties(0)
    assert key == f"{prop.gcnArchName} {prop.multi_processor_count}cu"
    with open(path, "w") as fh:
        fh.write(f"{key}|1 32 4 4 0.0001\n{key}|2 4 4 4 0.0001\n")
    assert autotune.tune([40, 72], path=path) == {1: (32, 4, 4), 2: (4, 4, 4)}
    with open(path) as fh:  # nothing re-measured, nothing rewritten
        assert fh.read() == f"{key}|1 32 4 4 0.0001\n{key}|2 4 4 4 0.0001\n"
