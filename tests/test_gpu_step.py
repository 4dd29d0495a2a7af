"""Band step on the GPU vs the FP64 oracle.

The same seeded inputs and the same tile list go to both sides (the list is
drawn by the test, not taken from either side).  FP32 agrees within the
rounding bound of ``gpu_util.fp32_step_bound``; FP64 agrees to a few ulp;
points with F = 0 and points outside the listed tiles keep their bits.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, fp32_step_bound, host, random_tiles, to_dev
from paper_1612_04040_amd import workloads as W
from paper_1612_04040_amd.band import BandGrid

pytestmark = pytest.mark.gpu

CASES = [
    # dims, tile, nsteps, tile fraction
    ((1, 1, 1), (8, 8, 8), 3, 1.0),
    ((5, 3, 2), (4, 3, 2), 2, 1.0),
    ((13, 9, 7), (4, 3, 2), 3, 0.6),
    ((64, 64, 64), (8, 8, 8), 10, 0.3),
    ((67, 45, 33), (8, 8, 8), 7, 0.5),
    ((100, 36, 20), (16, 4, 4), 4, 0.4),
    ((40, 40, 40), (32, 4, 4), 5, 0.5),
    ((48, 32, 24), (8, 8, 8), 1, 1.0),
]


def _inputs(rng, dims, dtype):
    nx, ny, nz = dims
    dx = 1.0 / max(dims)
    centers = rng.uniform(0.2, 0.8, size=(3, 3)) * np.array([nx, ny, nz]) * dx
    phi = W.sphere_union((nz, ny, nx), dx, centers, rng.uniform(0.1, 0.3, 3) * max(dims) * dx)
    phi += rng.uniform(-0.2, 0.2, phi.shape) * dx  # not an exact SDF
    F = rng.uniform(-1, 1, phi.shape)
    F[rng.random(phi.shape) < 0.1] = 0.0
    F[rng.random(phi.shape) < 0.05] = -0.0
    dt = 0.5 * dx / np.max(np.abs(F))
    return phi.astype(dtype), F.astype(dtype), dx, float(dtype(dt))


def _run_gpu(precision, dims, tile, phi, F, dx, dt, tiles, nsteps):
    bg = BandGrid(dims, tile, precision)
    t = torch.zeros(bg.capacity, dtype=torch.int32, device=dev())
    t[: tiles.size] = torch.from_numpy(tiles).to(dev())
    n = torch.tensor([tiles.size], dtype=torch.int32, device=dev())
    pd, fd = to_dev(phi), to_dev(F)
    bg.step(pd, fd, dx, dt, nsteps, tiles=t, ntiles=n)
    return host(pd)


def _outside_mask(dims, tile, tiles):
    nx, ny, nz = dims
    tx, ty, tz = tile
    ntx, nty = -(-nx // tx), -(-ny // ty)
    inside = np.zeros((nz, ny, nx), dtype=bool)
    for t in tiles:
        ti, tj, tk = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        inside[tk * tz:(tk + 1) * tz, tj * ty:(tj + 1) * ty, ti * tx:(ti + 1) * tx] = True
    return ~inside


@pytest.mark.parametrize("dims,tile,nsteps,frac", CASES)
def test_step_f32_parity(dims, tile, nsteps, frac):
    rng = np.random.default_rng(abs(hash((dims, tile, nsteps))) % 2**32)
    phi, F, dx, dt = _inputs(rng, dims, np.float32)
    tiles = random_tiles(rng, oracle.tile_count(dims, tile), frac)
    got = _run_gpu("f32", dims, tile, phi, F, dx, dt, tiles, nsteps)
    want = oracle.upwind_steps(phi, F, dx, dt, tiles, nsteps, tile)
    bound = fp32_step_bound(phi, F, dx, dt, nsteps)
    err = np.abs(got.astype(np.float64) - want)
    assert err.max() <= bound, (err.max(), bound)
    out = _outside_mask(dims, tile, tiles)
    assert np.array_equal(got[out].view(np.uint32), phi[out].view(np.uint32))


@pytest.mark.parametrize("dims,tile,nsteps,frac", CASES[2:6])
def test_step_f64_parity(dims, tile, nsteps, frac):
    rng = np.random.default_rng(abs(hash((dims, nsteps))) % 2**32)
    phi, F, dx, dt = _inputs(rng, dims, np.float64)
    tiles = random_tiles(rng, oracle.tile_count(dims, tile), frac)
    got = _run_gpu("f64", dims, tile, phi, F, dx, dt, tiles, nsteps)
    want = oracle.upwind_steps(phi, F, dx, dt, tiles, nsteps, tile)
    scale = np.max(np.abs(phi)) + 1.0
    assert np.max(np.abs(got - want)) <= 8 * nsteps * np.finfo(np.float64).eps * scale


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_zero_speed_bitwise(precision):
    dtype = np.float32 if precision == "f32" else np.float64
    rng = np.random.default_rng(4)
    dims = (37, 21, 18)
    phi = rng.standard_normal((18, 21, 37)).astype(dtype)
    phi.flat[::9] = 0.0
    phi.flat[1::9] = -0.0
    phi.flat[2::13] = np.finfo(dtype).tiny / 4  # subnormal
    F = np.zeros_like(phi)
    F.flat[::2] = -0.0
    tiles = np.arange(oracle.tile_count(dims, (8, 8, 8)), dtype=np.int32)
    for nsteps in (1, 4):
        got = _run_gpu(precision, dims, (8, 8, 8), phi, F, 0.1, 0.05, tiles, nsteps)
        assert got.tobytes() == phi.tobytes()


def test_zero_speed_bitwise_f16s():
    rng = np.random.default_rng(5)
    dims = (40, 24, 16)
    s = np.float32(0.1)
    h = (rng.standard_normal((16, 24, 40)) * 3).astype(np.float16)
    h.flat[::7] = np.float16(-0.0)
    F = np.zeros(h.shape, dtype=np.float32)
    bg = BandGrid(dims, (8, 8, 8), "f16s")
    bg.build(torch.from_numpy(h).to(dev()), float("inf"), dilate=False, scale=float(s))
    hd = torch.from_numpy(h).to(dev())
    bg.step(hd, to_dev(F), 0.1, 0.05, 3, scale=float(s))
    assert host(hd).tobytes() == h.tobytes()


def test_empty_band_changes_nothing():
    rng = np.random.default_rng(6)
    dims = (24, 24, 24)
    phi, F, dx, dt = _inputs(rng, dims, np.float32)
    bg = BandGrid(dims, (8, 8, 8), "f32")
    bg.ntiles.zero_()
    pd = to_dev(phi)
    bg.step(pd, to_dev(F), dx, dt, 5)
    assert host(pd).tobytes() == phi.tobytes()


def test_step_is_deterministic_and_odd_even_consistent():
    """Same call twice -> same bits; 3 + 4 steps == 7 steps (copy-back path)."""
    rng = np.random.default_rng(8)
    dims = (72, 56, 40)
    phi, F, dx, dt = _inputs(rng, dims, np.float32)
    tiles = random_tiles(rng, oracle.tile_count(dims, (8, 8, 8)), 0.5)
    a = _run_gpu("f32", dims, (8, 8, 8), phi, F, dx, dt, tiles, 7)
    b = _run_gpu("f32", dims, (8, 8, 8), phi, F, dx, dt, tiles, 7)
    assert a.tobytes() == b.tobytes()
    mid = _run_gpu("f32", dims, (8, 8, 8), phi, F, dx, dt, tiles, 3)
    c = _run_gpu("f32", dims, (8, 8, 8), mid, F, dx, dt, tiles, 4)
    assert a.tobytes() == c.tobytes()


def test_plane_front_exact_on_gpu():
    """Closed form: a plane advances by dt*F*|g| per step (FP32 rounding only)."""
    n = 64
    dx = 1.0 / n
    dt = 0.5 * dx
    phi = W.plane((n, n, n), dx, (0.48, -0.6, 0.64), 0.3).astype(np.float32)
    F = np.full(phi.shape, 0.8, dtype=np.float32)
    tiles = np.arange(oracle.tile_count((n, n, n), (8, 8, 8)), dtype=np.int32)
    steps = 6
    got = _run_gpu("f32", (n, n, n), (8, 8, 8), phi, F, dx, np.float32(dt), tiles, steps)
    expect = phi.astype(np.float64) - steps * 0.8 * float(np.float32(dt))
    inner = (slice(steps + 1, -steps - 1),) * 3
    bound = fp32_step_bound(phi, F, dx, float(np.float32(dt)), steps)
    assert np.max(np.abs(got[inner] - expect[inner])) <= bound


@pytest.mark.parametrize("dims", [(96, 100, 92), (64, 64, 64), (128, 72, 80)])
@pytest.mark.parametrize("run_width", [32, 64])
def test_vector_and_scalar_kernels_agree_bitwise(dims, run_width):
    """The vectorised FP32 step (16-byte rows) and the scalar fast step give
    the same bits, also with partial tiles at the high y/z faces and both run
    widths; both stay within the FP32 bound of the oracle."""
    from paper_1612_04040_amd import ls

    rng = np.random.default_rng(sum(dims) + run_width)
    nx, ny, nz = dims
    phi = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
    F = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
    F[rng.random(F.shape) < 0.05] = 0.0
    dx = 1.0 / nx
    dt = float(np.float32(W.stable_dt(F, dx)))
    tile = (8, 8, 8)
    ntiles = -(-nx // 8) * -(-ny // 8) * -(-nz // 8)
    tiles = random_tiles(rng, ntiles, 0.4)
    out = {}
    try:
        for vec in (0, 1):
            ls.ls_set_tuning(run_width, 0, 0, vec)
            bg = BandGrid(dims, tile, "f32")
            pd = to_dev(phi)
            bg.step(pd, to_dev(F), dx, dt, 3, tiles=to_dev(tiles),
                    ntiles=to_dev(np.array([tiles.size], np.int32)))
            out[vec] = host(pd)
    finally:
        ls.ls_set_tuning(0, 0, 0, 0)
    assert out[0].tobytes() == out[1].tobytes()
    want = oracle.upwind_steps(phi.astype(np.float64), F, dx, dt, tiles, 3, tile)
    assert np.max(np.abs(out[0] - want)) <= fp32_step_bound(phi, F, dx, dt, 3)


@pytest.mark.parametrize("dims", [(96, 100, 92), (128, 72, 80)])
@pytest.mark.parametrize("run_width", [32, 64])
def test_vector_and_scalar_kernels_agree_bitwise_f16s(dims, run_width):
    """Scaled-FP16 storage: the vectorised step (8-byte rows of four halves)
    and the scalar fast step give the same bits, F = 0 points keep theirs, and
    both stay within the FP16 storage bound of the FP64 oracle run on the
    dequantised input."""
    from paper_1612_04040_amd import ls

    rng = np.random.default_rng(sum(dims) + 7 * run_width)
    nx, ny, nz = dims
    s = np.float32(0.05)
    h = (rng.uniform(-1, 1, (nz, ny, nx)) / float(s)).astype(np.float16)
    h.flat[::11] = np.float16(-0.0)
    F = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
    zero = rng.random(F.shape) < 0.05
    F[zero] = 0.0
    phi = oracle.dequant_f16s(h, s)
    dx = 1.0 / nx
    dt = float(np.float32(W.stable_dt(F, dx)))
    tile = (8, 8, 8)
    ntiles = -(-nx // 8) * -(-ny // 8) * -(-nz // 8)
    tiles = random_tiles(rng, ntiles, 0.4)
    steps = 3
    out = {}
    try:
        for vec in (0, 1):
            ls.ls_set_tuning(run_width, 0, 0, vec)
            bg = BandGrid(dims, tile, "f16s")
            hd = torch.from_numpy(h.copy()).to(dev())
            bg.step(hd, to_dev(F), dx, dt, steps, scale=float(s), tiles=to_dev(tiles),
                    ntiles=to_dev(np.array([tiles.size], np.int32)))
            out[vec] = host(hd)
    finally:
        ls.ls_set_tuning(0, 0, 0, 0)
    assert out[0].tobytes() == out[1].tobytes()
    assert out[0][zero].tobytes() == h[zero].tobytes()
    want = oracle.upwind_steps(phi.astype(np.float64), F, dx, dt, tiles, steps, tile)
    got = oracle.dequant_f16s(out[0], s).astype(np.float64)
    # one FP16 store rounding per step (half an ulp of the largest |phi|/s
    # reached, times s) on top of the FP32 arithmetic bound; non-expansive
    reach = max(float(np.abs(want).max()), float(np.abs(got).max())) / float(s)
    half_ulp = 2.0 ** (np.floor(np.log2(reach)) - 11)
    bound = steps * half_ulp * float(s) + fp32_step_bound(phi, F, dx, dt, steps)
    assert np.max(np.abs(got - want)) <= bound


@pytest.mark.parametrize("precision", ["f32", "f16s"])
@pytest.mark.parametrize("dims", [(100, 64, 72), (128, 72, 80), (64, 64, 64)])
@pytest.mark.parametrize("run_width", [32, 64])
def test_two_step_launches_equal_one_step_launches(precision, dims, run_width):
    """Two steps per launch (temporal blocking, a tuning option on grids of
    whole y/z tiles) against one step per launch: the same bits after 1, 2, 3 and 6
    steps, on random band lists (tiles at every face of the grid, holes, a
    ragged x tile), with F = 0 points; and within the rounding bound of the
    FP64 oracle (FP32)."""
    from paper_1612_04040_amd import ls

    rng = np.random.default_rng(sum(dims) + run_width + (7 if precision == "f16s" else 0))
    nx, ny, nz = dims
    F = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
    F[rng.random(F.shape) < 0.05] = 0.0
    dx = 1.0 / nx
    dt = float(np.float32(W.stable_dt(F, dx)))
    s = np.float32(0.05)
    if precision == "f32":
        phi = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
    else:
        phi = (rng.uniform(-1, 1, (nz, ny, nx)) / float(s)).astype(np.float16)
    tile = (8, 8, 8)
    ntiles = -(-nx // 8) * -(-ny // 8) * -(-nz // 8)
    tiles = random_tiles(rng, ntiles, 0.5)
    for steps in (1, 2, 3, 6):
        out = {}
        try:
            for temporal in (0, 1):
                ls.ls_set_tuning(run_width, 0, 0, 0, temporal)
                bg = BandGrid(dims, tile, precision)
                pd = torch.from_numpy(phi.copy()).to(dev())
                bg.step(pd, to_dev(F), dx, dt, steps, scale=float(s) if precision == "f16s" else None,
                        tiles=to_dev(tiles), ntiles=to_dev(np.array([tiles.size], np.int32)))
                out[temporal] = host(pd)
        finally:
            ls.ls_set_tuning(0, 0, 0, 0, 0)
        assert out[0].tobytes() == out[1].tobytes(), f"{steps} steps"
    if precision == "f32":
        want = oracle.upwind_steps(phi.astype(np.float64), F, dx, dt, tiles, 6, tile)
        assert np.max(np.abs(out[0] - want)) <= fp32_step_bound(phi, F, dx, dt, 6)
