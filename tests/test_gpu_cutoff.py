"""The cut-off step and driver (Eq. 8) on the GPU against the FP64 oracle.

Inputs are seeded and drawn by the test; the oracle starts from the same
stored values and never sees a GPU result.

Error bound of n steps.  One cut-off step is the plain step with the speed
c(phi^n) F, 0 <= c <= 1, so the plain step's rounding bound holds for it.  A
perturbation d of the step-n field changes the centre's c by at most
1.5 / (gamma - beta) |d| (c is the smoothstep 3u^2 - 2u^3 of
u = (gamma - |phi|) / (gamma - beta), whose slope is at most 3/2), hence the
increment by at most dt max|F| G 1.5 / (gamma - beta) |d|, with G the upwind
gradient norm, at most sqrt(6) D / dx for D the largest difference of
neighbouring values.  So e_{n+1} <= (1 + L_n) e_n + r_n with
L_n = 1.5 sqrt(6) dt max|F| (D_n + 2 e_n) / ((gamma - beta) dx), D_n taken
from the oracle's step-n field, and r_n the one-step rounding: FP32
4 (eps/2 reach + 8 eps incr) with incr = sqrt(6) dt max|F| (D_n + 2 e_n) / dx
(the FP32 evaluation of c adds a few eps of the increment, inside the factor
8); scaled FP16 adds half an FP16 ulp of the reach per step; FP64 8 eps
(max|phi| + 1).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_util import EPS32, dev, host, random_tiles, report, to_dev
from paper_1612_04040_amd import workloads as W
from paper_1612_04040_amd.band import BandGrid

pytestmark = pytest.mark.gpu

EPS64 = float(np.finfo(np.float64).eps)

CASES = [
    # dims, tile, nsteps, tile fraction
    ((13, 9, 7), (4, 3, 2), 3, 0.6),      # run-time-shape kernel
    ((64, 64, 64), (8, 8, 8), 1, 0.3),    # vectorised kernel, one step
    ((64, 64, 64), (8, 8, 8), 6, 0.3),
    ((68, 45, 33), (8, 8, 8), 4, 0.5),    # vectorised, partial tiles in y and z
    ((67, 45, 33), (8, 8, 8), 4, 0.5),    # nx odd: the scalar fast kernel
    ((100, 36, 20), (16, 4, 4), 3, 0.4),
    ((40, 40, 40), (32, 4, 4), 2, 0.5),
]


def _inputs(rng, dims, dtype):
    nx, ny, nz = dims
    dx = 1.0 / max(dims)
    centers = rng.uniform(0.2, 0.8, size=(3, 3)) * np.array([nx, ny, nz]) * dx
    phi = W.sphere_union((nz, ny, nx), dx, centers, rng.uniform(0.1, 0.3, 3) * max(dims) * dx)
    phi += rng.uniform(-0.2, 0.2, phi.shape) * dx
    F = rng.uniform(-1, 1, phi.shape)
    F[rng.random(phi.shape) < 0.1] = 0.0
    dt = 0.5 * dx / np.max(np.abs(F))
    return phi.astype(dtype), F.astype(dtype), dx, float(dtype(dt))


def _max_neighbour_diff(p):
    return max(float(np.abs(np.diff(p, axis=a)).max()) if p.shape[a] > 1 else 0.0
               for a in range(3))


def _oracle_run(phi, F, dx, dt, tiles, nsteps, beta, gamma, tile):
    """The oracle's cut-off steps one at a time: the final field and, for
    steps 0..nsteps-1, (largest neighbour difference, max |phi|)."""
    p = np.asarray(phi, dtype=np.float64)
    stats = []
    for _ in range(nsteps):
        stats.append((_max_neighbour_diff(p), float(np.max(np.abs(p)))))
        p = oracle.cutoff_steps(p, F, dx, dt, tiles, 1, beta, gamma, tile)
    return p, stats


def _bound(stats, F, dx, dt, beta, gamma, kind, scale=None):
    fmax = float(np.max(np.abs(F)))
    e = 0.0
    for dmax, pmax in stats:
        d = dmax + 2 * e
        lip = 1.5 * math.sqrt(6) * dt * fmax * d / ((gamma - beta) * dx)
        incr = math.sqrt(6) * dt * fmax * d / dx
        reach = pmax + incr + e
        if kind == "f64":
            r = 8 * EPS64 * (pmax + 1.0)
        else:
            r = 4 * (0.5 * EPS32 * reach + 8 * EPS32 * incr)
            if kind == "f16s":
                r += 2.0 ** (math.floor(math.log2(reach / scale)) - 11) * scale
        e = (1 + lip) * e + r
    return e


def _run_gpu(precision, dims, tile, phi, F, dx, dt, tiles, nsteps, cut, scale=None):
    bg = BandGrid(dims, tile, precision)
    t = torch.zeros(bg.capacity, dtype=torch.int32, device=dev())
    t[: tiles.size] = torch.from_numpy(tiles).to(dev())
    n = torch.tensor([tiles.size], dtype=torch.int32, device=dev())
    pd, fd = to_dev(phi), to_dev(F)
    bg.step(pd, fd, dx, dt, nsteps, scale=scale, tiles=t, ntiles=n, cutoff=cut)
    return host(pd)


@pytest.mark.parametrize("dims,tile,nsteps,frac", CASES)
def test_cutoff_step_f32_parity(dims, tile, nsteps, frac):
    rng = np.random.default_rng(sum(dims) * 31 + nsteps)
    phi, F, dx, dt = _inputs(rng, dims, np.float32)
    tiles = random_tiles(rng, oracle.tile_count(dims, tile), frac)
    beta, gamma = float(np.float32(3 * dx)), float(np.float32(6 * dx))
    got = _run_gpu("f32", dims, tile, phi, F, dx, dt, tiles, nsteps, (beta, gamma))
    want, stats = _oracle_run(phi, F, dx, dt, tiles, nsteps, beta, gamma, tile)
    bound = _bound(stats, F, dx, dt, beta, gamma, "f32")
    err = np.abs(got.astype(np.float64) - want)
    assert err.max() <= bound, (err.max(), bound)
    # the cut-off acted: the plain steps land far outside the bound
    plain = oracle.upwind_steps(phi, F, dx, dt, tiles, nsteps, tile)
    assert np.abs(plain - want).max() > 100 * bound
    # |phi| >= gamma never moves (c = 0 there, and the value stays put)
    far = np.abs(phi) >= np.float32(gamma)
    assert got[far].tobytes() == phi[far].tobytes()


@pytest.mark.parametrize("dims,tile,nsteps,frac", [CASES[0], CASES[3], CASES[5]])
def test_cutoff_step_f64_parity(dims, tile, nsteps, frac):
    rng = np.random.default_rng(sum(dims) * 17 + nsteps)
    phi, F, dx, dt = _inputs(rng, dims, np.float64)
    tiles = random_tiles(rng, oracle.tile_count(dims, tile), frac)
    beta, gamma = 3 * dx, 6 * dx
    got = _run_gpu("f64", dims, tile, phi, F, dx, dt, tiles, nsteps, (beta, gamma))
    want, stats = _oracle_run(phi, F, dx, dt, tiles, nsteps, beta, gamma, tile)
    bound = _bound(stats, F, dx, dt, beta, gamma, "f64")
    err = np.abs(got - want).max()
    assert err <= bound, (err, bound)


@pytest.mark.parametrize("dims", [(64, 64, 64), (68, 45, 33)])
def test_cutoff_step_f16s_parity(dims):
    rng = np.random.default_rng(sum(dims) + 5)
    phi, F, dx, dt = _inputs(rng, dims, np.float32)
    s = np.float32(0.25 * dx)
    h = W.quantize_f16s(phi, s)
    phi0 = oracle.dequant_f16s(h, s)
    tiles = random_tiles(rng, oracle.tile_count(dims, (8, 8, 8)), 0.5)
    beta, gamma = float(np.float32(3 * dx)), float(np.float32(6 * dx))
    nsteps = 4
    bg = BandGrid(dims, (8, 8, 8), "f16s")
    hd = torch.from_numpy(h.copy()).to(dev())
    bg.step(hd, to_dev(F), dx, dt, nsteps, scale=float(s), tiles=to_dev(tiles),
            ntiles=to_dev(np.array([tiles.size], np.int32)), cutoff=(beta, gamma))
    got = oracle.dequant_f16s(host(hd), s).astype(np.float64)
    want, stats = _oracle_run(phi0, F, dx, dt, tiles, nsteps, beta, gamma, (8, 8, 8))
    bound = _bound(stats, F, dx, dt, beta, gamma, "f16s", float(s))
    err = np.abs(got - want).max()
    assert err <= bound, (err, bound)


@pytest.mark.parametrize("precision", ["f32", "f64", "f16s"])
def test_unit_cutoff_equals_plain_step_bitwise(precision):
    """beta above every |phi|: c = 1 exactly, so the cut-off kernels give the
    plain kernels' bits."""
    rng = np.random.default_rng(9)
    dims = (72, 40, 36)
    dtype = np.float64 if precision == "f64" else np.float32
    phi, F, dx, dt = _inputs(rng, dims, dtype)
    tiles = random_tiles(rng, oracle.tile_count(dims, (8, 8, 8)), 0.6)
    scale = None
    if precision == "f16s":
        scale = float(np.float32(0.25 * dx))
        phi = W.quantize_f16s(phi, scale)
    a = _run_gpu(precision, dims, (8, 8, 8), phi, F, dx, dt, tiles, 5, (50.0, 100.0), scale)
    b = _run_gpu(precision, dims, (8, 8, 8), phi, F, dx, dt, tiles, 5, None, scale)
    assert a.tobytes() == b.tobytes()


def test_cutoff_driver_equals_oracle_driver():
    """ls_band_run_cutoff_f32 (band rebuilds every 10 steps, tube and cut-off
    with the same gamma) against the oracle's driver with the cut-off: every
    window's band list bit-exact, values within the n-step bound."""
    n = 96
    rng = np.random.default_rng(21)
    phi, F, dx, dt = _inputs(rng, (n, n, n), np.float32)
    beta, gamma = float(np.float32(3 * dx)), float(np.float32(6 * dx))
    steps, window = 30, 10
    bg = BandGrid((n, n, n), (8, 8, 8), "f32")
    pd, fd = to_dev(phi), to_dev(F)
    lists = []
    for _ in range(steps // window):  # window by window, to compare the lists
        p2 = pd.clone()
        bg.run(p2, fd, dx, dt, gamma, window, window, beta=beta)
        lists.append(bg.band_list().numpy())
        pd = p2
    got = host(pd)
    # the one-call driver gives the same bits
    p1 = to_dev(phi)
    bg.run(p1, fd, dx, dt, gamma, steps, window, beta=beta)
    assert host(p1).tobytes() == got.tobytes()

    want, ref_lists = oracle.run_band(phi, F, dx, dt, np.float32(gamma), steps, window=window,
                                      record_tiles=True, beta=beta)
    for w, (a, b) in enumerate(zip(lists, ref_lists)):
        assert a.tolist() == b.tolist(), f"band list differs at window {w}"
    p, stats = phi.astype(np.float64), []
    for w in range(steps // window):
        p, st = _oracle_run(p, F, dx, dt, ref_lists[w], window, beta, gamma, (8, 8, 8))
        stats += st
    assert p.tobytes() == want.tobytes()
    bound = _bound(stats, F, dx, dt, beta, gamma, "f32")
    err = np.abs(got.astype(np.float64) - want)
    report("cutoff_driver_96", max_err_dx=float(err.max() / dx), bound_dx=bound / dx)
    assert err.max() <= bound, (err.max(), bound)


@pytest.mark.timeout(600)
def test_spheres512_cutoff_full_size_first_window():
    """The 512^3 three-sphere workload at full size, in the launch
    configuration the bench times (8^3 tiles, 32-point rows, the vectorised
    step with the cut-off, beta = 3 dx, gamma = 6 dx): one window of 10 steps
    of the driver against the oracle's driver, on every point."""
    wl = W.three_spheres_f32(512, 10)
    g32 = np.float32(wl.gamma)
    beta = float(np.float32(3 * wl.dx))
    bg = BandGrid((512,) * 3, wl.tile, "f32")
    pd, fd = to_dev(wl.phi), to_dev(wl.F)
    bg.run(pd, fd, wl.dx, wl.dt, float(g32), 10, 10, beta=beta)
    got_list = bg.band_list().numpy()
    got = host(pd)
    del pd
    # the oracle's driver for one window: the band of phi^0 (decided in FP32),
    # then 10 cut-off steps on it
    band = oracle.band_tiles(wl.phi, wl.tile, g32, dilate=True)
    assert got_list.tolist() == band.tolist()
    want, stats = _oracle_run(wl.phi, wl.F, wl.dx, wl.dt, band, 10, beta, float(g32), wl.tile)
    bound = _bound(stats, wl.F, wl.dx, wl.dt, beta, float(g32), "f32")
    err = np.abs(got.astype(np.float64) - want)
    report("spheres512_cutoff_first_window", band_tiles=int(got_list.size),
           max_err_dx=float(err.max() / wl.dx), bound_dx=bound / wl.dx)
    assert err.max() <= bound, (err.max(), bound)
    far = np.abs(wl.phi) >= g32
    assert got[far].tobytes() == wl.phi[far].tobytes()
