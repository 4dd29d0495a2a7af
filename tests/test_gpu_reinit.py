"""Reinitialisation (Eq. 12-13), clamp (Eq. 10) and the Steps 1-3 driver on the
GPU against the FP64 oracle.

Inputs are seeded and drawn by the test; the oracle starts from the same
stored values and never sees a GPU result.

FP64 follows the oracle's operations in the oracle's order (the smoothed sign,
the upwind term, the added dtau S, the clamp), so the FP64 results are equal
in value, point for point, over many steps and whole driver runs.

FP32 bound.  One step rounds the stored value (eps/2 of the reach) and
evaluates two increments of size at most dtau (G + 1), G <= sqrt(6) D / dx
the upwind gradient norm (D the largest neighbour difference), with a few eps
each, and S with a few eps (the reciprocal square root): r = 4 (eps/2 reach +
8 eps dtau (G + 1)).  Over several steps a perturbation e of the field moves S
by at most (1 + sqrt(3)/2) e / sqrt(c^2 + q) (q = |Dd|^2 dx^2; the partial
derivatives of c (c^2 + q)^-1/2), hence the increment by dtau (G + 1) times
that; the upwind part with S fixed is non-expansive under the CFL condition.
So e_{k+1} <= (1 + L_k) e_k + r_k with L_k = dtau (G_k + 1)(1 + sqrt(3)/2) / m_k,
m_k the smallest sqrt(c^2 + q) over the updated points of the oracle's step-k
field.
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

CASES = [
    # dims, tile, niter, tile fraction, clamp
    ((13, 9, 7), (4, 3, 2), 3, 0.6, False),   # run-time-shape kernel
    ((64, 64, 64), (8, 8, 8), 1, 0.3, False),  # vectorised kernel
    ((64, 64, 64), (8, 8, 8), 6, 0.3, True),
    ((68, 45, 33), (8, 8, 8), 5, 0.5, True),   # vectorised, partial tiles in y and z
    ((67, 45, 33), (8, 8, 8), 4, 0.5, False),  # nx odd: the scalar fast kernel
    ((100, 36, 20), (16, 4, 4), 3, 0.4, True),
    ((40, 40, 40), (32, 4, 4), 2, 0.5, False),
]


def _field(rng, dims, dtype):
    """A union of spheres with its gradient scaled by 1.5 and noise: not a
    distance function, so the reinitialisation moves every value."""
    nx, ny, nz = dims
    dx = 1.0 / max(dims)
    centers = rng.uniform(0.2, 0.8, size=(3, 3)) * np.array([nx, ny, nz]) * dx
    phi = W.sphere_union((nz, ny, nx), dx, centers, rng.uniform(0.1, 0.3, 3) * max(dims) * dx)
    phi = 1.5 * phi + rng.uniform(-0.2, 0.2, phi.shape) * dx
    return phi.astype(dtype), dx


def _gpu_reinit(precision, dims, tile, phi, dx, dtau, gamma, tiles, niter, scale=None):
    bg = BandGrid(dims, tile, precision)
    t = torch.zeros(bg.capacity, dtype=torch.int32, device=dev())
    t[: tiles.size] = torch.from_numpy(tiles).to(dev())
    n = torch.tensor([tiles.size], dtype=torch.int32, device=dev())
    pd = to_dev(phi)
    bg.reinit(pd, dx, dtau, niter, gamma=gamma, scale=scale, tiles=t, ntiles=n)
    return host(pd)


def _stats(p, dx, mask):
    """(largest neighbour difference, smallest sqrt(c^2 + q) over mask, max|p|)."""
    dmax = max(float(np.abs(np.diff(p, axis=a)).max()) if p.shape[a] > 1 else 0.0
               for a in range(3))
    q = np.zeros_like(p)
    for axis in range(3):
        n = p.shape[axis]
        up = np.take(p, np.minimum(np.arange(n) + 1, n - 1), axis=axis)
        dn = np.take(p, np.maximum(np.arange(n) - 1, 0), axis=axis)
        q += 0.25 * (up - dn) ** 2
    m = np.sqrt(p ** 2 + q)[mask & (p != 0)]
    return dmax, float(m.min()) if m.size else 1.0, float(np.abs(p).max())


def _fp32_bound(phi, dx, dtau, tiles, niter, tile, gamma):
    """The oracle's result after niter steps and the FP32 bound (module doc)."""
    nz, ny, nx = phi.shape
    mask = oracle.tile_mask((nx, ny, nz), tiles, tile)
    p = np.asarray(phi, dtype=np.float64)
    e = 0.0
    for k in range(niter):
        dmax, mmin, pmax = _stats(p, dx, mask)
        g = math.sqrt(6) * (dmax + 2 * e) / dx
        lip = dtau * (g + 1) * (1 + math.sqrt(3) / 2) / max(mmin - 2 * e, 1e-300)
        r = 4 * (0.5 * EPS32 * (pmax + dtau * (g + 1) + e) + 8 * EPS32 * dtau * (g + 1))
        e = (1 + lip) * e + r
        last = k == niter - 1
        p = oracle.reinit_steps(p, dx, dtau, tiles, 1, tile, gamma=gamma if last else None)
    return p, e


@pytest.mark.parametrize("dims,tile,niter,frac,clamp", CASES)
def test_reinit_f64_equals_oracle(dims, tile, niter, frac, clamp):
    rng = np.random.default_rng(sum(dims) * 13 + niter)
    phi, dx = _field(rng, dims, np.float64)
    tiles = random_tiles(rng, oracle.tile_count(dims, tile), frac)
    gamma = 4 * dx if clamp else None
    got = _gpu_reinit("f64", dims, tile, phi, dx, 0.5 * dx, gamma, tiles, niter)
    want = oracle.reinit_steps(phi, dx, 0.5 * dx, tiles, niter, tile, gamma=gamma)
    err = float(np.max(np.abs(got - want)))
    assert np.array_equal(got, want), err
    assert np.max(np.abs(want - phi)) > 0.1 * dx  # the steps moved values


@pytest.mark.parametrize("dims,tile,niter,frac,clamp", [c for c in CASES if c[2] <= 4])
def test_reinit_f32_parity(dims, tile, niter, frac, clamp):
    rng = np.random.default_rng(sum(dims) * 7 + niter)
    phi, dx = _field(rng, dims, np.float32)
    tiles = random_tiles(rng, oracle.tile_count(dims, tile), frac)
    gamma = float(np.float32(4 * dx)) if clamp else None
    dtau = float(np.float32(0.5 * dx))
    got = _gpu_reinit("f32", dims, tile, phi, dx, dtau, gamma, tiles, niter)
    want, bound = _fp32_bound(phi, dx, dtau, tiles, niter, tile, gamma)
    err = np.abs(got.astype(np.float64) - want)
    assert err.max() <= bound, (err.max(), bound)
    assert np.abs(want - phi).max() > 20 * bound  # the check is not vacuous
    out = ~oracle.tile_mask(dims, tiles, tile)
    assert got[out].tobytes() == phi[out].tobytes()
    if clamp:
        assert np.all(np.abs(got[~out]) <= np.float32(gamma))


def test_reinit_f16s_parity():
    """Scaled FP16 storage, one step: the FP32 bound plus half an FP16 ulp of
    the reach (the store)."""
    rng = np.random.default_rng(41)
    dims = (72, 40, 36)
    phi, dx = _field(rng, dims, np.float32)
    s = np.float32(0.25 * dx)
    h = W.quantize_f16s(phi, s)
    phi0 = oracle.dequant_f16s(h, s)
    tiles = random_tiles(rng, oracle.tile_count(dims, (8, 8, 8)), 0.5)
    dtau = float(np.float32(0.5 * dx))
    got = oracle.dequant_f16s(
        _gpu_reinit("f16s", dims, (8, 8, 8), h, dx, dtau, None, tiles, 1, scale=float(s)), s)
    want, bound = _fp32_bound(phi0, dx, dtau, tiles, 1, (8, 8, 8), None)
    reach = float(np.abs(want).max()) / float(s)
    bound += 2.0 ** (math.floor(math.log2(reach)) - 11) * float(s)
    err = np.abs(got.astype(np.float64) - want).max()
    assert err <= bound, (err, bound)


def test_driver_f64_equals_oracle_driver():
    """ls_band_run_reinit_f64 (Steps 1-3 in windows of 10 steps: band, cut-off
    steps, 24 reinitialisation steps, clamp) against the oracle's driver:
    band lists and values equal, on an expanding/shrinking union of spheres."""
    n = 64
    rng = np.random.default_rng(5)
    dx = 1.0 / n
    centers = rng.uniform(0.3, 0.7, size=(3, 3))
    phi = W.sphere_union((n, n, n), dx, centers, rng.uniform(0.1, 0.2, 3))
    F = rng.uniform(-1, 1, (n, n, n))
    dt = 0.5 * dx / float(np.max(np.abs(F)))
    beta, gamma, dtau = 3 * dx, 6 * dx, 0.5 * dx
    bg = BandGrid((n, n, n), (8, 8, 8), "f64")
    pd, fd = to_dev(phi), to_dev(F)
    acc = torch.zeros(1, dtype=torch.int64, device=dev())
    bg.run(pd, fd, dx, dt, gamma, 30, 10, tile_steps=acc, beta=beta, reinit=(dtau, 24))
    got = host(pd)
    want, lists = oracle.run_band(phi, F, dx, dt, gamma, 30, window=10, precision="f64",
                                  record_tiles=True, beta=beta, reinit=(dtau, 24))
    assert bg.band_list().numpy().tolist() == lists[-1].tolist()
    assert int(acc.item()) == sum(int(x.size) for x in lists) * 10
    err = float(np.max(np.abs(got - want)))
    report("reinit_driver_f64_64", max_err=err)
    assert np.array_equal(got, want), err


def test_driver_f32_equals_its_steps():
    """The one-call FP32 driver equals build + cut-off steps + reinitialisation
    with clamp, window by window, bit for bit; and with no reinitialisation
    steps it is the cut-off driver."""
    n = 96
    rng = np.random.default_rng(6)
    dx = 1.0 / n
    centers = rng.uniform(0.3, 0.7, size=(3, 3))
    phi = W.sphere_union((n, n, n), dx, centers, rng.uniform(0.1, 0.2, 3)).astype(np.float32)
    F = (0.5 * np.sin(7 * np.arange(n ** 3)).reshape(n, n, n)).astype(np.float32)
    dt = float(np.float32(dx))
    beta, gamma, dtau = float(np.float32(3 * dx)), float(np.float32(6 * dx)), float(np.float32(0.5 * dx))
    bg = BandGrid((n, n, n), (8, 8, 8), "f32")
    fd = to_dev(F)
    p1 = to_dev(phi)
    bg.run(p1, fd, dx, dt, gamma, 30, 10, beta=beta, reinit=(dtau, 24))
    p2 = to_dev(phi)
    for _ in range(3):
        bg.build(p2, gamma, dilate=True)
        bg.step(p2, fd, dx, dt, 10, cutoff=(beta, gamma))
        bg.reinit(p2, dx, dtau, 24, gamma=gamma)
    assert host(p1).tobytes() == host(p2).tobytes()
    p3, p4 = to_dev(phi), to_dev(phi)
    bg.run(p3, fd, dx, dt, gamma, 30, 10, beta=beta, reinit=(dtau, 0))
    bg.run(p4, fd, dx, dt, gamma, 30, 10, beta=beta)
    assert host(p3).tobytes() == host(p4).tobytes()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_spheres512_reinit_full_size_window(precision):
    """The 512^3 three-sphere workload with Step 3 (beta = 3 dx, gamma = 6 dx,
    24 reinitialisation steps of dx / 2) for one window, in the bench's
    launch configuration (FP32) and in FP64.  At any size: the band list is
    the oracle's, the band values are clamped to gamma and every point outside
    the band keeps its bits.  FP64 also against the oracle on every point of
    a sampled 48^3 block: the oracle runs the window on a 128^3 crop around
    it (the crop's part of the band, zero-gradient crop faces), and the 34
    launches of the window carry no information from a crop face to the
    block, so the values are the same."""
    wl = W.three_spheres_f32(512, 10)
    dtype = np.float64 if precision == "f64" else np.float32
    g = dtype(wl.gamma)
    beta, dtau = float(dtype(3 * wl.dx)), float(dtype(0.5 * wl.dx))
    phi0 = wl.phi.astype(dtype)
    F = wl.F.astype(dtype)
    bg = BandGrid((512,) * 3, wl.tile, precision)
    pd, fd = to_dev(phi0), to_dev(F)
    bg.run(pd, fd, wl.dx, float(wl.dt), float(g), 10, 10, beta=beta, reinit=(dtau, 24))
    band = bg.band_list().numpy()
    got = host(pd)
    del pd, fd
    want_band = oracle.band_tiles(phi0, wl.tile, g, dilate=True)
    assert band.tolist() == want_band.tolist()
    m = oracle.tile_mask((512,) * 3, want_band)
    assert np.all(np.abs(got[m]) <= g)
    assert got[~m].tobytes() == phi0[~m].tobytes()
    moved = np.abs(got[m].astype(np.float64) - phi0[m]).max()
    assert moved > wl.dx
    if precision == "f32":
        report("spheres512_reinit_f32_window", band_tiles=int(band.size))
        return
    rng = np.random.default_rng(1)
    near = np.argwhere(np.abs(phi0) < 0.5 * wl.dx)
    c = near[rng.integers(len(near))]
    lo = np.clip((c - 64) // 8 * 8, 0, 512 - 128)
    crop = tuple(slice(int(a), int(a) + 128) for a in lo)
    t = np.array(want_band, dtype=np.int64)
    ti, tj, tk = t % 64, (t // 64) % 64, t // 4096
    lt = lo // 8
    keep = ((ti >= lt[2]) & (ti < lt[2] + 16) & (tj >= lt[1]) & (tj < lt[1] + 16)
            & (tk >= lt[0]) & (tk < lt[0] + 16))
    local = ((tk[keep] - lt[0]) * 16 + (tj[keep] - lt[1])) * 16 + (ti[keep] - lt[2])
    local = np.sort(local).astype(np.int32)
    sub = oracle.cutoff_steps(phi0[crop], F[crop], wl.dx, float(wl.dt), local, 10, beta, float(g))
    sub = oracle.reinit_steps(sub, wl.dx, dtau, local, 24, gamma=float(g))
    inner = (slice(40, 88),) * 3
    a, b = got[crop][inner], sub[inner]
    err = float(np.abs(a - b).max())
    report("spheres512_reinit_f64_block", band_tiles=int(band.size), block_origin=lo.tolist(),
           max_err=err)
    assert np.array_equal(a, b), err


def test_driver_f16s_equals_its_steps():
    """Scaled FP16 storage: the cut-off driver and the Steps 1-3 driver equal
    build + cut-off steps (+ reinitialisation with clamp), window by window,
    bit for bit."""
    n = 64
    rng = np.random.default_rng(8)
    dx = 1.0 / n
    centers = rng.uniform(0.3, 0.7, size=(3, 3))
    phi = W.sphere_union((n, n, n), dx, centers, rng.uniform(0.1, 0.2, 3))
    s = float(np.float32(6 * dx))
    h = W.quantize_f16s(phi, s)
    F = rng.uniform(-1, 1, (n, n, n)).astype(np.float32)
    dt = float(np.float32(0.5 * dx))
    beta, gamma, dtau = float(np.float32(3 * dx)), float(np.float32(6 * dx)), float(np.float32(0.5 * dx))
    bg = BandGrid((n, n, n), (8, 8, 8), "f16s")
    fd = to_dev(F)
    for reinit in (None, (dtau, 6)):
        a = torch.from_numpy(h.copy()).to(dev())
        bg.run(a, fd, dx, dt, gamma, 20, 10, scale=s, beta=beta, reinit=reinit)
        b = torch.from_numpy(h.copy()).to(dev())
        for _ in range(2):
            bg.build(b, gamma, dilate=True, scale=s)
            bg.step(b, fd, dx, dt, 10, scale=s, cutoff=(beta, gamma))
            if reinit is not None:
                bg.reinit(b, dx, dtau, 6, gamma=gamma, scale=s)
        assert host(a).tobytes() == host(b).tobytes(), reinit
        assert not np.array_equal(host(a), h)


def test_empty_band_changes_nothing():
    """An empty band list: the cut-off steps, the reinitialisation steps (with
    the clamp) and the gather leave every byte as it was."""
    rng = np.random.default_rng(12)
    dims = (40, 32, 24)
    phi, dx = _field(rng, dims, np.float32)
    bg = BandGrid(dims, (8, 8, 8), "f32")
    bg.ntiles.zero_()
    pd = to_dev(phi)
    F = to_dev(rng.uniform(-1, 1, phi.shape).astype(np.float32))
    bg.step(pd, F, dx, 0.5 * dx, 3, cutoff=(3 * dx, 6 * dx))
    bg.reinit(pd, dx, 0.5 * dx, 4, gamma=2 * dx)
    assert host(pd).tobytes() == phi.tobytes()
    out = torch.full((bg.capacity * 512,), 3.0, device=dev())
    ids = torch.full((bg.capacity,), -2, dtype=torch.int32, device=dev())
    bg.gather(pd, out, ids=ids)
    assert np.all(host(out) == 3.0) and np.all(host(ids) == -2)
