"""The tile-major ("brick") layout on the GPU.

* The conversions are the permutation the layout defines (checked against a
  numpy reshape of the grid into 8^3 tiles), and they invert each other.
* The band build on bricks gives the x-fastest build's list.
* The brick driver (plain steps, the cut-off of Eq. 8, Steps 1-3 with the
  reinitialisation of Eq. 12-13 and the clamp of Eq. 10) gives the x-fastest
  driver's fields, band lists and tile-step counts bit for bit, in FP32 and
  scaled FP16, on grids whose tile rows are not a multiple of the 4-tile work
  item and with an odd step count per window (the copy-back); and it matches
  the oracle directly within the FP32 bound.
* At full size (the 512^3 three-sphere workload, 200 steps; the 1024^3 torus
  in FP32, 200 steps, and in scaled FP16, 500 steps) the brick driver equals
  the x-fastest driver bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, fp32_step_bound, host, to_dev
from paper_1612_04040_amd import ls
from paper_1612_04040_amd import workloads as W
from paper_1612_04040_amd.band import BandGrid

pytestmark = pytest.mark.gpu


def brick_order(a):
    """(nz, ny, nx) grid -> flat tile-major order (tiles in id order, x fastest inside)."""
    nz, ny, nx = a.shape
    t = a.reshape(nz // 8, 8, ny // 8, 8, nx // 8, 8).transpose(0, 2, 4, 1, 3, 5)
    return np.ascontiguousarray(t).reshape(-1)


DIMS = [(48, 40, 56), (72, 64, 80)]  # (nx, ny, nz): 6 and 9 tiles along x


@pytest.mark.parametrize("dims", DIMS)
def test_conversions_are_the_tile_major_permutation(dims):
    nx, ny, nz = dims
    rng = np.random.default_rng(sum(dims))
    a = rng.standard_normal((nz, ny, nx)).astype(np.float32)
    g = ls.grid(dims)
    src = to_dev(a)
    b = torch.empty_like(src)
    ls.ls_bricks_from_dense_f32(src, g, b)
    assert host(b).reshape(-1).tobytes() == brick_order(a).tobytes()
    back = torch.full_like(src, -9.0)
    ls.ls_bricks_to_dense_f32(b, g, back)
    assert host(back).tobytes() == a.tobytes()
    h = rng.integers(0, 1 << 16, size=(nz, ny, nx), dtype=np.uint16)
    hs = torch.from_numpy(h.view(np.float16)).to(dev())
    hb = torch.empty_like(hs)
    ls.ls_bricks_from_dense_f16s(hs, g, hb)
    assert host(hb).view(np.uint16).reshape(-1).tobytes() == brick_order(h).tobytes()
    hback = torch.zeros_like(hs)
    ls.ls_bricks_to_dense_f16s(hb, g, hback)
    assert host(hback).view(np.uint16).tobytes() == h.tobytes()


def _spheres(dims, seed):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    dx = 1.0 / max(dims)
    ext = np.array([nx, ny, nz]) * dx
    centers = rng.uniform(0.3, 0.7, size=(3, 3)) * ext
    radii = rng.uniform(0.1, 0.2, size=3) * min(ext)
    phi = W.sphere_union((nz, ny, nx), dx, centers, radii, dtype=np.float32)
    F = W.sinusoid3((nz, ny, nx), dx, amp=0.8, dtype=np.float32)
    F[rng.random(F.shape) < 0.02] = 0.0  # exact zeros keep their bits
    dt = float(np.float32(W.stable_dt(F, dx)))
    return phi, F, dx, dt, float(np.float32(6 * dx))


@pytest.mark.parametrize("precision", ["f32", "f16s"])
@pytest.mark.parametrize("dims", DIMS)
def test_brick_build_equals_build(precision, dims):
    phi, F, dx, dt, gamma = _spheres(dims, 3)
    bg = BandGrid(dims, (8, 8, 8), precision)
    scale = None
    if precision == "f32":
        pd = to_dev(phi)
    else:
        scale = float(np.float32(gamma))
        pd = torch.from_numpy(W.quantize_f16s(phi, np.float32(scale))).to(dev())
    for dil in (True, False):
        bg.build(pd, gamma, dilate=dil, scale=scale)
        want = bg.band_list().numpy().tolist()
        pb = torch.empty_like(pd)
        bg.to_bricks(pd, pb)
        bg.build_bricks(pb, gamma, dilate=dil, scale=scale)
        assert bg.band_list().numpy().tolist() == want
        assert len(want) > 0


MODES = [("plain", None, None), ("cutoff", 0.5, None), ("reinit", 0.5, 12)]


@pytest.mark.parametrize("mode,beta_dx,reinit_iters", MODES)
@pytest.mark.parametrize("precision", ["f32", "f16s"])
@pytest.mark.parametrize("dims", DIMS)
def test_brick_driver_equals_driver(dims, precision, mode, beta_dx, reinit_iters):
    """25 steps in windows of 7 (odd: the copy-back of the band after every
    window); x-fastest and tile-major drivers from the same fields."""
    phi, F, dx, dt, gamma = _spheres(dims, 11)
    beta = None if beta_dx is None else float(np.float32(beta_dx * gamma))
    reinit = None if reinit_iters is None else (float(np.float32(0.5 * dx)), reinit_iters)
    scale = None
    if precision == "f32":
        p0 = to_dev(phi)
    else:
        scale = float(np.float32(gamma))
        p0 = torch.from_numpy(W.quantize_f16s(phi, np.float32(scale))).to(dev())
    Fd = to_dev(F)
    dense = BandGrid(dims, (8, 8, 8), precision)
    bricks = BandGrid(dims, (8, 8, 8), precision)
    pd = p0.clone()
    acc_d = torch.zeros(1, dtype=torch.int64, device=dev())
    dense.run(pd, Fd, dx, dt, gamma, 25, 7, scale=scale, tile_steps=acc_d,
              beta=beta if (beta is not None or reinit is None) else None, reinit=reinit)
    pb = torch.empty_like(p0)
    bricks.to_bricks(p0, pb)
    Fb = torch.empty_like(Fd)
    bricks.to_bricks(Fd, Fb)
    acc_b = torch.zeros(1, dtype=torch.int64, device=dev())
    bricks.run_bricks(pb, Fb, dx, dt, gamma, 25, 7, scale=scale, tile_steps=acc_b, beta=beta,
                      reinit=reinit)
    out = torch.empty_like(p0)
    bricks.from_bricks(pb, out)
    assert host(out).tobytes() == host(pd).tobytes()
    assert bricks.band_list().numpy().tolist() == dense.band_list().numpy().tolist()
    assert int(acc_b.item()) == int(acc_d.item()) > 0


@pytest.mark.parametrize("dims", DIMS)
def test_brick_driver_matches_oracle(dims):
    phi, F, dx, dt, gamma = _spheres(dims, 21)
    bg = BandGrid(dims, (8, 8, 8), "f32")
    pb, Fb = torch.empty_like(to_dev(phi)), torch.empty_like(to_dev(F))
    bg.to_bricks(to_dev(phi), pb)
    bg.to_bricks(to_dev(F), Fb)
    bg.run_bricks(pb, Fb, dx, dt, gamma, 30, 10)
    got = torch.empty_like(pb)
    bg.from_bricks(pb, got)
    want, lists = oracle.run_band(phi, F, dx, dt, np.float32(gamma), 30, window=10,
                                  record_tiles=True)
    assert bg.band_list().numpy().tolist() == lists[-1].tolist()
    err = np.abs(host(got).astype(np.float64) - want)
    assert err.max() <= fp32_step_bound(phi, F, dx, dt, 30)


@pytest.mark.timeout(600)
def test_brick_driver_512_equals_driver():
    """The bench workload at full size: 512^3 three spheres, 200 steps."""
    n = 512
    wl = W.three_spheres_f32(n, 200)
    g32 = float(np.float32(wl.gamma))
    bg = BandGrid((n,) * 3, wl.tile, "f32")
    p0, Fd = to_dev(wl.phi), to_dev(wl.F)
    pd = p0.clone()
    acc_d = torch.zeros(1, dtype=torch.int64, device=dev())
    bg.run(pd, Fd, wl.dx, wl.dt, g32, 200, 10, tile_steps=acc_d)
    want = host(pd)
    want_list = bg.band_list().numpy().tolist()
    del pd
    pb, Fb = torch.empty_like(p0), torch.empty_like(Fd)
    bg.to_bricks(p0, pb)
    bg.to_bricks(Fd, Fb)
    acc_b = torch.zeros(1, dtype=torch.int64, device=dev())
    bg.run_bricks(pb, Fb, wl.dx, wl.dt, g32, 200, 10, tile_steps=acc_b)
    bg.from_bricks(pb, p0)
    assert host(p0).tobytes() == want.tobytes()
    assert bg.band_list().numpy().tolist() == want_list
    assert int(acc_b.item()) == int(acc_d.item())


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,steps", [("f32", 200), ("f16s", 500)])
def test_brick_driver_1024_torus_equals_driver(precision, steps):
    """The 1024^3 torus workloads at full size, as the bench runs them (FP32:
    200 steps, two steps per launch; scaled FP16: 500 steps, one step per
    launch): the brick driver equals the x-fastest driver bit for bit, band
    list and tile-step count included."""
    n = 1024
    wl = W.torus_grf(n, steps)
    g32 = float(np.float32(wl.gamma))
    scale = None
    if precision == "f32":
        p0 = to_dev(wl.phi)
    else:
        scale = float(np.float32(wl.scale))
        p0 = torch.from_numpy(W.quantize_f16s(wl.phi, np.float32(scale))).to(dev())
    wl.phi = None
    Fd = to_dev(wl.F)
    wl.F = None
    bg = BandGrid((n,) * 3, wl.tile, precision)
    pd = p0.clone()
    acc_d = torch.zeros(1, dtype=torch.int64, device=dev())
    bg.run(pd, Fd, wl.dx, wl.dt, g32, steps, wl.window, scale=scale, tile_steps=acc_d)
    want = host(pd)
    want_list = bg.band_list().numpy().tolist()
    del pd
    pb, Fb = torch.empty_like(p0), torch.empty_like(Fd)
    bg.to_bricks(p0, pb)
    bg.to_bricks(Fd, Fb)
    del Fd
    acc_b = torch.zeros(1, dtype=torch.int64, device=dev())
    bg.run_bricks(pb, Fb, wl.dx, wl.dt, g32, steps, wl.window, scale=scale, tile_steps=acc_b)
    bg.from_bricks(pb, p0)
    assert host(p0).tobytes() == want.tobytes()
    assert bg.band_list().numpy().tolist() == want_list
    assert int(acc_b.item()) == int(acc_d.item())


@pytest.mark.parametrize("mode,beta_dx,reinit_iters", MODES)
@pytest.mark.parametrize("precision", ["f32", "f16s"])
def test_brick_two_step_launches_equal_one_step_launches(precision, mode, beta_dx, reinit_iters):
    """Two steps per launch (ls_tuning.temporal = 1; the default on bricks in
    FP32) and one step per launch (temporal = 2; the FP16s default) give the
    same bits: windows of 10 (five pairs) and of 7 (three pairs and a single
    step)."""
    dims = DIMS[1]
    phi, F, dx, dt, gamma = _spheres(dims, 5)
    beta = None if beta_dx is None else float(np.float32(beta_dx * gamma))
    reinit = None if reinit_iters is None else (float(np.float32(0.5 * dx)), reinit_iters)
    scale = None
    if precision == "f32":
        p0 = to_dev(phi)
    else:
        scale = float(np.float32(gamma))
        p0 = torch.from_numpy(W.quantize_f16s(phi, np.float32(scale))).to(dev())
    bg = BandGrid(dims, (8, 8, 8), precision)
    Fb = torch.empty_like(to_dev(F))
    bg.to_bricks(to_dev(F), Fb)
    outs = {}
    try:
        for temporal in (1, 2):
            ls.ls_set_tuning(0, 0, 0, 0, temporal)
            for window in (10, 7):
                pb = torch.empty_like(p0)
                bg.to_bricks(p0, pb)
                bg.run_bricks(pb, Fb, dx, dt, gamma, 30, window, scale=scale, beta=beta,
                              reinit=reinit)
                outs[(temporal, window)] = (host(pb).tobytes(), bg.band_list().numpy().tolist())
    finally:
        ls.ls_set_tuning(0, 0, 0, 0, 0)
    for window in (10, 7):
        assert outs[(1, window)] == outs[(2, window)], window
