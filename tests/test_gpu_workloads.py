"""The full-size workloads on the GPU against the oracle.

* 64^3 FP64 sphere, full grid, F = 1, 50 steps: the oracle's result, and the
  front radius r0 + t within 1.5 dx.
* 512^3 FP32 three spheres, band 6 dx in 8^3 tiles, rebuilt every 10 steps,
  200 steps: every window's band list bit-exact; final max|err| <= 1e-4 dx
  over the tube T = {|phi| < gamma} (the band of Eq. 6), and over every
  point within the accumulated FP32 storage-rounding bound
  sum_n 1/2 ulp(|phi_n|) (points of the dilated margin carry |phi| up to
  ~30 dx, whose half-ulp is ~1e-6 dx per step).
* The one-call driver equals build + step window by window, bit for bit.
* A reduced torus (the 1024^3 scaled-FP16 recipe at 128^3): the FP16-stored
  run stays within the FP16 rounding bound of the FP64 oracle near the front.
* The 1024^3 FP16 torus at full size: the band list of phi^0 bit-exact and the
  first step within the FP16 storage bound of the oracle on every band point.
* The 256-grid batch at full size: sampled grids equal their single-grid runs,
  bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import EPS32, dev, error_by_band_distance, host, report, to_dev
from paper_1612_04040_amd import workloads as W
from paper_1612_04040_amd.band import BandGrid

pytestmark = pytest.mark.gpu


def _crossing_radii(phi, dx, center):
    out = []
    for ax in range(3):
        n = phi.shape[ax]
        lo = np.take(phi, np.arange(n - 1), axis=ax)
        hi = np.take(phi, np.arange(1, n), axis=ax)
        idx = np.nonzero((lo < 0) != (hi < 0))
        t = lo[idx] / (lo[idx] - hi[idx])
        pos = [(idx[d] + 0.5) * dx for d in range(3)]
        pos[ax] = pos[ax] + t * dx
        z, y, x = pos
        out.append(np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2))
    return np.concatenate(out)


def test_sphere64_f64_full_grid():
    wl = W.sphere_full_f64(64, 50)
    n = 64
    bg = BandGrid((n, n, n), wl.tile, "f64")
    bg.build(to_dev(wl.phi), float("inf"), dilate=False)  # every tile
    assert int(bg.ntiles.item()) == 512
    pd = to_dev(wl.phi)
    bg.step(pd, to_dev(wl.F), wl.dx, wl.dt, wl.nsteps)
    got = host(pd)
    want = oracle.run_full(wl.phi, wl.F, wl.dx, wl.dt, wl.nsteps)
    assert np.max(np.abs(got - want)) <= 1e-13
    r = _crossing_radii(got, wl.dx, (0.5, 0.5, 0.5))
    assert np.max(np.abs(r - (0.25 + wl.nsteps * wl.dt))) <= 1.5 * wl.dx


@pytest.mark.timeout(900)
def test_three_spheres_512_f32_200_steps():
    wl = W.three_spheres_f32(512, 200)
    g32 = np.float32(wl.gamma)
    dims = (512, 512, 512)
    bg = BandGrid(dims, wl.tile, "f32")
    pd, fd = to_dev(wl.phi), to_dev(wl.F)
    lists = []
    for _ in range(wl.nsteps // wl.window):
        bg.build(pd, float(g32), dilate=True)
        lists.append(bg.band_list().numpy())
        bg.step(pd, fd, wl.dx, wl.dt, wl.window)
    got = host(pd)
    print(f"[512^3] band tiles per window: {[int(x.size) for x in lists]}", flush=True)

    want, ref_lists = oracle.run_band(wl.phi, wl.F, wl.dx, wl.dt, g32, wl.nsteps,
                                      window=wl.window, record_tiles=True)
    for w, (a, b) in enumerate(zip(lists, ref_lists)):
        assert a.tolist() == b.tolist(), f"band list differs at window {w}"
    err = np.abs(got.astype(np.float64) - want)
    tube = np.abs(want) < wl.gamma
    by_dist = error_by_band_distance(err, want, wl.dx)
    report("three_spheres_512_f32", max_err_dx=float(err.max() / wl.dx),
           tube_max_err_dx=float(err[tube].max() / wl.dx), by_abs_phi_dx=by_dist,
           tiles_per_window=[int(x.size) for x in lists])
    print(f"[512^3] max|err| = {err.max() / wl.dx:.3e} dx, in tube "
          f"{err[tube].max() / wl.dx:.3e} dx, by |phi|/dx: {by_dist}", flush=True)
    assert err[tube].max() <= 1e-4 * wl.dx
    # everywhere: at most half an ulp of the largest |phi| per step, plus the
    # FP32 evaluation of the increment (a few eps of dt*|F|*|grad phi| <= dx/2)
    moved = err > 0
    pmax = float(max(np.abs(want[moved]).max(), np.abs(wl.phi[moved]).max())) if moved.any() else 0.0
    bound = wl.nsteps * (0.5 * np.spacing(np.float32(pmax)) + 4 * EPS32 * 0.5 * wl.dx)
    assert err.max() <= bound, (err.max(), bound)

    # the one-call driver (incremental rebuilds) gives the same bits and counts
    pd2 = to_dev(wl.phi)
    acc = torch.zeros(1, dtype=torch.int64, device=dev())
    bg.run(pd2, fd, wl.dx, wl.dt, float(g32), wl.nsteps, wl.window, tile_steps=acc)
    assert host(pd2).tobytes() == got.tobytes()
    assert bg.band_list().numpy().tolist() == lists[-1].tolist()
    assert int(acc.item()) == sum(int(x.size) for x in lists) * wl.window


@pytest.mark.timeout(600)
def test_incremental_rebuild_equals_full_build():
    """Window by window on the 512^3 workload: the rebuild from the previous
    band equals the full scan, bit for bit (and the step plan it leaves is
    the one the steps use)."""
    wl = W.three_spheres_f32(512, 60)
    g32 = float(np.float32(wl.gamma))
    full = BandGrid((512,) * 3, wl.tile, "f32")
    inc = BandGrid((512,) * 3, wl.tile, "f32")
    pd, fd = to_dev(wl.phi), to_dev(wl.F)
    inc.build(pd, g32, dilate=True)
    for w in range(wl.nsteps // wl.window):
        full.build(pd, g32, dilate=True)
        if w > 0:
            inc.rebuild(pd, g32, prev_t, prev_n)
        assert inc.band_list().numpy().tolist() == full.band_list().numpy().tolist(), w
        prev_t, prev_n = inc.tiles.clone(), inc.ntiles.clone()
        full.step(pd, fd, wl.dx, wl.dt, wl.window)


def test_rebuild_random_fields():
    """A random band whose complement holds no tube point: rebuild == build."""
    rng = np.random.default_rng(12)
    dims, tile = (67, 45, 33), (8, 8, 8)
    nz, ny, nx = 33, 45, 67
    gamma = 0.25
    phi = np.where(rng.random((nz, ny, nx)) < 0.5, 1.0, -1.0).astype(np.float32)
    phi[10:14, 20:22, 30:40] = rng.uniform(-0.3, 0.3, (4, 2, 10))  # a small tube
    bg = BandGrid(dims, tile, "f32")
    bg.build(to_dev(phi), gamma, dilate=True)
    prev_t, prev_n = bg.tiles.clone(), bg.ntiles.clone()
    # move values only inside the band, as a step would (the oracle's steps)
    band = oracle.band_tiles(phi, tile, np.float32(gamma), True)
    assert bg.band_list().numpy().tolist() == band.tolist()
    F = rng.uniform(-1, 1, phi.shape).astype(np.float32)
    moved = oracle.upwind_steps(phi, F, 0.05, 0.01, band, 3, tile).astype(np.float32)
    bg.rebuild(to_dev(moved), gamma, prev_t, prev_n)
    got = bg.band_list().numpy()
    assert got.tolist() == oracle.band_tiles(moved, tile, np.float32(gamma), True).tolist()


def test_torus_f16s_reduced():
    n, steps = 128, 50
    wl = W.torus_grf(n, steps, base=64)
    s = np.float32(wl.scale)
    h = W.quantize_f16s(wl.phi, s)
    bg = BandGrid((n, n, n), wl.tile, "f16s")
    hd = torch.from_numpy(h).to(dev())
    bg.run(hd, to_dev(wl.F), wl.dx, wl.dt, wl.gamma, steps, wl.window, scale=float(s))
    got = oracle.dequant_f16s(host(hd), s).astype(np.float64)
    want = oracle.run_band(wl.phi.astype(np.float64), wl.F, wl.dx, wl.dt, np.float32(wl.gamma),
                           steps, window=wl.window)
    front = np.abs(want) < wl.dx
    err = np.abs(got - want)[front]
    # per store at most 1/2 ulp of fp16(|phi|/s) <= 2^-12 s near the front (|phi| < dx < s/4)
    bound = steps * 2.0 ** -12 * float(s)
    print(f"[f16s {n}^3] max|err| near front {err.max() / wl.dx:.3e} dx, "
          f"bound {bound / wl.dx:.3e} dx", flush=True)
    assert err.max() <= bound


@pytest.mark.timeout(900)
@pytest.mark.parametrize("n", [256])
def test_torus_f16s_error_report(n):
    """The scaled-FP16 torus recipe, 500 steps, against the FP64 oracle run on
    the unquantised inputs with its own band decisions: the errors near the
    front and in the tube, and the Hausdorff distance of the fronts, are
    reported; asserted: the tube error stays within the FP16 storage bound
    (steps + 1) x half an FP16 ulp of the largest |phi|/s in the band, times s
    (the update is non-expansive in the max norm and each step adds at most
    one store rounding; the band lists of the two runs can differ at the band
    margin, outside the tube), and the fronts lie within 1 dx."""
    from paper_1612_04040_amd import metrics as M

    steps = 500
    wl = W.torus_grf(n, steps, base=128)
    s = np.float32(wl.scale)
    h = W.quantize_f16s(wl.phi, s)
    bg = BandGrid((n, n, n), wl.tile, "f16s")
    hd, Fd = torch.from_numpy(h).to(dev()), to_dev(wl.F)
    lists = []
    for _ in range(steps // wl.window):
        bg.build(hd, wl.gamma, dilate=True, scale=float(s))
        lists.append(bg.band_list().numpy())
        bg.step(hd, Fd, wl.dx, wl.dt, wl.window, scale=float(s))
    got = oracle.dequant_f16s(host(hd), s).astype(np.float64)
    want, own_lists = oracle.run_band(wl.phi.astype(np.float64), wl.F, wl.dx, wl.dt,
                                      np.float32(wl.gamma), steps, window=wl.window,
                                      record_tiles=True)
    err = np.abs(got - want)
    front = np.abs(want) < wl.dx
    tube = np.abs(want) < wl.gamma
    rec = dict(n=n, steps=steps,
               windows_with_other_lists=int(sum(a.tolist() != b.tolist()
                                                for a, b in zip(lists, own_lists))),
               max_err_front_dx=float(err[front].max() / wl.dx),
               max_err_tube_dx=float(err[tube].max() / wl.dx),
               rms_err_front_dx=float(np.sqrt(np.mean(err[front] ** 2)) / wl.dx),
               hausdorff_dx=M.hausdorff(M.zero_crossings(got, wl.dx),
                                        M.zero_crossings(want, wl.dx)) / wl.dx,
               by_abs_phi_dx=error_by_band_distance(err, want, wl.dx))
    band = np.zeros((n // 8,) * 3, bool)
    for tl in own_lists:
        band.reshape(-1)[tl] = True
    mask = np.repeat(np.repeat(np.repeat(band, 8, 0), 8, 1), 8, 2)
    hmax = float(max(np.abs(want[mask]).max(), np.abs(wl.phi[mask]).max())) / float(s)
    half_ulp = 2.0 ** (np.floor(np.log2(hmax)) - 11)
    rec["bound_dx"] = (steps + 1) * half_ulp * float(s) / wl.dx
    report("torus_f16s_error", **rec)
    print(f"[f16s torus {n}^3] {rec}", flush=True)
    assert rec["max_err_tube_dx"] <= rec["bound_dx"]
    assert rec["hausdorff_dx"] <= 1.0


@pytest.mark.timeout(1200)
def test_torus1024_f16s_full_size_first_step():
    """The 1024^3 scaled-FP16 torus at full size, in the launch configuration
    the bench times (8^3 tiles, 64-point item rows, the vectorised FP16 step):
    the band list of phi^0 equals the oracle's bit for bit, and one step
    matches the FP64 oracle's step of the dequantised phi^0 on every band
    point within one FP16 storage rounding (half an ulp of |phi|/s, times s)
    plus the FP32 arithmetic bound."""
    from gpu_util import fp32_step_bound

    n = 1024
    wl = W.torus_grf(n, 500)
    s = np.float32(wl.scale)
    h = W.quantize_f16s(wl.phi, s)
    wl.phi = None
    bg = BandGrid((n, n, n), wl.tile, "f16s")
    hd, Fd = torch.from_numpy(h).to(dev()), to_dev(wl.F)
    bg.build(hd, wl.gamma, dilate=True, scale=float(s))
    got_list = bg.band_list().numpy()
    phi0 = oracle.dequant_f16s(h, s)
    want_list = oracle.band_tiles(phi0, wl.tile, np.float32(wl.gamma), True)
    assert got_list.tolist() == want_list.tolist()
    bg.step(hd, Fd, wl.dx, wl.dt, 1, scale=float(s))
    got = oracle.dequant_f16s(host(hd), s)
    want = oracle.upwind_steps(phi0, wl.F, wl.dx, wl.dt, want_list, 1, wl.tile)
    mask = np.zeros((n // 8,) * 3, bool)
    mask.reshape(-1)[want_list] = True
    g = got.reshape(n // 8, 8, n // 8, 8, n // 8, 8).transpose(0, 2, 4, 1, 3, 5)[mask]
    w = want.reshape(n // 8, 8, n // 8, 8, n // 8, 8).transpose(0, 2, 4, 1, 3, 5)[mask]
    del got, want
    # per point: half an FP16 ulp of |want|/s (2^-25 s in the subnormal range),
    # the FP32 roundings of v / s and of the decode h * s, and the FP32
    # arithmetic of the step (global bound)
    mag = np.maximum(np.abs(w) / float(s), 2.0 ** -14)
    bound = (2.0 ** (np.floor(np.log2(mag)) - 11) * float(s) + 4 * EPS32 * np.abs(w) +
             fp32_step_bound(phi0, wl.F, wl.dx, wl.dt, 1))
    err = np.abs(g.astype(np.float64) - w)
    report("torus1024_f16s_first_step", band_tiles=int(want_list.size),
           max_err_dx=float(err.max() / wl.dx), max_err_over_bound=float((err / bound).max()))
    assert np.all(err <= bound)


@pytest.mark.timeout(900)
def test_batch256_full_size_grids_equal_single_runs():
    """The 256-grid batch at full size (32^3..192^3), with the autotuner's
    shapes and pitched rows as the bench runs it: two windows; every eighth
    grid, run alone through the single-grid driver (dense rows), gives the same
    bits and the same band list."""
    from paper_1612_04040_amd.autotune import shape_for, tune
    from paper_1612_04040_amd.batch import Batch

    insts = W.ellipsoid_batch()
    table = tune([it.n for it in insts])
    specs = [((it.n,) * 3, shape_for(it.n, table), it.dx, it.dt, it.gamma) for it in insts]
    b = Batch(specs, device=dev())
    b.load([it.phi for it in insts], [it.F for it in insts])
    b.run(20, 10)
    lists = b.band_lists()
    for i in range(0, len(insts), 8):
        dims, tile, dx, dt, gamma = specs[i]
        bg = BandGrid(dims, tile, "f32")
        pd = to_dev(insts[i].phi)
        bg.run(pd, to_dev(insts[i].F), dx, dt, gamma, 20, 10)
        assert host(b.view(b.phi, i)).tobytes() == host(pd).tobytes(), f"grid {i} {dims} {tile}"
        assert lists[i].tolist() == bg.band_list().numpy().tolist(), f"grid {i}"


@pytest.mark.parametrize("precision", ["f32", "f64", "f16s"])
@pytest.mark.parametrize("dims", [(96, 80, 72), (100, 84, 76)])
def test_incremental_rebuild_equals_full_build_all_storages(precision, dims):
    """Every storage precision, whole and partial tiles at the high faces:
    window by window of a moving sphere union, the rescan of the previous band
    gives the full scan's list, bit for bit."""
    nx, ny, nz = dims
    rng = np.random.default_rng(sum(dims))
    dx = 1.0 / max(dims)
    centers = rng.uniform(0.3, 0.7, size=(3, 3)) * np.array([nx, ny, nz]) * dx
    phi = W.sphere_union((nz, ny, nx), dx, centers, rng.uniform(0.1, 0.2, 3) * max(dims) * dx)
    F = (0.8 * rng.uniform(-1, 1, phi.shape)).astype(np.float32)
    gamma = 6 * dx
    s = np.float32(gamma)
    if precision == "f32":
        host_phi, Fh, scale = phi.astype(np.float32), F, None
    elif precision == "f64":
        host_phi, Fh, scale = phi, F.astype(np.float64), None
    else:
        host_phi, Fh, scale = W.quantize_f16s(phi.astype(np.float32), s), F, float(s)
    dt = 0.5 * dx
    full = BandGrid(dims, (8, 8, 8), precision)
    inc = BandGrid(dims, (8, 8, 8), precision)
    pd, fd = torch.from_numpy(np.ascontiguousarray(host_phi)).to(dev()), to_dev(Fh)
    inc.build(pd, gamma, dilate=True, scale=scale)
    for w in range(5):
        full.build(pd, gamma, dilate=True, scale=scale)
        if w > 0:
            inc.rebuild(pd, gamma, prev_t, prev_n, scale=scale)
        assert inc.band_list().numpy().tolist() == full.band_list().numpy().tolist(), w
        prev_t, prev_n = inc.tiles.clone(), inc.ntiles.clone()
        full.step(pd, fd, dx, dt, 10, scale=scale)
