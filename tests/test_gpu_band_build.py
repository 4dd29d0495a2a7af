"""Band build on the GPU vs the oracle: the tile lists are bit-exact.

Shapes span several tiles with ragged (partial) tiles on every axis, tile
shapes include non-cubic and odd ones, fields carry exact ties |phi| = gamma,
signed zeros and NaN, and the full 512^3 / 1024^3 shapes are covered.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, to_dev
from paper_1612_04040_amd import workloads as W
from paper_1612_04040_amd.band import BandGrid

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (5, 3, 2), (13, 9, 7), (64, 64, 64), (67, 45, 33), (130, 17, 9)]
TILES = [(8, 8, 8), (4, 3, 2), (16, 4, 4), (1, 1, 1)]


def _field(rng, dims, gamma, dtype):
    nx, ny, nz = dims
    phi = rng.uniform(-4 * gamma, 4 * gamma, size=(nz, ny, nx))
    r = rng.random(phi.shape)
    phi[r < 0.6] = np.where(phi[r < 0.6] > 0, 1.0, -1.0)  # most points far from the tube
    phi[(r >= 0.6) & (r < 0.65)] = gamma
    phi[(r >= 0.65) & (r < 0.7)] = -gamma
    phi[(r >= 0.7) & (r < 0.71)] = -0.0
    phi[(r >= 0.71) & (r < 0.72)] = np.nan
    return phi.astype(dtype)


def _gpu_list(bg, phi_dev, gamma, dilate, scale=None):
    bg.build(phi_dev, gamma, dilate=dilate, scale=scale)
    return bg.band_list().numpy()


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("tile", TILES)
def test_band_build_f32_bitexact(dims, tile):
    rng = np.random.default_rng(hash((dims, tile)) % 2**32)
    g32 = np.float32(0.25)
    phi = _field(rng, dims, g32, np.float32)
    bg = BandGrid(dims, tile, "f32")
    pd = to_dev(phi)
    for dilate in (False, True):
        got = _gpu_list(bg, pd, float(g32), dilate)
        want = oracle.band_tiles(phi, tile, g32, dilate=dilate)
        assert got.tolist() == want.tolist(), (dims, tile, dilate)


@pytest.mark.parametrize("dims", [(13, 9, 7), (67, 45, 33)])
def test_band_build_f64_bitexact(dims):
    rng = np.random.default_rng(7)
    phi = _field(rng, dims, 0.25, np.float64)
    bg = BandGrid(dims, (8, 8, 8), "f64")
    for dilate in (False, True):
        got = _gpu_list(bg, to_dev(phi), 0.25, dilate)
        assert got.tolist() == oracle.band_tiles(phi, (8, 8, 8), 0.25, dilate).tolist()


@pytest.mark.parametrize("dims", [(64, 64, 64), (72, 40, 24), (13, 9, 7)])
def test_band_build_f16s_bitexact(dims):
    rng = np.random.default_rng(9)
    s = np.float32(6.0 / 64)
    phi = _field(rng, dims, s, np.float32)
    h = W.quantize_f16s(phi, s)
    deq = oracle.dequant_f16s(h, s)
    bg = BandGrid(dims, (8, 8, 8), "f16s")
    hd = torch.from_numpy(h).to(dev())
    for dilate in (False, True):
        got = _gpu_list(bg, hd, float(s), dilate, scale=float(s))
        assert got.tolist() == oracle.band_tiles(deq, (8, 8, 8), s, dilate).tolist()


def test_band_build_empty_and_full():
    dims = (40, 24, 16)
    phi = np.ones((16, 24, 40), dtype=np.float32)
    bg = BandGrid(dims, (8, 8, 8), "f32")
    assert _gpu_list(bg, to_dev(phi), 0.5, True).size == 0
    assert _gpu_list(bg, to_dev(phi), float("inf"), False).tolist() == list(range(5 * 3 * 2))


def test_band_build_sphere_512():
    """Full-size shape of the three-sphere workload (512^3, 8^3 tiles)."""
    wl = W.three_spheres_f32(512, steps=0)
    bg = BandGrid((512,) * 3, (8, 8, 8), "f32")
    got = _gpu_list(bg, to_dev(wl.phi), wl.gamma, True)
    want = oracle.band_tiles(wl.phi, (8, 8, 8), np.float32(wl.gamma), True)
    assert got.tolist() == want.tolist()
    assert 10_000 < got.size < 60_000


def test_band_build_unaligned_scalar_path():
    """nx not a multiple of the vector width and an unaligned base pointer."""
    rng = np.random.default_rng(2)
    dims = (33, 20, 12)
    phi = _field(rng, dims, 0.25, np.float32)
    buf = torch.empty(phi.size + 1, dtype=torch.float32, device=dev())
    buf[1:] = to_dev(phi.reshape(-1))
    bg = BandGrid(dims, (8, 8, 8), "f32")
    bg.build(buf[1:], 0.25, dilate=True)
    got = bg.band_list().numpy()
    assert got.tolist() == oracle.band_tiles(phi, (8, 8, 8), np.float32(0.25), True).tolist()
    host(buf)
