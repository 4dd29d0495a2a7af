"""Pins of the oracle's band tile lists (Eq. 6, and Eq. 11 in tile form).

Checked against a closed form (a plane front: the active tile columns follow
from |x - x0| < gamma interval arithmetic) and against enumeration from the
tile's point of view on tiny random grids with exact ties |phi| = gamma.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import tiny
from paper_1612_04040_amd import workloads as W


@pytest.mark.parametrize("x0", [0.4, 0.377, 0.5])
@pytest.mark.parametrize("tile", [(8, 8, 8), (16, 4, 4), (5, 3, 7)])
def test_plane_band_closed_form(x0, tile):
    n = 64
    dx = 1.0 / n
    gamma = 6 * dx
    phi = W.plane((n, n, n), dx, (1.0, 0.0, 0.0), x0)
    tx, ty, tz = tile
    ntx, nty, ntz = math.ceil(n / tx), math.ceil(n / ty), math.ceil(n / tz)
    # points in the tube: |(i + 1/2) dx - x0| < gamma  <=>  i in (lo, hi)
    pts = [i for i in range(n) if abs(phi[0, 0, i]) < gamma]
    cols_a = sorted({i // tx for i in pts})
    cols_u = sorted({c + d for c in cols_a for d in (-1, 0, 1) if 0 <= c + d < ntx})
    for dilate, cols in ((False, cols_a), (True, cols_u)):
        expect = sorted((tk * nty + tj) * ntx + ti for tk in range(ntz) for tj in range(nty) for ti in cols)
        got = oracle.band_tiles(phi, tile, gamma, dilate=dilate)
        assert got.tolist() == expect


def _tiny_phi(rng, dims, gamma):
    nx, ny, nz = dims
    phi = rng.uniform(-3 * gamma, 3 * gamma, size=(nz, ny, nx))
    r = rng.random(phi.shape)
    phi[r < 0.1] = gamma          # ties: |phi| = gamma is outside (strict)
    phi[(r >= 0.1) & (r < 0.2)] = -gamma
    phi[(r >= 0.2) & (r < 0.22)] = 0.0
    phi[(r >= 0.22) & (r < 0.24)] = -0.0
    phi[(r >= 0.24) & (r < 0.6)] = np.sign(phi[(r >= 0.24) & (r < 0.6)]) * (gamma + 1e-3)
    return phi


@pytest.mark.parametrize("dims", [(1, 1, 1), (5, 3, 2), (13, 9, 7), (8, 8, 8), (17, 17, 17), (33, 9, 20)])
@pytest.mark.parametrize("tile", [(8, 8, 8), (4, 3, 2), (1, 1, 1), (16, 4, 4)])
@pytest.mark.parametrize("dilate", [False, True])
def test_band_bruteforce(dims, tile, dilate):
    rng = np.random.default_rng(sum(dims) * 7 + sum(tile))
    gamma = 0.25
    phi = _tiny_phi(rng, dims, gamma)
    # sparsify so that some tiles are empty
    nz, ny, nx = phi.shape
    mask = rng.random(phi.shape) < 0.93
    phi[mask] = np.where(phi[mask] >= 0, 1.0, -1.0)
    got = oracle.band_tiles(phi, tile, gamma, dilate=dilate)
    expect = tiny.band_tiles(phi.tolist(), gamma, tile, dilate=dilate)
    assert got.tolist() == expect


def test_band_f32_decision_matches_f32_compare():
    """FP32 phi and FP32 gamma promoted exactly give the FP32 comparison."""
    rng = np.random.default_rng(3)
    g32 = np.float32(6.0 / 512)
    phi = rng.uniform(-2 * g32, 2 * g32, size=(16, 16, 16)).astype(np.float32)
    phi.flat[::5] = g32
    phi.flat[1::5] = np.nextafter(g32, np.float32(0))
    got = oracle.band_tiles(phi, (4, 4, 4), g32, dilate=False)
    flags = (np.abs(phi) < g32).reshape(4, 4, 4, 4, 4, 4).any(axis=(1, 3, 5))
    assert got.tolist() == np.flatnonzero(flags.reshape(-1)).tolist()


def test_band_empty_and_full():
    phi = np.full((20, 20, 20), 1.0)
    assert oracle.band_tiles(phi, (8, 8, 8), 0.5).size == 0
    assert oracle.band_tiles(phi, (8, 8, 8), np.inf).tolist() == list(range(27))
    nan = np.full((8, 8, 8), np.nan)
    assert oracle.band_tiles(nan, (8, 8, 8), 1.0).size == 0  # NaN is never in the tube


def test_f16s_dequant_is_fp32_product():
    h = np.array([0.0, -0.0, 1.0, -1.5, 65504.0, 6e-8, 0.333], dtype=np.float16)
    s = np.float32(6.0 / 1024)
    got = oracle.dequant_f16s(h, s)
    assert got.dtype == np.float32
    assert np.array_equal(got.view(np.uint32), (h.astype(np.float32) * s).view(np.uint32))
