"""GPU test of the allocation-free band build (ls_band_build_f32_noalloc).

Two calls in a row on one device, the second on a smaller grid (so it runs on
the fixed array the first call left its contents in), each compared bit for
bit with ls_band_build_f32 on a workspace the caller allocates: the band
list, its count, and the unused tail of the caller's list buffer left as it
was.  The first grid is the largest kind the array holds (512^3 in 8^3 tiles).
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, to_dev
from paper_1612_04040_amd import ls
from paper_1612_04040_amd import workloads as W

pytestmark = pytest.mark.gpu


def _reference(phi_d, g, gamma, dilate):
    cap = ls.ls_grid_tiles(g)
    tiles = torch.full((cap,), -7, dtype=torch.int32, device=dev())
    cnt = torch.zeros(1, dtype=torch.int32, device=dev())
    wsb = ls.ls_workspace_bytes(g)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev())
    ls.ls_band_build_f32(phi_d, g, gamma, dilate, tiles, cap, cnt, ws, wsb)
    torch.cuda.synchronize()
    return tiles.cpu().numpy(), int(cnt.item())


def _noalloc(phi_d, g, gamma, dilate):
    cap = ls.ls_grid_tiles(g)
    tiles = torch.full((cap,), -7, dtype=torch.int32, device=dev())
    cnt = torch.zeros(1, dtype=torch.int32, device=dev())
    ls.ls_band_build_f32_noalloc(phi_d, g, gamma, dilate, tiles, cap, cnt)
    torch.cuda.synchronize()
    return tiles.cpu().numpy(), int(cnt.item())


def _inputs():
    wl = W.three_spheres_f32(512, 10)
    big = (wl.phi, (512, 512, 512), float(np.float32(wl.gamma)))
    rng = np.random.default_rng(71)
    dims = (90, 77, 61)  # ragged: partial tiles on every high face
    phi = (rng.standard_normal((dims[2], dims[1], dims[0])) * 0.2).astype(np.float32)
    phi[5, 7, 11] = 0.05  # exactly gamma: outside (strict)
    small = (phi, dims, 0.05)
    return big, small


@pytest.mark.parametrize("dilate", [1, 0])
def test_noalloc_build_matches_build_twice(dilate):
    for phi, dims, gamma in _inputs():  # large first, then smaller
        g = ls.grid(dims)
        print(f"noalloc build: dims {dims} dilate {dilate}", flush=True)
        phi_d = to_dev(phi)
        want, nwant = _reference(phi_d, g, gamma, dilate)
        got, ngot = _noalloc(phi_d, g, gamma, dilate)
        assert nwant > 0
        assert ngot == nwant
        np.testing.assert_array_equal(got, want)  # list and untouched tail


def test_noalloc_rejects_oversized_grid_on_device():
    g = ls.grid((1024, 1024, 512))
    assert ls.ls_workspace_bytes(g) > ls.ls_band_build_noalloc_max_bytes()
    phi_d = torch.zeros(1, dtype=torch.float32, device=dev())
    tiles = torch.zeros(1, dtype=torch.int32, device=dev())
    with pytest.raises(ls.LsError) as e:
        ls.ls_band_build_f32_noalloc(phi_d, g, 0.1, 1, tiles, ls.ls_grid_tiles(g), tiles)
    assert e.value.status == ls.LS_ERR_CAPACITY
