"""Pins of the interface metrics (zero crossings, Hausdorff distance,
trilinear upsampling) that judge the learned closure and the FP16 front.

* Linear interpolation along a grid edge is exact for a linear field, so the
  crossings of a plane lie on the plane: an axis-aligned plane x = x0 gives
  one crossing per grid row at x0 with y, z at the cell centres, an oblique
  plane gives points with n.p = c to rounding.
* Two concentric exact sphere distances: the crossings of each lie within
  O(dx^2) of their sphere, and the Hausdorff distance between the two point
  sets is the radius difference up to the lateral spacing of the samples.
* The Hausdorff distance equals a brute-force max-min over all pairs, and is
  symmetric (a one-sided distance misses the far point of the larger set).
* Trilinear upsampling reproduces a linear field exactly wherever the fine
  point lies between coarse centres, and extends the edge values beyond.
"""
import numpy as np

from paper_1612_04040_amd import metrics as M
from paper_1612_04040_amd import workloads as W


def test_plane_crossings_at_known_positions():
    n = 24
    dx = 1.0 / n
    x0 = 0.4321
    phi = W.plane((n, n, n), dx, (1.0, 0.0, 0.0), x0)
    p = M.zero_crossings(phi, dx)
    assert p.shape == (n * n, 3)
    assert np.max(np.abs(p[:, 0] - x0)) < 1e-12
    centres = (np.arange(n) + 0.5) * dx
    assert np.array_equal(np.unique(np.round(p[:, 1] / dx - 0.5)), np.arange(n))
    assert np.max(np.abs(p[:, 1][:, None] - centres[None, :]).min(axis=1)) < 1e-12
    assert np.max(np.abs(p[:, 2][:, None] - centres[None, :]).min(axis=1)) < 1e-12


def test_oblique_plane_crossings_lie_on_the_plane():
    n = 20
    dx = 1.0 / n
    g = np.array([0.3, -0.5, 0.8])
    g /= np.linalg.norm(g)
    c = float(g @ np.array([0.5, 0.5, 0.5])) + 0.03
    phi = W.plane((n, n, n), dx, tuple(g), c)
    p = M.zero_crossings(phi, dx)
    assert len(p) > 3 * n
    assert np.max(np.abs(p @ g - c)) < 1e-12
    # every crossing sits on a grid edge: two of its coordinates are cell centres
    on_centre = np.abs((p / dx - 0.5) - np.round(p / dx - 0.5)) < 1e-9
    assert np.all(on_centre.sum(axis=1) >= 2)


def _sphere_cloud(n, r):
    dx = 1.0 / n
    phi = W.sphere((n, n, n), dx, (0.5, 0.5, 0.5), r)
    return M.zero_crossings(phi, dx), dx


def test_sphere_crossings_and_concentric_hausdorff():
    n = 64
    r1, r2 = 0.2, 0.2 + 5.0 / n
    a, dx = _sphere_cloud(n, r1)
    b, _ = _sphere_cloud(n, r2)
    for p, r in ((a, r1), (b, r2)):
        rad = np.linalg.norm(p - 0.5, axis=1)
        # chord of a circle through two points at distance <= dx: sag <= dx^2 / (8 r)
        assert np.max(np.abs(rad - r)) <= dx * dx / (8 * r) + 1e-12
    h = M.hausdorff(a, b)
    d = r2 - r1
    # at least the radius difference less both sags; at most the radius
    # difference combined with half a cell diagonal of lateral offset
    assert d - dx * dx / (4 * r1) <= h <= np.hypot(d, 0.5 * np.sqrt(3) * dx)
    assert M.hausdorff(a, a) == 0.0


def test_hausdorff_brute_force_and_symmetry():
    rng = np.random.default_rng(7)
    a = rng.standard_normal((37, 3))
    b = rng.standard_normal((23, 3)) + 0.3
    d = np.linalg.norm(a[:, None, :] - b[None, :, :], axis=2)
    want = max(d.min(axis=1).max(), d.min(axis=0).max())
    assert abs(M.hausdorff(a, b) - want) < 1e-12
    assert abs(M.hausdorff(b, a) - want) < 1e-12
    # hand values: a far point present in one set only decides the distance
    one = np.array([[0.0, 0.0, 0.0]])
    two = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    assert M.hausdorff(one, two) == 5.0 and M.hausdorff(two, one) == 5.0
    assert M.hausdorff(np.zeros((0, 3)), one) == float("inf")


def test_upsample_trilinear_is_exact_on_a_linear_field():
    nc, factor = 8, 4
    dxc = 1.0 / nc
    g = (0.7, -0.2, 0.45)
    coarse = W.plane((nc, nc, nc), dxc, g, 0.1)
    fine = M.upsample_trilinear(coarse, factor)
    nf = nc * factor
    want = W.plane((nf, nf, nf), 1.0 / nf, g, 0.1)
    assert fine.shape == (nf, nf, nf)
    # fine points between the first and last coarse centres on every axis
    u = (np.arange(nf) + 0.5) / factor - 0.5
    inner = (u >= 0) & (u <= nc - 1)
    m = inner[:, None, None] & inner[None, :, None] & inner[None, None, :]
    assert np.max(np.abs(fine[m] - want[m])) < 1e-13
    # beyond the outer centres the edge value is extended (constant along the axis)
    assert np.array_equal(fine[:, :, 0], fine[:, :, 1])
    assert np.array_equal(fine[:, :, -1], fine[:, :, -2])


def test_upsample_trilinear_hand_value():
    """Factor 2 on a 3^3 field: fine point (z, y, x) = (1, 2, 3) has coarse
    coordinates (0.25, 0.75, 1.25), i.e. weights 3/4, 1/4 between coarse
    planes 0 and 1 in z, 1/4, 3/4 between rows 0 and 1 in y, 3/4, 1/4
    between columns 1 and 2 in x."""
    rng = np.random.default_rng(3)
    c = rng.standard_normal((3, 3, 3))
    wz = {0: 0.75, 1: 0.25}
    wy = {0: 0.25, 1: 0.75}
    wx = {1: 0.75, 2: 0.25}
    want = sum(wz[k] * wy[j] * wx[i] * c[k, j, i] for k in wz for j in wy for i in wx)
    got = M.upsample_trilinear(c, 2)[1, 2, 3]
    assert abs(got - want) < 1e-14
