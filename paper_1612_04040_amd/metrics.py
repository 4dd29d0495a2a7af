"""Interface metrics on the host (numpy / scipy): zero crossings of a level-set
field, their radius about a centre, and the symmetric Hausdorff distance
between two fronts.  Used to judge runs (not part of the update itself).

Fields are arrays of shape (nz, ny, nx) on the cell-centred grid
x_i = (i + 1/2) dx.
"""
import numpy as np
from scipy.spatial import cKDTree


def zero_crossings(phi, dx, origin=0.0):
    """Points where phi changes sign along grid edges (linear interpolation),
    as an (m, 3) array of (x, y, z)."""
    phi = np.asarray(phi, dtype=np.float64)
    pts = []
    for ax in range(3):  # array axes (z, y, x)
        n = phi.shape[ax]
        if n < 2:
            continue
        lo = np.take(phi, np.arange(n - 1), axis=ax)
        hi = np.take(phi, np.arange(1, n), axis=ax)
        idx = np.nonzero((lo < 0) != (hi < 0))
        t = lo[idx] / (lo[idx] - hi[idx])
        pos = [(idx[d] + 0.5) * dx + origin for d in range(3)]
        pos[ax] = pos[ax] + t * dx
        z, y, x = pos
        pts.append(np.stack([x, y, z], axis=1))
    return np.concatenate(pts) if pts else np.zeros((0, 3))


def radius_error(phi, dx, center, radius):
    """Crossing radii minus the expected radius."""
    p = zero_crossings(phi, dx)
    r = np.sqrt(((p - np.asarray(center)[None, :]) ** 2).sum(axis=1))
    return r - radius


def hausdorff(a, b):
    """Symmetric Hausdorff distance between two point sets (same units)."""
    if len(a) == 0 or len(b) == 0:
        return float("inf") if len(a) != len(b) else 0.0
    da, _ = cKDTree(b).query(a)
    db, _ = cKDTree(a).query(b)
    return float(max(da.max(), db.max()))


def upsample_trilinear(phi_c, factor):
    """Trilinear interpolation of a cell-centred coarse field onto the fine
    grid `factor` times finer (edge values extended)."""
    phi_c = np.asarray(phi_c, dtype=np.float64)
    nz, ny, nx = phi_c.shape

    def coords(n):
        u = (np.arange(n * factor) + 0.5) / factor - 0.5
        i0 = np.clip(np.floor(u).astype(np.int64), 0, n - 1)
        i1 = np.clip(i0 + 1, 0, n - 1)
        w = np.clip(u - np.floor(u), 0.0, 1.0)
        w = np.where(u < 0, 0.0, np.where(u > n - 1, 1.0, w))
        return i0, i1, w

    x0, x1, wx = coords(nx)
    y0, y1, wy = coords(ny)
    z0, z1, wz = coords(nz)
    t = phi_c[:, :, x0] * (1 - wx) + phi_c[:, :, x1] * wx
    t = t[:, y0, :] * (1 - wy)[None, :, None] + t[:, y1, :] * wy[None, :, None]
    return t[z0] * (1 - wz)[:, None, None] + t[z1] * wz[:, None, None]
