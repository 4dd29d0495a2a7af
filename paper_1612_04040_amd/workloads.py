"""Seeded synthetic inputs: initial level-set functions and speed fields.

This module holds no arithmetic of the method itself.  It only draws the
inputs (Step 0 of the narrow-band algorithm: the signed distance to an
initial front, Eq. 1, and a speed field F), and it is the one module that
both the GPU path's tests and the oracle's tests take inputs from.

Grid convention: cell-centred points x_i = (i + 1/2) dx on [0, N dx]^3,
arrays of shape (nz, ny, nx) with x fastest.
"""
from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------
# coordinates


def axis(n, dx):
    return (np.arange(n, dtype=np.float64) + 0.5) * dx


def _slabs(nz, max_points, plane):
    step = max(1, int(max_points // max(plane, 1)))
    for z0 in range(0, nz, step):
        yield z0, min(nz, z0 + step)


# ----------------------------------------------------------------------------
# signed distance functions (Eq. 1)


def sphere(shape, dx, center, radius, dtype=np.float64):
    """phi = |x - c| - r (exact signed distance)."""
    nz, ny, nx = shape
    out = np.empty(shape, dtype=dtype)
    x, y = axis(nx, dx), axis(ny, dx)
    zs = axis(nz, dx)
    for z0, z1 in _slabs(nz, 1 << 24, nx * ny):
        z = zs[z0:z1, None, None]
        d = np.sqrt((x[None, None, :] - center[0]) ** 2 + (y[None, :, None] - center[1]) ** 2
                    + (z - center[2]) ** 2) - radius
        out[z0:z1] = d
    return out


def sphere_union(shape, dx, centers, radii, dtype=np.float64):
    """phi = min_i (|x - c_i| - r_i): exact outside, sign-correct inside."""
    nz, ny, nx = shape
    out = np.empty(shape, dtype=dtype)
    x, y = axis(nx, dx), axis(ny, dx)
    zs = axis(nz, dx)
    for z0, z1 in _slabs(nz, 1 << 23, nx * ny):
        z = zs[z0:z1, None, None]
        best = None
        for c, r in zip(centers, radii):
            d = np.sqrt((x[None, None, :] - c[0]) ** 2 + (y[None, :, None] - c[1]) ** 2
                        + (z - c[2]) ** 2) - r
            best = d if best is None else np.minimum(best, d)
        out[z0:z1] = best
    return out


def torus(shape, dx, major, minor, center=(0.5, 0.5, 0.5), dtype=np.float64):
    """Torus about the z axis through ``center``: exact signed distance."""
    nz, ny, nx = shape
    out = np.empty(shape, dtype=dtype)
    x, y = axis(nx, dx) - center[0], axis(ny, dx) - center[1]
    zs = axis(nz, dx) - center[2]
    rho = np.sqrt(x[None, :] ** 2 + y[:, None] ** 2) - major  # (ny, nx)
    for z0, z1 in _slabs(nz, 1 << 24, nx * ny):
        z = zs[z0:z1, None, None]
        out[z0:z1] = np.sqrt(rho[None] ** 2 + z ** 2) - minor
    return out


def ellipsoid(shape, dx, center, semi_axes, rotation, dtype=np.float64):
    """phi = (|R^T (x - c) / a| - 1) * min(a): sign-correct, not exact."""
    nz, ny, nx = shape
    out = np.empty(shape, dtype=dtype)
    x, y = axis(nx, dx), axis(ny, dx)
    zs = axis(nz, dx)
    a = np.asarray(semi_axes, dtype=np.float64)
    R = np.asarray(rotation, dtype=np.float64)
    for z0, z1 in _slabs(nz, 1 << 23, nx * ny):
        z = zs[z0:z1, None, None]
        px = np.broadcast_to(x[None, None, :] - center[0], (z1 - z0, ny, nx))
        py = np.broadcast_to(y[None, :, None] - center[1], (z1 - z0, ny, nx))
        pz = np.broadcast_to(z - center[2], (z1 - z0, ny, nx))
        acc = 0.0
        for col in range(3):  # body coordinates R^T p, scaled by the semi-axes
            q = R[0, col] * px + R[1, col] * py + R[2, col] * pz
            acc = acc + (q / a[col]) ** 2
        out[z0:z1] = (np.sqrt(acc) - 1.0) * a.min()
    return out


def plane(shape, dx, normal, offset, dtype=np.float64):
    """phi = g . x - offset (a linear field; exact distance when |g| = 1)."""
    nz, ny, nx = shape
    g = np.asarray(normal, dtype=np.float64)
    x, y, z = axis(nx, dx), axis(ny, dx), axis(nz, dx)
    v = g[0] * x[None, None, :] + g[1] * y[None, :, None] + g[2] * z[:, None, None] - offset
    return v.astype(dtype)


def random_rotation(rng):
    """Uniform random rotation matrix (QR of a Gaussian matrix, sign-fixed)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# ----------------------------------------------------------------------------
# speed fields


def sinusoid3(shape, dx, amp=0.5, k=(1, 1, 1), phase=(0.0, 0.0, 0.0), bias=0.0, dtype=np.float64):
    """F = amp * prod_d sin(2 pi k_d x_d + p_d) + bias."""
    nz, ny, nx = shape
    sx = np.sin(2 * np.pi * k[0] * axis(nx, dx) + phase[0])
    sy = np.sin(2 * np.pi * k[1] * axis(ny, dx) + phase[1])
    sz = np.sin(2 * np.pi * k[2] * axis(nz, dx) + phase[2])
    out = np.empty(shape, dtype=dtype)
    for z0, z1 in _slabs(nz, 1 << 24, nx * ny):
        out[z0:z1] = amp * sz[z0:z1, None, None] * sy[None, :, None] * sx[None, None, :] + bias
    return out


def grf_periodic(rng, base, ell):
    """Unit-variance Gaussian random field on a periodic base^3 grid of [0,1]^3.

    Covariance exp(-r^2 / (2 ell^2)): white noise filtered by the square root
    of its spectral density, exp(-|k|^2 ell^2 / 4).
    """
    noise = rng.standard_normal((base, base, base))
    k1 = 2 * np.pi * np.fft.fftfreq(base, d=1.0 / base)
    kk = k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + k1[None, None, :] ** 2
    field_ = np.real(np.fft.ifftn(np.fft.fftn(noise) * np.exp(-kk * ell * ell / 4.0)))
    field_ -= field_.mean()
    field_ /= field_.std()
    return field_


def upsample_periodic(src, shape, dtype=np.float32):
    """Trilinear interpolation of a periodic cell-centred field onto ``shape``."""
    bz, by, bx = src.shape
    nz, ny, nx = shape

    def idx(n, b):
        u = (np.arange(n) + 0.5) * (b / n) - 0.5
        i0 = np.floor(u).astype(np.int64)
        w = u - i0
        return i0 % b, (i0 + 1) % b, w

    xi0, xi1, xw = idx(nx, bx)
    yi0, yi1, yw = idx(ny, by)
    zi0, zi1, zw = idx(nz, bz)
    # x then y on every base plane (small), then z per output slab
    tx = src[:, :, xi0] * (1 - xw) + src[:, :, xi1] * xw            # (bz, by, nx)
    txy = tx[:, yi0, :] * (1 - yw)[None, :, None] + tx[:, yi1, :] * yw[None, :, None]  # (bz, ny, nx)
    out = np.empty(shape, dtype=dtype)
    for z0, z1 in _slabs(nz, 1 << 24, nx * ny):
        w = zw[z0:z1, None, None]
        out[z0:z1] = txy[zi0[z0:z1]] * (1 - w) + txy[zi1[z0:z1]] * w
    return out


def stable_dt(F, dx, cfl=0.5):
    """dt = cfl * dx / max|F|, in FP64 from the stored F."""
    fmax = float(np.max(np.abs(np.asarray(F, dtype=np.float64))))
    return cfl * dx / fmax if fmax > 0 else cfl * dx


# ----------------------------------------------------------------------------
# the five workloads


@dataclass
class Workload:
    name: str
    phi: np.ndarray            # initial level-set function (storage precision or f64)
    F: np.ndarray              # speed
    dx: float
    dt: float
    gamma: float               # band half-width (0 for the full-grid run)
    nsteps: int
    window: int = 10
    tile: tuple = (8, 8, 8)
    scale: float = 0.0         # scaled-FP16 storage factor (0: not FP16)
    extra: dict = field(default_factory=dict)


def sphere_full_f64(n=64, steps=50, speed=1.0):
    """Single sphere r = 0.25 at the centre, F constant, dt = dx/2, full grid, FP64."""
    dx = 1.0 / n
    phi = sphere((n, n, n), dx, (0.5, 0.5, 0.5), 0.25)
    F = np.full((n, n, n), speed, dtype=np.float64)
    return Workload(f"sphere{n}_f64_full", phi, F, dx, 0.5 * dx, 0.0, steps, window=steps)


def three_spheres_f32(n=512, steps=200, seed=2, spheres=3):
    """Union of spheres (radii U(0.1,0.2), centres U(0.25,0.75)^3),
    F = 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z), band 6 dx, 8^3 tiles, FP32."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.25, 0.75, size=(spheres, 3))
    radii = rng.uniform(0.1, 0.2, size=spheres)
    dx = 1.0 / n
    phi = sphere_union((n, n, n), dx, centers, radii, dtype=np.float32)
    F = sinusoid3((n, n, n), dx, amp=0.5, dtype=np.float32)
    dt = float(np.float32(stable_dt(F, dx)))
    return Workload(f"spheres{n}_f32_band", phi, F, dx, dt, float(np.float32(6 * dx)), steps,
                    extra={"centers": centers, "radii": radii})


def torus_grf(n=1024, steps=500, seed=3, base=128, dtype_phi=np.float32):
    """Torus R = 0.3, r = 0.1 about z, F = 1 + 0.3 GRF(ell = 0.05), band 6 dx.

    ``phi`` is returned unquantised (``dtype_phi``); the scaled-FP16 copy is
    made by the caller with scale = 6 dx.
    """
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    phi = torus((n, n, n), dx, 0.3, 0.1, dtype=dtype_phi)
    eta = grf_periodic(rng, base, 0.05)
    F = upsample_periodic(eta, (n, n, n), dtype=np.float32)
    F *= np.float32(0.3)
    F += np.float32(1.0)
    dt = float(np.float32(stable_dt(F, dx)))
    gamma = float(np.float32(6 * dx))
    return Workload(f"torus{n}_band", phi, F, dx, dt, gamma, steps, scale=gamma)


def quantize_f16s(phi, scale):
    """Scaled-FP16 storage h = fp16(phi / s), round to nearest even."""
    s = np.float32(scale)
    out = np.empty(phi.shape, dtype=np.float16)
    flat_in = phi.reshape(-1)
    flat_out = out.reshape(-1)
    step = 1 << 24
    for a in range(0, flat_in.size, step):
        v = flat_in[a:a + step].astype(np.float32) / s
        flat_out[a:a + step] = v.astype(np.float16)
    return out


@dataclass
class Instance:
    n: int
    phi: np.ndarray
    F: np.ndarray
    dx: float
    dt: float
    gamma: float


def ellipsoid_batch(count=256, nmin=32, nmax=192, seed=4, steps=100, base=64, sizes=None):
    """Uneven batch: cubic sizes U{nmin..nmax}, random ellipsoids, F = u + 0.2 GRF."""
    rng = np.random.default_rng(seed)
    if sizes is None:
        sizes = rng.integers(nmin, nmax + 1, size=count)
    out = []
    for n in sizes:
        n = int(n)
        dx = 1.0 / n
        a = rng.uniform(0.1, 0.3, size=3)
        c = rng.uniform(0.35, 0.65, size=3)
        R = random_rotation(rng)
        u = rng.uniform(-1.0, 1.0)
        phi = ellipsoid((n, n, n), dx, c, a, R, dtype=np.float32)
        eta = grf_periodic(rng, base, 0.05)
        F = upsample_periodic(eta, (n, n, n), dtype=np.float32)
        F *= np.float32(0.2)
        F += np.float32(u)
        dt = float(np.float32(stable_dt(F, dx)))
        out.append(Instance(n, phi, F, dx, dt, float(np.float32(6 * dx))))
    return out


class ClosureCase:
    """One closure problem: 1-4 spheres (radii U(0.1, 0.2), centres
    U(0.25, 0.75)^3) and F = a prod_d sin(2 pi k_d x_d + p_d) + b with
    k_d in {1, 2}, a in [0.3, 1], b in [-0.5, 0.5]; the same analytic fields
    sampled on a fine grid and on the grid `ratio` times coarser (both
    cell-centred on [0, 1]^3).  dt_fine = 0.5 dx_fine / max|F| (FP32),
    dt_coarse = ratio * dt_fine (the same CFL number)."""

    def __init__(self, seed, n_fine=512, ratio=4):
        rng = np.random.default_rng(seed)
        count = int(rng.integers(1, 5))
        self.seed = seed
        self.centers = rng.uniform(0.25, 0.75, size=(count, 3))
        self.radii = rng.uniform(0.1, 0.2, size=count)
        self.k = tuple(int(v) for v in rng.integers(1, 3, size=3))
        self.phase = tuple(float(v) for v in rng.uniform(0, 2 * np.pi, size=3))
        self.amp = float(rng.uniform(0.3, 1.0))
        self.bias = float(rng.uniform(-0.5, 0.5))
        self.n_fine, self.ratio = n_fine, ratio
        self.n_coarse = n_fine // ratio
        self.dx_fine = 1.0 / n_fine
        self.dx_coarse = ratio / n_fine
        # max|F| over the continuum bounds every sample; the same scalar serves both grids
        self.fmax = float(np.float32(self.amp + abs(self.bias)))
        self.dt_fine = float(np.float32(0.5 * self.dx_fine / self.fmax))
        self.dt_coarse = float(np.float32(ratio * self.dt_fine))
        self.gamma_fine = float(np.float32(6 * self.dx_fine))
        self.gamma_coarse = float(np.float32(6 * self.dx_coarse))

    def phi(self, n):
        return sphere_union((n, n, n), 1.0 / n, self.centers, self.radii, dtype=np.float32)

    def F(self, n):
        return sinusoid3((n, n, n), 1.0 / n, amp=self.amp, k=self.k, phase=self.phase,
                         bias=self.bias, dtype=np.float32)


class PlaneCase(ClosureCase):
    """A closure problem with a plane front phi = n.x - c (random unit normal,
    c in [0.35, 0.65]) and a constant speed of either sign (|F| in [0.3, 1]):
    the first-order scheme advances it exactly away from the grid faces, so
    the correction it asks for is zero there."""

    def __init__(self, seed, n_fine=512, ratio=4):
        super().__init__(seed, n_fine, ratio)
        rng = np.random.default_rng(10_000 + seed)
        v = rng.standard_normal(3)
        self.normal = v / np.linalg.norm(v)
        self.offset = float(np.dot(self.normal, [0.5, 0.5, 0.5])) + float(rng.uniform(-0.15, 0.15))
        self.speed = float(rng.uniform(0.3, 1.0)) * (1.0 if rng.random() < 0.5 else -1.0)
        self.fmax = float(np.float32(abs(self.speed)))
        self.dt_fine = float(np.float32(0.5 * self.dx_fine / self.fmax))
        self.dt_coarse = float(np.float32(ratio * self.dt_fine))

    def phi(self, n):
        return plane((n, n, n), 1.0 / n, tuple(self.normal), self.offset, dtype=np.float32)

    def F(self, n):
        return np.full((n, n, n), self.speed, dtype=np.float32)
