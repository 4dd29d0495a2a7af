"""Brute force for tiny grids, in pure Python (test infrastructure only).

Two independent evaluations of one Jacobi step of Eq. 3-5, point by point:
Python floats (IEEE double, one rounding per operation, the same as the C
oracle) and 50-digit decimals (the exact result to well below double
precision).  Plus the band tile sets by point enumeration, written from the
point of view of a tile (Eq. 6 and the tile form of Eq. 11) rather than from
the point of view of a grid point as the C oracle does.

Arrays are nested Python lists indexed [k][j][i] (x fastest).
"""
import decimal
import math

_CTX = decimal.Context(prec=50)


def _clamp(v, lo, hi):
    return lo if v < lo else (hi if v > hi else v)


def _point(phi, F, i, j, k, dx, dt, num):
    """One point of Eq. 3 with Eq. 4 / Eq. 5; ``num`` supplies the arithmetic."""
    nz, ny, nx = len(phi), len(phi[0]), len(phi[0][0])
    c = phi[k][j][i]
    f = F[k][j][i]
    if f == 0:
        return c
    nb = {
        "x": (phi[k][j][_clamp(i - 1, 0, nx - 1)], phi[k][j][_clamp(i + 1, 0, nx - 1)]),
        "y": (phi[k][_clamp(j - 1, 0, ny - 1)][i], phi[k][_clamp(j + 1, 0, ny - 1)][i]),
        "z": (phi[_clamp(k - 1, 0, nz - 1)][j][i], phi[_clamp(k + 1, 0, nz - 1)][j][i]),
    }
    total = num.zero
    for axis in ("x", "y", "z"):
        lo, hi = nb[axis]
        d_minus = num.div(num.sub(c, lo), dx)   # backward difference D^-
        d_plus = num.div(num.sub(hi, c), dx)    # forward difference D^+
        if f > 0:
            term = num.add(num.sq(max(d_minus, num.zero)), num.sq(min(d_plus, num.zero)))
        else:
            term = num.add(num.sq(max(d_plus, num.zero)), num.sq(min(d_minus, num.zero)))
        total = num.add(total, term)
    return num.sub(c, num.mul(num.mul(dt, f), num.sqrt(total)))


class _Float:
    zero = 0.0

    @staticmethod
    def add(a, b):
        return a + b

    @staticmethod
    def sub(a, b):
        return a - b

    @staticmethod
    def mul(a, b):
        return a * b

    @staticmethod
    def div(a, b):
        return a / b

    @staticmethod
    def sq(a):
        return a * a

    @staticmethod
    def sqrt(a):
        return math.sqrt(a)


class _Dec:
    zero = decimal.Decimal(0)

    @staticmethod
    def add(a, b):
        return _CTX.add(a, b)

    @staticmethod
    def sub(a, b):
        return _CTX.subtract(a, b)

    @staticmethod
    def mul(a, b):
        return _CTX.multiply(a, b)

    @staticmethod
    def div(a, b):
        return _CTX.divide(a, b)

    @staticmethod
    def sq(a):
        return _CTX.multiply(a, a)

    @staticmethod
    def sqrt(a):
        return _CTX.sqrt(a)


def _tile_points(t, dims, tile):
    nx, ny, nz = dims
    tx, ty, tz = tile
    ntx, nty = -(-nx // tx), -(-ny // ty)
    ti, tj, tk = t % ntx, (t // ntx) % nty, t // (ntx * nty)
    for k in range(tk * tz, min((tk + 1) * tz, nz)):
        for j in range(tj * ty, min((tj + 1) * ty, ny)):
            for i in range(ti * tx, min((ti + 1) * tx, nx)):
                yield i, j, k


def steps(phi, F, dx, dt, tiles, tile, nsteps, exact=False):
    """``nsteps`` Jacobi steps on the points of ``tiles``; nested lists in/out.

    With ``exact`` the arithmetic is 50-digit decimal (inputs converted
    exactly from their binary values), otherwise Python float.
    """
    num = _Dec if exact else _Float
    conv = (lambda v: decimal.Decimal(v)) if exact else float
    cur = [[[conv(v) for v in row] for row in plane] for plane in phi]
    f = [[[conv(v) for v in row] for row in plane] for plane in F]
    dxv, dtv = conv(dx), conv(dt)
    dims = (len(cur[0][0]), len(cur[0]), len(cur))
    for _ in range(nsteps):
        new = [[list(row) for row in plane] for plane in cur]
        for t in tiles:
            for i, j, k in _tile_points(int(t), dims, tile):
                new[k][j][i] = _point(cur, f, i, j, k, dxv, dtv, num)
        cur = new
    return cur


def band_tiles(phi, gamma, tile, dilate=True):
    """Band tile ids by enumeration over tiles.

    A tile is in A if one of its own points has |phi| < gamma; in U (dilate)
    if one of the points of the up to 27 tiles around it, itself included,
    has.  ``phi`` values and ``gamma`` are compared exactly as given.
    """
    nz, ny, nx = len(phi), len(phi[0]), len(phi[0][0])
    tx, ty, tz = tile
    ntx, nty, ntz = -(-nx // tx), -(-ny // ty), -(-nz // tz)
    out = []
    for t in range(ntx * nty * ntz):
        ti, tj, tk = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        reach = 1 if dilate else 0
        i0, i1 = max(0, (ti - reach) * tx), min(nx, (ti + 1 + reach) * tx)
        j0, j1 = max(0, (tj - reach) * ty), min(ny, (tj + 1 + reach) * ty)
        k0, k1 = max(0, (tk - reach) * tz), min(nz, (tk + 1 + reach) * tz)
        hit = any(abs(phi[k][j][i]) < gamma
                  for k in range(k0, k1) for j in range(j0, j1) for i in range(i0, i1))
        if hit:
            out.append(t)
    return out
