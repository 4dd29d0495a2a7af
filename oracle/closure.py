"""FP64 reference of the learned closure (test infrastructure only).

A small 3-layer 3^3-conv network corrects the coarse first-order upwind step
(Eq. 3-5) toward fine-grid runs of the same scheme restricted 4x.  Every
function here is the plain definition in numpy float64; the pins are in
tests/test_oracle_closure.py (finite-difference gradients, scipy
correlation, closed forms of the restriction, the zero-network identity).

Conventions (readings for an addition to the method; the paper has no network):
  restriction  coarse cell (I,J,K) = mean of the 2x2x2 fine points 4I+1..4I+2
               (the coarse cell centre lies midway between them).
  features     c0 = clip(phi / gamma, -2, 2), c1 = F / Fmax,
               c2 = (plain step increment) / dx_c.
  network      conv3^3(3->16) + b, SiLU, conv3^3(16->16) + b, SiLU,
               conv3^3(16->1) + b; zero padding at the grid faces;
               cross-correlation: out[o,z,y,x] = sum_{c,dz,dy,dx}
               w[o,c,dz,dy,dx] * in[c, z+dz-1, y+dy-1, x+dx-1].
  gate         the correction is weighted by the cut-off function of Eq. 8,
               c(phi) = 1 for |phi| <= beta, (|phi| - gamma)^2 (2|phi| + gamma
               - 3 beta) / (gamma - beta)^3 for beta < |phi| <= gamma, 0 beyond,
               with beta = gamma / 2: it acts near the front only.
  update       on the active tiles: phi + delta_plain + k, with the correction
               k = dx_c * c(phi) * r limited to |k| <= |delta_plain| / 2 (it
               never reverses or stalls the plain step); elsewhere in the band
               the plain step; a tile where some c(phi) * r is non-finite or
               exceeds 1/2 in magnitude falls back to the plain step.
  loss         mean over active points of (phi_pred - phi_target)^2 / dx_c^2
               = mean (c r - r*)^2 with r* = (phi_target - phi - delta_plain)/dx_c.
  judge        the plain scheme judges the corrected run: a shadow plain run
               advances beside it, and after every window each tile whose
               zero-crossing state (points of both signs, phi < 0 and
               phi >= 0, present or not) differs from the shadow's takes the
               shadow's values.
"""
import numpy as np

import oracle

CHANNELS = (3, 16, 16, 1)


def restrict4(phi_f):
    """Coarse field: mean of the 2x2x2 fine points around each coarse centre."""
    f = np.asarray(phi_f, dtype=np.float64)
    nz, ny, nx = f.shape
    assert nz % 4 == 0 and ny % 4 == 0 and nx % 4 == 0
    sub = f.reshape(nz // 4, 4, ny // 4, 4, nx // 4, 4)[:, 1:3, :, 1:3, :, 1:3]
    return sub.mean(axis=(1, 3, 5))


def plain_increment(phi_c, F_c, dx, dt, tiles, tile=(8, 8, 8)):
    """delta = (one plain step of Eq. 3 on the listed tiles) - phi."""
    nxt = oracle.upwind_steps(phi_c, F_c, dx, dt, tiles, 1, tile)
    return nxt - np.asarray(phi_c, dtype=np.float64)


def features(phi_c, F_c, delta, dx, gamma, fmax):
    c0 = np.clip(np.asarray(phi_c, np.float64) / gamma, -2.0, 2.0)
    c1 = np.asarray(F_c, np.float64) / fmax
    c2 = np.asarray(delta, np.float64) / dx
    return np.stack([c0, c1, c2])


def conv3(x, w, b):
    """3^3 cross-correlation with zero padding: x (C,Z,Y,X), w (O,C,3,3,3)."""
    C, Z, Y, X = x.shape
    O = w.shape[0]
    xp = np.zeros((C, Z + 2, Y + 2, X + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((O, Z, Y, X))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                patch = xp[:, dz:dz + Z, dy:dy + Y, dx:dx + X]
                out += np.einsum("oc,czyx->ozyx", w[:, :, dz, dy, dx], patch)
    return out + b[:, None, None, None]


def conv3_backward(x, w, gout):
    """Gradients of conv3 w.r.t. x, w, b for an upstream gradient gout (O,Z,Y,X)."""
    C, Z, Y, X = x.shape
    xp = np.zeros((C, Z + 2, Y + 2, X + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                patch = xp[:, dz:dz + Z, dy:dy + Y, dx:dx + X]
                gw[:, :, dz, dy, dx] = np.einsum("ozyx,czyx->oc", gout, patch)
                gxp[:, dz:dz + Z, dy:dy + Y, dx:dx + X] += np.einsum("oc,ozyx->czyx",
                                                                    w[:, :, dz, dy, dx], gout)
    gb = gout.sum(axis=(1, 2, 3))
    return gxp[:, 1:-1, 1:-1, 1:-1], gw, gb


# The cut-off function of Eq. 8 (defined with the band driver's steps).
cutoff = oracle.cutoff


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(rng, scale=None):
    """Weights ~ N(0, 1/fan_in) (scaled), zero biases; last layer zero, so the
    network starts as the plain scheme (r = 0)."""
    params = {}
    for l in range(3):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        std = (1.0 / (27 * cin)) ** 0.5 if scale is None else scale
        w = rng.standard_normal((cout, cin, 3, 3, 3)) * std
        if l == 2:
            w[:] = 0.0
        params[f"w{l}"] = w
        params[f"b{l}"] = np.zeros(cout)
    return params


def forward(params, feat):
    """r (Z,Y,X) and the cache the backward pass needs."""
    z0 = conv3(feat, params["w0"], params["b0"])
    a0 = silu(z0)
    z1 = conv3(a0, params["w1"], params["b1"])
    a1 = silu(z1)
    r = conv3(a1, params["w2"], params["b2"])[0]
    return r, (feat, z0, a0, z1, a1)


def loss_and_grad(params, feat, rstar, mask, gate=None):
    """Mean over mask of (c r - r*)^2 (c = gate, 1 if None) and its gradient
    w.r.t. every parameter."""
    r, (x, z0, a0, z1, a1) = forward(params, feat)
    m = mask.astype(np.float64)
    c = np.ones_like(r) if gate is None else np.asarray(gate, np.float64)
    cnt = max(m.sum(), 1.0)
    diff = (c * r - rstar) * m
    loss = float((diff ** 2).sum() / cnt)
    gr = (2.0 / cnt) * diff * c
    g = {}
    ga1, g["w2"], g["b2"] = conv3_backward(a1, params["w2"], gr[None])
    gz1 = ga1 * silu_grad(z1)
    ga0, g["w1"], g["b1"] = conv3_backward(a0, params["w1"], gz1)
    gz0 = ga0 * silu_grad(z0)
    _, g["w0"], g["b0"] = conv3_backward(x, params["w0"], gz0)
    return loss, g


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of every parameter, in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[:] = beta1 * m + (1 - beta1) * grads[k]
        v[:] = beta2 * v + (1 - beta2) * grads[k] ** 2
        mhat = m / (1 - beta1 ** t)
        vhat = v / (1 - beta2 ** t)
        params[k] -= lr * mhat / (np.sqrt(vhat) + eps)
    return params


def closure_step(params, phi_c, F_c, dx, dt, gamma, fmax, band, active, tile=(8, 8, 8)):
    """One corrected coarse step: plain on the band, plus dx*c(phi)*r (limited
    to half the plain increment) on the active tiles whose gated correction is
    finite and at most 1/2 (else plain)."""
    delta = plain_increment(phi_c, F_c, dx, dt, band, tile)
    feat = features(phi_c, F_c, delta, dx, gamma, fmax)
    r, _ = forward(params, feat)
    r = cutoff(phi_c, 0.5 * gamma, gamma) * r
    out = np.asarray(phi_c, np.float64) + delta
    nz, ny, nx = out.shape
    tx, ty, tz = tile
    ntx, nty = -(-nx // tx), -(-ny // ty)
    fallbacks = 0
    for t in active:
        ti, tj, tk = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        sl = (slice(tk * tz, (tk + 1) * tz), slice(tj * ty, (tj + 1) * ty),
              slice(ti * tx, (ti + 1) * tx))
        rt = r[sl]
        if not np.all(np.isfinite(rt)) or np.max(np.abs(rt)) > 0.5:
            fallbacks += 1
            continue
        lim = 0.5 * np.abs(delta[sl])
        out[sl] += np.clip(dx * rt, -lim, lim)
    return out, fallbacks


def crossing_tiles(phi, tile=(8, 8, 8)):
    """Boolean per tile (tile id order, x fastest): the tile holds a point with
    phi < 0 and a point with phi >= 0 (NaN counts as not negative)."""
    nz, ny, nx = phi.shape
    tx, ty, tz = tile
    ntx, nty, ntz = -(-nx // tx), -(-ny // ty), -(-nz // tz)
    out = np.zeros(ntx * nty * ntz, bool)
    for t in range(out.size):
        ti, tj, tk = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        blk = phi[tk * tz:(tk + 1) * tz, tj * ty:(tj + 1) * ty, ti * tx:(ti + 1) * tx]
        neg = blk < 0
        out[t] = bool(neg.any()) and bool((~neg).any())
    return out


def judge(phi, shadow, tile=(8, 8, 8), dx=None, tau=0.0):
    """The judge after a window: (phi with every tile whose crossing state
    differs from the shadow's replaced by the shadow's values, the number of
    such tiles).  With tau > 0 (and the spacing dx) a tile is replaced as
    well when the two fronts lie apart by more than tau dx there: some point
    next to either front (|phi| < dx or |shadow| < dx) has
    |phi - shadow| > tau dx (both fields are distance-like near the front, so
    the difference of the values there is the distance between the fronts)."""
    out = np.array(phi, copy=True)
    bad = crossing_tiles(phi, tile) != crossing_tiles(shadow, tile)
    nz, ny, nx = phi.shape
    tx, ty, tz = tile
    ntx, nty = -(-nx // tx), -(-ny // ty)

    def block(t):
        ti, tj, tk = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        return (slice(tk * tz, (tk + 1) * tz), slice(tj * ty, (tj + 1) * ty),
                slice(ti * tx, (ti + 1) * tx))

    if tau > 0:
        for t in range(bad.size):
            sl = block(t)
            a, b = phi[sl], shadow[sl]
            near = (np.abs(a) < dx) | (np.abs(b) < dx)
            if np.any(near & (np.abs(a - b) > tau * dx)):
                bad[t] = True
    idx = np.flatnonzero(bad)
    for t in idx:
        sl = block(t)
        out[sl] = shadow[sl]
    return out, int(idx.size)
