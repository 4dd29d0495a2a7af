"""Learned closure of the coarse first-order step: device buffers and thin
wrappers over the closure C-ABI (``ls_closure_*``, ``ls_adam_step``,
``ls_restrict4_f32``).  Arguments are marshalled here; the network, its
gradients, the optimiser and the restriction run in libls's HIP kernels.

Parameter vector layout (FP32, 8673 values): w0 (16,3,3,3,3), b0 (16),
w1 (16,16,3,3,3), b1 (16), w2 (1,16,3,3,3), b2 (1); weights indexed
(out, in, dz, dy, dx).
"""
import numpy as np
import torch

from . import ls
from .band import BandGrid

CHANNELS = (3, 16, 16, 1)
PARAM_SHAPES = (("w0", (16, 3, 3, 3, 3)), ("b0", (16,)), ("w1", (16, 16, 3, 3, 3)), ("b1", (16,)),
                ("w2", (1, 16, 3, 3, 3)), ("b2", (1,)))
NPARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


def flatten(params):
    """Flat FP32 vector from a dict of the shapes in PARAM_SHAPES."""
    return np.concatenate([np.asarray(params[k], np.float32).reshape(-1) for k, _ in PARAM_SHAPES])


def unflatten(vec):
    vec = np.asarray(vec)
    out, o = {}, 0
    for k, s in PARAM_SHAPES:
        n = int(np.prod(s))
        out[k] = vec[o:o + n].reshape(s)
        o += n
    return out


def init_params(rng):
    """Weights ~ N(0, 1/fan_in), zero biases, last layer zero (so the network
    starts as the plain scheme: r = 0)."""
    params = {}
    for l in range(3):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        w = rng.standard_normal((cout, cin, 3, 3, 3)) * (1.0 / (27 * cin)) ** 0.5
        if l == 2:
            w[:] = 0.0
        params[f"w{l}"] = w
        params[f"b{l}"] = np.zeros(cout)
    return flatten(params)


def _aligned(nbytes, device):
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf[off:off + nbytes]


class ClosureGrid:
    """Buffers of the closure on one coarse grid (8^3 tiles): the band
    buffers of a BandGrid plus the closure workspace."""

    def __init__(self, dims, device="cuda"):
        self.bg = BandGrid(dims, (8, 8, 8), "f32", device)
        self.device = self.bg.device
        self.g = self.bg.g
        self.cws_bytes = ls.ls_closure_workspace_bytes(self.g)
        self._cbuf, self.cws = _aligned(self.cws_bytes, self.device)
        self.grad = torch.zeros(NPARAMS, dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.fallbacks = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.resets = torch.zeros(1, dtype=torch.int32, device=self.device)

    def _band(self):
        b = self.bg
        return b.tiles, b.capacity, b.ntiles, b.ws, b.ws_bytes

    def forward(self, phi, F, dx, dt, gamma, fmax, params, r=None, plain=None, stream=None):
        t, cap, n, ws, wsb = self._band()
        ls.ls_closure_forward_f32(phi, F, self.g, dx, dt, gamma, fmax, params, r, plain, t, cap, n,
                                  ws, wsb, self.cws, self.cws_bytes, stream)

    def backward(self, phi, target, F, dx, dt, gamma, fmax, params, stream=None):
        """Fills self.grad and self.loss (device)."""
        t, cap, n, ws, wsb = self._band()
        ls.ls_closure_backward_f32(phi, target, F, self.g, dx, dt, gamma, fmax, params, self.grad,
                                   self.loss, t, cap, n, ws, wsb, self.cws, self.cws_bytes, stream)

    def run(self, phi, F, dx, dt, gamma, fmax, params, nsteps, window=10, judge=True,
            stream=None):
        """Corrected narrow-band run, judged by a plain shadow run unless
        judge=False (0): True (1) judges the interface's topology per tile, 2
        its position as well (the fronts within one grid spacing), 3 the same
        within half a grid spacing;
        self.fallbacks and self.resets accumulate (zero them first)."""
        t, cap, n, ws, wsb = self._band()
        ls.ls_closure_run_f32(phi, F, self.g, dx, dt, gamma, fmax, params, nsteps, window, int(judge),
                              t, cap, n, self.fallbacks, self.resets, ws, wsb, self.cws,
                              self.cws_bytes, stream)

    def band_list(self):
        return self.bg.band_list()


class Adam:
    """Adam state of a device parameter vector (update in ls_adam_step)."""

    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.t = 0
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps

    def step(self, grad, lr=None, stream=None):
        self.t += 1
        ls.ls_adam_step(self.params, grad, self.m, self.v, self.params.numel(),
                        self.lr if lr is None else lr, self.beta1, self.beta2, self.eps, self.t,
                        stream)


def restrict4(fine, coarse=None, stream=None):
    """Device restriction of a (nz, ny, nx) FP32 field by 4 in every axis."""
    nz, ny, nx = fine.shape
    if coarse is None:
        coarse = torch.empty((nz // 4, ny // 4, nx // 4), dtype=torch.float32, device=fine.device)
    ls.ls_restrict4_f32(fine, ls.grid((nx, ny, nz)), coarse, stream)
    return coarse
