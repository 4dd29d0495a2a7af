"""Helpers of the GPU tests: device placement, tolerance bounds, reports."""
import json
import os

import numpy as np
import torch

EPS32 = float(np.finfo(np.float32).eps)


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def fp32_step_bound(phi, F, dx, dt, nsteps):
    """A bound on |FP32 - FP64| after nsteps of the upwind update.

    Each step rounds the stored value (1/2 ulp of the largest |phi| it can
    reach) and evaluates the increment dt*F*|grad| with a relative error of a
    few FP32 epsilons; the update is non-expansive in the max norm under the
    CFL condition, so the per-step errors add up.  Generous by a factor 4.
    """
    pmax = float(np.max(np.abs(phi)))
    gmax = 2 * np.sqrt(3) * pmax / dx  # largest one-sided difference norm
    incr = dt * float(np.max(np.abs(F))) * gmax
    reach = pmax + nsteps * incr
    return 4 * nsteps * (0.5 * EPS32 * reach + 8 * EPS32 * incr)


def random_tiles(rng, ntiles, frac):
    k = max(1, int(ntiles * frac))
    return np.sort(rng.choice(ntiles, size=min(k, ntiles), replace=False)).astype(np.int32)


def report(name, **fields):
    """Append a JSON record to $LS_REPORT_DIR/reports.jsonl when that variable
    names an existing folder."""
    out = os.environ.get("LS_REPORT_DIR", "")
    if out and os.path.isdir(out):
        with open(os.path.join(out, "reports.jsonl"), "a") as fh:
            fh.write(json.dumps({"test": name, **fields}) + "\n")


def error_by_band_distance(err, ref, dx, edges=(0, 1, 2, 4, 6, 8, 12, 16, 24, 32, 1e9)):
    """Max |err| (in dx) per |phi_ref| / dx bin."""
    d = np.abs(ref) / dx
    out = {}
    for lo, hi in zip(edges[:-1], edges[1:]):
        m = (d >= lo) & (d < hi)
        if m.any():
            out[f"{lo}-{hi if hi < 1e8 else 'inf'}"] = float(err[m].max() / dx)
    return out
