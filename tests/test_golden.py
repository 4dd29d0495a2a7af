"""Stored expected values (tests/golden/, written by make_golden.py from the
oracle alone): the oracle must still produce them bit for bit, and so must
the GPU's FP64 path (a regression fixture: it pins nothing the oracle pins
do not, but any change of either side's arithmetic shows here first)."""
import importlib.util
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "sphere40_f64.json")


def _maker():
    spec = importlib.util.spec_from_file_location("make_golden",
                                                  os.path.join(HERE, "golden", "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_oracle_reproduces_golden():
    with open(GOLDEN) as fh:
        want = json.load(fh)
    assert _maker().compute() == want


@pytest.mark.gpu
def test_gpu_f64_reproduces_golden():
    import torch

    from paper_1612_04040_amd.band import BandGrid

    with open(GOLDEN) as fh:
        want = json.load(fh)
    mk = _maker()
    phi, F, dx, dt = mk.sphere_case()
    n = phi.shape[0]
    dev = torch.device("cuda:0")
    bg = BandGrid((n, n, n), (8, 8, 8), "f64", device=dev)
    pd = torch.from_numpy(phi).to(dev)
    Fd = torch.from_numpy(F).to(dev)
    every = torch.arange(bg.capacity, dtype=torch.int32, device=dev)
    count = torch.tensor([bg.capacity], dtype=torch.int32, device=dev)
    bg.step(pd, Fd, dx, dt, want["steps"], tiles=every, ntiles=count)
    got = pd.cpu().numpy()
    for k, j, i, v in want["samples"]:
        assert repr(float(got[k, j, i])) == v, (k, j, i)
    f32 = torch.from_numpy(got.astype(np.float32)).to(dev)
    b32 = BandGrid((n, n, n), (8, 8, 8), "f32", device=dev)
    gamma = float(np.float32(3 * dx))
    b32.build(f32, gamma, dilate=True)
    assert b32.band_list().tolist() == want["band_u"]
    b32.build(f32, gamma, dilate=False)
    assert b32.band_list().tolist() == want["band_a"]
