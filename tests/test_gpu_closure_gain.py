"""What the trained closure gains over the plain coarse scheme.

The network is trained on the GPU by the library's own kernels (forward,
backward, Adam) on restricted fine trajectories of six seeds (256^3 fine,
64^3 coarse, 60 coarse steps), then judged on two held-out seeds, teacher
forced: from the restricted fine field at coarse step n, one corrected coarse
step (the full driver: cut-off gate, limiter, per-tile fallback) against the
restricted fine field at n + 1.  Asserted: the training loss on the held-out
pairs falls, and the mean error of the step near the front (points with
|target| < dx_coarse) falls by at least 30 %.  Reported, not asserted: the
Hausdorff distance of 60-step roll-outs (plain, corrected, corrected with the
plain judge) to the restricted fine trajectory, on the coarse grid.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, report
from paper_1612_04040_amd import closure as C
from paper_1612_04040_amd import closure_train as T
from paper_1612_04040_amd import metrics as M
from paper_1612_04040_amd.band import BandGrid

pytestmark = pytest.mark.gpu

N_FINE, STEPS = 256, 60


@pytest.mark.timeout(600)
def test_trained_closure_beats_plain_step():
    d = dev()
    train_p = [T.Problem(s, N_FINE, STEPS, d) for s in range(100, 106)]
    val_p = [T.Problem(s, N_FINE, STEPS, d) for s in (200, 201)]
    nc = N_FINE // 4
    cg = C.ClosureGrid((nc,) * 3, d)
    zero = torch.from_numpy(C.init_params(np.random.default_rng(0)).astype(np.float32)).to(d)
    loss_plain = T.one_step_loss(cg, val_p, zero)
    front_plain = T.front_error(cg, val_p, zero)
    params = zero.clone()
    T.train(cg, train_p, params, 1500, 1e-3, seed=0, log_every=500, rollout_prob=0.0)
    loss_learned = T.one_step_loss(cg, val_p, params)
    front_learned = T.front_error(cg, val_p, params)

    rec = dict(n_fine=N_FINE, coarse_steps=STEPS, iters=1500, loss_plain=loss_plain,
               loss_learned=loss_learned, front_err_plain_dx_c=front_plain,
               front_err_learned_dx_c=front_learned, rollouts=[])
    bg = BandGrid((nc,) * 3, (8, 8, 8), "f32", d)
    for p in val_p:
        c = p.case
        target = M.zero_crossings(p.snaps[STEPS].cpu().numpy(), c.dx_coarse)
        out = {"seed": c.seed}
        for name in ("plain", "learned", "judged"):
            phi = p.snaps[0].clone()
            if name == "plain":
                bg.run(phi, p.F, c.dx_coarse, c.dt_coarse, c.gamma_coarse, STEPS, 10)
            else:
                cg.run(phi, p.F, c.dx_coarse, c.dt_coarse, c.gamma_coarse, c.fmax, params, STEPS,
                       10, judge=name == "judged")
            got = M.zero_crossings(phi.cpu().numpy(), c.dx_coarse)
            out[f"hausdorff_{name}_dx_c"] = M.hausdorff(got, target) / c.dx_coarse
        rec["rollouts"].append(out)
    report("closure_gain", **rec)
    print(f"[closure gain] {rec}", flush=True)

    assert loss_learned < 0.95 * loss_plain
    assert front_learned < 0.7 * front_plain
