"""Training and evaluation of the learned closure on the GPU.

Orchestration only: fine runs, restriction, forward, backward and Adam all run
in libls (``ls_upwind_step_f32``, ``ls_restrict4_f32``,
``ls_closure_backward_f32``, ``ls_adam_step``, ``ls_closure_run_f32``); the
host picks training pairs, schedules the learning rate and computes interface
metrics (zero crossings and Hausdorff distances, numpy / scipy).

Data: for every seed a fine grid (n_fine^3) is advanced by the plain scheme
over the whole grid (every tile updated, so the restricted field is a valid
target everywhere on the coarse band), and the fine field restricted 4x is
kept after every `ratio` fine steps (= one coarse step at the same CFL
number).  A training pair is (restricted field at coarse step n, at n + 1).

    python -m paper_1612_04040_amd.closure_train --out closure.json
"""
import argparse
import json
import math
import time

import numpy as np
import torch

from . import closure as C
from . import ls
from . import metrics
from . import workloads as W
from .band import BandGrid


def _dev(a, device):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def fine_trajectory(case, nsteps, device):
    """Restricted fine fields at coarse steps 0..nsteps, shape (nsteps+1, nc, nc, nc)."""
    nf, nc, ratio = case.n_fine, case.n_coarse, case.ratio
    phi = _dev(case.phi(nf), device)
    F = _dev(case.F(nf), device)
    bg = BandGrid((nf, nf, nf), (8, 8, 8), "f32", device)
    every = torch.arange(bg.capacity, dtype=torch.int32, device=device)
    count = torch.tensor([bg.capacity], dtype=torch.int32, device=device)
    snaps = torch.empty((nsteps + 1, nc, nc, nc), dtype=torch.float32, device=device)
    for k in range(nsteps):
        C.restrict4(phi, snaps[k])
        bg.step(phi, F, case.dx_fine, case.dt_fine, ratio, tiles=every, ntiles=count)
    C.restrict4(phi, snaps[nsteps])
    del phi, F, bg
    return snaps


class Problem:
    """Device inputs of one seed on the coarse grid (plane=True: a plane front)."""

    def __init__(self, seed, n_fine, nsteps, device, with_trajectory=True, plane=False):
        self.case = (W.PlaneCase if plane else W.ClosureCase)(seed, n_fine)
        nc = self.case.n_coarse
        self.F = _dev(self.case.F(nc), device)
        self.snaps = fine_trajectory(self.case, nsteps, device) if with_trajectory else None


def train(cg, problems, params, iters, lr, seed=0, log_every=200, rollout_max=8,
          rollout_from=0.25, rollout_prob=0.5):
    """Adam on random (seed, step) pairs; returns the loss log.

    After the first `rollout_from` of the iterations, with probability
    `rollout_prob` the input of a pair is not the restricted fine field but the
    corrected coarse run of the current network started k <= rollout_max steps
    earlier from it (no gradient through the roll-out), so the network also
    learns to correct its own drift; the target stays the restricted fine
    field one step later."""
    rng = np.random.default_rng(seed)
    opt = C.Adam(params, lr=lr)
    log = []
    acc = torch.zeros(1, dtype=torch.float32, device=params.device)
    tmp = torch.empty_like(problems[0].snaps[0])
    for it in range(iters):
        p = problems[rng.integers(len(problems))]
        n = int(rng.integers(p.snaps.shape[0] - 1))
        c = p.case
        x = p.snaps[n]
        if it >= rollout_from * iters and rng.random() < rollout_prob:
            k = int(rng.integers(1, rollout_max + 1))
            if n >= k:
                tmp.copy_(p.snaps[n - k])
                cg.run(tmp, p.F, c.dx_coarse, c.dt_coarse, c.gamma_coarse, c.fmax, params, k,
                       10, judge=False)
                x = tmp
        cg.backward(x, p.snaps[n + 1], p.F, c.dx_coarse, c.dt_coarse, c.gamma_coarse, c.fmax,
                    params)
        # cosine decay to lr / 100
        lr_t = lr * (0.01 + 0.99 * 0.5 * (1 + math.cos(math.pi * it / max(1, iters))))
        opt.step(cg.grad, lr=lr_t)
        acc += cg.loss
        if (it + 1) % log_every == 0:
            log.append((it + 1, float(acc.item()) / log_every))
            acc.zero_()
            if (it + 1) % (5 * log_every) == 0:
                print(f"train: iter {it + 1}, mean loss {log[-1][1]:.4g}", flush=True)
    return log


def one_step_loss(cg, problems, params, every=10):
    """Mean training loss over every `every`-th pair of the given problems."""
    tot, cnt = 0.0, 0
    for p in problems:
        c = p.case
        for n in range(0, p.snaps.shape[0] - 1, every):
            cg.backward(p.snaps[n], p.snaps[n + 1], p.F, c.dx_coarse, c.dt_coarse,
                        c.gamma_coarse, c.fmax, params)
            tot += float(cg.loss.item())
            cnt += 1
    return tot / max(cnt, 1)


def front_error(cg, problems, params, every=10):
    """Teacher-forced error of one corrected coarse step (the driver with
    gate, limiter and fallback; no judge) near the front: mean |phi^{n+1} - target| over
    the points with |target| < dx_coarse, in dx_coarse, over every `every`-th
    pair.  With the zero parameters it is the plain scheme's error."""
    tot, cnt = 0.0, 0
    x = torch.empty_like(problems[0].snaps[0])
    for p in problems:
        c = p.case
        for n in range(0, p.snaps.shape[0] - 1, every):
            x.copy_(p.snaps[n])
            cg.run(x, p.F, c.dx_coarse, c.dt_coarse, c.gamma_coarse, c.fmax, params, 1, 10,
                   judge=False)
            t = p.snaps[n + 1]
            front = t.abs() < c.dx_coarse
            tot += float(((x - t).abs()[front]).sum().item()) / c.dx_coarse
            cnt += int(front.sum().item())
    return tot / max(cnt, 1)


def _timed(fn, stream, reps=3):
    """Median wall time (ms) of fn() between HIP events on `stream`."""
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out))


def _graph_timed(body, stream, reps=3):
    """Captures body(stream) into a HIP graph (every launch of the run, the
    reset of phi included), then times its replays; also times one eager
    call.  Returns (graph ms, eager ms)."""
    eager = _timed(lambda: body(stream), stream, 1)
    torch.cuda.synchronize()
    ls.ls_graph_begin(stream)
    body(stream)
    graph = ls.ls_graph_end(stream)
    try:
        ms = _timed(lambda: ls.ls_graph_launch(graph, stream), stream, reps)
    finally:
        ls.ls_graph_destroy(graph)
    return ms, eager


def evaluate(seed, n_fine, nsteps, params, device, reps=3):
    """Plain fine (band) vs plain coarse vs learned coarse (without and with
    the plain judge), from the same restricted initial field; each whole run
    captured in a HIP graph and timed on replay; Hausdorff distances in fine
    dx, also for the restricted fine result (what a coarse grid can hold)."""
    case = W.ClosureCase(seed, n_fine)
    nf, nc, ratio = case.n_fine, case.n_coarse, case.ratio
    phi_f0 = _dev(case.phi(nf), device)
    F_f = _dev(case.F(nf), device)
    F_c = _dev(case.F(nc), device)
    phi_c0 = C.restrict4(phi_f0)
    out = {"seed": seed, "n_fine": nf, "n_coarse": nc, "coarse_steps": nsteps,
           "fine_steps": nsteps * ratio}
    stream = torch.cuda.Stream(device)

    bgf = BandGrid((nf,) * 3, (8, 8, 8), "f32", device)
    phi_f = torch.empty_like(phi_f0)

    def fine_run(s):
        ls.ls_copy_f32(phi_f, phi_f0, phi_f.numel(), s)
        bgf.run(phi_f, F_f, case.dx_fine, case.dt_fine, case.gamma_fine, nsteps * ratio, 10,
                stream=s)

    out["fine_ms"], out["fine_eager_ms"] = _graph_timed(fine_run, stream, reps)
    fine = phi_f.cpu().numpy()
    # what a coarse grid can hold at best: the fine result restricted
    best = C.restrict4(phi_f).cpu().numpy()
    del bgf, F_f

    bgc = BandGrid((nc,) * 3, (8, 8, 8), "f32", device)
    phi_p = torch.empty_like(phi_c0)

    def plain_run(s):
        ls.ls_copy_f32(phi_p, phi_c0, phi_p.numel(), s)
        bgc.run(phi_p, F_c, case.dx_coarse, case.dt_coarse, case.gamma_coarse, nsteps, 10,
                stream=s)

    out["plain_coarse_ms"], out["plain_coarse_eager_ms"] = _graph_timed(plain_run, stream, reps)
    plain = phi_p.cpu().numpy()

    cg = C.ClosureGrid((nc,) * 3, device)
    phi_l = torch.empty_like(phi_c0)
    zero_i = torch.zeros(1, dtype=torch.int32, device=device)
    fields = {}
    # the product run is "judged" (the plain shadow judges the topology and the
    # position of the front per tile, judge mode 2); the topology judge alone
    # (mode 1), the position bound at half a grid spacing (mode 3) and no judge
    # are reported beside it
    for name, judge in (("learned", 0), ("judged_topology", 1), ("judged", 2),
                        ("judged_half", 3)):
        def learned_run(s):
            ls.ls_copy_f32(phi_l, phi_c0, phi_l.numel(), s)
            ls.ls_copy_f32(cg.fallbacks, zero_i, 1, s)  # int32 zeros, same width
            ls.ls_copy_f32(cg.resets, zero_i, 1, s)
            cg.run(phi_l, F_c, case.dx_coarse, case.dt_coarse, case.gamma_coarse, case.fmax,
                   params, nsteps, 10, judge=judge, stream=s)

        out[f"{name}_coarse_ms"], out[f"{name}_coarse_eager_ms"] = _graph_timed(
            learned_run, stream, reps)
        out[f"{name}_fallbacks"] = int(cg.fallbacks.item())
        if judge:
            out[f"{name}_resets"] = int(cg.resets.item())
        fields[name] = phi_l.cpu().numpy()

    dxf = case.dx_fine
    pf = metrics.zero_crossings(fine, dxf)
    for name, field in (("restricted_fine", best), ("plain_coarse", plain),
                        ("learned_coarse", fields["learned"]),
                        ("judged_topology_coarse", fields["judged_topology"]),
                        ("judged_coarse", fields["judged"]),
                        ("judged_half_coarse", fields["judged_half"])):
        up = metrics.upsample_trilinear(field, ratio)
        pc = metrics.zero_crossings(up, dxf)
        out[f"hausdorff_{name}_dx_fine"] = metrics.hausdorff(pc, pf) / dxf
        del up
    # against what the coarse grid can hold: the restricted fine result, on the
    # coarse lattice (in fine dx)
    pb = metrics.zero_crossings(best, case.dx_coarse)
    for name, field in (("plain_coarse", plain), ("learned_coarse", fields["learned"]),
                        ("judged_topology_coarse", fields["judged_topology"]),
                        ("judged_coarse", fields["judged"]),
                        ("judged_half_coarse", fields["judged_half"])):
        pc = metrics.zero_crossings(field, case.dx_coarse)
        out[f"hausdorff_{name}_to_restricted_dx_fine"] = metrics.hausdorff(pc, pb) / dxf
    out["speedup_judged_vs_fine"] = out["fine_ms"] / out["judged_coarse_ms"]
    return out


def _seeds(spec):
    lo, hi = (int(v) for v in spec.split("-"))
    return list(range(lo, hi + 1))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n-fine", type=int, default=512)
    ap.add_argument("--coarse-steps", type=int, default=400)
    ap.add_argument("--train-seeds", default="100-131")
    ap.add_argument("--val-seeds", default="200-203")
    ap.add_argument("--eval-seed", type=int, default=5)
    ap.add_argument("--iters", type=int, default=20000)
    ap.add_argument("--rollout-max", type=int, default=4)
    ap.add_argument("--rollout-prob", type=float, default=0.5)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--params-out", default=None, help="save the trained parameters (.npy)")
    ap.add_argument("--out", default=None, help="write the JSON report here")
    args = ap.parse_args(argv)
    device = torch.device("cuda:0")
    report = {"args": vars(args)}

    t0 = time.time()
    train_p, val_p = [], []
    for s in _seeds(args.train_seeds) + _seeds(args.val_seeds):
        (train_p if len(train_p) < len(_seeds(args.train_seeds)) else val_p).append(
            Problem(s, args.n_fine, args.coarse_steps, device))
        print(f"data: seed {s} ready ({time.time() - t0:.1f} s)", flush=True)
    torch.cuda.synchronize()
    report["data_s"] = time.time() - t0
    print(f"data: {len(train_p)} train / {len(val_p)} val seeds in {report['data_s']:.1f} s",
          flush=True)

    nc = args.n_fine // 4
    cg = C.ClosureGrid((nc,) * 3, device)
    zero = _dev(C.init_params(np.random.default_rng(args.init_seed)).astype(np.float32), device)
    params = zero.clone()
    report["val_loss_plain"] = one_step_loss(cg, val_p, zero)
    t0 = time.time()
    report["train_log"] = train(cg, train_p, params, args.iters, args.lr, seed=args.init_seed,
                                rollout_max=args.rollout_max, rollout_prob=args.rollout_prob)
    torch.cuda.synchronize()
    report["train_s"] = time.time() - t0
    report["val_loss_learned"] = one_step_loss(cg, val_p, params)
    report["val_front_err_plain_dx_c"] = front_error(cg, val_p, zero)
    report["val_front_err_learned_dx_c"] = front_error(cg, val_p, params)
    print(f"train: {args.iters} iters in {report['train_s']:.1f} s, val loss "
          f"{report['val_loss_plain']:.4g} (plain) -> {report['val_loss_learned']:.4g}, one-step "
          f"front error {report['val_front_err_plain_dx_c']:.4g} -> "
          f"{report['val_front_err_learned_dx_c']:.4g} dx_c", flush=True)
    del train_p, val_p
    torch.cuda.empty_cache()

    gate = []
    for s in _seeds(args.val_seeds):
        e = evaluate(s, args.n_fine, args.coarse_steps, params, device, reps=1)
        gate.append(e)
        print(f"val seed {s}: H restricted fine {e['hausdorff_restricted_fine_dx_fine']:.3f}, "
              f"plain {e['hausdorff_plain_coarse_dx_fine']:.3f}, "
              f"learned {e['hausdorff_learned_coarse_dx_fine']:.3f}, "
              f"judged {e['hausdorff_judged_coarse_dx_fine']:.3f} dx_f; to the restricted fine "
              f"result: plain {e['hausdorff_plain_coarse_to_restricted_dx_fine']:.3f}, "
              f"judged {e['hausdorff_judged_coarse_to_restricted_dx_fine']:.3f} dx_f", flush=True)
    report["validation"] = gate
    # the product run is the judged one: enabled if it beats the plain coarse
    # scheme on the held-out seeds (mean Hausdorff distance to the fine run)
    report["model_enabled"] = bool(np.mean([e["hausdorff_judged_coarse_dx_fine"] for e in gate]) <
                                   np.mean([e["hausdorff_plain_coarse_dx_fine"] for e in gate]))
    ev = evaluate(args.eval_seed, args.n_fine, args.coarse_steps, params, device)
    report["evaluation"] = ev
    print(json.dumps(ev), flush=True)
    if args.params_out:
        np.save(args.params_out, params.cpu().numpy())
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(report, fh, indent=1)
    return report


if __name__ == "__main__":
    main()
