"""Learned warm start for runs to steady state: training data from the
solver, training of the network on the GPU, and the warm-versus-cold
comparison.  Every step runs in the library's kernels (the batch solver of
``lem.h`` and the network of ``lem_surrogate.h``); this module only moves
arrays and drives the loops.

    python -m paper_1803_02977_amd.warmstart train --samples 20000 --out weights.npz
    python -m paper_1803_02977_amd.warmstart evaluate --weights weights.npz --grids 100

Training targets are steady states of the solver (no cell changes by more
than 1e-6 of the grid's largest height in one step) from seeded (K, U, h0)
realizations at the workload's dt = 1000 yr.  They are reached by
steady-state projections (every cell set to where the implicit update leaves
it, given the routing of the current heights; lem_batch_project_to_steady)
until the heights stop changing, then confirmed by the method's own steps;
``--gen steps`` uses steps alone.  The evaluation times, on held-out
realizations, the cold start (noise surface) and the warm start (the
network's prediction), each by steps alone and by projections then steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

from .lem import Batch  # noqa: E402
from .surrogate import Surrogate, init_params, load_params, save_params  # noqa: E402

DX = 100.0
M = 0.5
DT = 1000.0
RTOL = 1e-6
WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warmstart_weights.npz")


def _log(msg):
    print(f"[warmstart] {msg}", flush=True)


def _grids(u, ny, nx, dt):
    """Batch descriptors; u holds each grid's uplift rate (its field is
    passed separately, as is K)."""
    return [W.Realization(ny, nx, DX, DX, dt, M, float(v), 1e-5, 0) for v in u]


def steady_states(K, U, h0, dt=DT, check_every=10, max_steps=200000, chunk=None,
                  label="steady", project=False, stats=None):
    """Runs the batch solver from h0 (device tensors [n, ny, nx]) with the K
    and U fields until every grid is steady; returns (h, steps per grid).
    With ``project`` the run starts with steady-state projections until they
    stop changing the heights (lem_batch_project_to_steady), then the
    method's steps confirm the steady state; ``stats`` (a dict) receives the
    projections per grid and the seconds of both parts."""
    import torch
    n, ny, nx = K.shape
    b = Batch(_grids(U[:, 0, 0].cpu().numpy(), ny, nx, dt), device=K.device)
    h = h0.reshape(-1).clone()
    t0 = time.perf_counter()

    def progress(done, conv):
        _log(f"{label}: {done} steps, {conv}/{n} grids steady, {time.perf_counter() - t0:.1f} s")

    if project:
        its = b.project_to_steady(h, rtol=RTOL, check_every=check_every, max_iters=max_steps,
                                  K=K.reshape(-1), U=U.reshape(-1))
        torch.cuda.synchronize()
        if stats is not None:
            stats["projections"] = its
            stats["project_s"] = time.perf_counter() - t0
        _log(f"{label}: projections done ({int(np.max(its))} at most), "
             f"{time.perf_counter() - t0:.1f} s")
    t1 = time.perf_counter()
    steps = b.run_to_steady(h, rtol=RTOL, check_every=check_every, max_steps=max_steps,
                            K=K.reshape(-1), U=U.reshape(-1), chunk=chunk, progress=progress)
    torch.cuda.synchronize()
    if stats is not None:
        stats["steps_s"] = time.perf_counter() - t1
    b.close()
    return h.reshape(K.shape), steps


def steady_states_queue(K, U, h_init, slots, dt=DT, check_every=10, chunk=500,
                        max_steps=200000, label="queue"):
    """Runs many realizations to steady state through a batch of `slots`
    identical grids: whenever a grid converges its slot is refilled with the
    next realization (heights, K and U fields), so the batch stays full and
    the run's time follows the total number of steps rather than the
    slowest realization.  Each realization evolves exactly as it would
    alone (grids of a batch are independent), so results and step counts
    equal those of steady_states().  Returns (h, steps per realization)."""
    import torch

    from .lem import lem_batch_run_to_steady
    n, ny, nx = K.shape
    if chunk % check_every:
        raise ValueError("chunk must be a multiple of check_every")
    S = min(slots, n)
    cells = ny * nx
    b = Batch(_grids(np.full(S, 1e-3), ny, nx, dt), device=K.device)
    hs = torch.zeros(S * cells, dtype=torch.float64, device=K.device)
    Ks = torch.full_like(hs, 1e-5)
    Us = torch.zeros_like(hs)
    hv, Kv, Uv = hs.view(S, ny, nx), Ks.view(S, ny, nx), Us.view(S, ny, nx)
    state = np.zeros(S, np.int64)   # >= 0: idle or converged (not stepped); -1: running
    item = np.full(S, -1)
    age = np.zeros(S, np.int64)
    steps = np.full(n, -1, np.int64)
    h_out = torch.empty_like(K)
    nxt = 0
    t0 = time.perf_counter()

    def load(g):
        nonlocal nxt
        hv[g].copy_(h_init[nxt])
        Kv[g].copy_(K[nxt])
        Uv[g].copy_(U[nxt])
        item[g], age[g], state[g] = nxt, 0, -1
        nxt += 1

    for g in range(S):
        load(g)
    rounds = 0
    while (state < 0).any():
        got = lem_batch_run_to_steady(b.ctx, hs.data_ptr(), Ks.data_ptr(), Us.data_ptr(), RTOL,
                                      check_every, chunk, S, steps_in=state)
        for g in range(S):
            if state[g] >= 0:
                continue
            if got[g] >= 0 or age[g] + chunk >= max_steps:
                steps[item[g]] = age[g] + got[g] if got[g] >= 0 else -1
                h_out[item[g]].copy_(hv[g])
                if nxt < n:
                    load(g)
                else:
                    state[g] = 0
            else:
                age[g] += chunk
        rounds += 1
        if rounds % 8 == 0:
            _log(f"{label}: {int((steps >= 0).sum())}/{n} steady, "
                 f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    b.close()
    return h_out, steps


def make_dataset(count, first_seed, device, piece=1000):
    """Seeded realizations uploaded to the device in pieces of `piece`."""
    import torch
    side = W.WARMSTART_SIDE
    K = torch.empty((count, side, side), dtype=torch.float64, device=device)
    U = torch.empty_like(K)
    h0 = torch.empty_like(K)
    for i in range(0, count, piece):
        k = min(piece, count - i)
        a, b, c = W.warmstart_inputs(k, first_seed + i)
        K[i:i + k].copy_(torch.from_numpy(a))
        U[i:i + k].copy_(torch.from_numpy(b))
        h0[i:i + k].copy_(torch.from_numpy(c))
    return K, U, h0


def validation_loss(net, K, U, h0, target, batch):
    """Mean loss over held-out samples (whole batches only)."""
    n = (K.shape[0] // batch) * batch
    acc = 0.0
    for i in range(0, n, batch):
        loss, _ = net.loss_grad(K[i:i + batch].contiguous(), U[i:i + batch].contiguous(),
                                h0[i:i + batch].contiguous(), target[i:i + batch].contiguous())
        acc += loss
    return acc / max(n // batch, 1)


def train(net, K, U, h0, target, epochs, batch, lr, lr_min, seed=0, log_every=200, val=None):
    """Adam with a cosine learning-rate decay over all steps; returns the
    per-epoch mean losses (and, with val = (K, U, h0, target) of held-out
    samples, their loss after each epoch)."""
    import torch
    n = K.shape[0]
    rng = np.random.default_rng(seed)
    per_epoch = n // batch
    total = epochs * per_epoch
    losses, val_losses = [], []
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(n)).to(K.device)
        acc = 0.0
        for j in range(per_epoch):
            idx = order[j * batch:(j + 1) * batch]
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * step / max(total, 1)))
            loss = net.train_step(K[idx].contiguous(), U[idx].contiguous(), h0[idx].contiguous(),
                                  target[idx].contiguous(), lr=lr_t)
            acc += loss
            step += 1
            if step % log_every == 0:
                _log(f"epoch {ep} step {step}/{total} loss {loss:.5f} lr {lr_t:.2e} "
                     f"{time.perf_counter() - t0:.1f} s")
        losses.append(acc / per_epoch)
        if val is not None:
            val_losses.append(validation_loss(net, *val, batch))
            _log(f"epoch {ep} mean loss {losses[-1]:.5f}, held-out loss {val_losses[-1]:.5f}")
        else:
            _log(f"epoch {ep} mean loss {losses[-1]:.5f}")
    return (losses, val_losses) if val is not None else losses


def predict(net, K, U, h0, batch):
    import torch
    out = torch.empty_like(K)
    for i in range(0, K.shape[0], batch):
        j = min(i + batch, K.shape[0])
        out[i:j] = net.predict(K[i:j].contiguous(), U[i:j].contiguous(), h0[i:j].contiguous())
    return out


def evaluate(net, grids, first_seed=W.WARMSTART_TEST_SEED, batch=16, dt=DT, check_every=10,
             max_steps=200000, chunk=2000, device="cuda:0", slots=None, plain_sample=0,
             project=False):
    """Steps and device time to steady state from the noise surface (cold)
    and from the network's prediction (warm), on held-out realizations, with
    the same solver, dt and stopping rule.  slots=None runs all realizations
    as one batch (time = slowest realization); otherwise a batch of `slots`
    grids is refilled as realizations converge (steady_states_queue).
    plain_sample > 0 also runs that many realizations from the noise surface
    one after another through the single-grid path (the plain solver).
    project=True also times both starts with steady-state projections before
    the steps (one batch)."""
    import torch
    dev = torch.device(device)
    K, U, h0 = make_dataset(grids, first_seed, dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    hp = predict(net, K, U, h0, batch)
    torch.cuda.synchronize()
    t_pred = time.perf_counter() - t

    def run(h_start, label):
        if slots:
            return steady_states_queue(K, U, h_start, slots, dt=dt, check_every=check_every,
                                       chunk=min(chunk, 500), max_steps=max_steps, label=label)
        return steady_states(K, U, h_start, dt=dt, check_every=check_every,
                             max_steps=max_steps, chunk=chunk, label=label)

    t = time.perf_counter()
    h_cold, s_cold = run(h0, "cold")
    t_cold = time.perf_counter() - t
    t = time.perf_counter()
    h_warm, s_warm = run(hp, "warm")
    t_warm = time.perf_counter() - t
    plain = None
    if plain_sample:
        t = time.perf_counter()
        ps = []
        for i in range(plain_sample):
            _, st = steady_states(K[i:i + 1].contiguous(), U[i:i + 1].contiguous(),
                                  h0[i:i + 1].contiguous(), dt=dt, check_every=check_every,
                                  max_steps=max_steps, chunk=chunk, label=f"plain {i}")
            ps.append(int(st[0]))
        t_plain = time.perf_counter() - t
        plain = {"realizations": plain_sample, "s": t_plain,
                 "s_per_realization": t_plain / plain_sample,
                 "steps_match_batch": ps == [int(v) for v in s_cold[:plain_sample]]}
    rel = lambda a, b: float((torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item())
    projected = None
    if project:
        projected = {}
        for label, h_start, extra in (("cold", h0, 0.0), ("warm", hp, t_pred)):
            st = {}
            t = time.perf_counter()
            h_fin, s_fin = steady_states(K, U, h_start, dt=dt, check_every=check_every,
                                         max_steps=max_steps, chunk=chunk,
                                         label=f"{label}+projection", project=True, stats=st)
            total = time.perf_counter() - t + extra
            its = st["projections"]
            projected[label] = {
                "s": total, "project_s": st["project_s"], "steps_s": st["steps_s"],
                "projections_mean": float(np.mean(its)), "projections_max": int(np.max(its)),
                "steps_after_mean": float(np.mean(s_fin)), "steps_after_max": int(np.max(s_fin)),
                "all_converged": bool((its >= 0).all() and (s_fin >= 0).all()),
                "rel_l2_vs_cold_steady": rel(h_fin, h_cold)}
        projected["time_ratio_warm_over_cold"] = projected["warm"]["s"] / projected["cold"]["s"]
        projected["time_ratio_warm_projected_over_cold_steps"] = projected["warm"]["s"] / t_cold
    return {
        "projected": projected,
        "plain": plain,
        "grids": grids, "side": int(K.shape[1]), "dt": dt, "rtol": RTOL,
        "check_every": check_every,
        "cold_steps": s_cold.tolist(), "warm_steps": s_warm.tolist(),
        "slots": slots or grids,
        "cold_steps_mean": float(np.mean(s_cold)), "warm_steps_mean": float(np.mean(s_warm)),
        "cold_steps_pct": [int(v) for v in np.percentile(s_cold, [10, 50, 90, 100])],
        "warm_steps_pct": [int(v) for v in np.percentile(s_warm, [10, 50, 90, 100])],
        "steps_ratio_warm_over_cold": float(np.sum(s_warm) / np.sum(s_cold)),
        "warm_fewer_steps_frac": float(np.mean(s_warm < s_cold)),
        "all_converged": bool((s_cold >= 0).all() and (s_warm >= 0).all()),
        "cold_s": t_cold, "warm_s": t_warm + t_pred, "predict_s": t_pred,
        "time_ratio_warm_over_cold": (t_warm + t_pred) / t_cold,
        "prediction_rel_l2_vs_cold_steady": rel(hp, h_cold),
        "noise_rel_l2_vs_cold_steady": rel(h0, h_cold),
        "warm_steady_rel_l2_vs_cold_steady": rel(h_warm, h_cold),
    }


def main():
    import torch
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--samples", type=int, default=20000)
    t.add_argument("--epochs", type=int, default=4)
    t.add_argument("--batch", type=int, default=16)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--lr-min", type=float, default=5e-5)
    t.add_argument("--gen-dt", type=float, default=DT)
    t.add_argument("--gen", choices=("project", "steps"), default="project",
                   help="targets: fixed points of steady-state projections (then confirmed by "
                        "steps), or runs of steps alone")
    t.add_argument("--val", type=int, default=1000, help="held-out samples for the validation loss")
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--out", default=WEIGHTS_PATH)
    t.add_argument("--report", default=None)
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", default=WEIGHTS_PATH)
    e.add_argument("--grids", type=int, default=100)
    e.add_argument("--report", default=None)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    side = W.WARMSTART_SIDE
    report = {}
    if args.cmd == "train":
        t0 = time.perf_counter()
        total = args.samples + args.val
        # Training seeds, then the validation seeds right after them (the
        # evaluation's held-out seeds start far above both).
        K, U, h0 = make_dataset(total, W.WARMSTART_TRAIN_SEED, dev)
        _log(f"inputs for {total} realizations on the device, {time.perf_counter() - t0:.1f} s")
        t0 = time.perf_counter()
        st = {}
        hs, steps = steady_states(K, U, h0, dt=args.gen_dt, chunk=200, label="data",
                                  project=args.gen == "project", stats=st)
        t_gen = time.perf_counter() - t0
        its = st.get("projections", np.zeros_like(steps))
        ok = (steps >= 0) & (its >= 0)
        _log(f"steady states: {int(ok.sum())}/{total} converged, mean {steps[ok].mean():.0f} "
             f"steps after {its[ok].mean():.0f} projections, {t_gen:.1f} s")
        tr = np.nonzero(ok[:args.samples])[0]
        va = args.samples + np.nonzero(ok[args.samples:])[0]
        sel = lambda idx: tuple(a[torch.from_numpy(idx).to(dev)] for a in (K, U, h0, hs))
        Kt, Ut, h0t, hst = sel(tr)
        val = sel(va) if len(va) else None
        del K, U, h0, hs
        net = Surrogate(args.batch, side, side, device=dev)
        net.set_params(init_params(args.seed))
        t0 = time.perf_counter()
        out = train(net, Kt, Ut, h0t, hst, args.epochs, args.batch, args.lr, args.lr_min,
                    seed=args.seed, val=val)
        losses, val_losses = out if val is not None else (out, [])
        t_train = time.perf_counter() - t0
        p = net.get_params().cpu().numpy()
        save_params(args.out, p)
        report = {"samples": args.samples, "validation_samples": int(len(va)),
                  "converged": int(ok.sum()), "gen": args.gen, "gen_dt": args.gen_dt,
                  "gen_projections_mean": float(its[ok].mean()),
                  "gen_steps_mean": float(steps[ok].mean()), "gen_s": t_gen,
                  "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
                  "epoch_losses": losses, "validation_losses": val_losses, "train_s": t_train,
                  "train_steps_per_s": args.epochs * (len(tr) // args.batch) / t_train}
        _log(json.dumps(report))
    else:
        net = Surrogate(16, side, side, device=dev)
        net.set_params(load_params(args.weights))
        report = evaluate(net, args.grids)
        _log(json.dumps({k: v for k, v in report.items() if not isinstance(v, list)}))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
