"""Learned initial guess for the steady-state solver (not part of the paper).

The data path, all on the GPU through the library:
  1. solve cavities to steady state with the batched solver;
  2. resample u / U_char, v / U_char and theta = T + 1/2 of each steady
     cavity onto the res x res canvas (lf_resample, bilinear, cell-centred);
  3. train the network (lf_net_*) on (log10 Ra, Pr, A) -> fields;
  4. for new cavities, predict the canvas fields, resample them onto each
     cavity's grid, initialise f = f_eq(1, u_pred) and T = T_pred
     (lf_batch_init_device) and run to steady state as usual.

This module only sequences library calls and moves device pointers; random
draws (sample order, initial weights, perturbations) are inputs.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import Batch, Context, Net, resample

CHANNELS = ("u", "v", "T")


def features(cases) -> np.ndarray:
    """[n][3] float32: log10 Ra, Pr, aspect nx / ny."""
    return np.array([[math.log10(c["Ra"]), c["Pr"], c["nx"] / c["ny"]] for c in cases],
                    np.float32)


def solve(ctx: Context, cases, T0=None, tol=1e-8, check_every=1000, max_steps=2_000_000,
          chunk=100_000, log=None, batch: Batch | None = None):
    """Run a batch of cavities to steady state (FP32, stop rule of
    lf_batch_run_to_steady), in calls of growing step limit so that progress
    can be reported.  Returns (batch, steps, rules, residuals, seconds)."""
    b = batch if batch is not None else Batch(ctx, cases, "f32")
    if batch is None:
        b.init(T0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    limit = 0
    while True:
        limit = min(limit + chunk, max_steps)
        steps, rules, r = b.run_to_steady(tol, check_every, limit, raise_on_notconv=False)
        done = int(np.count_nonzero(rules != 0))
        if log:
            log(f"  {done}/{len(cases)} cavities steady after up to {limit} steps, "
                f"{time.perf_counter() - t0:.1f} s")
        if done == len(cases) or limit >= max_steps or np.any(rules < 0):
            break
    torch.cuda.synchronize()
    return b, steps, rules, r, time.perf_counter() - t0


def dataset_from_batch(ctx: Context, b: Batch, cases, res=128) -> torch.Tensor:
    """Target planes [n][3][res][res] (float32, device) from a batch's fields."""
    out = torch.empty(len(cases), 3, res, res, dtype=torch.float32, device=f"cuda:{ctx.device}")
    for k, c in enumerate(cases):
        U = b.params(k)["U_char"]
        tmp = torch.empty(c["ny"], c["nx"], dtype=torch.float32, device=out.device)
        for ch, name in enumerate(CHANNELS):
            b.fetch_device(k, name, tmp)
            scale, off = (1.0 / U, 0.0) if name != "T" else (1.0, 0.5)
            resample(ctx, tmp, out[k, ch], scale, off)
        ctx.stream.synchronize()  # tmp is reused
    return out


def lr_at(step, total, lr0, warmup=100):
    """Linear warm-up then cosine decay to lr0 / 50."""
    if step < warmup:
        return lr0 * (step + 1) / warmup
    x = (step - warmup) / max(1, total - warmup)
    return lr0 * (0.02 + 0.98 * 0.5 * (1.0 + math.cos(math.pi * min(1.0, x))))


def train(net: Net, feat: torch.Tensor, target: torch.Tensor, order: np.ndarray, lr0=2e-3,
          log=None, log_every=500):
    """Adam steps over the rows of order ([steps][batch] sample indices);
    returns the loss read back every log_every steps."""
    order_dev = torch.tensor(np.ascontiguousarray(order, np.int32), device=feat.device)
    hist = []
    total = order.shape[0]
    t0 = time.perf_counter()
    for s in range(total):
        net.train_step(feat, target, order_dev[s], lr_at(s, total, lr0))
        if (s + 1) % log_every == 0 or s + 1 == total:
            loss = net.loss()
            hist.append((s + 1, loss))
            if log:
                log(f"  step {s + 1}/{total}: loss {loss:.3e}, {time.perf_counter() - t0:.1f} s")
    return hist


def warm_init(ctx: Context, net: Net, b: Batch, cases, antisym=True):
    """Predict the fields of every cavity of b and initialise it with them.
    antisym: keep only the part of each predicted field that is odd under the
    180-degree rotation of the cavity, as the side-heated cavity's steady
    state is (hot and cold walls opposite, T_ref midway): the cold start
    from T ~ 0 never leaves that class, and prediction errors outside it
    excite slowly decaying modes."""
    dev = f"cuda:{ctx.device}"
    feat = torch.tensor(features(cases), device=dev)
    R = net.res
    pred = torch.empty(len(cases), 3, R, R, dtype=torch.float32, device=dev)
    for k0 in range(0, len(cases), net.max_batch):
        nb = min(net.max_batch, len(cases) - k0)
        idx = torch.arange(k0, k0 + nb, dtype=torch.int32, device=dev)
        net.forward(feat, idx, pred=pred[k0:k0 + nb])
    T0, u0, v0 = [], [], []
    for k, c in enumerate(cases):
        U = b.params(k)["U_char"]
        fields = [torch.empty(c["ny"], c["nx"], dtype=torch.float64, device=dev) for _ in range(3)]
        resample(ctx, pred[k, 0], fields[0], U, 0.0, antisym)
        resample(ctx, pred[k, 1], fields[1], U, 0.0, antisym)
        resample(ctx, pred[k, 2], fields[2], 1.0, -0.5, antisym)
        u0.append(fields[0])
        v0.append(fields[1])
        T0.append(fields[2])
    b.init_device(T0, u0, v0)
    ctx.stream.synchronize()  # the staging tensors may be released afterwards
    return b


def compare(ctx: Context, net: Net, cases, T0_cold, tol=1e-8, check_every=1000,
            max_steps=2_000_000, chunk=200_000, log=None, antisym=True):
    """Cold start (T0_cold, u = 0) against the learned start, same stop rule.
    Times include the prediction and resampling of the warm start."""
    bc, sc, rc, _, tc = solve(ctx, cases, T0_cold, tol, check_every, max_steps, chunk, log)
    nu_c = np.array([bc.nusselt(k)["nu_hot"] for k in range(len(cases))])
    del bc
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bw = Batch(ctx, cases, "f32")
    warm_init(ctx, net, bw, cases, antisym)
    t_pred = time.perf_counter() - t0
    bw, sw, rw, _, tw = solve(ctx, cases, None, tol, check_every, max_steps, chunk, log, batch=bw)
    nu_w = np.array([bw.nusselt(k)["nu_hot"] for k in range(len(cases))])
    del bw
    return {"steps_cold": sc, "steps_warm": sw, "rules_cold": rc, "rules_warm": rw,
            "nu_cold": nu_c, "nu_warm": nu_w, "seconds_cold": tc,
            "seconds_warm": tw + t_pred, "seconds_predict": t_pred}
