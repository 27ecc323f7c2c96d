"""Train the learned initial guess and compare warm and cold starts.

    python -m paper_1908_08386_amd.train_warmstart --out weights.npz [--report r.json]
    python -m paper_1908_08386_amd.train_warmstart --eval-only weights.npz [--heldout-n N]

1. Draw the training cavities (heterogeneous side-heated cavities: ny from
   64..512 capped at --max-ny-train, A in 1..4, log10 Ra in [3, 6], Pr 0.71
   or 7) and solve them to steady state with the batched FP32 solver.
2. Resample the steady fields onto the res x res canvas and train the
   network with Adam on mini-batches in seeded random order.
3. Save the FP32 weights, then solve held-out cavities (their own seed, full
   drawn sizes unless --max-ny-eval caps them) from the cold start and from
   the network's prediction with the same stop rule, and report steps, wall
   time (the warm side includes prediction and resampling) and the Nusselt
   numbers of both.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1908_08386_amd as lf  # noqa: E402
from paper_1908_08386_amd import warmstart as ws  # noqa: E402
from synth_inputs import SEED_HELDOUT, SEED_TRAIN, cavity_sweep, perturbation, uniform01  # noqa: E402


def log(msg):
    print(msg, flush=True)


def orders(n, batch, epochs, seed):
    """[epochs * (n // batch)][batch] sample indices: one seeded permutation
    per epoch, cut into mini-batches."""
    rows = []
    for e in range(epochs):
        perm = np.argsort(uniform01(seed * 1000 + e, n), kind="stable")
        for k in range(n // batch):
            rows.append(perm[k * batch:(k + 1) * batch])
    return np.array(rows, np.int32)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--train-n", type=int, default=2000)
    ap.add_argument("--max-ny-train", type=int, default=128)
    ap.add_argument("--heldout-n", type=int, default=128)
    ap.add_argument("--max-ny-eval", type=int, default=0, help="0 = full drawn sizes")
    ap.add_argument("--heldout-range", default="",
                    help="evaluate only draws A:B of the held-out set (split long evaluations)")
    ap.add_argument("--res", type=int, default=128)
    ap.add_argument("--widths", default="32,32,64,64,128")
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--max-steps", type=int, default=3_000_000)
    ap.add_argument("--out", default="", help="where to save the trained weights (.npz)")
    ap.add_argument("--report", default="")
    ap.add_argument("--skip-eval", action="store_true")
    ap.add_argument("--eval-only", default="",
                    help="skip solving and training: evaluate these saved weights")
    a = ap.parse_args(argv)
    widths = tuple(int(x) for x in a.widths.split(","))
    if not a.eval_only and not a.out:
        ap.error("--out is required unless --eval-only is given")
    ctx = lf.Context(0)
    report = {"train_n": a.train_n, "max_ny_train": a.max_ny_train, "res": a.res,
              "widths": widths, "epochs": a.epochs, "batch": a.batch, "lr": a.lr}

    if a.eval_only:
        W = np.load(a.eval_only)
        net = lf.Net(ctx, int(W["res"]), tuple(int(x) for x in W["widths"]), int(W["cout"]),
                     max_batch=a.batch)
        net.set_weights(W["weights"])
        report = {"weights": a.eval_only}
        evaluate(a, ctx, net, report)
        return

    log(f"step: solve {a.train_n} training cavities")
    cases = cavity_sweep(a.train_n, SEED_TRAIN, max_ny=a.max_ny_train)
    T0 = [perturbation(c["nx"], c["ny"], c["seed"]) for c in cases]
    b, steps, rules, _, sec = ws.solve(ctx, cases, T0, max_steps=a.max_steps, chunk=50_000,
                                       log=log)
    report["train_solve"] = {"seconds": round(sec, 2), "nodes": int(sum(c["nx"] * c["ny"] for c in cases)),
                             "steps_median": int(np.median(steps)), "steps_max": int(steps.max()),
                             "rules": {str(k): int(np.count_nonzero(rules == k)) for k in (-1, 0, 1, 2)}}
    log(f"  solved in {sec:.1f} s: {report['train_solve']}")
    target = ws.dataset_from_batch(ctx, b, cases, a.res)
    del b
    feat = torch.tensor(ws.features(cases), device="cuda")

    log("step: train")
    net = lf.Net(ctx, a.res, widths, 8, max_batch=a.batch)
    net.set_weights(net.he_uniform(uniform01(SEED_TRAIN * 7 + 1, net.nparam)))
    order = orders(a.train_n, a.batch, a.epochs, SEED_TRAIN)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = ws.train(net, feat, target, order, a.lr, log=log, log_every=500)
    torch.cuda.synchronize()
    tt = time.perf_counter() - t0
    fwd, trn = net.flops()
    report["train"] = {"seconds": round(tt, 2), "steps": int(order.shape[0]),
                       "tflops": round(trn * a.batch * order.shape[0] / tt / 1e12, 2),
                       "params": int(net.nparam), "loss": hist}
    # full-data loss of the final weights
    net.backward(feat, target, torch.arange(min(a.batch, a.train_n), dtype=torch.int32,
                                            device="cuda"))
    report["train"]["final_batch_loss"] = net.loss()
    log(f"  trained in {tt:.1f} s ({report['train']['tflops']} TFLOP/s), "
        f"loss {hist[-1][1]:.3e}")
    w = net.weights()
    np.savez(a.out, weights=w, res=a.res, widths=np.array(widths), cout=8,
             meta=json.dumps({k: v for k, v in report.items() if k != "train"} |
                             {"final_loss": hist[-1][1], "train_steps": int(order.shape[0])}))
    log(f"  weights -> {a.out}")

    if not a.skip_eval:
        evaluate(a, ctx, net, report)
        return
    if a.report:
        with open(a.report, "w") as f:
            json.dump(report, f, indent=1, default=float)
    log("done")


def evaluate(a, ctx, net, report):
    held = cavity_sweep(a.heldout_n, SEED_HELDOUT, max_ny=a.max_ny_eval or None)
    lo, hi = 0, len(held)
    if a.heldout_range:
        lo, hi = (int(x) for x in a.heldout_range.split(":"))
        held = held[lo:hi]
    log(f"step: held-out comparison (draws {lo}..{hi - 1} of {a.heldout_n})")
    T0h = [perturbation(c["nx"], c["ny"], c["seed"]) for c in held]
    res = ws.compare(ctx, net, held, T0h, max_steps=a.max_steps, log=log)
    dnu = np.abs(res["nu_warm"] - res["nu_cold"]) / np.abs(res["nu_cold"])
    ratio = res["steps_warm"] / np.maximum(res["steps_cold"], 1)
    report["heldout"] = {
        "n": a.heldout_n, "draws": [lo, hi], "max_ny": a.max_ny_eval or 512,
        "max_steps": a.max_steps,
        "seconds_cold": round(res["seconds_cold"], 2), "seconds_warm": round(res["seconds_warm"], 2),
        "seconds_predict": round(res["seconds_predict"], 3),
        "speedup_wall": round(res["seconds_cold"] / res["seconds_warm"], 3),
        "step_ratio_median": round(float(np.median(ratio)), 3),
        "step_ratio_min": round(float(ratio.min()), 3), "step_ratio_max": round(float(ratio.max()), 3),
        "steps_cold_total": int(res["steps_cold"].sum()), "steps_warm_total": int(res["steps_warm"].sum()),
        "dnu_rel_max": float(dnu.max()), "dnu_rel_median": float(np.median(dnu)),
        "rules_cold": res["rules_cold"].tolist(), "rules_warm": res["rules_warm"].tolist(),
        "steps_cold": res["steps_cold"].tolist(), "steps_warm": res["steps_warm"].tolist(),
        "nu_cold": res["nu_cold"].tolist(), "nu_warm": res["nu_warm"].tolist()}
    both = (res["rules_cold"] > 0) & (res["rules_warm"] > 0)
    report["heldout"]["stopped_both"] = int(both.sum())
    report["heldout"]["dnu_rel_max_stopped_both"] = float(dnu[both].max()) if both.any() else None
    log(json.dumps({k: v for k, v in report["heldout"].items()
                    if not k.startswith(("rules", "steps_c", "steps_w", "nu_"))}))
    if a.report:
        with open(a.report, "w") as f:
            json.dump(report, f, indent=1, default=float)
    log("done")


if __name__ == "__main__":
    main()
