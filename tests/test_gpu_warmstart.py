"""The learned warm start end to end: the dataset path (steady fields
resampled onto the canvas), the prediction path (network output resampled
onto a cavity) against the FP64 references, and warm against cold starts
under the same stop rule with the committed weights."""
import os

import numpy as np
import pytest
import torch

from oracle import net as onet
from synth_inputs import SEED_HELDOUT, cavity_sweep, perturbation

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1908_08386_amd", "weights", "warmstart_r128.npz")


@pytest.fixture(scope="module")
def lf():
    import paper_1908_08386_amd as lf
    return lf


@pytest.fixture(scope="module")
def ws():
    from paper_1908_08386_amd import warmstart
    return warmstart


@pytest.fixture(scope="module")
def ctx(lf):
    return lf.Context(0)


def test_dataset_path_vs_fp64(lf, ws, ctx):
    cases = [dict(nx=96, ny=48, Ra=2e4, Pr=0.71), dict(nx=40, ny=40, Ra=1e5, Pr=7.0)]
    b = lf.Batch(ctx, cases, "f32").init([perturbation(c["nx"], c["ny"], 7, 0.1) for c in cases])
    b.step(3000)
    b.residual()  # moments of the current state
    tgt = ws.dataset_from_batch(ctx, b, cases, 64).cpu().numpy()
    for k, c in enumerate(cases):
        U = b.params(k)["U_char"]
        for ch, (f, sc, off) in enumerate((("u", 1 / U, 0.0), ("v", 1 / U, 0.0), ("T", 1.0, 0.5))):
            ref = onet.bilinear(b.fetch(k, f), 64, 64) * sc + off
            assert np.abs(tgt[k, ch] - ref).max() <= 2e-6 * max(np.abs(ref).max(), 1.0), (k, f)


@pytest.fixture(scope="module")
def net(lf, ctx):
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights in the package")
    W = np.load(WEIGHTS)
    n = lf.Net(ctx, int(W["res"]), tuple(int(x) for x in W["widths"]), int(W["cout"]),
               max_batch=8)
    n.set_weights(W["weights"])
    return n


def test_prediction_path_vs_fp64(lf, ws, ctx, net):
    """Predicted initial fields on two cavity grids against the FP64 network
    on the same bf16-rounded weights, resampled by the FP64 bilinear rule and
    reduced to the part that is odd under the 180-degree rotation."""
    cases = [dict(nx=150, ny=50, Ra=3e5, Pr=0.71), dict(nx=64, ny=64, Ra=2e3, Pr=7.0)]
    b = lf.Batch(ctx, cases, "f32")
    ws.warm_init(ctx, net, b, cases)
    w = net.weights().astype(np.float64)
    k = 0
    for o, i in net.layer_shapes():
        w[k:k + o * 9 * i] = onet.bf16_round(w[k:k + o * 9 * i])
        k += o * 9 * i + o
    x = onet.bf16_round(onet.net_inputs(ws.features(cases).astype(np.float64), net.res))
    y, _ = onet.forward(w, x, net.widths, net.cout)
    for k, c in enumerate(cases):
        U = b.params(k)["U_char"]
        for ch, (f, sc, off) in enumerate((("u", U, 0.0), ("v", U, 0.0), ("T", 1.0, -0.5))):
            d = onet.bilinear(y[k, :, :, ch], c["ny"], c["nx"]) * sc + off
            ref = 0.5 * (d - d[::-1, ::-1])  # the rotation-odd part (warm_init's default)
            got = b.fetch(k, f)
            scale = U if f != "T" else 1.0
            assert np.abs(got - ref).max() <= 1e-2 * scale * max(np.abs(y[k, :, :, ch]).max(), 0.5), (k, f)


def test_warm_and_cold_reach_the_same_steady_state(lf, ws, ctx, net):
    """Six held-out sweep cavities (ny <= 64) from the cold and from the
    learned start, each run to the same stop rule: every run stops by the
    rule (not the step limit), warm and cold Nusselt numbers agree to 1e-4,
    and the learned start gains: the median warm/cold step ratio is below
    0.8."""
    held = cavity_sweep(6, SEED_HELDOUT, max_ny=64)
    T0 = [perturbation(c["nx"], c["ny"], c["seed"]) for c in held]
    res = ws.compare(ctx, net, held, T0, max_steps=1_500_000, chunk=500_000)
    for rules in (res["rules_cold"], res["rules_warm"]):
        assert np.all((rules == lf.STOP_TOL) | (rules == lf.STOP_FLOOR)), res
    dnu = np.abs(res["nu_warm"] - res["nu_cold"]) / np.abs(res["nu_cold"])
    assert dnu.max() <= 1e-4, (dnu, res)
    ratio = res["steps_warm"] / res["steps_cold"]
    print(f"warm/cold steps {ratio.round(3).tolist()}, max dNu/Nu {dnu.max():.2e}", flush=True)
    assert np.median(ratio) < 0.8, (ratio, res)
