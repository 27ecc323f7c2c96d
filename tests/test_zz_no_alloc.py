"""lf_case_residual_noalloc (the residual with its per-block partials and its
fold's output in the library's static per-GPU scratch, for callers that
cannot allocate) against lf_case_residual, which takes them from the bound
workspace, through the C-ABI on twin cases: bitwise equal residuals and the
same re-snapshot, over calls in a row whose cases shrink, so each call finds
more partials in the shared scratch than it writes (700, then 90, then 64
blocks), and on a split-mode case whose residual goes through its dense
output fields."""
import numpy as np
import pytest

from synth_inputs import perturbation

pytestmark = pytest.mark.gpu


def twins(lf, ctx, nx, ny, prec, mode, seed):
    out = []
    for _ in range(2):
        c = lf.Case(ctx, nx, ny, prec, mode=mode).set_physics(1e5, 0.71).set_cavity_walls()
        c.init(perturbation(nx, ny, seed, amp=0.05) if mode == lf.MODE_HYBRID else None)
        out.append(c)
    return out


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_residual_matches_the_workspace_residual(prec):
    import paper_1908_08386_amd as lf
    ctx = lf.Context(0)
    for nx, ny, mode, seed in ((300, 700, lf.MODE_HYBRID, 71), (130, 90, lf.MODE_HYBRID, 72),
                               (64, 64, lf.MODE_SPLIT, 0)):
        print(f"noalloc residual: {prec} {nx}x{ny} mode {mode}", flush=True)
        a, b = twins(lf, ctx, nx, ny, prec, mode, seed)
        for _ in range(3):
            a.step(150)
            b.step(150)
            ra, rb = a.residual(), b.residual_noalloc()
            assert np.all(ra > 0) and np.array_equal(ra, rb), (nx, ny, ra, rb)
        # both re-snapshotted the same fields: the next residuals agree too
        a.step(10)
        b.step(10)
        assert np.array_equal(a.residual(), b.residual())
        a.close()
        b.close()
