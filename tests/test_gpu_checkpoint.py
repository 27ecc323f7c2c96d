"""Checkpoint and resume (lf_case_save / lf_case_load): a case restored into
a fresh handle continues bit for bit, in Mode H and in the split mode."""
import numpy as np
import pytest

from synth_inputs import perturbation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    import paper_1908_08386_amd as lf
    return lf


@pytest.fixture(scope="module")
def ctx(lf):
    return lf.Context(0)


@pytest.mark.parametrize("mode,prec,nx,ny", [(0, "f32", 70, 48), (0, "f64", 64, 64), (1, "f64", 64, 32),
                                             (1, "f32", 96, 40)])
def test_resume_is_bitwise(lf, ctx, mode, prec, nx, ny):
    T0 = perturbation(nx, ny, 77, amp=0.05)
    a = lf.Case(ctx, nx, ny, prec, mode=mode).set_physics(2e5, 0.71).set_cavity_walls().init(T0)
    a.step(300)
    blob = a.save()
    a.step(250)
    b = lf.Case(ctx, nx, ny, prec, mode=mode).load(blob)
    assert b.steps == 300 and b.params() == a.params()
    b.step(250)
    for f in ("u", "v", "T"):
        assert np.array_equal(a.fetch(f), b.fetch(f)), f
    assert a.nusselt() == b.nusselt()


def test_load_rejects_other_geometry(lf, ctx):
    a = lf.Case(ctx, 64, 32, "f32").set_physics(1e4, 0.71).set_cavity_walls().init()
    blob = a.save()
    for other in (lf.Case(ctx, 64, 33, "f32"), lf.Case(ctx, 64, 32, "f64"),
                  lf.Case(ctx, 64, 32, "f32", mode=lf.MODE_SPLIT)):
        with pytest.raises(lf.LFError) as e:
            other.load(blob)
        assert e.value.status == lf.LF_EINVAL
    with pytest.raises(lf.LFError):
        lf.Case(ctx, 64, 32, "f32").load(blob[:100])
    with pytest.raises(lf.LFError) as e:
        lf.Case(ctx, 64, 32, "f32").save()
    assert e.value.status == lf.LF_ESTATE


@pytest.mark.parametrize("mode", ["gs2", "mcm"])
def test_resume_keeps_cycle_settings(lf, ctx, mode):
    """Grid setting 2 and LBM-MCM carry their cycle settings (and, for the
    walkers, the stream seed) in the checkpoint: a restored case continues
    bit for bit although the target case was created with the defaults."""
    nx, ny = 32, 24
    T0 = perturbation(nx, ny, 81, amp=0.2)
    m = lf.MODE_HYBRID_GS2 if mode == "gs2" else lf.MODE_LBM_MCM

    def make():
        return lf.Case(ctx, nx, ny, "f64", mode=m).set_physics(1e4, 0.71).set_cavity_walls()

    a = make()
    if mode == "gs2":
        a.set_subcycle(7, 3)
    else:
        a.set_mcm(9, 64, 12345, 1 << 20)
    a.init(T0).step(20)
    blob = a.save()
    b = make()
    b.init(T0).load(blob)
    a.step(25)
    b.step(25)
    for f in ("u", "v", "T"):
        assert np.array_equal(a.fetch(f), b.fetch(f)), f
