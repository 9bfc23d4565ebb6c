"""The launch schedules of a context (mgseg_set_schedule) compute the same bits,
and the autotuner (mgseg_tune) keeps the solve where it stood: every schedule
of the tuner's set, from the same start, gives a finest phi identical to the
default schedule's after three V-cycles (config-1 image, a 256 x 384 image
whose lines take the two-half and single-half sweep kernels, and a 64 x 1280
image whose rows take the long-line kernel, a 1152 x 64 image whose columns
do, and a 768 x 64 image whose columns take the 1024-thread kernel, split or
not), and tuning
leaves phi, the cycle count and the residual unchanged."""
import itertools
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1807_02137_amd import mgseg, synth  # noqa: E402

SCHEDULES = list(itertools.product((0, 16, 32, 64), (0, 1), (0, 1), (0, 1)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(inst, levels, sched, cycles=3, **kw):
    s = mgseg.Solver(inst.image, inst.markers, mgseg.Params(levels=levels, **kw))
    if sched is not None:
        s.set_schedule(*sched)
    for _ in range(cycles):
        s.vcycle()
    phi = s.get("phi64")
    s.close()
    return phi


@pytest.mark.parametrize("shape,levels,smoother", [((128, 128), 6, 0), ((256, 384), 6, 0), ((128, 128), 6, 3),
                                                   ((64, 1280), 5, 0), ((1152, 64), 5, 0), ((768, 64), 5, 0)])
def test_every_schedule_gives_the_same_bits(shape, levels, smoother):
    say("case schedules", shape, "smoother", smoother)
    inst = synth.shapes_instance(11, shape[0], shape[1], 4, 1.0, 0.05, 4, "sched", min_count=3)
    ref = run(inst, levels, None, smoother=smoother)
    for sc in SCHEDULES:
        phi = run(inst, levels, sc, smoother=smoother)
        same = np.array_equal(phi, ref)
        say("  schedule", sc, "identical" if same else f"differs by {np.abs(phi - ref).max():.3e}")
        assert same


def test_tune_restores_the_state():
    say("case tune")
    inst = synth.config1(1001)
    s = mgseg.Solver(inst.image, inst.markers, mgseg.Params(levels=6))
    s.vcycle()
    s.vcycle()
    before, st0 = s.get("phi64"), s.stats()
    sched, ms = s.tune(1)
    after, st1 = s.get("phi64"), s.stats()
    say("chosen", sched, f"{ms:.3f} ms per cycle")
    assert tuple(sched.values()) in SCHEDULES and ms > 0
    assert np.array_equal(before, after)
    assert st0["cycles"] == st1["cycles"] and st0["rel_res"] == st1["rel_res"]
    s.close()
