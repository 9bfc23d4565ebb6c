"""GPU AOS solver against the oracle's AOS (both FP64): the state after a few
steps element by element, the region means, the stopping step of a run to
the paper's relative-change tolerance, a non-square grid, the Rada-Chen area
term, and the hand-over of the AOS result to the multigrid cycle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import Oracle, OracleParams  # noqa: E402
from paper_1807_02137_amd import mgseg, synth  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pair(inst, levels=1, **kw):
    s = mgseg.Solver(inst.image, inst.markers, mgseg.Params(levels=levels, **kw))
    o = Oracle(inst.image, inst.markers, OracleParams(levels=levels, **kw))
    return s, o


@pytest.mark.parametrize("tau", [0.5, 50.0])
def test_aos_steps_match_the_oracle(tau):
    say("case AOS steps config-1 seed 1000 tau", tau)
    inst = synth.config1(1000)
    s, o = pair(inst)
    for k in range(4):
        it, eta_g, rel_g, _ = s.aos(tau, eta_tol=0.0, max_iters=1)
        eta_o = o.aos_step(tau)
        pg, po = s.get("phi64"), o.get("phi")
        d = np.abs(pg - po).max()
        say(f"step {k}: eta gpu {eta_g:.6e} oracle {eta_o:.6e} max|dphi| {d:.3e}")
        assert it == 1
        assert d <= 1e-10
        assert abs(eta_g - eta_o) <= 1e-9 * max(eta_o, 1e-300)
    sg, so = s.scalars(), o.scalars()
    assert abs(sg["c1"] - so["c1"]) <= 1e-11 and abs(sg["c2"] - so["c2"]) <= 1e-11
    s.close()


def test_aos_run_to_tolerance_and_rada_chen_area_term():
    say("case AOS run Rada-Chen seed 1001")
    inst = synth.config1(1001)
    s, o = pair(inst, model=1)
    it, eta, rel, ok = s.aos(20.0, eta_tol=1e-4, max_iters=400)
    k, hist = o.aos(20.0, 1e-4, 400)
    pg, po = s.get("phi64"), o.get("phi")
    say(f"gpu {it} steps eta {eta:.3e} rel {rel:.3e}; oracle {k} steps; max|dphi| {np.abs(pg - po).max():.3e}")
    assert ok and k > 0 and it == k
    assert np.abs(pg - po).max() <= 1e-8
    assert abs(rel - o.res_norm() / o.scalars()["res0"]) <= 1e-6 * max(rel, 1e-12)
    s.close()


def test_aos_non_square_grid():
    say("case AOS 96 x 160")
    inst = synth.shapes_instance(7, 96, 160, 3, 1.0, 0.05, 4, "aos_ragged", min_count=3)
    s, o = pair(inst)
    s.aos(8.0, eta_tol=0.0, max_iters=3)
    for _ in range(3):
        o.aos_step(8.0)
    d = np.abs(s.get("phi64") - o.get("phi")).max()
    say("max|dphi|", d)
    assert d <= 1e-10
    s.close()


def test_multigrid_cycle_continues_from_the_aos_result():
    say("case AOS then V-cycle seed 1002")
    inst = synth.config1(1002)
    s, o = pair(inst, levels=6)
    s.aos(10.0, eta_tol=0.0, max_iters=3)
    for _ in range(3):
        o.aos_step(10.0)
    rg = s.vcycle()
    ro, _ = o.vcycle()
    pg, po = s.get("phi64"), o.get("phi")
    flips = int(((pg > 0) != (po > 0)).sum())
    say(f"after AOS: cycle rel gpu {rg:.4e} oracle {ro:.4e} max|dphi| {np.abs(pg - po).max():.3e} flips {flips}")
    assert abs(rg - ro) <= 1e-3 * ro
    assert flips == 0 and np.abs(pg - po).max() <= 1e-4
    s.close()
