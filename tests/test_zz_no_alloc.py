"""The entry point that allocates nothing (mgseg_solve_noalloc), called
through the C ABI, against the allocating path (mgseg_setup + mgseg_solve +
mgseg_get_phi) on the same inputs: two calls in a row, the second on a
smaller image, then an image too large for the static scratch."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1807_02137_amd import mgseg, synth  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def reference(image, markers, params):
    s = mgseg.Solver(image, markers, params)
    cyc, rel, ok = s.solve(1e-6, 60)
    phi = s.phi().cpu().numpy()
    s.close()
    return phi, cyc, rel


def test_noalloc_matches_the_allocating_path_twice():
    cases = [("config1 seed 1000, 128x128", synth.config1(1000), 6),
             ("tiny 48x80", synth.tiny_instance(5, 48, 80), 0)]
    for name, inst, lev in cases:
        say("case no-alloc", name)
        params = mgseg.Params(levels=lev)
        phi_n, cyc_n, rel_n, code = mgseg.solve_noalloc(inst.image, inst.markers, params, 1e-6, 60)
        torch.cuda.synchronize()
        phi_r, cyc_r, rel_r = reference(inst.image, inst.markers, params)
        pn = phi_n.cpu().numpy()
        agree = (pn > 0) == (phi_r > 0)
        flips = int((~agree).sum())
        dmax = float(np.abs(pn - phi_r).max())
        say(f"  no-alloc {cyc_n} cycles rel {rel_n:.3e}; allocating {cyc_r} cycles rel {rel_r:.3e}; "
            f"max|dphi| {dmax:.3e} flips {flips}")
        assert code == 0 and rel_n <= 1e-6
        assert cyc_n == cyc_r
        assert flips == 0 and dmax <= 1e-4


def test_noalloc_refuses_an_image_beyond_the_scratch():
    say("case no-alloc 1024x1024 (beyond the scratch)")
    inst = synth.config2(2000)
    with pytest.raises(mgseg.MgsegError) as e:
        mgseg.solve_noalloc(inst.image, inst.markers, mgseg.Params(levels=9), 1e-6, 5)
    assert e.value.code == 8
