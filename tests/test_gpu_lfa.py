"""GPU local Fourier analysis of the smoothers over a whole image (Sec. 3.3,
Table 1's mu~_max and mu~_avg) against the oracle's LFA (oracle/lfa.py) on
the oracle's own frozen coefficients at the same phi: every pixel of a
128 x 128 image for GSLEX-I, sampled pixels (with the worst ones) for
GSLINE-I, NEWT-I and Hybrid Smoother 2, and the image aggregates."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import Oracle, OracleParams, lfa  # noqa: E402
from paper_1807_02137_amd import mgseg, synth  # noqa: E402

NEW = {1: {"B", "D"}, 3: {"A", "B", "D"}, 4: {"B", "D"}}
TOL = 2e-4          # FP32 couplings and angle table against FP64


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def state(seed, model):
    """GPU solver and oracle at the same phi: a few oracle cycles from phi0."""
    inst = synth.config1(seed)
    o = Oracle(inst.image, inst.markers, OracleParams(levels=6, model=model))
    for _ in range(3):
        o.vcycle()
    s = mgseg.Solver(inst.image, inst.markers, mgseg.Params(levels=6, model=model))
    phi = o.get("phi")
    s.set("phi64", phi)
    o.freeze(0)
    coef = np.stack([o.get(k) for k in "ABCD"], axis=-1)
    return s, o, coef


def oracle_rate(coef, smoother, lab=0, q=0.0):
    if smoother == 0:
        new = set("ABCD") - {"ABCD"[int(np.log2(lab))]} if lab else {"B", "D"}
    else:
        new = NEW[smoother]
    return lfa.rate(coef, new, q=q)


@pytest.mark.parametrize("model", [0, 1])
def test_gslex_rates_every_pixel(model):
    say("case LFA GSLEX-I every pixel, model", model)
    s, o, coef = state(1000, model)
    agg, mu = s.smoothing_rates(1, per_pixel=True)
    n, m = mu.shape
    want = np.array([[oracle_rate(coef[i, j], 1) for j in range(m)] for i in range(n)])
    d = np.abs(mu - want).max()
    say(f"max|dmu| {d:.2e}; gpu mu~ max {agg['mu_max']:.4f} avg {agg['mu_avg']:.4f}; "
        f"oracle max {want.max():.4f} avg {want.mean():.4f}")
    assert d <= TOL
    assert abs(agg["mu_max"] - want.max()) <= TOL and abs(agg["mu_avg"] - want.mean()) <= TOL
    s.close()


@pytest.mark.parametrize("smoother,model", [(3, 0), (3, 1), (4, 1), (0, 0), (0, 1)])
def test_rates_sampled_pixels(smoother, model):
    say("case LFA smoother", smoother, "model", model)
    s, o, coef = state(1001, model)
    agg, mu = s.smoothing_rates(smoother, per_pixel=True)
    lab = o.labels()
    q = o.newton_qprime(0) if smoother == 4 else np.zeros(mu.shape)
    rng = np.random.default_rng(smoother * 10 + model)
    n, m = mu.shape
    pts = {tuple(rng.integers(0, [n, m])) for _ in range(150)}
    pts |= {tuple(np.unravel_index(k, mu.shape)) for k in np.argsort(mu, axis=None)[-20:]}
    pts |= {tuple(p) for p in np.argwhere(lab > 0)[:60]}
    worst = 0.0
    for (i, j) in pts:
        want = oracle_rate(coef[i, j], smoother, int(lab[i, j]) if smoother == 0 else 0, q[i, j])
        worst = max(worst, abs(mu[i, j] - want))
    say(f"{len(pts)} pixels, max|dmu| {worst:.2e}; mu~ {agg}")
    assert worst <= TOL
    assert abs(agg["share_D"] - (lab > 0).mean()) <= 1e-12 + 3.0 / lab.size
    jump = s.get("labels") > 0
    assert abs(agg["share_D"] - jump.mean()) <= 1e-12
    if jump.any():
        assert abs(agg["mu_max_D"] - mu[jump].max()) <= 1e-6
        assert abs(agg["mu_avg_D"] - mu[jump].mean()) <= 1e-6
    s.close()
