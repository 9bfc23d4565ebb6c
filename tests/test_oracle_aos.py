"""Pins of the oracle's AOS solver (additive operator splitting, the
competitor of the timing comparison in Sec. 5 and a coarsest-grid solver
named in Algorithm 1), each against something other than the AOS code: a
library banded solver, the explicit step of the same PDE (the oracle's
separately written operator N), the maximum principle of the implicit
factors, and the closed form of a state that varies along one axis only."""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import Oracle, OracleParams, tridiag_solve
from paper_1807_02137_amd import synth


def _banded(lo, di, up):
    n = len(di)
    ab = np.zeros((3, n))
    ab[0, 1:] = up[:-1]
    ab[1] = di
    ab[2, :-1] = lo[1:]
    return ab


@pytest.mark.parametrize("n", [1, 2, 7, 64])
def test_tridiag_solve_matches_a_banded_library_solve(n):
    rng = np.random.default_rng(n)
    lo, up = -rng.uniform(0, 1, n), -rng.uniform(0, 1, n)
    lo[0], up[-1] = 0.0, 0.0
    di = 1.0 + np.abs(lo) + np.abs(up) + rng.uniform(0, 0.1, n)
    b = rng.normal(size=n)
    x = tridiag_solve(lo, di, up, b)
    assert np.abs(x - sl.solve_banded((1, 1), _banded(lo, di, up), b)).max() <= 1e-13


def _tiny(seed=3, **kw):
    inst = synth.tiny_instance(seed, 24, 24)
    return Oracle(inst.image, inst.markers, OracleParams(levels=1, **kw))


def test_small_step_is_the_explicit_step_of_the_same_pde():
    """(phi^1 - phi^0) / tau -> N(phi^0) as tau -> 0 (the splitting is consistent
    with phi_t = N(phi)), at the cells the box does not clamp; the gap shrinks
    in proportion to tau."""
    gaps = []
    for tau_hat in (1e-4, 1e-5):
        o = _tiny()
        phi0 = o.get("phi")
        N0 = o.operator(0)
        n, m, h = o.shape(0)
        tau = tau_hat * h / 0.5
        o.aos_step(tau_hat)
        phi1 = o.get("phi")
        free = np.abs(phi1) < 4.0 - 1e-9
        d = (phi1 - phi0) / tau
        gaps.append(np.abs(d - N0)[free].max() / np.abs(N0[free]).max())
    assert gaps[0] <= 1e-2 and gaps[1] <= 0.2 * gaps[0]


def test_constants_kept_and_maximum_principle_without_forcing():
    """With no fitting force (fit = 0, F = 0) every implicit factor has unit row
    sums and a non-negative inverse, so a step keeps a constant field and keeps
    any field within its own minimum and maximum."""
    o = _tiny()
    n, m, _ = o.shape(0)
    rng = np.random.default_rng(1)
    phi = rng.uniform(-1.0, 1.0, (n, m))
    o.set("phi", phi)
    o.set("fit", np.zeros((n, m)))
    o.aos_step(50.0)
    out = o.get("phi")
    assert out.min() >= phi.min() - 1e-14 and out.max() <= phi.max() + 1e-14
    assert np.abs(out - phi).max() > 1e-3                 # it did smooth
    o.set("phi", np.full((n, m), 0.37))
    o.set("fit", np.zeros((n, m)))
    o.aos_step(50.0)
    assert np.abs(o.get("phi") - 0.37).max() <= 1e-14


def test_state_constant_along_rows_has_the_closed_form():
    """phi, w and the fitting term depend on the row index i only.  The row
    systems then return their right-hand side unchanged (their coupling acts on
    differences along j, which vanish), and the step is the average of the
    right-hand side and one column solve: phi^1 = clamp((r + T^{-1} r) / 2),
    r = phi - tau fit, T the column system built from the frozen A, B."""
    o = _tiny()
    n, m, h = o.shape(0)
    i = np.arange(n)[:, None] * np.ones((1, m))
    phi = 2.0 * np.tanh((i - n / 2.0) / 3.0)
    w = 0.3 + 0.6 * np.exp(-((i - 8.0) ** 2) / 10.0)
    fit = 0.4 * np.sin(i / 3.0)
    o.set("phi", phi)
    o.set("w", w)
    o.set("fit", fit)
    o.freeze(0)
    A, B = o.get("A"), o.get("B")
    tau_hat = 3.0
    tau = tau_hat * h / 0.5
    r = phi[:, 0] - tau * fit[:, 0]
    lo, up = -2 * tau * B[:, 0], -2 * tau * A[:, 0]
    di = 1.0 + 2 * tau * (A[:, 0] + B[:, 0])
    y1 = sl.solve_banded((1, 1), _banded(lo, di, up), r)
    want = np.clip(0.5 * (r + y1), -4.0, 4.0)
    o.set("phi", phi)
    o.set("fit", fit)
    o.aos_step(tau_hat)
    got = o.get("phi")
    assert np.abs(got - want[:, None]).max() <= 1e-12


def test_fixed_point_gap_shrinks_with_the_step():
    """The splitting's fixed point is not exactly N(phi) = 0 (the two factors see
    different states); the gap vanishes with the step: run AOS to stagnation at
    two steps and compare the projected residual of the paper's rows there."""
    rel = []
    for tau_hat in (2.0, 1.0):
        o = _tiny()
        k, hist = o.aos(tau_hat, eta_tol=1e-13, max_iters=40000)
        assert k > 0
        rel.append(o.res_norm() / o.scalars()["res0"])
    assert rel[0] < 5e-6
    assert rel[1] < 0.6 * rel[0]
