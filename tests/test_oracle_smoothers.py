"""Pins of the oracle's standard smoothers of Sec. 3.2 (GSLEX-I/II,
GSLINE-I/II, NEWT-I/II, beside Hybrid Smoothers 1 and 2), each against
something other than the smoother's own code: the discrete solution (found
by the multigrid solve and checked with the separately written operator N)
is a fixed point of every smoother; the line smoothers equal column solves
by a banded library routine; the local ("-II") variants equal a plain
Python loop that refreshes a pixel's (or a column's) coefficients with the
oracle's freeze right before using them; and NEWT reduces to GSLEX where the
model has no area term."""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import Oracle, OracleParams
from paper_1807_02137_amd import synth

STEP = {"gsline1": 6, "newt1": 7, "gslex2": 8, "gsline2": 9, "newt2": 10}


def _tiny(seed=3, n=16, **kw):
    inst = synth.tiny_instance(seed, n, n)
    return Oracle(inst.image, inst.markers, OracleParams(**kw))


@pytest.mark.parametrize("smoother", [0, 1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("model", [0, 1])
def test_the_discrete_solution_is_a_fixed_point_of_every_smoother(smoother, model):
    o = _tiny(levels=2, model=model, order=0)
    k, _ = o.solve(1e-13, 200)
    assert k > 0
    phi = o.get("phi")
    t = _tiny(levels=2, model=model, order=0, smoother=smoother)
    t.set("phi", phi)
    t.update_c()
    rel = t.res_norm() / o.scalars()["res0"]
    assert rel <= 1e-12
    t.smooth(1, 0)
    assert np.abs(t.get("phi") - phi).max() <= 1e-9


def _banded(lo, di, up):
    n = len(di)
    ab = np.zeros((3, n))
    ab[0, 1:] = up[:-1]
    ab[1] = di
    ab[2, :-1] = lo[1:]
    return ab


def _column_solve(A, B, C, D, S, f, phi, j):
    """Column j's rows with its neighbours' current values, solved by a banded
    library routine (no bound is active: the box is wide)."""
    n, m = phi.shape
    rhs = f[:, j].copy()
    if j + 1 < m:
        rhs -= C[:, j] * phi[:, j + 1]
    if j > 0:
        rhs -= D[:, j] * phi[:, j - 1]
    lo = np.r_[0.0, B[1:, j]]
    up = np.r_[A[:-1, j], 0.0]
    return sl.solve_banded((1, 1), _banded(lo, -S[:, j], up), rhs)


def _moved(seed=3, n=12, M=1e6, **kw):
    """A tiny instance with a smooth level set of moderate slope (a tilted
    tanh front); with the wide box no bound is active in one line sweep."""
    o = _tiny(seed, n, levels=1, M=M, order=0, **kw)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    o.set("phi", 2.0 * np.tanh((0.8 * i - 0.5 * j - 2.0) / 3.0) + 0.05 * np.sin(1.7 * i + 0.9 * j))
    o.update_c()
    return o


@pytest.mark.parametrize("model", [0, 1])
def test_gsline1_is_column_solves_with_frozen_coefficients(model):
    o = _moved(model=model)
    phi = o.get("phi")
    o.freeze(0)
    A, B, C, D, S, f = (o.get(k) for k in "ABCDSf")
    o.sweep(STEP["gsline1"], 0)
    want = phi.copy()
    for j in range(phi.shape[1]):
        want[:, j] = _column_solve(A, B, C, D, S, f, want, j)
    assert np.abs(o.get("phi") - want).max() <= 1e-10


def _fresh(o, phi):
    """The coefficients of eq. abcdrc at phi (the oracle's freeze)."""
    o.set("phi", phi)
    o.freeze(0)
    return [o.get(k) for k in "ABCDSf"]


@pytest.mark.parametrize("model", [0, 1])
def test_gsline2_refreshes_each_column_before_its_solve(model):
    o = _moved(model=model)
    phi = o.get("phi")
    probe = _moved(model=model)
    want = phi.copy()
    for j in range(phi.shape[1]):
        A, B, C, D, S, f = _fresh(probe, want)
        want[:, j] = _column_solve(A, B, C, D, S, f, want, j)
    o.freeze(0)
    o.sweep(STEP["gsline2"], 0)
    assert np.abs(o.get("phi") - want).max() <= 1e-10


def _point(A, B, C, D, S, f, v, i, j, qp=0.0, M=4.0):
    n, m = v.shape
    r = -f[i, j] + qp * v[i, j]
    if i + 1 < n:
        r += A[i, j] * v[i + 1, j]
    if i > 0:
        r += B[i, j] * v[i - 1, j]
    if j + 1 < m:
        r += C[i, j] * v[i, j + 1]
    if j > 0:
        r += D[i, j] * v[i, j - 1]
    return min(max(r / (S[i, j] + qp), -M), M)


@pytest.mark.parametrize("model", [0, 1])
def test_gslex2_refreshes_each_pixel_before_its_update(model):
    """(with the paper's box |phi| <= 4: the local refresh alone is not stable)"""
    o = _moved(model=model, M=4.0)
    phi = o.get("phi")
    probe = _moved(model=model, M=4.0)
    want = phi.copy()
    for i in range(phi.shape[0]):
        for j in range(phi.shape[1]):
            A, B, C, D, S, f = _fresh(probe, want)
            want[i, j] = _point(A, B, C, D, S, f, want, i, j)
    o.freeze(0)
    o.sweep(STEP["gslex2"], 0)
    got = o.get("phi")
    assert np.abs(got - want).max() <= 1e-10
    # and it is not GSLEX-I: the frozen sweep differs after the first pixel
    g = _moved(model=model, M=4.0)
    g.freeze(0)
    g.sweep(4, 0)
    assert abs(g.get("phi")[0, 0] - got[0, 0]) <= 1e-14
    assert np.abs(g.get("phi") - got).max() > 1e-9


def test_newt_is_gslex_without_an_area_term():
    for step_newt, step_gslex in ((STEP["newt1"], 4), (STEP["newt2"], STEP["gslex2"])):
        a, b = _moved(model=0), _moved(model=0)
        a.freeze(0); b.freeze(0)
        a.sweep(step_newt, 0)
        b.sweep(step_gslex, 0)
        assert np.abs(a.get("phi") - b.get("phi")).max() == 0.0


def test_newt_first_pixel_is_the_newton_weighted_average():
    """Rada-Chen, rows scaled by delta: at the first pixel of the sweep (nothing
    updated before it) NEWT-I is Newton's step on the pixel's own row, whose
    derivative adds Q' (the derivative of the area term in phi_00, here by a
    central difference of the oracle's area term) to S:
        x_N = (S x_G + Q' x_0) / (S + Q'),
    x_G the GSLEX-I value and x_0 the old value."""
    a, g = _moved(model=1, M=4.0), _moved(model=1, M=4.0)
    phi = a.get("phi")
    x0 = phi[0, 0]
    probe = _moved(model=1, M=4.0)

    def area(x):
        v = phi.copy()
        v[0, 0] = x
        probe.set("phi", v)
        return probe.area_term(0)

    qp = (area(x0 + 1e-4) - area(x0 - 1e-4)) / 2e-4
    assert qp > 0
    a.freeze(0); g.freeze(0)
    S = a.get("S")[0, 0]
    a.sweep(STEP["newt1"], 0)
    g.sweep(4, 0)
    xg, xn = g.get("phi")[0, 0], a.get("phi")[0, 0]
    want = (S * xg + qp * x0) / (S + qp)
    assert abs(xn - want) <= 1e-9 * max(1.0, abs(want))
    assert abs(xn - xg) > 0.0
