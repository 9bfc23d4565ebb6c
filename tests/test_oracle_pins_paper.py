"""More pins of the FP64 oracle, each against something other than the
oracle itself: hand-made fields with labels worked out by hand, closed forms,
a library routine (scipy's Gaussian filter), the pinned visit orders, the
monotone-multigrid property of the coarse bounds, brute-force projected
time-marching from the initial level set, and the local Fourier analysis
against the oracle's own Hybrid Smoother 2 sweep."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import Oracle, OracleParams, prolong, setup_maps, visit_order
from oracle import lfa
from paper_1807_02137_amd import synth


def _blank(n, m, **kw):
    """An oracle on a flat image (its maps are overwritten by the tests)."""
    img = np.zeros((n, m))
    mk = np.array([[n / 2, m / 2]])
    return Oracle(img, mk, OracleParams(levels=1, **kw))


# ------------------------------------------------- jump set and labels (Sec. 4.1, Sec. 5.2)
def _labels_for(w, psi=None, Sigma=2.0):
    n, m = w.shape
    o = _blank(n, m, Sigma=Sigma)
    o.set("w", w)
    o.set("phi", np.zeros((n, m)) if psi is None else psi)
    o.freeze(0)
    return o.labels()


def test_labels_threshold_argmin_ties_and_boundary():
    """Flat psi (every face value is its w average over e = 1): the cell (2, 2)
    with w = 0.9 and a neighbour below of w = 0 has faces A = 0.45 and
    B = C = D = 0.95, a ratio 2.11 > Sigma = 2, so it is in the jump set
    labelled A (bit 0); with w = 1 the ratio is exactly 2 and it is not
    (strict test).  Two equal smallest faces take the first of A, B, C, D.
    A corner cell compares its two interior faces only."""
    w = np.ones((5, 5))
    w[2, 2], w[3, 2] = 0.9, 0.0
    lab = _labels_for(w)
    assert lab[2, 2] == 1                     # A is the smallest: starred in sweep A
    w[2, 2] = 1.0
    lab = _labels_for(w)
    assert lab[2, 2] == 0                     # ratio exactly Sigma: not in the jump set
    # ties: cell (2, 2) with w = 0.9 below and right neighbours of w = 0: A = C = 0.45
    w = np.ones((5, 5))
    w[2, 2], w[3, 2], w[2, 3] = 0.9, 0.0, 0.0
    lab = _labels_for(w)
    assert lab[2, 2] == 1                     # A before C
    # corner (0, 0): faces A (to (1, 0)) and C (to (0, 1)) only; the missing B, D do not count
    w = np.ones((5, 5))
    w[0, 0], w[1, 0] = 0.9, 0.0               # A = 0.45, C = 0.95: ratio 2.11
    lab = _labels_for(w)
    assert lab[0, 0] == 1
    w[1, 0] = 0.5                             # A = 0.7, C = 0.95: ratio 1.36
    assert _labels_for(w)[0, 0] == 0


def test_labels_zero_face_is_an_infinite_ratio():
    """A face between two cells of w = 0 carries 0: the ratio is infinite, the cell
    is in the jump set with that face as its label; a cell whose faces are all 0
    has no ratio and is not."""
    w = np.ones((6, 6))
    w[2, 2] = w[2, 1] = 0.0                   # face D of (2, 2) is 0, the others 0.5
    lab = _labels_for(w)
    assert lab[2, 2] == 8                     # bit 3 = D
    w = np.zeros((6, 6))
    assert (_labels_for(w) == 0).all()


def test_labels_follow_the_gradient_of_psi():
    """w = 1 and psi a vertical step of height 8 between rows 2 and 3: the face
    A of row 2 is 1/sqrt(64 + 1), the others 1 (flat along the row), so row 2 is
    labelled A and row 3 is labelled B; rows away from the step are not starred."""
    n, m = 6, 6
    psi = np.zeros((n, m))
    psi[3:, :] = 8.0
    lab = _labels_for(np.ones((n, m)), psi)
    assert (lab[2, :] == 1).all() and (lab[3, :] == 2).all()
    assert (lab[[0, 1, 4, 5], :] == 0).all()


# ------------------------------------------------- the sweeps follow the pinned visit orders (Fig. 4)
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("s", [0, 1, 2, 3])
def test_sweep_without_stars_is_point_gauss_seidel_in_visit_order(s, order):
    """With no starred cell a sweep is point Gauss-Seidel (eq. gslexrc) in its visit
    order; replaying the pinned visit order cell by cell gives the same result."""
    inst = synth.tiny_instance(4, 12, 16)
    o = Oracle(inst.image, inst.markers, OracleParams(levels=1, order=order))
    o.smooth(1, 0)
    o.freeze(0)
    o.set_labels(np.zeros((12, 16), np.uint8))
    A, B, C, D, S, f = (o.get(k) for k in ("A", "B", "C", "D", "S", "f"))
    phi = o.get("phi").ravel().copy()
    n, m = 12, 16
    for q in visit_order(s, n, m, order):
        i, j = divmod(int(q), m)
        v = -f[i, j]
        if i < n - 1: v += A[i, j] * phi[q + m]
        if i > 0: v += B[i, j] * phi[q - m]
        if j < m - 1: v += C[i, j] * phi[q + 1]
        if j > 0: v += D[i, j] * phi[q - 1]
        phi[q] = min(4.0, max(-4.0, v / S[i, j]))
    o.sweep(s, 0)
    assert np.abs(o.get("phi").ravel() - phi).max() <= 1e-13


# ------------------------------------------------- c1, c2 (eq. c1c2) in closed form
def test_region_means_closed_form():
    """A two-valued image (a inside a rectangle R, b outside) with phi = +M on R and
    -M outside: H takes two values h+ = 1/2 + atan(M)/pi and h- = 1 - h+, so
    c1 = (h+ a |R| + h- b |R^c|) / (h+ |R| + h- |R^c|) and c2 likewise with
    1 - H."""
    n, m, a, b = 20, 24, 0.8, 0.1
    R = np.zeros((n, m), bool)
    R[5:12, 3:17] = True
    img = np.where(R, a, b)
    o = Oracle(img, np.array([[8.5, 8.5]]), OracleParams(levels=1))
    o.set("phi", np.where(R, 4.0, -4.0))
    o.update_c()
    hp = 0.5 + math.atan(4.0) / math.pi
    hm = 1.0 - hp
    nR, nC = R.sum(), (~R).sum()
    c1 = (hp * a * nR + hm * b * nC) / (hp * nR + hm * nC)
    c2 = (hm * a * nR + hp * b * nC) / (hm * nR + hp * nC)
    sc = o.scalars()
    assert abs(sc["c1"] - c1) <= 1e-14 and abs(sc["c2"] - c2) <= 1e-14


# ------------------------------------------------- energy (eq. scfunc / rcfunc)
def test_energy_length_term_is_the_interface_length():
    """Coarea: with w = 1, no data or selection term and phi the signed distance to
    a circle of radius R (pixels, clamped to +-M), the length term sums to
    mu * (2 pi R h) * (2/pi) atan(M): the circle's length in domain units times
    the mass of delta_eps between -M and M.  Discretisation error O(1/R)."""
    n = m = 96
    R = 30.0
    yy, xx = np.mgrid[0:n, 0:m] + 0.5
    sd = R - np.hypot(yy - 48.0, xx - 48.0)
    img = np.zeros((n, m))
    o = Oracle(img, np.array([[48.5, 48.5]]),
               OracleParams(levels=1, beta=0.0, theta=0.0, lambda1=0.0, lambda2=0.0, mu=0.5))
    o.set("phi", np.clip(sd, -4.0, 4.0))
    h = 1.0 / n
    want = 0.5 * 2.0 * math.pi * R * h * (2.0 / math.pi) * math.atan(4.0)
    assert abs(o.energy() - want) <= 0.005 * want


def test_energy_region_terms_closed_form():
    """phi constant (no length term): the Spencer-Chen energy is the cell area times
    the sum of H lambda1 (z - c1)^2 + (1 - H) lambda2 (z - c2)^2 + H theta d, which
    for z two-valued and d given is a closed form in the counts; Rada-Chen adds
    nu ((h^2 sum H - A1)^2 + (h^2 sum (1 - H) - (1 - A1))^2)."""
    n, m, a, b = 16, 20, 0.7, 0.2
    R = np.zeros((n, m), bool)
    R[4:10, 5:15] = True
    img = np.where(R, a, b)
    mk = np.array([[6.5, 7.5], [6.5, 12.5], [8.5, 10.5]])
    for model in (0, 1):
        o = Oracle(img, mk, OracleParams(levels=1, model=model))
        o.set("phi", np.full((n, m), 1.5))
        c1, c2, A1 = (o.scalars()[k] for k in ("c1", "c2", "A1"))
        H = 0.5 + math.atan(1.5) / math.pi
        h2 = 1.0 / (n * m)
        lam = 6.5025
        per = lambda z: H * lam * (z - c1) ** 2 + (1 - H) * lam * (z - c2) ** 2
        want = h2 * (R.sum() * per(a) + (~R).sum() * per(b))
        if model == 0:
            want += h2 * H * 4.0 * o.get("d").sum()
        else:
            want += (h2 * n * m * H - A1) ** 2 + (h2 * n * m * (1 - H) - (1 - A1)) ** 2
        assert abs(o.energy() - want) <= 1e-12 * abs(want)


# ------------------------------------------------- setup maps against a library routine / closed forms
@pytest.mark.parametrize("sigma", [0.7, 1.0, 1.5])
def test_edge_detector_matches_scipy_gaussian_filter(sigma):
    """g = 1/(1 + beta |grad(G_sigma * z)|^2): the blur against scipy's Gaussian
    filter (half-sample mirror = 'reflect', truncation at 4 sigma) and central
    differences with mirrored edges, on a random image."""
    rng = np.random.default_rng(11)
    img = rng.random((24, 30))
    out = setup_maps(img, np.array([[5.5, 5.5], [12.5, 20.5], [18.5, 8.5]]), OracleParams(sigma_g=sigma))
    zb = ndimage.gaussian_filter(img, sigma, mode="reflect", truncate=4.0)
    zp = np.pad(zb, 1, mode="symmetric")
    gx = (zp[1:-1, 2:] - zp[1:-1, :-2]) / 2.0
    gy = (zp[2:, 1:-1] - zp[:-2, 1:-1]) / 2.0
    g = 1.0 / (1.0 + 16384.0 * (gx ** 2 + gy ** 2))
    assert np.abs(out["g"] - g).max() <= 1e-12


def test_marker_distance_at_sigma():
    """One marker: d = 1 - exp(-r^2 / (2 sigma_d^2)) in domain units; at r = sigma_d
    (4 px on a 40 x 40 grid, h0 = 1/40, sigma_d = 0.1) d = 1 - exp(-1/2), at the
    marker 0, and d grows with r."""
    out = setup_maps(np.zeros((40, 40)), np.array([[10.5, 10.5]]), OracleParams())
    assert out["d"][10, 10] == 0.0
    assert abs(out["d"][10, 14] - (1.0 - math.exp(-0.5))) <= 1e-15
    assert abs(out["d"][14, 10] - (1.0 - math.exp(-0.5))) <= 1e-15
    assert abs(out["d"][13, 14] - (1.0 - math.exp(-25.0 / 32.0))) <= 1e-15   # r = 5 px
    assert out["d"][10, 20] > out["d"][10, 15] > out["d"][10, 12]


# ------------------------------------------------- coarse bounds: corrections never cut back
def test_coarse_corrections_within_bounds_are_never_clipped():
    """The coarse bounds let every coarse unknown move only as far as each fine
    cell its interpolated correction reaches can follow inside its own box:
    any coarse correction within the bounds, prolongated, leaves every fine cell
    inside its box (bilinear weights are non-negative and sum to one), and each
    bound is tight (moving one coarse unknown past it pushes a fine cell out)."""
    inst = synth.config1(1001)
    o = Oracle(inst.image, inst.markers, OracleParams(levels=3))
    o.vcycle()
    o.smooth(2, 0)
    for l in (0, 1):
        if l == 1:
            o.smooth(2, 1)
        o.to_coarse(l)
        phi, lo, hi = o.get("phi", l), o.get("lo", l), o.get("hi", l)
        pc, loc, hic = o.get("phic", l + 1), o.get("lo", l + 1), o.get("hi", l + 1)
        rng = np.random.default_rng(l)
        for trial in range(4):
            t = rng.random(pc.shape) if trial < 2 else np.full(pc.shape, float(trial == 3))
            e = (loc - pc) + t * (hic - loc)
            f = phi + prolong(e)
            assert (f >= lo - 1e-12).all() and (f <= hi + 1e-12).all()
        # tightness on a sample of coarse unknowns
        nc, mc = pc.shape
        for I, J in [(1, 1), (nc // 2, mc // 3), (nc - 1, mc - 1)]:
            e = np.zeros_like(pc)
            e[I, J] = hic[I, J] - pc[I, J] + 1e-6
            f = phi + prolong(e)
            assert (f > hi + 1e-9).any(), (l, I, J)


# ------------------------------------------------- fixed point vs time-marching from phi0 (brute force)
@pytest.mark.parametrize("seed", [1, 6, 9])
def test_time_marching_from_phi0_reaches_the_multigrid_fixed_point(seed):
    """Projected explicit time-marching of the same discrete system, started from
    the initial level set (not from the multigrid result), reaches the FAS
    fixed point on tiny same-basin instances (one disc, 24 x 24): seed 1 is the
    binary segmentation of the whole disc, seeds 6 and 9 fixed points with free
    interior cells."""
    inst = synth.tiny_instance(seed, 24, 24)
    o = Oracle(inst.image, inst.markers, OracleParams(levels=3))
    k, hist = o.solve(1e-12, 80)
    assert k > 0
    t = Oracle(inst.image, inst.markers, OracleParams(levels=3))
    rel = 1.0
    for _ in range(4):
        rel = t.timemarch(20000, cfl=0.2, crefresh=50, tol=1e-13)
        if rel <= 1e-13:
            break
    assert rel <= 1e-13
    assert np.abs(t.get("phi") - o.get("phi")).max() <= 1e-8


# ------------------------------------------------- LFA against the oracle's own Hybrid Smoother 2 sweep
def _frozen_problem(coef, n, order, bit):
    """An n x n grid with the frozen coefficients (A, B, C, D) at every cell, S their
    sum, f = F = 0 (the error equation), a wide box, and every cell starred in
    the sweep `bit` (so that sweep solves whole lines collectively)."""
    o = _blank(n, n, M=1e6, order=order)
    o.freeze(0)
    for name, v in zip("ABCD", coef):
        o.set(name, np.full((n, n), float(v)))
    o.set("S", np.full((n, n), float(sum(coef))))
    o.set("f", np.zeros((n, n)))
    o.set_labels(np.full((n, n), 1 << bit, np.uint8))
    return o


def _measured_sweep_rate(coef, s, n=96, sweeps=40):
    """Power iteration of one oracle sweep on a frozen-coefficient error equation,
    with the low frequencies (max(|a1|, |a2|) <= pi/2) removed after each sweep:
    the asymptotic high-frequency reduction per sweep, away from the edges."""
    o = _frozen_problem(coef, n, 0, s)
    rng = np.random.default_rng(0)
    e = rng.standard_normal((n, n))
    k = np.fft.fftfreq(n) * 2 * np.pi
    lf = (np.abs(k)[:, None] <= np.pi / 2) & (np.abs(k)[None, :] <= np.pi / 2)
    win = np.zeros((n, n), bool)
    win[n // 4: 3 * n // 4, n // 4: 3 * n // 4] = True
    r = 0.0
    for it in range(sweeps):
        E = np.fft.fft2(e)
        E[lf] = 0.0
        e = np.real(np.fft.ifft2(E))
        e /= np.linalg.norm(e[win])
        o.set("phi", e)
        o.sweep(s, 0)
        e2 = o.get("phi")
        E2 = np.fft.fft2(e2)
        E2[lf] = 0.0
        r = np.linalg.norm(np.real(np.fft.ifft2(E2))[win])
        e = e2
    return r


def test_lfa_hybrid2_rate_matches_the_oracles_own_sweep():
    """At a jump pixel (Table 2's first rows: one coupling much smaller than the
    rest) Hybrid Smoother 2's sweep along the smallest coupling's lines lags only
    that coupling; the oracle's own sweep (lexicographic line order, every cell
    starred, each line one superpixel) reduces high-frequency error at the rate
    the single-harmonic LFA of "lag only the smallest" gives."""
    coef_sets = [(0.05, 1.0, 1.0, 1.0), (1.0, 1.0, 0.08, 1.0), (0.3, 1.0, 0.8, 0.9)]
    for coef in coef_sets:
        s = int(np.argmin(coef))
        want = lfa.rate_hybrid2(np.array(coef))
        got = _measured_sweep_rate(coef, s)
        assert abs(got - want) <= 0.015, (coef, got, want)


# ------------------------------------------------- Hybrid Smoother 1 (Sec. 4.2, Algorithm 2)
from oracle import box_dense  # noqa: E402


def _arrow(rng, k):
    """A random arrow matrix (centre coupled to k - 1 leaves, leaves to the centre
    only) with a negative, strictly dominant diagonal, as eqs. caseAlagged-caseDlagged."""
    M = np.zeros((k, k))
    for a in range(1, k):
        M[0, a] = rng.uniform(0.1, 1.0)
        M[a, 0] = rng.uniform(0.1, 1.0)
    for a in range(k):
        M[a, a] = -(np.abs(M[a]).sum() + rng.uniform(0.05, 1.0))
    return M


def test_box_dense_unconstrained_matches_linalg():
    rng = np.random.default_rng(5)
    for _ in range(50):
        k = int(rng.integers(2, 5))
        M, b = _arrow(rng, k), rng.normal(0, 2, k)
        x = box_dense(M, b, np.full(k, -1e9), np.full(k, 1e9))
        assert np.abs(x - np.linalg.solve(M, b)).max() <= 1e-12 * (1 + np.abs(x).max())


def test_box_dense_matches_projected_gauss_seidel():
    """Against brute force: projected Gauss-Seidel iterated to a fixed point (the
    unique solution of the box-constrained M-matrix problem)."""
    rng = np.random.default_rng(6)
    for _ in range(200):
        k = int(rng.integers(2, 5))
        M, b = _arrow(rng, k), rng.normal(0, 3, k)
        lo, hi = rng.uniform(-2, 0, k), rng.uniform(0, 2, k)
        x = box_dense(M, b, lo, hi)
        y = np.zeros(k)
        for _ in range(5000):
            for a in range(k):
                v = (b[a] - M[a] @ y + M[a, a] * y[a]) / M[a, a]
                y[a] = min(hi[a], max(lo[a], v))
        assert np.abs(x - y).max() <= 1e-10


def test_eight_class_order_keeps_blocks_apart():
    """Two jump pixels of one class (i + 3 j) mod 8 are at least four cells apart
    (L1), so their blocks (the pixel and its neighbours) share no pixel and neither
    reads a pixel the other writes (a block reads up to two cells from its centre)."""
    for di in range(-4, 5):
        for dj in range(-4, 5):
            if (di, dj) != (0, 0) and (di + 3 * dj) % 8 == 0:
                assert abs(di) + abs(dj) >= 4


def test_hybrid1_fixed_point_is_projected_solution():
    """Iterated on one grid, Hybrid Smoother 1 (GSLINE-I on every column, then the
    blocks at the jump pixels) stops at a point where the projected residual of
    the discrete equations vanishes."""
    inst = synth.tiny_instance(8, 20, 24)
    o = Oracle(inst.image, inst.markers, OracleParams(levels=1, smoother=2))
    o.smooth(400, 0)
    r = o.residual(0, True)
    assert np.abs(r).max() <= 1e-9


@pytest.mark.parametrize("seed", [1000, 1001, 1002])
def test_hybrid1_paper_order_and_parallel_order_agree(seed):
    """Algorithm 2 with the paper's order and with the parallel order (four column
    classes, eight block classes) reach 1e-6 and the same segmentation."""
    inst = synth.config1(seed)
    out = []
    for order in (0, 1):
        o = Oracle(inst.image, inst.markers, OracleParams(levels=6, smoother=2, order=order))
        k, hist = o.solve(1e-6, 40)
        assert k > 0
        out.append(o.get("phi") > 0)
    assert np.array_equal(out[0], out[1])
