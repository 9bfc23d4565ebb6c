"""Local Fourier analysis of the frozen-coefficient smoothers (Sec. 3.3, Sec. 4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

With the coefficients A, B, C, D (couplings to i+1, i-1, j+1, j-1) frozen at a
pixel and S = A + B + C + D, a smoother that takes the couplings in ``new``
at the updated iterate and the others at the old one has the error equation
    sum_{new} c e^{(k+1)}_nb + sum_{old} c e^{(k)}_nb - S e^{(k+1)} = 0,
so a Fourier mode exp(i(a1 i + a2 j)) is amplified by
    mu(a1, a2) = |sum_{old} c E_c| / |S - sum_{new} c E_c|,
with E_A = e^{i a1}, E_B = e^{-i a1}, E_C = e^{i a2}, E_D = e^{-i a2}.
The smoothing rate is the maximum over the high frequencies (Sec. 3.3).
GSLEX (point lexicographic): new = {B, D} (the formula after eq. errorform);
GSLINE (column lines, eq. gslinelfa): new = {A, B, D};
Hybrid-2 sweep lagging s (Sec. 4.3): new = every coupling except s.

For the parallel sweep, whose lines are taken in four classes (line index mod
4), rate_lines4 gives the 4-harmonic LFA, and measured_rate measures any of
these smoothers directly (power iteration of one sweep on a periodic
frozen-coefficient grid with the low frequencies removed), which pins the
analysis to the smoother it describes.

The frequencies are sampled on the discrete grid theta in {-n/2 .. n/2},
alpha = 2 pi theta / n (Sec. 3.3) with n = 128, and the high-frequency set is
max(|a1|, |a2|) > pi/2 (strict): this sampling reproduces the printed rates
of Table 2.
"""
from __future__ import annotations

import numpy as np

COUPLINGS = "ABCD"


def freq_grid(n: int = 128, strict: bool = True):
    th = np.arange(-(n // 2), n // 2 + 1)
    a = 2.0 * np.pi * th / n
    a1, a2 = np.meshgrid(a, a, indexing="ij")
    amax = np.maximum(np.abs(a1), np.abs(a2))
    hf = amax > np.pi / 2 if strict else amax >= np.pi / 2
    return a1, a2, hf


def symbol(coef, new, a1, a2, q=0.0):
    """Amplification of each Fourier mode for frozen ``coef`` = (A, B, C, D);
    q: a term added to the diagonal (NEWT's derivative of the area term)."""
    A, B, C, D = (float(c) for c in coef)
    S = A + B + C + D + float(q)
    E = {"A": np.exp(1j * a1), "B": np.exp(-1j * a1), "C": np.exp(1j * a2), "D": np.exp(-1j * a2)}
    cf = {"A": A, "B": B, "C": C, "D": D}
    num = sum(cf[k] * E[k] for k in COUPLINGS if k not in new)
    den = S - sum(cf[k] * E[k] for k in COUPLINGS if k in new)
    num = np.abs(num) if not np.isscalar(num) else abs(num) * np.ones_like(a1)
    den = np.abs(den) * np.ones_like(a1)
    # a mode with no coupling at all (both sums empty: a pixel without faces) is not amplified
    out = np.zeros_like(num)
    np.divide(num, den, out=out, where=den > 0)
    return np.where((den == 0) & (num > 0), np.inf, out)


def rate(coef, new, n: int = 128, strict: bool = True, q: float = 0.0) -> float:
    """Smoothing rate mu-hat: maximum of the symbol over high frequencies."""
    a1, a2, hf = freq_grid(n, strict)
    return float(symbol(coef, set(new), a1, a2, q)[hf].max())


def rate_gslex(coef, n=128, strict=True):
    return rate(coef, {"B", "D"}, n, strict)


def rate_gsline(coef, n=128, strict=True):
    return rate(coef, {"A", "B", "D"}, n, strict)


def rate_lag(coef, lagged, n=128):
    """Rate of the adapted scheme that lags the couplings in ``lagged``."""
    return rate(coef, set(COUPLINGS) - set(lagged), n)


def rate_hybrid2(coef, n=128):
    """Hybrid Smoother 2 at a jump pixel: one of its four sweeps lags only the
    smallest coupling (Sec. 4.2, "lag only the smallest"); that sweep's rate."""
    s = COUPLINGS[int(np.argmin(coef))]
    return rate_lag(coef, s, n)


def iterations_for(mu: float, reduction: float = 0.1) -> int:
    """Sweeps needed to reduce high-frequency error by ``reduction`` (Sec. 4.1)."""
    return int(np.ceil(np.log(reduction) / np.log(mu)))


# --------------------------------------------------------------------------
# Line orderings, with the lines along j (rows) and the cross-line index i.
# In a sweep every line is relaxed once: point Gauss-Seidel along the line
# (the in-line predecessor D new, the successor C old) or the whole line at
# once (C and D both new); the cross-line neighbours A (i+1) and B (i-1) enter
# at their current values.  Lines are taken either lexicographically
# (i = 0, 1, ...) or in the four classes i mod 4 (all lines of a class, then
# the next class), the order of the parallel sweep.  A column sweep is the
# same with (A, B, C, D) -> (C, D, A, B).

def _line_gain(coef, in_new, beta, a2):
    """Amplification g of one harmonic on a line being relaxed, its cross-line
    neighbours held at the harmonic's current values."""
    A, B, C, D = (float(c) for c in coef)
    S = A + B + C + D
    Ec, Ed = np.exp(1j * a2), np.exp(-1j * a2)
    num = A * np.exp(1j * beta) + B * np.exp(-1j * beta)
    den = S + 0j
    if "C" in in_new:
        den = den - C * Ec
    else:
        num = num + C * Ec
    if "D" in in_new:
        den = den - D * Ed
    else:
        num = num + D * Ed
    return num / den


def _hf(a1, a2):
    w = lambda a: (a + np.pi) % (2 * np.pi) - np.pi
    return np.maximum(np.abs(w(a1)), np.abs(w(a2))) > np.pi / 2


def rate_lines4(coef, in_new=("D",), classes=(0, 1, 2, 3), n: int = 64) -> float:
    """Smoothing rate of the 4-class line sweep by 4-harmonic LFA.

    The cross-line frequencies beta_m = a1 + 2 pi m / 4 (m = 0..3) are coupled
    by the class pattern: relaxing the lines of class c multiplies harmonic m
    by g_m on those lines only, and the indicator of the class,
    (1/4) sum_k w^{k (i - c)} with w = e^{2 pi i / 4}, moves it to the
    harmonics m + k; so the partial step is P_c = I + (1/4) W_c diag(g - 1),
    W_c[p, m] = w^{-(p - m) c}, and the sweep is the product of the P_c in
    class order.  The rate is the largest spectral radius of the sweep with
    the low-frequency harmonics projected out, over the n x n frequency grid
    (a1 in one quarter of the circle, a2 on the whole circle)."""
    w = np.exp(2j * np.pi / 4)
    idx = np.arange(4)
    best = 0.0
    th1 = np.arange(-(n // 8), n // 8) * 2 * np.pi / n
    th2 = np.arange(-(n // 2), n // 2) * 2 * np.pi / n
    for a1 in th1:
        beta = a1 + 2 * np.pi * idx / 4
        for a2 in th2:
            g = _line_gain(coef, in_new, beta, a2)
            Sm = np.eye(4, dtype=complex)
            for c in classes:
                Wc = w ** (-((idx[:, None] - idx[None, :]) * c))
                Sm = (np.eye(4) + 0.25 * Wc * (g - 1.0)[None, :]) @ Sm
            q = _hf(beta, np.full(4, a2)).astype(float)
            if not q.any():
                continue
            rho = np.abs(np.linalg.eigvals(q[:, None] * Sm)).max()
            best = max(best, float(rho))
    return best


def _sweep_periodic(e, coef, in_new, line_order):
    """One sweep of the frozen-coefficient smoother on the periodic grid e
    (zero right-hand side), lines (rows) in ``line_order``."""
    A, B, C, D = (float(c) for c in coef)
    S = A + B + C + D
    n, m = e.shape
    for i in line_order:
        up, dn = e[(i + 1) % n], e[(i - 1) % n]
        rhs = A * up + B * dn
        if "C" in in_new and "D" in in_new:
            # the periodic line at once: S x_j - C x_{j+1} - D x_{j-1} = rhs_j (circulant solve)
            lam = S - C * np.exp(2j * np.pi * np.arange(m) / m) - D * np.exp(-2j * np.pi * np.arange(m) / m)
            e[i] = np.real(np.fft.ifft(np.fft.fft(rhs) / lam))
        else:
            row = e[i]
            for j in range(m):
                row[j] = (rhs[j] + C * row[(j + 1) % m] + D * row[j - 1]) / S
    return e


def measured_rate(coef, in_new=("D",), order="classes", n: int = 64, sweeps: int = 60, seed: int = 0) -> float:
    """Worst high-frequency reduction per sweep of the smoother itself, by
    power iteration: a random error, one sweep, the low frequencies removed
    (FFT), renormalised; the rate is the geometric mean of the last third of
    the per-sweep norm ratios.  order: "lex" (rows 0..n-1) or "classes"
    (rows of class 0, 1, 2, 3)."""
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((n, n))
    k = np.fft.fftfreq(n) * 2 * np.pi
    lf = (np.abs(k)[:, None] <= np.pi / 2) & (np.abs(k)[None, :] <= np.pi / 2)
    proj = lambda x: np.real(np.fft.ifft2(np.where(lf, 0.0, np.fft.fft2(x))))
    lines = list(range(n)) if order == "lex" else [i for c in range(4) for i in range(c, n, 4)]
    e = proj(e)
    e /= np.linalg.norm(e)
    ratios = []
    for _ in range(sweeps):
        e = proj(_sweep_periodic(e, coef, set(in_new), lines))
        r = np.linalg.norm(e)
        ratios.append(r)
        e /= r
    tail = np.array(ratios[-(sweeps // 3):])
    return float(np.exp(np.log(tail).mean()))
