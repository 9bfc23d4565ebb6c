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


def symbol(coef, new, a1, a2):
    """Amplification of each Fourier mode for frozen ``coef`` = (A, B, C, D)."""
    A, B, C, D = (float(c) for c in coef)
    S = A + B + C + D
    E = {"A": np.exp(1j * a1), "B": np.exp(-1j * a1), "C": np.exp(1j * a2), "D": np.exp(-1j * a2)}
    cf = {"A": A, "B": B, "C": C, "D": D}
    num = sum(cf[k] * E[k] for k in COUPLINGS if k not in new)
    den = S - sum(cf[k] * E[k] for k in COUPLINGS if k in new)
    num = np.abs(num) if not np.isscalar(num) else abs(num) * np.ones_like(a1)
    return num / np.abs(den)


def rate(coef, new, n: int = 128, strict: bool = True) -> float:
    """Smoothing rate mu-hat: maximum of the symbol over high frequencies."""
    a1, a2, hf = freq_grid(n, strict)
    return float(symbol(coef, set(new), a1, a2)[hf].max())


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
