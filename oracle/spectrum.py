"""Linear power spectrum and its sigma_8 normalisation (oracle side; test infrastructure only).

Section "Collapse times": the power spectrum of the linear field delta_l comes from the
cosmological model, and <delta_l^2> = sigma_8^2 when the field is top-hat smoothed on 8 Mpc/h.

The paper's runs use the MICE cosmology with an external initial-conditions generator, neither of
which is available; the workloads here use the BBKS transfer function (Bardeen, Bond, Kaiser &
Szalay 1986) with shape parameter Gamma, a primordial slope n and sigma_8 at z = 0:

    P(k) = A k^n T(k/Gamma)^2,
    T(q) = ln(1 + 2.34 q)/(2.34 q) * [1 + 3.89 q + (16.1 q)^2 + (5.46 q)^3 + (6.71 q)^4]^(-1/4),
    sigma^2(R) = 1/(2 pi^2) * Int k^2 P(k) W_TH(k R)^2 dk,   W_TH(x) = 3 (sin x - x cos x)/x^3,

with k in h/Mpc and A fixed by sigma^2(8) = sigma_8^2.  The integral is done with
scipy.integrate.quad in ln k.
"""

import numpy as np
from scipy import integrate


def bbks_transfer(k, gamma):
    """BBKS transfer function T(k/Gamma), k in h/Mpc; T -> 1 as k -> 0."""
    k = np.asarray(k, dtype=np.float64)
    q = k / gamma
    x = 2.34 * q
    # ln(1+x)/x with its k -> 0 limit
    with np.errstate(divide="ignore", invalid="ignore"):
        lead = np.where(x > 1e-8, np.log1p(x) / np.where(x > 0, x, 1.0), 1.0 - 0.5 * x)
    poly = 1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4
    return lead * poly ** -0.25


def tophat_window(x):
    """Fourier transform of a unit-volume top-hat: 3 (sin x - x cos x)/x^3 (series for small x)."""
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 1e-3
    xs = np.where(small, 1.0, x)
    full = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
    series = 1.0 - x * x / 10.0 + x ** 4 / 280.0
    return np.where(small, series, full)


def unnormalised_power(k, gamma, ns):
    """k^n T(k/Gamma)^2 (A = 1)."""
    k = np.asarray(k, dtype=np.float64)
    return k ** ns * bbks_transfer(k, gamma) ** 2


def sigma2_tophat(radius, gamma, ns, amplitude=1.0):
    """sigma^2(R) = 1/(2 pi^2) Int k^2 P(k) W_TH(kR)^2 dk, integrated in ln k with quad."""

    def integrand(lnk):
        k = np.exp(lnk)
        return k ** 3 * amplitude * unnormalised_power(k, gamma, ns) * tophat_window(k * radius) ** 2

    # The integrand is negligible outside [1e-7, 1e3] h/Mpc for R = O(1..100) Mpc/h.  The range is
    # split into eighth-decades so quad resolves the window's oscillations, and a first coarse pass
    # sets the absolute tolerance of the second.
    edges = np.log(np.logspace(-7, 3, 81))
    scale = sum(integrate.quad(integrand, a, b, limit=200)[0] for a, b in zip(edges[:-1], edges[1:]))
    total = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        val, _ = integrate.quad(integrand, a, b, epsabs=1e-15 * scale, epsrel=1e-13, limit=400)
        total += val
    return total / (2.0 * np.pi ** 2)


def sigma2_tophat_many(radii, gamma, ns, amplitude=1.0, intervals=1 << 18):
    """sigma^2(R) for many radii at once: the same integral by composite Simpson in ln k over
    [1e-7, 1e3] h/Mpc with `intervals` panels (the window's oscillations are resolved wherever the
    integrand is not negligible)."""
    lnk = np.linspace(np.log(1e-7), np.log(1e3), intervals + 1)
    h = lnk[1] - lnk[0]
    w = np.full(intervals + 1, 2.0)
    w[1::2] = 4.0
    w[0] = w[-1] = 1.0
    k = np.exp(lnk)
    base = k ** 3 * amplitude * unnormalised_power(k, gamma, ns) * w * (h / 3.0)
    return np.array([float(np.sum(base * tophat_window(k * r) ** 2)) for r in np.atleast_1d(radii)]) / (2.0 * np.pi ** 2)


def amplitude_for_sigma8(sigma8, gamma, ns):
    """A such that sigma^2(8 Mpc/h) = sigma_8^2."""
    return sigma8 ** 2 / sigma2_tophat(8.0, gamma, ns, 1.0)


def power(k, amplitude, gamma, ns):
    """P(k) = A k^n T(k/Gamma)^2 in (Mpc/h)^3, k in h/Mpc; P(0) = 0 for n > 0."""
    return amplitude * unnormalised_power(k, gamma, ns)
