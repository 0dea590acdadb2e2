"""Growing-mode clock and smoothing-radius ladder (oracle side; test infrastructure only).

Section "Collapse times": the linear growing mode D, normalised to 1 at z = 0, is the time
coordinate in which collapse is computed, F = 1/D at collapse; and the smoothing radii are
chosen so that the mass variances sigma^2(R) of the smoothed field are logarithmically spaced by
0.15 dex.  Section "Simulations": the runs use a flat LambdaCDM cosmology (Omega_m = 0.25).

Readings (the paper gives neither formula):

* D is the growing mode of a flat LambdaCDM universe without radiation,
      D(a) = (5 Omega_m / 2) E(a) Int_0^a da' / (a' E(a'))^3,   E(a) = sqrt(Omega_m a^-3 + 1 - Omega_m),
  normalised to D(1) = 1 (EdS, Omega_m = 1: D = a).  The collapse redshift of a point with
  inverse collapse time F solves D(z_c) = 1/F; D grows monotonically to a finite limit
  D_inf = D(a -> inf), so F = 0 or 1/F >= D_inf means no collapse, reported as z_c = -1.
* sigma^2(R) = 1/(2 pi^2) Int k^2 P(k) exp(-k^2 R^2) dk, the variance of the field smoothed with
  the Gaussian window of ``hessian`` (W^2 = exp(-k^2 R^2)), from the continuous spectrum of
  ``spectrum`` with the same sigma_8 normalisation.  From the largest radius R_0 the ladder takes
  R_{i+1} < R_i with sigma^2(R_{i+1}) = 10^0.15 sigma^2(R_i) while R_{i+1} >= R_min.
"""

import numpy as np
from scipy import integrate, optimize

from . import spectrum


def _e(a, om):
    return np.sqrt(om / a ** 3 + (1.0 - om))


def _integral(a, om):
    """Int_0^a dx/(x E(x))^3 = Int_0^a x^(3/2) (om + (1-om) x^3)^(-3/2) dx, split at x = 1: beyond
    it x = 1/u gives Int_{1/a}^1 u (om u^3 + 1 - om)^(-3/2) du, integrated in ln u."""
    ol = 1.0 - om
    lo, _ = integrate.quad(lambda x: x ** 1.5 * (om + ol * x ** 3) ** -1.5, 0.0, min(a, 1.0),
                           epsabs=0.0, epsrel=2e-14, limit=400)
    if a <= 1.0:
        return lo
    # in s = ln u the integrand u^2 (om u^3 + 1 - om)^(-3/2) is smooth for any omega_m
    f = lambda s: np.exp(2 * s) * (om * np.exp(3 * s) + ol) ** -1.5
    if not np.isfinite(a):
        hi, _ = integrate.quad(f, -np.inf, 0.0, epsabs=0.0, epsrel=2e-14, limit=400)
        return lo + hi
    # unit panels in ln u: the integrand varies by at most a factor e^2.5 across each
    edges = np.append(np.arange(-np.log(a), 0.0, 1.0), 0.0)
    hi = sum(integrate.quad(f, e0, e1, epsabs=0.0, epsrel=2e-14, limit=200)[0] for e0, e1 in zip(edges[:-1], edges[1:]))
    return lo + hi


def growth_unnormalised(a, om):
    """(5 Om/2) E(a) Int_0^a da'/(a' E(a'))^3 (-> a as a -> 0)."""
    return 2.5 * om * _e(a, om) * _integral(a, om)


def growth(a, om):
    """D(a) normalised to D(1) = 1."""
    return growth_unnormalised(a, om) / growth_unnormalised(1.0, om)


def growth_limit(om):
    """D(a -> inf) = (5 Om/2) sqrt(1 - Om) Int_0^inf da/(a E(a))^3 / D_unnorm(1)."""
    return 2.5 * om * np.sqrt(1.0 - om) * _integral(np.inf, om) / growth_unnormalised(1.0, om)


def collapse_redshift(F, om):
    """z_c with D(z_c) = 1/F for each F (array); -1 where there is no collapse."""
    F = np.asarray(F, dtype=np.float64)
    out = np.full(F.shape, -1.0)
    dinf = np.inf if om >= 1.0 else growth_limit(om)
    for i, f in np.ndenumerate(F):
        if not f > 0.0:
            continue
        target = 1.0 / f
        if target >= dinf:
            continue
        if om >= 1.0:
            out[i] = f - 1.0
            continue
        # bracket a in ln a: D increases monotonically from 0
        hi = 1.0
        while growth(hi, om) < target:
            hi *= 2.0
        lo = min(target, 1.0) * 1e-3
        ln_a = optimize.brentq(lambda x: growth(np.exp(x), om) - target, np.log(lo), np.log(hi), xtol=1e-15, rtol=1e-15)
        out[i] = np.exp(-ln_a) - 1.0
    return out


def sigma2_gaussian(radius, gamma, ns, amplitude):
    """sigma^2(R) = 1/(2 pi^2) Int k^2 P(k) exp(-k^2 R^2) dk (R in Mpc/h), quad in ln k."""

    def integrand(lnk):
        k = np.exp(lnk)
        return k ** 3 * spectrum.power(k, amplitude, gamma, ns) * np.exp(-(k * radius) ** 2)

    kmax = 40.0 / radius
    edges = np.linspace(np.log(1e-7), np.log(kmax), 60)
    total = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        val, _ = integrate.quad(integrand, a, b, epsabs=0.0, epsrel=1e-13, limit=400)
        total += val
    return total / (2.0 * np.pi ** 2)


def radius_ladder(n, box, r_max_cells, r_min_cells, dex=0.15, sigma8=0.8, gamma=0.21, ns=1.0):
    """Radii in cells, largest first, with sigma^2 spaced by `dex` decades."""
    amp = spectrum.amplitude_for_sigma8(sigma8, gamma, ns)
    cell = box / n
    radii = [float(r_max_cells)]
    s2 = sigma2_gaussian(r_max_cells * cell, gamma, ns, amp)
    while True:
        target = s2 * 10.0 ** dex
        r_prev = radii[-1]
        f = lambda lr: np.log(sigma2_gaussian(np.exp(lr) * cell, gamma, ns, amp)) - np.log(target)
        lo = np.log(r_prev)
        hi = lo
        while f(hi) < 0.0:
            hi -= 0.5
            if np.exp(hi) < 1e-3 * r_min_cells:
                return radii
        r_new = float(np.exp(optimize.brentq(f, hi, lo, xtol=1e-14, rtol=1e-15)))
        if r_new < r_min_cells:
            return radii
        radii.append(r_new)
        s2 = target
